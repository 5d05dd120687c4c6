// Device helpers shared by the gfx950 kernels: MFMA wrappers, lane
// broadcasts, subdomain indexing and the Robin-face rule.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mrcm {

// ---------------------------------------------------------------------------
// MFMA 16x16x4 wrappers.  Operand layout (both precisions): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator item v of lane l is
// D[row(v, l)][l % 16]; the row map differs between the FP64 and FP32
// instructions.
// ---------------------------------------------------------------------------
template <typename T> struct Mma;

template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int v, int lane) { return 4 * v + (lane >> 4); }
};

template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int v, int lane) { return 4 * (lane >> 4) + v; }
};

// Value of a VGPR in a given lane (lane index must be wave-uniform).
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  long long x = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ void set_status(DevStatus *st, int code, int where, double value) {
  if (atomicCAS(&st->code, 0, code) == 0) {
    st->where = where;
    st->value = value;
  }
}

// ---------------------------------------------------------------------------
// Subdomain indexing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void local_to_global(const SubDesc &S, int r, int x[3]) {
  const int t0 = r % S.n0;
  const int rr = r / S.n0;
  const int t1 = rr % S.n1;
  const int t2 = rr / S.n1;
  x[S.ax[0]] = S.lo[S.ax[0]] + t0;
  x[S.ax[1]] = S.lo[S.ax[1]] + t1;
  x[S.ax[2]] = S.lo[S.ax[2]] + t2;
}

__device__ __forceinline__ int local_row(const SubDesc &S, const int x[3]) {
  const int t0 = x[S.ax[0]] - S.lo[S.ax[0]];
  const int t1 = x[S.ax[1]] - S.lo[S.ax[1]];
  const int t2 = x[S.ax[2]] - S.lo[S.ax[2]];
  return t0 + S.n0 * (t1 + S.n1 * t2);
}

__device__ __forceinline__ long long cell_index(const Geom &g, const int x[3]) {
  return (long long)x[0] + (long long)g.nx * ((long long)x[1] + (long long)g.ny * x[2]);
}

// Robin face rule.  Face f (-x..+z) of the cell at global coordinates x in
// subdomain S lies on Gamma when the neighbour across it is outside the box
// but inside the domain.  Then: local patch lp, Robin parameter
// beta = alpha H_d / K_d(c), transmissibility T = A_d / (h_d / (2 K_d) + beta)
// and sigma = +1 on a + face (lower side of the interface), -1 on a - face.
__device__ __forceinline__ bool gamma_face(const Geom &g, const SubDesc &S, const int x[3], int f,
                                           double kd, int &lp, double &T, double &beta) {
  const int d = f >> 1;
  const int side = (f & 1) ? 1 : -1;
  const int xn = x[d] + side;
  if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) return false;
  const int ifc = S.face_if[f];
  if (ifc < 0) return false;
  const IfaceDesc I = g.ifc[ifc];
  const int ta = x[I.a] - S.lo[I.a];
  const int tb = x[I.b] - S.lo[I.b];
  lp = S.face_p0[f] + split_group(ta, I.la, I.na) + I.na * split_group(tb, I.lb, I.nb);
  const double H = S.ext[d] * g.h[d];
  beta = g.alpha * H / kd;
  T = g.area[d] / (g.h[d] / (2.0 * kd) + beta);
  return true;
}

}  // namespace mrcm
