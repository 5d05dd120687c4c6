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

// Value of lane n of each row of 16 lanes, for every lane of that row (DPP
// row_newbcast: a VGPR-to-VGPR move, no scalar registers involved; FP64 moves
// in one instruction).  n must fold to a constant after unrolling.
template <int n, typename T> __device__ __forceinline__ T row_bcast_c(T x) {
  return __builtin_amdgcn_mov_dpp(x, 0x150 + n, 0xf, 0xf, true);
}
template <typename T> __device__ __forceinline__ T row_bcast(T x, int n) {
  switch (n) {
    case 0: return row_bcast_c<0>(x);
    case 1: return row_bcast_c<1>(x);
    case 2: return row_bcast_c<2>(x);
    case 3: return row_bcast_c<3>(x);
    case 4: return row_bcast_c<4>(x);
    case 5: return row_bcast_c<5>(x);
    case 6: return row_bcast_c<6>(x);
    case 7: return row_bcast_c<7>(x);
    case 8: return row_bcast_c<8>(x);
    case 9: return row_bcast_c<9>(x);
    case 10: return row_bcast_c<10>(x);
    case 11: return row_bcast_c<11>(x);
    case 12: return row_bcast_c<12>(x);
    case 13: return row_bcast_c<13>(x);
    case 14: return row_bcast_c<14>(x);
    default: return row_bcast_c<15>(x);
  }
}

__device__ __forceinline__ void set_status(DevStatus *st, int code, int where, double value) {
  if (atomicCAS(&st->code, 0, code) == 0) {
    st->where = where;
    st->value = value;
  }
}

// ---------------------------------------------------------------------------
// Per-axis accessors.  Kernel arguments and small private arrays indexed with
// a run-time axis would be spilled to scratch; selects keep them in registers.
// ---------------------------------------------------------------------------
struct I3 {
  int v0, v1, v2;
  __device__ __forceinline__ int operator[](int d) const { return d == 0 ? v0 : (d == 1 ? v1 : v2); }
  __device__ __forceinline__ void set(int d, int x) {
    v0 = (d == 0) ? x : v0;
    v1 = (d == 1) ? x : v1;
    v2 = (d == 2) ? x : v2;
  }
};

__device__ __forceinline__ const double *kdir(const Geom &g, int d) {
  return d == 0 ? g.k[0] : (d == 1 ? g.k[1] : g.k[2]);
}
__device__ __forceinline__ double hdir(const Geom &g, int d) {
  return d == 0 ? g.h[0] : (d == 1 ? g.h[1] : g.h[2]);
}
__device__ __forceinline__ double adir(const Geom &g, int d) {
  return d == 0 ? g.area[0] : (d == 1 ? g.area[1] : g.area[2]);
}
__device__ __forceinline__ int ndir(const Geom &g, int d) {
  return d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
}
__device__ __forceinline__ int wall_type_of(const Geom &g, int f) {
  int w = g.wall_type[0];
  w = (f == 1) ? g.wall_type[1] : w;
  w = (f == 2) ? g.wall_type[2] : w;
  w = (f == 3) ? g.wall_type[3] : w;
  w = (f == 4) ? g.wall_type[4] : w;
  w = (f == 5) ? g.wall_type[5] : w;
  return w;
}
__device__ __forceinline__ const double *wall_value_of(const Geom &g, int f) {
  const double *w = g.wall_value[0];
  w = (f == 1) ? g.wall_value[1] : w;
  w = (f == 2) ? g.wall_value[2] : w;
  w = (f == 3) ? g.wall_value[3] : w;
  w = (f == 4) ? g.wall_value[4] : w;
  w = (f == 5) ? g.wall_value[5] : w;
  return w;
}
__device__ __forceinline__ const int *subof_dir(const Geom &g, int d) {
  return d == 0 ? g.sub_of[0] : (d == 1 ? g.sub_of[1] : g.sub_of[2]);
}

// ---------------------------------------------------------------------------
// Subdomain indexing (descriptors are read through references to global
// memory, never copied into private arrays).
// ---------------------------------------------------------------------------
__device__ __forceinline__ I3 local_to_global(const SubDesc &S, int r) {
  const int t0 = r % S.n0;
  const int rr = r / S.n0;
  const int t1 = rr % S.n1;
  const int t2 = rr / S.n1;
  const int a0 = S.ax[0], a1 = S.ax[1], a2 = S.ax[2];
  I3 x{0, 0, 0};
  x.set(a0, S.lo[a0] + t0);
  x.set(a1, S.lo[a1] + t1);
  x.set(a2, S.lo[a2] + t2);
  return x;
}

__device__ __forceinline__ int local_row(const SubDesc &S, const I3 &x) {
  const int a0 = S.ax[0], a1 = S.ax[1], a2 = S.ax[2];
  const int t0 = x[a0] - S.lo[a0];
  const int t1 = x[a1] - S.lo[a1];
  const int t2 = x[a2] - S.lo[a2];
  return t0 + S.n0 * (t1 + S.n1 * t2);
}

__device__ __forceinline__ long long cell_index(const Geom &g, const I3 &x) {
  return (long long)x.v0 + (long long)g.nx * ((long long)x.v1 + (long long)g.ny * x.v2);
}

// Robin parameter, eq. (3.1), of face f (on Gamma) of the cell at global
// coordinates x in subdomain S, whose permeability along the normal is kd:
// beta_mode 0, per side, beta = alpha H_d / K_d(c) with H_d the subdomain's
// extent along the normal; beta_mode 1, one value per face shared by both
// sides, with the harmonic means of the two sides' H_d and of the two cells'
// K_d across the face.
__device__ __forceinline__ double robin_beta(const Geom &g, const SubDesc &S, const I3 &x, int f, double kd) {
  const int d = f >> 1;
  const double hd = hdir(g, d);
  double H = S.ext[d] * hd, Kb = kd;
  if (g.beta_mode) {
    I3 y = x;
    y.set(d, x[d] + ((f & 1) ? 1 : -1));
    const double kn = kdir(g, d)[cell_index(g, y)];
    const IfaceDesc &I = g.ifc[S.face_if[f]];
    const double Ho = g.sub[(f & 1) ? I.hi_sub : I.lo_sub].ext[d] * hd;
    H = 2.0 * H * Ho / (H + Ho);
    Kb = 2.0 * kd * kn / (kd + kn);
  }
  return g.alpha * H / Kb;
}

// Robin face rule.  Face f (-x..+z) of the cell at global coordinates x in
// subdomain S lies on Gamma when the neighbour across it is outside the box
// but inside the domain.  Then: local patch lp, Robin parameter beta
// (robin_beta), transmissibility T = A_d / (h_d / (2 K_d(c)) + beta)
// and sigma = +1 on a + face (lower side of the interface), -1 on a - face.
__device__ __forceinline__ bool gamma_face(const Geom &g, const SubDesc &S, const I3 &x, int f,
                                           double kd, int &lp, double &T, double &beta) {
  const int d = f >> 1;
  const int side = (f & 1) ? 1 : -1;
  const int xn = x[d] + side;
  const int lo = S.lo[d], ext = S.ext[d];
  if (xn >= lo && xn < lo + ext) return false;
  const int ifc = S.face_if[f];
  if (ifc < 0) return false;
  const IfaceDesc &I = g.ifc[ifc];
  const int ta = x[I.a] - S.lo[I.a];
  const int tb = x[I.b] - S.lo[I.b];
  lp = S.face_p0[f] + split_group(ta, I.la, I.na) + I.na * split_group(tb, I.lb, I.nb);
  const double hd = hdir(g, d);
  beta = robin_beta(g, S, x, f, kd);
  T = adir(g, d) / (hd / (2.0 * kd) + beta);
  return true;
}

}  // namespace mrcm
