// Internal layout shared by the host runtime and the gfx950 kernels.
// Not part of the public ABI.
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace mrcm {

// Panel width of the local band Cholesky and of the band solves.
constexpr int kNB = 16;
// Largest local bandwidth the factor kernels accept, per precision: the LDS
// window of the factor holds (b + kNB) columns of 16*ceil(b/16) + 17 entries.
constexpr int kMaxBand64 = 112;
constexpr int kMaxBand32 = 176;
// Largest number of right-hand sides of one subdomain (2|I^l| + 1).
constexpr int kMaxRhs = 128;

// One subdomain.  Local row r = t0 + n0*(t1 + n1*t2) where t_k is the cell
// coordinate along global axis ax[k] measured from lo[ax[k]].
struct SubDesc {
  int32_t lo[3];
  int32_t ext[3];
  int32_t ax[3];
  int32_t n0, n1, n2;
  int32_t N;        // cells
  int32_t b;        // lower bandwidth n0*n1
  int32_t m;        // right-hand-side columns 2*npatch + 1
  int32_t npatch;   // |I^l|
  int32_t face_if[6];   // interface id on faces -x..+z, or -1 for a wall
  int32_t face_p0[6];   // position in I^l of the face's first patch
  int32_t patch_off;    // offset of I^l in the concatenated patch lists
  int32_t col_off;      // offset of the subdomain's columns in per-column arrays
  int32_t pin_local;    // local row of the pinned cell or -1
  int64_t cell_off;     // offset of the subdomain's rows in per-row arrays
  int64_t L_off;        // offset (elements) of the band factor, N*(b+1)
  int64_t D_off;        // offset (elements) of the inverted 16x16 diagonal blocks, ceil(N/16)*256
  int64_t X_off;        // offset (elements) of X, N*m
  int64_t F_off;        // offset (elements) of F / Fb, npatch*m
};

// Grid and fluids of the two-phase saturation step.
struct TwoPhaseGrid {
  int32_t nx, ny, nz;
  double hx, hy, hz;
  double mu_w, mu_o;
};

// One interface between subdomains lo_sub < hi_sub along axis d; tangential
// axes a < b with extents la, lb split into na x nb patches; first patch p0.
struct IfaceDesc {
  int32_t d, lo_sub, hi_sub, a, b, la, lb, na, nb, p0;
};

// Device view of the problem geometry and data used by every kernel.
struct Geom {
  int32_t nx, ny, nz;
  double h[3];
  double area[3];       // face areas V/h_d
  double alpha;
  int32_t beta_mode;    // 0 per side, 1 one value per face shared by both sides
  int32_t wall_type[6];
  const double *wall_value[6];
  const double *k[3];   // kx, ky, kz
  const double *q;
  int64_t pin;
  const SubDesc *sub;
  const IfaceDesc *ifc;
  const int32_t *sub_of[3];   // per axis: coordinate -> subdomain coordinate
  int32_t nd[3];
};

// Status codes kernels write (values of mrcm_status).
constexpr int kStatusSingular = -5;  // MRCM_ESINGULAR: zero pivot in the interface factorisation

// Status word written by kernels (first error wins).
struct DevStatus {
  int32_t code;     // 0 ok, else an mrcm_status value
  int32_t where;    // subdomain or row
  double value;     // pivot value or residual
};

// Balanced split of n cells into k groups, larger groups first: group of cell t.
__host__ __device__ inline int split_group(int t, int n, int k) {
  int q = n / k, r = n % k;
  int big = r * (q + 1);
  return t < big ? t / (q + 1) : r + (t - big) / q;
}
// First cell of group g.
__host__ __device__ inline int split_start(int g, int n, int k) {
  int q = n / k, r = n % k;
  return g < r ? g * (q + 1) : r * (q + 1) + (g - r) * q;
}

}  // namespace mrcm
