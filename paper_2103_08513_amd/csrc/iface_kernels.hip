// Interface system and reconstruction of the MRCM (Algorithm 2, "Assembly",
// "InterfaceSolver" and loop 2) on gfx950.
//
// The interface matrix is kept as a band in column-major LAPACK layout:
// entry (i, j), |i - j| <= w, lives at AB[j*ld + (w + i - j)], ld = 2w + 1.
// Unknowns are interleaved per patch after a bandwidth-reducing ordering:
// patch p at position pos[p] owns unknowns 2*pos[p] (pi^p) and 2*pos[p]+1 (pi^u).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "launch.h"

namespace mrcm {

__global__ void k_fill(double *__restrict__ a, long long n, double v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) a[i] = v;
}

__global__ void k_copy(const double *__restrict__ a, double *__restrict__ b, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Scatter of the per-subdomain flux blocks into A^int and b^int (one
// workgroup per subdomain, one thread per (row patch, column patch) pair).
// An entry receives one contribution per subdomain that contains both of its
// patches -- at most two -- so the FP64 atomic sums are order independent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_iface_scatter(Geom g, const int *__restrict__ patches,
                                                       const int *__restrict__ pos,
                                                       const double *__restrict__ F,
                                                       const double *__restrict__ Fb,
                                                       const double *__restrict__ SAb,
                                                       double *__restrict__ AB, int w,
                                                       double *__restrict__ bint) {
  const SubDesc S = g.sub[blockIdx.x];
  const int n = S.npatch, m = S.m;
  const int ld = 2 * w + 1;
  const double *Fs = F + S.F_off;
  const double *Fbs = Fb + S.F_off;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int li = e / n, lj = e % n;
    int fi = 0;
    for (int ff = 0; ff < 6; ++ff) {
      if (S.face_if[ff] < 0) continue;
      const IfaceDesc I = g.ifc[S.face_if[ff]];
      if (li >= S.face_p0[ff] && li < S.face_p0[ff] + I.na * I.nb) fi = ff;
    }
    const double sig = (fi & 1) ? 1.0 : -1.0;
    const long long rP = 2LL * pos[patches[S.patch_off + li]], rU = rP + 1;
    const long long cP = 2LL * pos[patches[S.patch_off + lj]], cU = cP + 1;
    const double *fr = Fs + (size_t)li * m;
    const double *br = Fbs + (size_t)li * m;
    double uu = sig * br[1 + n + lj];
    if (li == lj) uu -= SAb[S.patch_off + li];
    atomicAdd(&AB[cP * ld + (w + rP - cP)], fr[1 + lj]);
    atomicAdd(&AB[cU * ld + (w + rP - cU)], fr[1 + n + lj]);
    atomicAdd(&AB[cP * ld + (w + rU - cP)], sig * br[1 + lj]);
    atomicAdd(&AB[cU * ld + (w + rU - cU)], uu);
    if (lj == 0) {
      atomicAdd(&bint[rP], -fr[0]);
      atomicAdd(&bint[rU], -sig * br[0]);
    }
  }
}

// ---------------------------------------------------------------------------
// Band LU without pivoting, right-looking, blocks of kLU columns.
// Step k0 = panel kernel (every workgroup factors the kLU x kLU diagonal block
// in wave 0's registers; workgroup 0 stores it to `diag` and applies L11^{-1}
// to the right-hand side, the others compute a chunk of L21 = A21 U11^{-1} or
// U12 = L11^{-1} A12) followed by the update kernel A22 -= L21 U12 (MFMA
// FP64), which also copies the factored diagonal block into the band and
// updates the right-hand side, b2 -= L21 y1.
// ---------------------------------------------------------------------------
constexpr int kLU = 32;

__device__ __forceinline__ void lu_diag_block(const double *AB, int ld, int w, int k0, int kb,
                                              double *D /* [kLU][kLU+1] */, DevStatus *st) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int lane = tid;
    double row[kLU];
#pragma unroll
    for (int c = 0; c < kLU; ++c)
      row[c] = (lane < kb && c < kb && abs(lane - c) <= w) ? AB[(size_t)(k0 + c) * ld + (w + lane - c)]
                                                            : 0.0;
#pragma unroll
    for (int p = 0; p < kLU; ++p) {
      if (p < kb) {
        double piv = lane_bcast(row[p], p);
        if (piv == 0.0 || !isfinite(piv)) {
          if (lane == 0) set_status(st, -5, k0 + p, piv);
          piv = 1.0;
        }
        const double l = row[p] / piv;
        if (lane > p) row[p] = l;
#pragma unroll
        for (int c = p + 1; c < kLU; ++c) {
          const double upc = lane_bcast(row[c], p);
          if (lane > p) row[c] -= l * upc;
        }
      }
    }
    if (lane < kLU) {
#pragma unroll
      for (int c = 0; c < kLU; ++c) D[lane * (kLU + 1) + c] = row[c];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_lu_panel(double *__restrict__ AB, int n, int w, int k0,
                                                  double *__restrict__ diag,
                                                  double *__restrict__ bint, DevStatus *st) {
  __shared__ double D[kLU * (kLU + 1)];
  const int ld = 2 * w + 1;
  const int kb = min(kLU, n - k0);
  const int r0 = k0 + kb;
  const int nr = max(0, min(n, k0 + kb + w) - r0);  // rows of L21 / columns of U12
  const int nchunk = (nr + 255) / 256;
  lu_diag_block(AB, ld, w, k0, kb, D, st);
  const int tid = threadIdx.x;
  const int role = blockIdx.x;
  if (role == 0) {
    for (int e = tid; e < kb * kb; e += blockDim.x) {
      const int r = e / kb, c = e % kb;
      diag[r * kLU + c] = D[r * (kLU + 1) + c];
    }
    if (tid == 0) {
      // y1 = L11^{-1} b1 (unit lower)
      for (int r = 0; r < kb; ++r) {
        double s = bint[k0 + r];
        for (int p = 0; p < r; ++p) s -= D[r * (kLU + 1) + p] * bint[k0 + p];
        bint[k0 + r] = s;
      }
    }
    return;
  }
  if (role <= nchunk) {
    // L21 rows: l U11 = a, for row i = r0 + chunk*256 + tid
    const int i = r0 + (role - 1) * 256 + tid;
    if (i >= r0 + nr) return;
    double l[kLU];
#pragma unroll
    for (int c = 0; c < kLU; ++c) {
      const int j = k0 + c;
      l[c] = (c < kb && i - j <= w) ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kLU; ++c) {
      if (c < kb) {
        double s = l[c];
#pragma unroll
        for (int p = 0; p < c; ++p) s -= l[p] * D[p * (kLU + 1) + c];
        l[c] = s / D[c * (kLU + 1) + c];
      }
    }
#pragma unroll
    for (int c = 0; c < kLU; ++c) {
      const int j = k0 + c;
      if (c < kb && i - j <= w) AB[(size_t)j * ld + (w + i - j)] = l[c];
    }
    return;
  }
  {
    // U12 columns: L11 u = a (unit lower), for column j = r0 + chunk*256 + tid
    const int j = r0 + (role - 1 - nchunk) * 256 + tid;
    if (j >= r0 + nr) return;
    double u[kLU];
#pragma unroll
    for (int r = 0; r < kLU; ++r) {
      const int i = k0 + r;
      u[r] = (r < kb && j - i <= w) ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kLU; ++r) {
      if (r < kb) {
        double s = u[r];
#pragma unroll
        for (int p = 0; p < r; ++p) s -= D[r * (kLU + 1) + p] * u[p];
        u[r] = s;
      }
    }
#pragma unroll
    for (int r = 0; r < kLU; ++r) {
      const int i = k0 + r;
      if (r < kb && j - i <= w) AB[(size_t)j * ld + (w + i - j)] = u[r];
    }
  }
}

// A22 -= L21 U12 in 64x64 tiles (four waves, each 16 rows x 64 columns).
// Extra workgroups: one copies the factored diagonal block, the last ones
// update the right-hand side.
__global__ __launch_bounds__(256) void k_lu_update(double *__restrict__ AB, int n, int w, int k0,
                                                   const double *__restrict__ diag,
                                                   double *__restrict__ bint) {
  using M = Mma<double>;
  __shared__ double Ls[64 * (kLU + 1)];
  __shared__ double Us[kLU * (64 + 1)];
  const int ld = 2 * w + 1;
  const int kb = min(kLU, n - k0);
  const int r0 = k0 + kb;
  const int nr = max(0, min(n, k0 + kb + w) - r0);
  const int nt = (nr + 63) / 64;
  const int tid = threadIdx.x;
  const int bid = blockIdx.x;
  if (bid == nt * nt) {
    for (int e = tid; e < kb * kb; e += blockDim.x) {
      const int r = e / kb, c = e % kb;
      if (abs(r - c) <= w) AB[(size_t)(k0 + c) * ld + (w + r - c)] = diag[r * kLU + c];
    }
    return;
  }
  if (bid > nt * nt) {
    // b2 -= L21 y1 for rows r0 + chunk*256 + tid
    const int i = r0 + (bid - nt * nt - 1) * 256 + tid;
    if (i >= r0 + nr) return;
    double s = 0.0;
    for (int c = 0; c < kb; ++c) {
      const int j = k0 + c;
      if (i - j <= w) s += AB[(size_t)j * ld + (w + i - j)] * bint[j];
    }
    bint[i] -= s;
    return;
  }
  const int ti = bid / nt, tj = bid % nt;
  const int i0 = r0 + ti * 64, j0 = r0 + tj * 64;
  // stage L21 tile (64 x kb) and U12 tile (kb x 64)
  for (int e = tid; e < 64 * kLU; e += 256) {
    const int r = e % 64, c = e / 64;
    const int i = i0 + r, j = k0 + c;
    Ls[r * (kLU + 1) + c] = (c < kb && i < r0 + nr && i - j <= w) ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
  }
  for (int e = tid; e < 64 * kLU; e += 256) {
    const int r = e % kLU, c = e / kLU;
    const int i = k0 + r, j = j0 + c;
    Us[r * 65 + c] = (r < kb && j < r0 + nr && j - i <= w) ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
    typename M::v4 c;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wave * 16 + M::crow(v, lane), j = j0 + tc * 16 + lr;
      const bool ok = i < r0 + nr && j < r0 + nr && (i - j <= w) && (j - i <= w);
      c[v] = ok ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < kLU / 4; ++s) {
      const int kk = 4 * s + lk;
      const double a = Ls[(wave * 16 + lr) * (kLU + 1) + kk];
      const double b = Us[kk * 65 + tc * 16 + lr];
      c = M::mma(-a, b, c);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wave * 16 + M::crow(v, lane), j = j0 + tc * 16 + lr;
      const bool ok = i < r0 + nr && j < r0 + nr && (i - j <= w) && (j - i <= w);
      if (ok) AB[(size_t)j * ld + (w + i - j)] = c[v];
    }
  }
}

// Triangular sweeps with the band factors, one workgroup of 1024 lanes.
// lower: L y = b (unit lower), forward.  upper: U x = y, backward.  In place.
__global__ __launch_bounds__(1024) void k_lu_sweep(const double *__restrict__ AB, int n, int w,
                                                   double *__restrict__ x, int upper) {
  __shared__ double xb[kLU];
  const int ld = 2 * w + 1;
  const int tid = threadIdx.x;
  const int nblk = (n + kLU - 1) / kLU;
  for (int s = 0; s < nblk; ++s) {
    const int blk = upper ? (nblk - 1 - s) : s;
    const int k0 = blk * kLU;
    const int kb = min(kLU, n - k0);
    if (tid < 64) {
      const int lane = tid;
      double xv = (lane < kb) ? x[k0 + lane] : 0.0;
      if (upper) {
        for (int c = kb - 1; c >= 0; --c) {
          const double dc = AB[(size_t)(k0 + c) * ld + w];
          double xc = lane_bcast(xv, c) / dc;
          if (lane == c) xv = xc;
          if (lane < c && c - lane <= w) xv -= AB[(size_t)(k0 + c) * ld + (w + lane - c)] * xc;
        }
      } else {
        for (int c = 0; c < kb; ++c) {
          const double xc = lane_bcast(xv, c);
          if (lane > c && lane < kb && lane - c <= w) xv -= AB[(size_t)(k0 + c) * ld + (w + lane - c)] * xc;
        }
      }
      if (lane < kb) {
        xb[lane] = xv;
        x[k0 + lane] = xv;
      }
    }
    __syncthreads();
    // propagate the block to the rows it couples to
    if (upper) {
      const int ilo = max(0, k0 - w);
      for (int i = ilo + tid; i < k0; i += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < kb; ++c) {
          const int j = k0 + c;
          if (j - i <= w) acc += AB[(size_t)j * ld + (w + i - j)] * xb[c];
        }
        x[i] -= acc;
      }
    } else {
      const int ihi = min(n, k0 + kb + w);
      for (int i = k0 + kb + tid; i < ihi; i += blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < kb; ++c) {
          const int j = k0 + c;
          if (i - j <= w) acc += AB[(size_t)j * ld + (w + i - j)] * xb[c];
        }
        x[i] -= acc;
      }
    }
    __syncthreads();
  }
}

// r = b - A x with the unfactored band (one thread per row).
__global__ void k_band_residual(const double *__restrict__ AB, int n, int w,
                                const double *__restrict__ x, const double *__restrict__ b,
                                double *__restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ld = 2 * w + 1;
  double acc = 0.0;
  const int jlo = max(0, i - w), jhi = min(n - 1, i + w);
  for (int j = jlo; j <= jhi; ++j) acc += AB[(size_t)j * ld + (w + i - j)] * x[j];
  r[i] = b[i] - acc;
}

// Permutation between the natural order (pi^p then pi^u) and the band order.
__global__ void k_perm_to_natural(const double *__restrict__ y, const int *__restrict__ pos, int nv,
                                  double *__restrict__ X) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nv) return;
  X[p] = y[2 * pos[p]];
  X[nv + p] = y[2 * pos[p] + 1];
}
__global__ void k_perm_to_band(const double *__restrict__ X, const int *__restrict__ pos, int nv,
                               double *__restrict__ y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nv) return;
  y[2 * pos[p]] = X[p];
  y[2 * pos[p] + 1] = X[nv + p];
}

// Sum of squares of a vector into out[slot] (one workgroup).
__global__ __launch_bounds__(256) void k_norm2(const double *__restrict__ v, int n,
                                               double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i] * v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// ---------------------------------------------------------------------------
// Reconstruction, eq. (2.23): p^l = X_l [1, pi^p_{I^l}, pi^u_{I^l}].
// One workgroup per subdomain; the combination weights go to LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_recon_p(Geom g, const int *__restrict__ patches,
                                                 const double *__restrict__ Xg,
                                                 const double *__restrict__ pi, int nv,
                                                 double *__restrict__ p) {
  __shared__ double cw[kMaxRhs];
  const SubDesc S = g.sub[blockIdx.x];
  const int m = S.m, n = S.npatch;
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    double v = 1.0;
    if (c >= 1 && c <= n) v = pi[patches[S.patch_off + c - 1]];
    else if (c > n) v = pi[nv + patches[S.patch_off + c - 1 - n]];
    cw[c] = v;
  }
  __syncthreads();
  const double *X = Xg + S.X_off;
  for (int r = threadIdx.x; r < S.N; r += blockDim.x) {
    const double *row = X + (size_t)r * m;
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += row[c] * cw[c];
    int x[3];
    local_to_global(S, r, x);
    p[cell_index(g, x)] = s;
  }
}

// Per-cell outward normal velocities on the six faces, own side (one thread
// per cell): eq. (2.12) inside a subdomain, the Robin rule on Gamma with
// G_f = pi^p_i - sigma beta_f pi^u_i, the wall rules on the walls.
__global__ void k_recon_u(Geom g, const double *__restrict__ p, const double *__restrict__ pi,
                          int nv, double *__restrict__ U) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int x[3];
  x[0] = (int)(c % g.nx);
  x[1] = (int)((c / g.nx) % g.ny);
  x[2] = (int)(c / ((long long)g.nx * g.ny));
  const int s[3] = {g.sub_of[0][x[0]], g.sub_of[1][x[1]], g.sub_of[2][x[2]]};
  const int l = s[0] + g.nd[0] * (s[1] + g.nd[1] * s[2]);
  const SubDesc S = g.sub[l];
  const int n[3] = {g.nx, g.ny, g.nz};
  const double pc = p[c];
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const double kd = g.k[d][c];
    const int xn = x[d] + side;
    double u = 0.0;
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) {
      int y[3] = {x[0], x[1], x[2]};
      y[d] = xn;
      const long long cn = cell_index(g, y);
      const double kn = g.k[d][cn];
      u = (2.0 * kd * kn / (kd + kn)) * (pc - p[cn]) / g.h[d];
    } else if (xn >= 0 && xn < n[d]) {
      int lp;
      double T, beta;
      gamma_face(g, S, x, f, kd, lp, T, beta);
      const int patch = g.ifc[S.face_if[f]].p0 + (lp - S.face_p0[f]);
      const double G = pi[patch] - side * beta * pi[nv + patch];
      u = T * (pc - G) / g.area[d];
    } else {
      const int wt = g.wall_type[f];
      if (wt != 0) {
        const int a = (d == 0) ? 1 : 0;
        const int b = (d == 2) ? 1 : 2;
        const double gv = g.wall_value[f] ? g.wall_value[f][x[a] + (long long)n[a] * x[b]] : 0.0;
        u = (wt == 1) ? 2.0 * kd / g.h[d] * (pc - gv) : gv;
      }
    }
    U[(long long)f * N + c] = u;
  }
}

}  // namespace mrcm

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace mrcm {

static unsigned grid_for(long long n, int bs = 256) {
  long long b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

hipError_t launch_fill(double *a, long long n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, a, n, v);
  return hipGetLastError();
}

hipError_t launch_copy(const double *a, double *b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_iface_scatter(const Geom &g, int n_sub, const int *patches, const int *pos,
                                const double *F, const double *Fb, const double *SAb, double *AB,
                                int w, double *b, hipStream_t s) {
  hipLaunchKernelGGL(k_iface_scatter, dim3(n_sub), dim3(256), 0, s, g, patches, pos, F, Fb, SAb, AB,
                     w, b);
  return hipGetLastError();
}

hipError_t launch_band_lu(double *AB, int n, int w, double *diag, double *b, DevStatus *st,
                          hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += kLU) {
    const int kb = (n - k0 < kLU) ? n - k0 : kLU;
    const int nr = std::max(0, std::min(n, k0 + kb + w) - (k0 + kb));
    const int nchunk = (nr + 255) / 256;
    hipLaunchKernelGGL(k_lu_panel, dim3(1 + 2 * nchunk), dim3(256), 0, s, AB, n, w, k0, diag, b, st);
    const int nt = (nr + 63) / 64;
    hipLaunchKernelGGL(k_lu_update, dim3(nt * nt + 1 + nchunk), dim3(256), 0, s, AB, n, w, k0, diag,
                       b);
  }
  return hipGetLastError();
}

hipError_t launch_lu_sweep(const double *AB, int n, int w, double *x, int upper, hipStream_t s) {
  hipLaunchKernelGGL(k_lu_sweep, dim3(1), dim3(1024), 0, s, AB, n, w, x, upper);
  return hipGetLastError();
}

hipError_t launch_band_residual(const double *AB, int n, int w, const double *x, const double *b,
                                double *r, hipStream_t s) {
  hipLaunchKernelGGL(k_band_residual, dim3(grid_for(n)), dim3(256), 0, s, AB, n, w, x, b, r);
  return hipGetLastError();
}

hipError_t launch_perm(const double *src, const int *pos, int nv, double *dst, int to_natural,
                       hipStream_t s) {
  if (to_natural)
    hipLaunchKernelGGL(k_perm_to_natural, dim3(grid_for(nv)), dim3(256), 0, s, src, pos, nv, dst);
  else
    hipLaunchKernelGGL(k_perm_to_band, dim3(grid_for(nv)), dim3(256), 0, s, src, pos, nv, dst);
  return hipGetLastError();
}

hipError_t launch_norm2(const double *v, int n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

hipError_t launch_axpy(double *y, const double *x, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}

hipError_t launch_recon_p(const Geom &g, int n_sub, const int *patches, const double *X,
                          const double *pi, int nv, double *p, hipStream_t s) {
  hipLaunchKernelGGL(k_recon_p, dim3(n_sub), dim3(256), 0, s, g, patches, X, pi, nv, p);
  return hipGetLastError();
}

hipError_t launch_recon_u(const Geom &g, const double *p, const double *pi, int nv, double *U,
                          hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_recon_u, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, p, pi, nv, U);
  return hipGetLastError();
}

}  // namespace mrcm
