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
  const SubDesc &S = g.sub[blockIdx.x];
  const int n = S.npatch, m = S.m;
  const int ld = 2 * w + 1;
  const double *Fs = F + S.F_off;
  const double *Fbs = Fb + S.F_off;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int li = e / n, lj = e % n;
    int fi = 0;
    for (int ff = 0; ff < 6; ++ff) {
      const int ii = S.face_if[ff];
      if (ii < 0) continue;
      const IfaceDesc &I = g.ifc[ii];
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

// Unrolled LU of the kLU x kLU diagonal block held one row per lane
// (rows beyond kb and entries outside the band are zero).  Step P: the pivot
// row P is broadcast from lane P and every lower row eliminates column P.
template <int P>
__device__ __forceinline__ void lu_rows_step(double (&row)[kLU], int lane, int kb, int k0,
                                             DevStatus *st) {
  if (P < kb) {
    double piv = lane_bcast(row[P], P);
    if (piv == 0.0 || !isfinite(piv)) {
      if (lane == 0) set_status(st, -5, k0 + P, piv);
      piv = 1.0;
    }
    const double l = row[P] / piv;
    if (lane > P) row[P] = l;
#pragma unroll
    for (int c = P + 1; c < kLU; ++c) {
      const double u = lane_bcast(row[c], P);
      if (lane > P) row[c] -= l * u;
    }
  }
  if constexpr (P + 1 < kLU) lu_rows_step<P + 1>(row, lane, kb, k0, st);
}

// l U11 = a for one row l (U11 upper, from LDS D).
template <int C>
__device__ __forceinline__ void trsm_row_upper(double (&l)[kLU], const double *D, int kb) {
  if (C < kb) {
    double s = l[C];
#pragma unroll
    for (int p = 0; p < C; ++p) s -= l[p] * D[p * (kLU + 1) + C];
    l[C] = s / D[C * (kLU + 1) + C];
  }
  if constexpr (C + 1 < kLU) trsm_row_upper<C + 1>(l, D, kb);
}

// L11 u = a for one column u (L11 unit lower, from LDS D).
template <int R>
__device__ __forceinline__ void trsm_col_lower(double (&u)[kLU], const double *D, int kb) {
  if (R < kb) {
    double s = u[R];
#pragma unroll
    for (int p = 0; p < R; ++p) s -= D[R * (kLU + 1) + p] * u[p];
    u[R] = s;
  }
  if constexpr (R + 1 < kLU) trsm_col_lower<R + 1>(u, D, kb);
}

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
    lu_rows_step<0>(row, lane, kb, k0, st);
    if (lane < kLU) {
#pragma unroll
      for (int c = 0; c < kLU; ++c) D[lane * (kLU + 1) + c] = row[c];
    }
  }
  __syncthreads();
}

// One unit of the panel step at column k0 (role 0: diagonal block and
// right-hand side; roles 1..nchunk: 256 rows of L21; the rest: 256 columns of
// U12).  Every unit factors the diagonal block itself, from the unmodified
// band, so units need no ordering among themselves.
__device__ void lu_panel_unit(double *__restrict__ AB, int n, int w, int k0, int role,
                              double *__restrict__ diag, double *__restrict__ bint, DevStatus *st,
                              double *D) {
  const int ld = 2 * w + 1;
  const int kb = min(kLU, n - k0);
  const int r0 = k0 + kb;
  const int nr = max(0, min(n, k0 + kb + w) - r0);  // rows of L21 / columns of U12
  const int nchunk = (nr + 255) / 256;
  const int tid = threadIdx.x;
  // Each workgroup loads its row / column of the panel before factoring the
  // diagonal block, so the loads overlap the factorisation.
  double v[kLU];
  int idx = -1;
  if (role >= 1 && role <= nchunk) {
    const int i = r0 + (role - 1) * 256 + tid;
    if (i < r0 + nr) idx = i;
#pragma unroll
    for (int c = 0; c < kLU; ++c) {
      const int j = k0 + c;
      v[c] = (idx >= 0 && c < kb && idx - j <= w) ? AB[(size_t)j * ld + (w + idx - j)] : 0.0;
    }
  } else if (role > nchunk) {
    const int j = r0 + (role - 1 - nchunk) * 256 + tid;
    if (j < r0 + nr) idx = j;
#pragma unroll
    for (int r = 0; r < kLU; ++r) {
      const int i = k0 + r;
      v[r] = (idx >= 0 && r < kb && idx - i <= w) ? AB[(size_t)idx * ld + (w + i - idx)] : 0.0;
    }
  }
  lu_diag_block(AB, ld, w, k0, kb, D, st);
  if (role == 0) {
    for (int e = tid; e < kb * kb; e += blockDim.x) {
      const int r = e / kb, c = e % kb;
      diag[r * kLU + c] = D[r * (kLU + 1) + c];
    }
    if (tid == 0) {
      // y1 = L11^{-1} b1 (unit lower)
      for (int r = 0; r < kb; ++r) {
        double sum = bint[k0 + r];
        for (int p = 0; p < r; ++p) sum -= D[r * (kLU + 1) + p] * bint[k0 + p];
        bint[k0 + r] = sum;
      }
    }
    return;
  }
  if (idx < 0) return;
  if (role <= nchunk) {
    trsm_row_upper<0>(v, D, kb);
#pragma unroll
    for (int c = 0; c < kLU; ++c) {
      const int j = k0 + c;
      if (c < kb && idx - j <= w) AB[(size_t)j * ld + (w + idx - j)] = v[c];
    }
  } else {
    trsm_col_lower<0>(v, D, kb);
#pragma unroll
    for (int r = 0; r < kLU; ++r) {
      const int i = k0 + r;
      if (r < kb && idx - i <= w) AB[(size_t)idx * ld + (w + i - idx)] = v[r];
    }
  }
}

__global__ __launch_bounds__(256) void k_lu_panel(double *__restrict__ AB, int n, int w, int k0,
                                                  double *__restrict__ diag,
                                                  double *__restrict__ bint, DevStatus *st) {
  __shared__ double D[kLU * (kLU + 1)];
  lu_panel_unit(AB, n, w, k0, blockIdx.x, diag, bint, st, D);
}

// A22 -= L21 U12 in 64x64 tiles (four waves, each 16 rows x 64 columns).
// Extra workgroups: one copies the factored diagonal block, the last ones
// update the right-hand side.
// One unit of the update step at column k0: units 0..nt*nt-1 are 64x64 tiles
// of A22 -= L21 U12; unit nt*nt copies the factored diagonal block into the
// band; the last units update the right-hand side, b2 -= L21 y1.
__device__ void lu_update_unit(double *__restrict__ AB, int n, int w, int k0, int bid,
                               const double *__restrict__ diag, double *__restrict__ bint,
                               double *Ls, double *Us) {
  using M = Mma<double>;
  const int ld = 2 * w + 1;
  const int kb = min(kLU, n - k0);
  const int r0 = k0 + kb;
  const int nr = max(0, min(n, k0 + kb + w) - r0);
  const int nt = (nr + 63) / 64;
  const int tid = threadIdx.x;
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
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // the C tile is fetched first so its latency overlaps the staging below
  typename M::v4 cacc[4];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wave * 16 + M::crow(v, lane), j = j0 + tc * 16 + lr;
      const bool ok = i < r0 + nr && j < r0 + nr && (i - j <= w) && (j - i <= w);
      cacc[tc][v] = ok ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
    }
  }
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
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
    typename M::v4 c = cacc[tc];
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

__global__ __launch_bounds__(256) void k_lu_update(double *__restrict__ AB, int n, int w, int k0,
                                                   const double *__restrict__ diag,
                                                   double *__restrict__ bint) {
  __shared__ double Ls[64 * (kLU + 1)];
  __shared__ double Us[kLU * (64 + 1)];
  lu_update_unit(AB, n, w, k0, blockIdx.x, diag, bint, Ls, Us);
}

// Triangular sweeps with the band factors, one workgroup of 1024 lanes.
// lower: L y = b (unit lower), forward.  upper: U x = y, backward.  In place.
// Per block of kSW unknowns, wave 0 solves the diagonal block (one row per
// lane, broadcasts between lanes) while the other waves apply the block to
// the rows it couples to (one row per lane; beyond 960 rows a slower loop).
// The active part of x lives in an LDS ring of RW >= w + 2 kSW entries; the
// band entries of the next block and the x entries that enter the ring next
// are fetched one block ahead, so no global access sits on the critical path.
constexpr int kSW = 16;

template <int C>
__device__ __forceinline__ void sweep_upper_step(const double (&u)[kSW], double &xv, int lane, int kb) {
  constexpr int c = kSW - 1 - C;
  if (c < kb) {
    const double dc = lane_bcast(u[c], c);
    const double xc = lane_bcast(xv, c) / dc;
    if (lane == c) xv = xc;
    if (lane < c) xv -= u[c] * xc;
  }
  if constexpr (C + 1 < kSW) sweep_upper_step<C + 1>(u, xv, lane, kb);
}

template <int C>
__device__ __forceinline__ void sweep_lower_step(const double (&u)[kSW], double &xv, int lane, int kb) {
  if (C < kb) {
    const double xc = lane_bcast(xv, C);
    if (lane > C) xv -= u[C] * xc;
  }
  if constexpr (C + 1 < kSW) sweep_lower_step<C + 1>(u, xv, lane, kb);
}

constexpr int kSweepThreads = 1024;

__global__ __launch_bounds__(kSweepThreads) void k_lu_sweep(const double *__restrict__ AB, int n,
                                                            int w, double *__restrict__ x, int upper,
                                                            int RW) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *xr = reinterpret_cast<double *>(smem_raw);  // ring, entry i at i % RW
  __shared__ double xb[kSW];
  const int ld = 2 * w + 1;
  const int tid = threadIdx.x;
  const int nblk = (n + kSW - 1) / kSW;
  const int nprop = kSweepThreads - 64;
  double cur[kSW], nxt[kSW];
  double xin_cur = 0.0, xin_nxt = 0.0;  // entering x value (threads 64..64+kSW-1)
  // rows the block at k0 updates: [lo, hi)
  auto prop_lo = [&](int k0, int kb) { return upper ? max(0, k0 - w) : k0 + kb; };
  auto prop_hi = [&](int k0, int kb) { return upper ? k0 : min(n, k0 + kb + w); };
  auto fetch = [&](int blk, double (&dst)[kSW]) {
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    if (tid < 64) {
#pragma unroll
      for (int c = 0; c < kSW; ++c)
        dst[c] = (tid < kb && c < kb && abs(tid - c) <= w) ? AB[(size_t)(k0 + c) * ld + (w + tid - c)] : 0.0;
    } else {
      const int i = prop_lo(k0, kb) + (tid - 64);
      const bool ok = i < prop_hi(k0, kb);
#pragma unroll
      for (int c = 0; c < kSW; ++c) {
        const int j = k0 + c;
        const bool in = ok && c < kb && (upper ? (j - i <= w) : (i - j <= w));
        dst[c] = in ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
      }
    }
  };
  // x entries that enter the ring when block blk becomes current: for the
  // upper sweep the rows [lo(blk), lo(blk+1)), for the lower sweep the rows
  // [hi(blk-1), hi(blk)) -- at most kSW of them.
  auto enter_range = [&](int blk, int &a, int &b) {
    const int k0 = blk * kSW, kb = min(kSW, n - k0);
    if (upper) {
      a = prop_lo(k0, kb);
      const int k1 = (blk + 1) * kSW;
      b = (blk + 1 < nblk) ? prop_lo(k1, min(kSW, n - k1)) : a;
    } else {
      const int kp = (blk - 1) * kSW;
      a = (blk > 0) ? prop_hi(kp, kSW) : b;
      b = prop_hi(k0, kb);
      if (blk == 0) a = b;
    }
  };
  auto fetch_x = [&](int blk) {
    int a, b;
    enter_range(blk, a, b);
    const int i = a + (tid - 64);
    return (tid >= 64 && tid < 64 + kSW && i < b) ? x[i] : 0.0;
  };
  auto store_x = [&](int blk, double v) {
    int a, b;
    enter_range(blk, a, b);
    const int i = a + (tid - 64);
    if (tid >= 64 && tid < 64 + kSW && i < b) xr[i % RW] = v;
  };
  // initial ring: the first block's own rows and the rows it updates
  {
    const int blk = upper ? nblk - 1 : 0;
    const int k0 = blk * kSW, kb = min(kSW, n - k0);
    const int a = upper ? prop_lo(k0, kb) : k0;
    const int b = upper ? n : prop_hi(k0, kb);
    for (int i = a + tid; i < b; i += kSweepThreads) xr[i % RW] = x[i];
  }
  fetch(upper ? nblk - 1 : 0, cur);
  if (nblk > 1) xin_nxt = fetch_x(upper ? nblk - 2 : 1);
  __syncthreads();
  auto body = [&](int s, double (&cu)[kSW], double (&nx)[kSW]) {
    const int blk = upper ? (nblk - 1 - s) : s;
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    const int nb = upper ? blk - 1 : blk + 1;
    xin_cur = xin_nxt;
    if (s + 1 < nblk) fetch(nb, nx);
    if (s + 2 < nblk) xin_nxt = fetch_x(upper ? blk - 2 : blk + 2);
    if (tid < 64) {
      const int lane = tid;
      double xv = (lane < kb) ? xr[(k0 + lane) % RW] : 0.0;
      if (upper) sweep_upper_step<0>(cu, xv, lane, kb);
      else sweep_lower_step<0>(cu, xv, lane, kb);
      if (lane < kb) {
        xb[lane] = xv;
        x[k0 + lane] = xv;
      }
    }
    __syncthreads();
    if (tid >= 64) {
      const int ilo = prop_lo(k0, kb), ihi = prop_hi(k0, kb);
      const int i0 = ilo + (tid - 64);
      if (i0 < ihi) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kSW; ++c) acc += cu[c] * xb[c];
        xr[i0 % RW] -= acc;
      }
      for (int i = i0 + nprop; i < ihi; i += nprop) {
        double acc = 0.0;
        for (int c = 0; c < kb; ++c) {
          const int j = k0 + c;
          if (upper ? (j - i <= w) : (i - j <= w)) acc += AB[(size_t)j * ld + (w + i - j)] * xb[c];
        }
        xr[i % RW] -= acc;
      }
      // rows that the next block needs and no earlier block touched
      if (s + 1 < nblk) store_x(nb, xin_cur);
    }
    __syncthreads();
  };
  for (int s = 0; s < nblk; s += 2) {
    body(s, cur, nxt);
    if (s + 1 < nblk) body(s + 1, nxt, cur);
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
  const SubDesc &S = g.sub[blockIdx.x];
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
    p[cell_index(g, local_to_global(S, r))] = s;
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
  I3 x;
  x.v0 = (int)(c % g.nx);
  x.v1 = (int)((c / g.nx) % g.ny);
  x.v2 = (int)(c / ((long long)g.nx * g.ny));
  const int l = g.sub_of[0][x.v0] + g.nd[0] * (g.sub_of[1][x.v1] + g.nd[1] * g.sub_of[2][x.v2]);
  const SubDesc &S = g.sub[l];
  const double pc = p[c];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const double *karr = kdir(g, d);
    const double kd = karr[c];
    const double hd = hdir(g, d);
    const int xn = x[d] + side;
    double u = 0.0;
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) {
      I3 y = x;
      y.set(d, xn);
      const long long cn = cell_index(g, y);
      const double kn = karr[cn];
      u = (2.0 * kd * kn / (kd + kn)) * (pc - p[cn]) / hd;
    } else if (xn >= 0 && xn < ndir(g, d)) {
      int lp;
      double T, beta;
      gamma_face(g, S, x, f, kd, lp, T, beta);
      const int patch = g.ifc[S.face_if[f]].p0 + (lp - S.face_p0[f]);
      const double G = pi[patch] - side * beta * pi[nv + patch];
      u = T * (pc - G) / adir(g, d);
    } else {
      const int wt = wall_type_of(g, f);
      if (wt != 0) {
        const int a = (d == 0) ? 1 : 0;
        const int b = (d == 2) ? 1 : 2;
        const double *wv = wall_value_of(g, f);
        const double gv = wv ? wv[x[a] + (long long)ndir(g, a) * x[b]] : 0.0;
        u = (wt == 1) ? 2.0 * kd / hd * (pc - gv) : gv;
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
    const int kb = std::min(kLU, n - k0);
    const int nr = std::max(0, std::min(n, k0 + kb + w) - (k0 + kb));
    const int nchunk = (nr + 255) / 256;
    const int nt = (nr + 63) / 64;
    hipLaunchKernelGGL(k_lu_panel, dim3(1 + 2 * nchunk), dim3(256), 0, s, AB, n, w, k0, diag, b, st);
    hipLaunchKernelGGL(k_lu_update, dim3(nt * nt + 1 + nchunk), dim3(256), 0, s, AB, n, w, k0, diag,
                       b);
  }
  return hipGetLastError();
}

hipError_t launch_lu_sweep(const double *AB, int n, int w, double *x, int upper, hipStream_t s) {
  const int RW = w + 2 * kSW + 1;
  const size_t lds = (size_t)RW * sizeof(double);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)k_lu_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lu_sweep, dim3(1), dim3(kSweepThreads), lds, s, AB, n, w, x, upper, RW);
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
