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
#include "ldl16.h"

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
// Band LDL^T of the interface system.  With s = -1 on the pressure rows (even
// unknowns) and +1 on the velocity rows, M = diag(s) A^int is symmetric:
// A^UP = -(A^PU)^T, A^PP and A^UU symmetric (eqs. (2.19)-(2.22)), with
// -A^PP >= 0 and A^UU < 0, i.e. quasi-definite, which admits an LDL^T
// factorisation in any symmetric order without pivoting.  The factors are
// stored LU-fashion in the band -- L below the diagonal, D on it, U = D L^T
// above -- so the two triangular sweeps solve M x = diag(s) b.
//
// Column blocks of kLB = 16.  Block k is factored by one wave (each row of 16
// lanes holds the whole 16x16 block, so broadcasts are DPP row moves), which
// also forms L11^{-1} and 1/D into `inv` (272 entries per block: L11^{-1}
// row-major, then 1/D).  One kernel per block then applies it to the trailing
// band: every lower 64x64 tile (ti >= tj) forms W = A21 L11^{-T} for its
// row and column blocks on MFMA (L21 = W D^{-1}, U12 = W^T) and updates
// C -= L21 W^T; the tile holding the next diagonal block factors it at once.
// ---------------------------------------------------------------------------

__global__ void k_flip_copy(const double *__restrict__ AB0, double *__restrict__ AB,
                            const double *__restrict__ b0, double *__restrict__ b, int n, int w) {
  const int ld = 2 * w + 1;
  const long long total = (long long)n * ld;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; e < total; e += stride) {
    const int j = (int)(e / ld);
    const int i = j + (int)(e % ld) - w;
    AB[e] = (i & 1) ? AB0[e] : -AB0[e];
    if (e < n) b[e] = (e & 1) ? b0[e] : -b0[e];
  }
}

__global__ __launch_bounds__(64) void k_ldl_first(double *__restrict__ AB, int n, int w,
                                                  double *__restrict__ inv, DevStatus *st) {
  __shared__ double blk[2 * kLB * (kLB + 1)];
  __shared__ double T[kInvStride];
  const int ld = 2 * w + 1;
  const int lane = threadIdx.x;
  const int kb = min(kLB, n);
  for (int e = lane; e < kLB * kLB; e += 64) {
    const int r = e / kLB, c = e % kLB;
    blk[r * (kLB + 1) + c] = (r < kb && c <= r && r - c <= w) ? AB[(size_t)c * ld + (w + r - c)] : 0.0;
  }
  __syncthreads();
  auto store = [&](int t, int i, double v) {
    if (abs(i - t) <= w) AB[(size_t)t * ld + (w + i - t)] = v;
  };
  if (ldl_diag16(blk, kb, lane, store, inv, blk, T) && lane == 0) set_status(st, -5, 0, 0.0);
}

// y of the last block, y = L11^{-1} b (its rows of b are final after the
// last step).
__global__ __launch_bounds__(64) void k_ldl_tail_y(const double *__restrict__ inv_last, const double *__restrict__ b,
                                                   double *__restrict__ y, int n, int k0) {
  const int r = threadIdx.x;
  if (r >= kLB || k0 + r >= n) return;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < kLB; ++c) acc += inv_last[r * kLB + c] * (k0 + c < n ? b[k0 + c] : 0.0);
  y[k0 + r] = acc;
}

// Step for block k0 (factored; its L11^{-1}, 1/D in inv_k): the trailing rows
// and columns r0 = k0 + 16 .. r0 + nr - 1 in lower 64x64 tiles, one
// workgroup (four waves, 16 rows each) per tile, plus a fifth wave that, in
// the tile holding the next diagonal block, factors that block while the
// other waves finish the tile.  The forward substitution
// L y = b rides along: block k's y_k = L11^{-1} b_k (b_k is final once the
// previous steps have run) goes to y, and each diagonal tile applies
// b -= L21 y_k to its 64 rows.
constexpr int kStepThreads = 320;

__global__ __launch_bounds__(kStepThreads) void k_ldl_step(double *__restrict__ AB, int n, int w, int k0,
                                                  const double *__restrict__ inv_k,
                                                  double *__restrict__ inv_next, double *__restrict__ b,
                                                  double *__restrict__ y, DevStatus *st) {
  using M = Mma<double>;
  __shared__ double Li[kLB * (kLB + 1)];
  __shared__ double Dq[kLB];
  __shared__ double Wi[64 * (kLB + 1)];
  __shared__ double Wj[64 * (kLB + 1)];
  __shared__ double Dn[2 * kLB * (kLB + 1)];
  __shared__ double yk[kLB];
  __shared__ double bk[kLB];
  __shared__ double Ts[kInvStride];  // staging of the next block's inverse
  const int ld = 2 * w + 1;
  const int r0 = k0 + kLB;
  const int nr = min(n, k0 + kLB + w) - r0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // lower tile (ti, tj) of this workgroup
  int ti = 0, tj = blockIdx.x;
  while (tj > ti) {
    tj -= ti + 1;
    ++ti;
  }
  const int i0 = r0 + 64 * ti, j0 = r0 + 64 * tj;
  for (int e = tid; e < kLB * kLB; e += 256) Li[(e / kLB) * (kLB + 1) + (e % kLB)] = inv_k[e];
  if (tid < kLB) Dq[tid] = inv_k[kLB * kLB + tid];
  if (tid >= 64 && tid < 64 + kLB) bk[tid - 64] = (k0 + tid - 64 < n) ? b[k0 + tid - 64] : 0.0;
  // A21 rows of this wave for the row block (and the column block)
  auto a21 = [&](int i, int c) -> double {
    const int j = k0 + c;
    return (i < r0 + nr && i - j <= w) ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
  };
  // waves 0..3 own 16 rows of the tile each; wave 4 owns none
  const bool rows = wave < 4;
  double ai[4] = {0.0, 0.0, 0.0, 0.0}, aj[4] = {0.0, 0.0, 0.0, 0.0};
  // this lane's operands of L11^{-1} and 1/D, straight from global memory so
  // that W and the next diagonal block need no barrier
  double bl[4] = {0.0, 0.0, 0.0, 0.0}, dq[4] = {0.0, 0.0, 0.0, 0.0};
  typename M::v4 c[4];
  if (rows) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      ai[s] = a21(i0 + 16 * wave + lr, 4 * s + lk);
      aj[s] = a21(j0 + 16 * wave + lr, 4 * s + lk);
      bl[s] = inv_k[lr * kLB + 4 * s + lk];
      dq[s] = inv_k[kLB * kLB + 4 * s + lk];
    }
    // the C tile of this wave: rows i0 + 16 wave + .., columns j0 + 16 tc + ..
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * wave + M::crow(v, lane), j = j0 + 16 * tc + lr;
        const bool ok = i < r0 + nr && j < r0 + nr && i >= j && i - j <= w;
        c[tc][v] = ok ? AB[(size_t)j * ld + (w + i - j)] : 0.0;
      }
    }
  }
  // W = A21 L11^{-T}: lane supplies A[l%16][k] and B[k][l%16] = L11^{-1}[l%16][k]
  if (rows) {
    typename M::v4 wi = {0.0, 0.0, 0.0, 0.0}, wj = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      wi = M::mma(ai[s], bl[s], wi);
      wj = M::mma(aj[s], bl[s], wj);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wi[(16 * wave + M::crow(v, lane)) * (kLB + 1) + lr] = wi[v];
      Wj[(16 * wave + M::crow(v, lane)) * (kLB + 1) + lr] = wj[v];
    }
  }
  // C -= (W_i D^{-1}) W_j^T.  a = W_i D^{-1} comes from this wave's own rows
  // of Wi (no barrier needed).  In the tile holding the next diagonal block,
  // wave 0 updates that block right away -- its only columns on or below the
  // diagonal -- and hands it to wave 4 across the one barrier; wave 4 factors
  // it (the critical path from one step to the next) while the row waves
  // finish the tile.
  const bool has_next = ti == 0 && tj == 0;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (rows) {
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = Wi[(16 * wave + lr) * (kLB + 1) + 4 * s + lk] * dq[s];
  }
  if (has_next && wave == 0) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c[0] = M::mma(-a[s], Wj[lr * (kLB + 1) + 4 * s + lk], c[0]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + M::crow(v, lane), j = j0 + lr;
      const bool ok = i < r0 + nr && j < r0 + nr && i >= j && i - j <= w;
      Dn[(i - r0) * (kLB + 1) + (j - r0)] = ok ? c[0][v] : 0.0;
    }
  }
  __syncthreads();
  // forward substitution of block k in the diagonal tiles, by wave 1 (off
  // wave 0's path): y_k = L11^{-1} b_k on lanes 0..15, then b -= L21 y_k on
  // the tile's rows (the wave's LDS accesses complete in order)
  if (ti == tj && wave == 1) {
    if (lane < kLB) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < kLB; ++c) acc += Li[lane * (kLB + 1) + c] * bk[c];
      yk[lane] = acc;
      if (ti == 0 && k0 + lane < n) y[k0 + lane] = acc;
    }
    const int i = i0 + lane;
    if (i < r0 + nr) {
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < kLB; ++c) acc += Wi[lane * (kLB + 1) + c] * Dq[c] * yk[c];
      b[i] -= acc;
    }
  }
  if (has_next && wave == 4) {
    const int kb = min(kLB, n - r0);
    auto store = [&](int t, int i, double v) {
      if (abs(i - t) <= w) AB[(size_t)(r0 + t) * ld + (w + i - t)] = v;
    };
    if (ldl_diag16(Dn, kb, lane, store, inv_next, Dn, Ts) && lane == 0) set_status(st, -5, r0, 0.0);
  } else if (rows && !(has_next && wave == 0)) {
    // the first ntc tile columns of this wave's rows; in a diagonal tile the
    // columns past the wave's own 16 rows lie above the diagonal (and in the
    // tile of the next diagonal block wave 0 is already done)
    auto update_cols = [&](auto ntc_c) {
      constexpr int NTC = decltype(ntc_c)::value;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int tc = 0; tc < NTC; ++tc)
          c[tc] = M::mma(-a[s], Wj[(16 * tc + lr) * (kLB + 1) + 4 * s + lk], c[tc]);
      }
#pragma unroll
      for (int tc = 0; tc < NTC; ++tc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * wave + M::crow(v, lane), j = j0 + 16 * tc + lr;
          const bool ok = i < r0 + nr && j < r0 + nr && i >= j && i - j <= w;
          if (ok) AB[(size_t)j * ld + (w + i - j)] = c[tc][v];
        }
      }
    };
    const int ntc = (ti == tj) ? wave + 1 : 4;
    if (ntc == 4)
      update_cols(std::integral_constant<int, 4>{});
    else if (ntc == 3)
      update_cols(std::integral_constant<int, 3>{});
    else if (ntc == 2)
      update_cols(std::integral_constant<int, 2>{});
    else
      update_cols(std::integral_constant<int, 1>{});
  }
  // the diagonal tile of each row block stores U12 = W^T above the diagonal.
  // L21 = W D^{-1} is not stored here: the other tiles of this launch still
  // read A21 from those entries, and a workgroup that starts after this one
  // has finished would read L21 instead.  k_ldl_lower writes it once the
  // whole factorisation is done.
  if (ti == tj && rows) {
    for (int e = tid; e < 64 * kLB; e += 256) {
      const int rr = e / kLB, cc = e % kLB;
      const int i = i0 + rr, j = k0 + cc;
      if (i < r0 + nr && i - j <= w) AB[(size_t)i * ld + (w + j - i)] = Wi[rr * (kLB + 1) + cc];
    }
  }
}

// L below the diagonal blocks from the stored U = D L^T: L(i, j) = U(j, i) / D_j
// for j < i <= j + w outside j's own 16-block (whose L the block
// factorisation wrote).  One thread per band entry below the diagonal.
__global__ void k_ldl_lower(double *__restrict__ AB, const double *__restrict__ inv, int n, int w) {
  const int ld = 2 * w + 1;
  const long long total = (long long)n * w;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int j = (int)(e / w), t = 1 + (int)(e % w);
    const int i = j + t;
    if (i >= n || i / kLB == j / kLB) continue;
    const double dinv = inv[(size_t)(j / kLB) * kInvStride + kLB * kLB + (j % kLB)];
    AB[(size_t)j * ld + (w + t)] = AB[(size_t)i * ld + (w - t)] * dinv;
  }
}

// Triangular sweeps with the band factors, one workgroup of 1024 lanes.
// lower: L y = b (unit lower), forward.  upper: U x = y, backward.  In place.
// Per block of kSW = 16 unknowns, wave 0 solves the diagonal block as a
// product with its stored inverse -- L11^{-1} forward, U11^{-1} = L11^{-T} D^{-1}
// backward -- while the other waves apply the block to the rows it couples
// to (one row per lane; beyond 960 rows a slower loop).  The active part of x
// lives in an LDS ring of RW >= w + 2 kSW entries; the band entries and
// inverse of the next block and the x entries that enter the ring next are
// fetched one block ahead, so no global access sits on the critical path.
constexpr int kSW = kLB;

constexpr int kSweepThreads = 1024;

__global__ __launch_bounds__(kSweepThreads) void k_lu_sweep(const double *__restrict__ AB,
                                                            const double *__restrict__ inv, int n,
                                                            int w, double *__restrict__ x, int upper,
                                                            int RW) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *xr = reinterpret_cast<double *>(smem_raw);  // ring, entry i at i % RW
  __shared__ double xb[kSW];
  const int ld = 2 * w + 1;
  const int tid = threadIdx.x;
  const int nblk = (n + kSW - 1) / kSW;
  const int nprop = kSweepThreads - 64;
  // band entries of one block (diagonal-block inverse for wave 0; entry kSW
  // carries wave 0's 1/D_r)
  double cur[kSW + 1], nxt[kSW + 1];
  double xin_cur = 0.0, xin_nxt = 0.0;  // entering x value (threads 64..64+kSW-1)
  // rows the block at k0 updates: [lo, hi)
  auto prop_lo = [&](int k0, int kb) { return upper ? max(0, k0 - w) : k0 + kb; };
  auto prop_hi = [&](int k0, int kb) { return upper ? k0 : min(n, k0 + kb + w); };
  auto fetch = [&](int blk, double (&dst)[kSW + 1]) {
    dst[kSW] = 0.0;
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    if (tid < 64) {
      // row tid of the diagonal block's inverse: lower L11^{-1}, upper
      // L11^{-T} (applied to D^{-1} times the block, with 1/D_r in dst[kSW]);
      // rows and columns past the matrix are zero.  Nothing is computed on
      // the loaded values here, so the loads stay in flight.
      const double *iv = inv + (size_t)blk * kInvStride;
      const int r = tid & 15;
#pragma unroll
      for (int c = 0; c < kSW; ++c) {
        const bool in = r < kb && c < kb;
        dst[c] = !in ? 0.0 : (upper ? iv[c * kLB + r] : iv[r * kLB + c]);
      }
      dst[kSW] = (upper && r < kb) ? iv[kLB * kLB + r] : 0.0;
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
  auto body = [&](int s, double (&cu)[kSW + 1], double (&nx)[kSW + 1]) {
    const int blk = upper ? (nblk - 1 - s) : s;
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    const int nb = upper ? blk - 1 : blk + 1;
    xin_cur = xin_nxt;
    if (s + 1 < nblk) fetch(nb, nx);
    if (s + 2 < nblk) xin_nxt = fetch_x(upper ? blk - 2 : blk + 2);
    if (tid < 64) {
      const int lane = tid;
      double xo = (lane < kb) ? xr[(k0 + lane) % RW] : 0.0;
      if (upper) xo *= cu[kSW];
      double xv = 0.0, xw = 0.0;
#pragma unroll
      for (int c = 0; c < kSW; c += 2) {
        xv += cu[c] * row_bcast(xo, c);
        xw += cu[c + 1] * row_bcast(xo, c + 1);
      }
      xv += xw;
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

// Sweeps for systems whose right-hand side fits in LDS (n <= kSweepLdsMax):
// the whole vector stays in LDS, so no ring bookkeeping sits in the loop.
// Band loads are unconditional at clamped addresses with a validity mask
// applied at use, so nothing stops them from staying in flight while the
// previous block computes (a load under a branch makes the compiler wait for
// every outstanding load before the loop goes on).
constexpr int kSweepLdsMax = 14336;

template <int UPPER>
__global__ __launch_bounds__(kSweepThreads) void k_band_sweep(const double *__restrict__ AB,
                                                              const double *__restrict__ inv, int n,
                                                              int w, double *__restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *xs = reinterpret_cast<double *>(smem_raw);
  const int ld = 2 * w + 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int nblk = (n + kSW - 1) / kSW;
  const int q = tid - 64;  // propagation row offset of threads 64..
  for (int i = tid; i < n; i += kSweepThreads) xs[i] = x[i];
  // rows a block updates: lower [k0+kb, k0+kb+w), upper [k0-w, k0)
  auto fetch = [&](int blk, double (&dst)[kSW + 1], unsigned &mask) {
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    mask = 0u;
    if (tid < 64) {
      // diagonal-block inverse, row r (identity past the matrix): lower
      // L11^{-1}, upper L11^{-T} with 1/D_r in dst[kSW]
      const double *iv = inv + (size_t)blk * kInvStride;
      const int r = tid & 15;
#pragma unroll
      for (int c = 0; c < kSW; ++c) dst[c] = UPPER ? iv[c * kLB + r] : iv[r * kLB + c];
      dst[kSW] = iv[kLB * kLB + r];
    } else {
      const int i = UPPER ? k0 - w + q : k0 + kb + q;
      const bool row_ok = UPPER ? (i >= 0 && i < k0) : (i < min(n, k0 + kb + w));
#pragma unroll
      for (int c = 0; c < kSW; ++c) {
        const int j = k0 + c;
        const int off = UPPER ? (j - i) : (i - j);
        const bool in = row_ok && c < kb && off <= w;
        const long long e = in ? (long long)j * ld + (w + i - j) : 0;
        dst[c] = AB[e];
        mask |= in ? (1u << c) : 0u;
      }
      dst[kSW] = 0.0;
    }
  };
  double cu[kSW + 1], nx[kSW + 1];
  unsigned mcu = 0u, mnx = 0u;
  fetch(UPPER ? nblk - 1 : 0, cu, mcu);
  __syncthreads();
  auto body = [&](int s, double (&c0)[kSW + 1], unsigned m0, double (&c1)[kSW + 1], unsigned &m1) {
    const int blk = UPPER ? (nblk - 1 - s) : s;
    const int k0 = blk * kSW;
    const int kb = min(kSW, n - k0);
    if (s + 1 < nblk) fetch(UPPER ? blk - 1 : blk + 1, c1, m1);
    if (tid < 64) {
      double xo = (lane < kb) ? xs[k0 + lane] : 0.0;
      if (UPPER) xo *= c0[kSW];
      double xv = 0.0, xw = 0.0;
#pragma unroll
      for (int c = 0; c < kSW; c += 2) {
        xv += c0[c] * row_bcast(xo, c);
        xw += c0[c + 1] * row_bcast(xo, c + 1);
      }
      if (lane < kb) xs[k0 + lane] = xv + xw;
    }
    __syncthreads();
    if (tid >= 64) {
      const int i = UPPER ? k0 - w + q : k0 + kb + q;
      if (m0) {
        double acc = 0.0, acd = 0.0;
#pragma unroll
        for (int c = 0; c < kSW; c += 2) {
          acc += ((m0 >> c) & 1u ? c0[c] : 0.0) * xs[k0 + c];
          acd += ((m0 >> (c + 1)) & 1u ? c0[c + 1] : 0.0) * xs[k0 + c + 1];
        }
        xs[i] -= acc + acd;
      }
      // rows beyond the threads' reach (w > kSweepThreads - 64)
      const int lo = UPPER ? max(0, k0 - w) : k0 + kb;
      const int hi = UPPER ? k0 : min(n, k0 + kb + w);
      for (int i2 = (UPPER ? k0 - w : k0 + kb) + q + (kSweepThreads - 64); i2 < hi; i2 += kSweepThreads - 64) {
        if (i2 < lo) continue;
        double acc = 0.0;
        for (int c = 0; c < kb; ++c) {
          const int j = k0 + c;
          if (UPPER ? (j - i2 <= w) : (i2 - j <= w)) acc += AB[(size_t)j * ld + (w + i2 - j)] * xs[j];
        }
        xs[i2] -= acc;
      }
    }
    __syncthreads();
  };
  for (int s = 0; s < nblk; s += 2) {
    body(s, cu, mcu, nx, mnx);
    if (s + 1 < nblk) body(s + 1, nx, mnx, cu, mcu);
  }
  for (int i = tid; i < n; i += kSweepThreads) x[i] = xs[i];
}

// Backward sweep U x = y by chunks of kChunk = 128 unknowns, last chunk
// first, one launch per chunk.  The launch for the chunk at c0 also applies
// the chunk solved by the previous launch (at cn = c0 + 128):
//   workgroup 0 subtracts it from the chunk's own rows and then solves the
//     chunk's triangle: wave 0 solves each 16-block with the stored inverse,
//     U_bb^{-1} = L11^{-T} D^{-1}, while waves 1-4 subtract it from the rows
//     above it in the chunk;
//   workgroups 1.. subtract it from the rows above the chunk (up to w rows
//     above cn), 64 rows each -- nearly all of the band is read there, in
//     parallel rather than through a single compute unit.
// The two parts write disjoint rows and read only the finished chunk at cn.
constexpr int kChunk = 128;
constexpr int kChunkBlocks = kChunk / kSW;
constexpr int kStepT = 512;

// Rows [lo, hi) minus U(rows, cn .. cn+mn-1) x(cn ..): 64 rows from row0,
// one per lane, wave q taking columns 16q .. 16q+15 (eight waves).
__device__ __forceinline__ void usweep_far(const double *__restrict__ AB, int w, double *__restrict__ x,
                                           int cn, int mn, int row0, int hi, double *xc, double *part) {
  const int ld = 2 * w + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = row0 + lane;
  if (tid < kChunk) xc[tid] = tid < mn ? x[cn + tid] : 0.0;
  double a[kSW];
  unsigned msk = 0u;
#pragma unroll
  for (int c = 0; c < kSW; ++c) {
    const int j = cn + kSW * wave + c;
    const bool ok = i < hi && j < cn + mn && j - i <= w;
    a[c] = AB[ok ? (size_t)j * ld + (w + i - j) : 0];
    msk |= ok ? (1u << c) : 0u;
  }
  __syncthreads();
  double acc = 0.0, acd = 0.0;
#pragma unroll
  for (int c = 0; c < kSW; c += 2) {
    acc += ((msk >> c) & 1u ? a[c] : 0.0) * xc[kSW * wave + c];
    acd += ((msk >> (c + 1)) & 1u ? a[c + 1] : 0.0) * xc[kSW * wave + c + 1];
  }
  part[wave * 64 + lane] = acc + acd;
  __syncthreads();
  if (wave == 0 && i < hi) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kStepT / 64; ++q) t += part[q * 64 + lane];
    x[i] -= t;
  }
}

__global__ __launch_bounds__(kStepT) void k_usweep_step(const double *__restrict__ AB,
                                                        const double *__restrict__ inv, int n, int w,
                                                        double *__restrict__ x, int c0, int has_next) {
  __shared__ double xs[kChunk];
  __shared__ double lt[kChunkBlocks * kInvStride];
  __shared__ double part[kStepT];  // far: per-wave sums; near: 4 x 128 partial sums
  __shared__ double xcn[kChunk];   // near: the x of the chunk at cn
  const int ld = 2 * w + 1;
  const int m = min(kChunk, n - c0);
  const int cn = c0 + kChunk;
  const int mn = has_next ? min(kChunk, n - cn) : 0;
  if (blockIdx.x > 0) {
    const int lo = max(0, cn - w);
    usweep_far(AB, w, x, cn, mn, lo + 64 * (blockIdx.x - 1), c0, xs, part);
    return;
  }
  const int nbk = (m + kSW - 1) / kSW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // First the near update on all waves: row tid & 127 of the chunk against
  // columns 32 q .. 32 q + 31 of the chunk at cn, q = tid >> 7.  Then the
  // chunk's triangle on waves 1-4 (t = tid - 64): waves 1-2 hold row t & 127's
  // entries in blocks 1..4 of the chunk, waves 3-4 in blocks 5..7 (only
  // blocks above the row's own block are used).  The two phases' operands
  // are never live together.
  const bool rw = wave >= 1 && wave <= 4;
  const int t = tid - 64, row = t & 127, half = t >> 7;
  // global loads first: the block inverses, the chunk's right-hand side and
  // the x of the chunk at cn, the near band block
  constexpr int kLtPer = (kChunkBlocks * kInvStride + kStepT - 1) / kStepT;
  const double *iv = inv + (size_t)(c0 / kSW) * kInvStride;
  const int nlt = nbk * kInvStride;
  double ltv[kLtPer];
#pragma unroll
  for (int q = 0; q < kLtPer; ++q) ltv[q] = iv[min(tid + kStepT * q, nlt - 1)];
  const double xv0 = x[c0 + min(tid, m - 1)];
  const double xn0 = mn > 0 ? x[cn + min(tid, mn - 1)] : 0.0;
  const int nrow = tid & 127, nq = tid >> 7;
  double nb[32];
  unsigned nmsk = 0u;
  if (mn > 0) {
    const int i = c0 + nrow;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int j = cn + 32 * nq + c;
      const bool ok = nrow < m && j < cn + mn && j - i <= w;
      nb[c] = AB[ok ? (size_t)j * ld + (w + i - j) : 0];
      nmsk |= ok ? (1u << c) : 0u;
    }
  }
  if (tid < kChunk) {
    xs[tid] = tid < m ? xv0 : 0.0;
    xcn[tid] = tid < mn ? xn0 : 0.0;
  }
#pragma unroll
  for (int q = 0; q < kLtPer; ++q)
    if (tid + kStepT * q < nlt) lt[tid + kStepT * q] = ltv[q];
  __syncthreads();
  {
    double acc = 0.0, acd = 0.0;
    if (mn > 0) {
      const double *xc = xcn + 32 * nq;
#pragma unroll
      for (int c = 0; c < 32; c += 2) {
        acc += ((nmsk >> c) & 1u ? nb[c] : 0.0) * xc[c];
        acd += ((nmsk >> (c + 1)) & 1u ? nb[c + 1] : 0.0) * xc[c + 1];
      }
    }
    part[nq * kChunk + nrow] = acc + acd;
  }
  __builtin_amdgcn_sched_barrier(0);
  // the triangle's band entries: u[k][c] = U(c0 + row, c0 + 16 bb + c) with
  // bb = 1 + k (waves 1-2) or 5 + k (waves 3-4)
  double u[4][kSW];
  unsigned msk[4];
  if (rw) {
    const int i = c0 + row;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int bb = (half ? 5 : 1) + k;
      msk[k] = 0u;
#pragma unroll
      for (int c = 0; c < kSW; ++c) {
        const int j = c0 + kSW * bb + c;
        const bool ok = bb < kChunkBlocks && row < kSW * bb && j < c0 + m && j - i <= w;
        u[k][c] = AB[ok ? (size_t)j * ld + (w + i - j) : 0];
        msk[k] |= ok ? (1u << c) : 0u;
      }
    }
  }
  __syncthreads();
  if (tid < m) xs[tid] -= (part[tid] + part[kChunk + tid]) + (part[2 * kChunk + tid] + part[3 * kChunk + tid]);
  __syncthreads();
#pragma unroll
  for (int bb = kChunkBlocks - 1; bb >= 0; --bb) {
    if (bb < nbk) {
      const int b0 = kSW * bb;
      const int kb = min(kSW, m - b0);
      if (wave == 0) {
        const int r = lane & 15;
        const double *l = lt + bb * kInvStride;
        const double xo = (r < kb) ? xs[b0 + r] * l[kLB * kLB + r] : 0.0;
        double xv = 0.0, xw = 0.0;
#pragma unroll
        for (int c = 0; c < kSW; c += 2) {
          xv += l[c * kLB + r] * row_bcast(xo, c);
          xw += l[(c + 1) * kLB + r] * row_bcast(xo, c + 1);
        }
        if (lane < kb) xs[b0 + lane] = xv + xw;
      }
      __syncthreads();
      // block bb's owners: waves 1-2 for bb = 1..4, waves 3-4 for bb = 5..7
      if (bb > 0 && rw && half == (bb >= 5 ? 1 : 0) && row < b0) {
        const int k = bb - (bb >= 5 ? 5 : 1);
        double acc = 0.0, acd = 0.0;
#pragma unroll
        for (int c = 0; c < kSW; c += 2) {
          acc += ((msk[k] >> c) & 1u ? u[k][c] : 0.0) * xs[b0 + c];
          acd += ((msk[k] >> (c + 1)) & 1u ? u[k][c + 1] : 0.0) * xs[b0 + c + 1];
        }
        xs[row] -= acc + acd;
      }
      __syncthreads();
    }
  }
  if (tid < m) x[c0 + tid] = xs[tid];
}

// r = b - A x with the unfactored band (one thread per row).
__global__ void k_band_residual(const double *__restrict__ AB, int n, int w,
                                const double *__restrict__ x, const double *__restrict__ b,
                                double *__restrict__ r, int flip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ld = 2 * w + 1;
  double acc = 0.0;
  const int jlo = max(0, i - w), jhi = min(n - 1, i + w);
  for (int j = jlo; j <= jhi; ++j) acc += AB[(size_t)j * ld + (w + i - j)] * x[j];
  // flip: the residual of the symmetric form, diag(s) (b - A x)
  r[i] = (flip && !(i & 1)) ? acc - b[i] : b[i] - acc;
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

size_t ldl_inv_size(int n) { return (size_t)((n + kLB - 1) / kLB) * kInvStride; }

hipError_t launch_band_ldl(const double *AB0, double *AB, const double *b0, double *b, double *y, int n, int w,
                           double *inv, DevStatus *st, hipStream_t s) {
  hipLaunchKernelGGL(k_flip_copy, dim3(1024), dim3(256), 0, s, AB0, AB, b0, b, n, w);
  hipLaunchKernelGGL(k_ldl_first, dim3(1), dim3(64), 0, s, AB, n, w, inv, st);
  int k0 = 0;
  for (; k0 + kLB < n; k0 += kLB) {
    const int nr = std::min(n, k0 + kLB + w) - (k0 + kLB);
    const int nt = (nr + 63) / 64;
    hipLaunchKernelGGL(k_ldl_step, dim3(nt * (nt + 1) / 2), dim3(kStepThreads), 0, s, AB, n, w, k0,
                       inv + (size_t)(k0 / kLB) * kInvStride, inv + (size_t)(k0 / kLB + 1) * kInvStride, b, y, st);
  }
  hipLaunchKernelGGL(k_ldl_tail_y, dim3(1), dim3(64), 0, s, inv + (size_t)(k0 / kLB) * kInvStride, b, y, n, k0);
  if (w > 0) hipLaunchKernelGGL(k_ldl_lower, dim3(grid_for((long long)n * w)), dim3(256), 0, s, AB, inv, n, w);
  return hipGetLastError();
}

hipError_t launch_lu_sweep(const double *AB, const double *inv, int n, int w, double *x, int upper,
                           hipStream_t s) {
  if (upper) {
    const int last = ((n - 1) / kChunk) * kChunk;
    for (int c0 = last; c0 >= 0; c0 -= kChunk) {
      const int has_next = c0 < last;
      // rows above this chunk that the chunk at c0 + kChunk still reaches
      const int far = has_next ? c0 - std::max(0, c0 + kChunk - w) : 0;
      hipLaunchKernelGGL(k_usweep_step, dim3(1 + (far > 0 ? (far + 63) / 64 : 0)), dim3(kStepT), 0, s, AB, inv, n,
                         w, x, c0, has_next);
    }
    // the first chunk's contribution to rows above it: there are none

    return hipGetLastError();
  }
  if (n <= kSweepLdsMax) {
    const size_t lds = (size_t)n * sizeof(double);
    const void *k = upper ? (const void *)k_band_sweep<1> : (const void *)k_band_sweep<0>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (upper)
      hipLaunchKernelGGL(k_band_sweep<1>, dim3(1), dim3(kSweepThreads), lds, s, AB, inv, n, w, x);
    else
      hipLaunchKernelGGL(k_band_sweep<0>, dim3(1), dim3(kSweepThreads), lds, s, AB, inv, n, w, x);
    return hipGetLastError();
  }
  const int RW = w + 2 * kSW + 1;
  const size_t lds = (size_t)RW * sizeof(double);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)k_lu_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lu_sweep, dim3(1), dim3(kSweepThreads), lds, s, AB, inv, n, w, x, upper, RW);
  return hipGetLastError();
}

hipError_t launch_band_residual(const double *AB, int n, int w, const double *x, const double *b,
                                double *r, int flip, hipStream_t s) {
  hipLaunchKernelGGL(k_band_residual, dim3(grid_for(n)), dim3(256), 0, s, AB, n, w, x, b, r, flip);
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
