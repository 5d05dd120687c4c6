// Loop 1 of the MRCM (Algorithm 2) on gfx950: per-subdomain coefficients,
// band Cholesky of the local matrix A^H_l, the 2|I^l|+1 band solves of
// (2.25)/(2.26), the FP64 residual used by mixed-precision refinement, and
// the reduction of the MBF fluxes over each patch.
//
// One workgroup (256 lanes, four wave64s) owns one subdomain.  The local rows
// are ordered with the box's shortest axis fastest, so the lower bandwidth is
// b = n0*n1 and the factor of a 20x20x5 block has b = 100.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "launch.h"

namespace mrcm {

// ---------------------------------------------------------------------------
// Input check: permeabilities must be positive and finite.
// ---------------------------------------------------------------------------
__global__ void k_check_perm(const double *kx, const double *ky, const double *kz, long long n,
                             DevStatus *st) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double a = kx[c], b = ky[c], d = kz[c];
  const bool ok = (a > 0.0) && (b > 0.0) && (d > 0.0) && isfinite(a) && isfinite(b) && isfinite(d);
  if (!ok) set_status(st, -1, (int)c, a);
}

// ---------------------------------------------------------------------------
// Coefficients (one thread per local row).  Per row: the diagonal of A^H_l
// (TPFA transmissibilities of eq. (2.10) as total rates, Robin and wall
// terms), the transmissibilities towards the +ax0, +ax1, +ax2 neighbours
// inside the box (the off-diagonal entries are their negatives), the
// particular right-hand side (source plus wall data) and 1/sqrt(diagonal).
// The pinned row becomes the identity and its column is removed.
// ---------------------------------------------------------------------------
__global__ void k_coef(Geom g, double *__restrict__ coef, double *__restrict__ r0,
                       double *__restrict__ scal) {
  const SubDesc &S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.N) return;
  const I3 x = local_to_global(S, r);
  const long long c = cell_index(g, x);
  const double kc0 = g.k[0][c], kc1 = g.k[1][c], kc2 = g.k[2][c];
  const int a0 = S.ax[0], a1 = S.ax[1];
  double diag = 0.0, rhs = g.q[c];
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const double kd = d == 0 ? kc0 : (d == 1 ? kc1 : kc2);
    const int xn = x[d] + side;
    const int lo = S.lo[d], ext = S.ext[d];
    const double hd = hdir(g, d), ad = adir(g, d);
    if (xn >= lo && xn < lo + ext) {
      I3 y = x;
      y.set(d, xn);
      const long long cn = cell_index(g, y);
      const double kn = kdir(g, d)[cn];
      const double T = ad * (2.0 * kd * kn / (kd + kn)) / hd;
      diag += T;
      if (side > 0) {
        const double tv = (cn == g.pin) ? 0.0 : T;
        const int p = (d == a0) ? 0 : ((d == a1) ? 1 : 2);
        t0 = (p == 0) ? tv : t0;
        t1 = (p == 1) ? tv : t1;
        t2 = (p == 2) ? tv : t2;
      }
    } else if (xn >= 0 && xn < ndir(g, d)) {
      const double beta = robin_beta(g, S, x, f, kd);
      diag += ad / (hd / (2.0 * kd) + beta);
    } else {
      const int wt = wall_type_of(g, f);
      if (wt != 0) {
        const int a = (d == 0) ? 1 : 0;
        const int b = (d == 2) ? 1 : 2;
        const double *wv = wall_value_of(g, f);
        const double gv = wv ? wv[x[a] + (long long)ndir(g, a) * x[b]] : 0.0;
        if (wt == 1) {
          const double T = ad * 2.0 * kd / hd;
          diag += T;
          rhs += T * gv;
        } else {
          rhs -= ad * gv;
        }
      }
    }
  }
  if (c == g.pin) {
    diag = 1.0;
    t0 = t1 = t2 = 0.0;
    rhs = 0.0;
  }
  const long long o = S.cell_off + r;
  coef[4 * o + 0] = diag;
  coef[4 * o + 1] = t0;
  coef[4 * o + 2] = t1;
  coef[4 * o + 3] = t2;
  r0[o] = rhs;
  scal[o] = 1.0 / sqrt(diag);
}

// ---------------------------------------------------------------------------
// Right-hand sides of one local row: column 0 the particular problem, column
// 1+j the P-type MBF of local patch j (G = 1 on the patch), column 1+n+j the
// U-type MBF (G = -sigma beta_f); entry = T_f G_f per Robin face.  Calls
// emit(col, value) for each Robin entry of the row; the pinned row is zero.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void rhs_row_faces(const Geom &g, const SubDesc &S, int r, F emit) {
  if (r == S.pin_local) return;
  const I3 x = local_to_global(S, r);
  const long long c = cell_index(g, x);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int sigma = (f & 1) ? 1 : -1;
    const int xn = x[d] + sigma;
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) continue;
    int lp;
    double T, beta;
    if (gamma_face(g, S, x, f, kdir(g, d)[c], lp, T, beta)) {
      emit(1 + lp, T);
      emit(1 + S.npatch + lp, -sigma * beta * T);
    }
  }
}

// Right-hand sides of rows rbase .. rbase + kRowsPB - 1 of subdomain S into
// the LDS tile (row-major, stride m): one thread per row finds the row's
// Robin entries once, the rest of the tile is zero.  Ends with a barrier.
constexpr int kRowsPB = 64;

__device__ __forceinline__ void rhs_tile(const Geom &g, const SubDesc &S, const double *__restrict__ r0,
                                         int rbase, double *tile) {
  const int m = S.m, tid = threadIdx.x;
  for (int e = tid; e < kRowsPB * m; e += blockDim.x) tile[e] = 0.0;
  __syncthreads();
  if (tid < kRowsPB && rbase + tid < S.N) {
    const int r = rbase + tid;
    double *row = tile + tid * m;
    row[0] = r0[S.cell_off + r];
    rhs_row_faces(g, S, r, [&](int col, double v) { row[col] = v; });
  }
  __syncthreads();
}

// Dense right-hand sides R (row-major, N_l x m_l) of every subdomain,
// kRowsPB rows per workgroup, written out as one contiguous run.  The tile
// (kRowsPB rows of the largest column count, in dynamic LDS) is sized to the
// launch, so that small column counts leave room for more workgroups per CU
// to cover the latency of the coefficient loads.
__global__ __launch_bounds__(256) void k_rhs(Geom g, const double *__restrict__ r0,
                                             double *__restrict__ B, double *__restrict__ B2) {
  extern __shared__ double tile[];
  const SubDesc &S = g.sub[blockIdx.y];
  const int rbase = blockIdx.x * kRowsPB;
  if (rbase >= S.N) return;
  rhs_tile(g, S, r0, rbase, tile);
  const int ne = min(kRowsPB, S.N - rbase) * S.m;
  double *dst = B + S.X_off + (size_t)rbase * S.m;
  for (int e = threadIdx.x; e < ne; e += blockDim.x) dst[e] = tile[e];
  if (B2) {
    double *dst2 = B2 + S.X_off + (size_t)rbase * S.m;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) dst2[e] = tile[e];
  }
}

// ---------------------------------------------------------------------------
// Band Cholesky.  The active part of the band -- the current panel of kNB
// columns and the columns it updates -- lives in LDS as a ring of
// W = max(b, kNB) + kNB column slots, each holding the b+1 entries
// L[j..j+b][j] and zero padding beyond offset b.  Columns are assembled from
// the coefficients when they enter the ring, so A^H_l never exists in global
// memory.  Iteration k (panel k fully factored) has two phases separated by
// workgroup barriers:
//   P1  wave 0 applies panel k to the next panel's 16x16 diagonal block and
//       factors it in registers (lane broadcasts, reciprocal square roots),
//       inverting it on the way; the other waves -- and wave 0 once done --
//       take the rest of panel k's trailing update (MFMA tiles) and the
//       copies of panel k to global memory from a shared counter;
//   P2  all waves form the next panel's sub-diagonal rows
//       L21 = A21 L11^{-T} on MFMA, and the columns k+W .. k+W+15 (their
//       coefficients fetched one iteration earlier) take panel k's slots.
// The factor is written by column, (b+1) entries per column; the inverses of
// the 16x16 diagonal blocks (what the solves use) go to a separate array.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int s, int W) { return s >= W ? s - W : s; }

// Reciprocal and reciprocal square root from the hardware estimates (relative
// error near 2^-24 in FP64, about an ulp in FP32).  FP64 refines with one
// third-order step: with e = 1 - x y, 1/x = y (1 + e + e^2 + ...), so
// y (1 + e + e^2) leaves an error of order e^3; with e = 1 - x y^2,
// 1/sqrt(x) = y (1 + e/2 + 3e^2/8 + ...).  FP32 takes one Newton step.
// The estimate and the refinement are separate calls so that a caller can
// place independent work between them.
__device__ __forceinline__ double rcp_est(double x) { return __builtin_amdgcn_rcp(x); }
__device__ __forceinline__ float rcp_est(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsq_est(double x) { return __builtin_amdgcn_rsq(x); }
__device__ __forceinline__ float rsq_est(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }
// the correction factors: 1/x = y (1 + rcp_t(e)), 1/sqrt(x) = y (1 + rsq_t(e))
__device__ __forceinline__ double rcp_t(double e) { return fma(e, e, e); }
__device__ __forceinline__ float rcp_t(float e) { return e; }
__device__ __forceinline__ double rsq_t(double e) { return e * fma(0.375, e, 0.5); }
__device__ __forceinline__ float rsq_t(float e) { return 0.5f * e; }
template <typename T>
__device__ __forceinline__ T rcp_refine(T x, T y) {
  return fmat(y, rcp_t(fmat(-x, y, T(1))), y);
}
template <typename T>
__device__ __forceinline__ T rsq_refine(T x, T y) {
  return fmat(y, rsq_t(fmat(-x * y, y, T(1))), y);
}

// Diagonal block of panel k (kb <= 16 columns) on one wave: Cholesky factor
// L11, written back into the ring, and X = L11^{-1} into Xs (row-major
// 16x16; rows and columns past the matrix hold the identity).  Each row of
// 16 lanes holds the whole block (lane r: row r), so every broadcast stays
// within a row.  The elimination runs in the square-root-free form: with
// pivot D and column a (entries a_i = A'[i][jj]), the Schur update is
// A'[i][p] -= a_i a_p / D, so the chain from one pivot to the next needs only
// 1/D; the Cholesky column a / sqrt(D) and the step of the inverse are formed
// beside it.  The inverse rides along: lane c solves L11 x = e_c column by
// column, x_i -= L[i][jj] x_jj = a_i (x_jj / D) with x_jj taken before its
// own scaling by 1/sqrt(D).  The results of each pivot are written as soon as
// they are final, beside the chain; lanes with nothing to write put it into
// `junk` (kNB spare LDS entries).  Returns nonzero when a pivot was not
// positive.
template <typename T>
__device__ __forceinline__ int factor_diag(T *S, T *Xs, T *junk, int ldb, int k, int kb, int b, int W,
                                           int lane) {
  const int sk = k % W;
  int r = lane & 15;
  // opaque to the optimiser: values derived from the lane index (identity
  // entries, addresses) are recomputed per call instead of being hoisted out
  // of the panel loop and held in registers across it
  asm volatile("" : "+v"(r));
  T v[kNB], x[kNB];
#pragma unroll
  for (int jj = 0; jj < kNB; ++jj) {
    // all sixteen loads in flight at once: the offset is clamped into the
    // column and the entry selected afterwards
    const T a = S[wrap(sk + jj, W) * ldb + max(r - jj, 0)];
    v[jj] = (jj < kb && r < kb && jj <= r) ? a : ((r == jj) ? T(1) : T(0));
    x[jj] = (r == jj) ? T(1) : T(0);
  }
  T ok = T(1);
  T q, y;
  {
    const T d = row_bcast(v[0], 0);
    ok = (d > T(0)) ? ok : T(0);
    q = rcp_refine(d, rcp_est(d));
    y = rsq_refine(d, rsq_est(d));
  }
  // Software-pipelined: pivot jj finishes column jj + 1 first and starts the
  // reciprocals of the next pivot, whose latency the updates of the remaining
  // columns cover; the scheduling barriers keep this interleaving (and the
  // pivots in order: without them the scheduler may defer whole chains of
  // updates and hold their broadcast values in registers).
#pragma unroll
  for (int jj = 0; jj < kNB; ++jj) {
    const T w = v[jj] * q;
    const T xq = x[jj] * q;
    // entries above the diagonal of v collect garbage that is never read
    auto upd = [&](int i) {
      if (i < kNB) {
        const T a = row_bcast(v[jj], i);
        v[i] -= w * a;
        x[i] -= a * xq;
      }
    };
    T qn = T(0), yn = T(0);
    if (jj + 1 < kNB) {
      // column jj+1 first: it carries the next pivot
      // The next pivot, d = A'[jj+1][jj+1] - a^2 / D with a = A'[jj+1][jj],
      // formed in every lane from values final before this pivot, so that
      // only one FMA after 1/D sits on the chain (lane jj+1's own update of
      // v[jj+1] gives the same value up to rounding).
      const T a = row_bcast(v[jj], jj + 1);
      const T vd = row_bcast(v[jj + 1], jj + 1);
      const T d = fmat(-q, a * a, vd);
      v[jj + 1] -= w * a;
      x[jj + 1] -= a * xq;
      ok = (d > T(0)) ? ok : T(0);
      // the refinements step by step, two column updates between dependent
      // steps (the compiler would otherwise issue the chain back to back)
      const T q0 = rcp_est(d);
      const T y0 = rsq_est(d);
      upd(jj + 2);
      upd(jj + 3);
      __builtin_amdgcn_sched_barrier(0);
      const T e = fmat(-d, q0, T(1));
      const T xy = d * y0;
      upd(jj + 4);
      upd(jj + 5);
      __builtin_amdgcn_sched_barrier(0);
      const T t = rcp_t(e);
      const T ey = fmat(-xy, y0, T(1));
      upd(jj + 6);
      upd(jj + 7);
      __builtin_amdgcn_sched_barrier(0);
      qn = fmat(q0, t, q0);
      const T ty = rsq_t(ey);
      upd(jj + 8);
      upd(jj + 9);
      __builtin_amdgcn_sched_barrier(0);
      yn = fmat(y0, ty, y0);
#pragma unroll
      for (int i = jj + 10; i < kNB; ++i) upd(i);
    }
    // lane jj holds the pivot itself, so the same product gives it sqrt(D)
    v[jj] *= y;
    x[jj] *= y;
    // column jj of the factor and entry jj of lane r's column of the inverse
    // are final
    Xs[jj * kNB + r] = x[jj];
    {
      const bool mine = jj < kb && jj <= r && r - jj <= b;
      T *dst = mine ? S + (wrap(sk + jj, W) * ldb + r - jj) : junk + r;
      *dst = v[jj];
    }
    __builtin_amdgcn_sched_barrier(0);
    q = qn;
    y = yn;
  }
  return ok == T(1) ? 0 : 1;
}

// Tiles ti = ti0 + dt*t, t < NB (all >= 1; rows 16ti..16ti+15 of panel k) of
// L21 = A21 X^T, X = L11^{-1} from Xs, written back into the ring; slots
// t >= cnt repeat tile ti0 and store nothing.  Rows past the matrix or the
// band come out zero because the corresponding entries of A21 are zero.
// The MFMA chains of the tiles are interleaved without branches.
template <typename T, int NB>
__device__ __forceinline__ void panel_l21_tiles(T *S, const T *Xs, int ldb, int k, int kb, int b, int W,
                                                int lane, int ti0, int dt, int cnt) {
  using M = Mma<T>;
  const int sk = k % W;
  const int r = lane & 15, lk = lane >> 4;
  T bx[4];
  int colk[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = 4 * s + lk;
    bx[s] = Xs[r * kNB + kk];
    colk[s] = wrap(sk + kk, W) * ldb - kk + r;
  }
  int ti[NB];
  T a[NB][4];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    ti[t] = t < cnt ? ti0 + dt * t : ti0;
#pragma unroll
    for (int s = 0; s < 4; ++s) a[t][s] = S[colk[s] + 16 * ti[t]];
  }
  __builtin_amdgcn_sched_barrier(0);
  typename M::v4 acc[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    acc[t] = typename M::v4{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s) a[t][s] = (4 * s + lk < kb) ? a[t][s] : T(0);
  }
  if constexpr (NB == 1) {
    // a lone tile: four independent MFMAs summed
    typename M::v4 p1 = M::mma(a[0][1], bx[1], acc[0]);
    typename M::v4 p2 = M::mma(a[0][2], bx[2], acc[0]);
    typename M::v4 p3 = M::mma(a[0][3], bx[3], acc[0]);
    acc[0] = M::mma(a[0][0], bx[0], acc[0]);
    acc[0] = (acc[0] + p1) + (p2 + p3);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int t = 0; t < NB; ++t) acc[t] = M::mma(a[t][s], bx[s], acc[t]);
    }
  }
  T *col = S + wrap(sk + r, W) * ldb - r;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * ti[t] + M::crow(q, lane);
      if (t < cnt && r < kb && i - r <= b) col[i] = acc[t][q];
    }
  }
}

// NB tiles (ti[t], tp[t]) of the trailing update C -= L21 L21^T after panel k
// (rows and columns counted from k + kNB); slots t >= cnt repeat a valid tile
// and store nothing.  All operands are loaded first and the MFMA chains of
// the tiles are interleaved without branches: a single chain would wait out
// the full MFMA latency at every step.  Each ring column is padded with zeros
// beyond offset b up to 16*(nT+1), so operand reads outside the band or below
// the matrix need no test; colA[s] is the slot offset of panel column
// k + 4s + lane/16.  Accumulator loads clamp the offset so that the strictly
// upper half of diagonal tiles and columns past the band need no branch; only
// their stores are masked.
template <typename T, int NB>
__device__ __forceinline__ void factor_tiles(T *S, int ldb, int b, int W, int sk, int lane, const int (&ti)[NB],
                                             const int (&tp)[NB], int cnt, const int (&colA)[4]) {
  using M = Mma<T>;
  const int lr = lane & 15, lk = lane >> 4;
  typename M::v4 c[NB];
  T a[NB][4], bb[NB][4];
  int cs[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int pp = tp[t] * 16 + lr;
    cs[t] = wrap(sk + kNB + pp, W) * ldb;
#pragma unroll
    for (int v = 0; v < 4; ++v) c[t][v] = S[cs[t] + max(ti[t] * 16 + M::crow(v, lane) - pp, 0)];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a[t][s] = S[colA[s] + kNB + ti[t] * 16 + lr - (4 * s + lk)];
      bb[t][s] = S[colA[s] + kNB + pp - (4 * s + lk)];
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (NB == 1) {
    // a lone tile: four independent MFMAs summed, instead of one dependent
    // chain of four
    typename M::v4 p1 = M::mma(-a[0][1], bb[0][1], typename M::v4{T(0), T(0), T(0), T(0)});
    typename M::v4 p2 = M::mma(-a[0][2], bb[0][2], typename M::v4{T(0), T(0), T(0), T(0)});
    typename M::v4 p3 = M::mma(-a[0][3], bb[0][3], typename M::v4{T(0), T(0), T(0), T(0)});
    c[0] = M::mma(-a[0][0], bb[0][0], c[0]);
    c[0] = (c[0] + p1) + (p2 + p3);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int t = 0; t < NB; ++t) c[t] = M::mma(-a[t][s], bb[t][s], c[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int pp = tp[t] * 16 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int off = ti[t] * 16 + M::crow(v, lane) - pp;
      // the loaded accumulator of a masked entry is never stored, so it need
      // not be zero
      if (t < cnt && pp < b && (ti[t] != tp[t] || off >= 0)) S[cs[t] + off] = c[t][v];
    }
  }
}

// Coefficient of the entering column j at band offset t (kind = which of the
// offsets 0, 1, n0, b; duplicates of an earlier kind load nothing).  The
// loads are issued one iteration ahead; the value is formed when the column
// enters.
struct ColFetch {
  double c0, c1, c2, c3, s1, s2;
  int slot;
};

__device__ __forceinline__ ColFetch fetch_column_entry(const double *cf, const double *sc, int j, int t,
                                                       bool first, int N, int n0, int b) {
  ColFetch f{0.0, 0.0, 0.0, 0.0, 1.0, 1.0, -1};
  if (j < N && j + t < N && first) {
    if (t == 0) f.c0 = cf[4 * j];
    if (t == 1) f.c1 = cf[4 * j + 1];
    if (t == n0) f.c2 = cf[4 * j + 2];
    if (t == b) f.c3 = cf[4 * j + 3];
    f.s1 = sc[j];
    f.s2 = sc[j + t];
    f.slot = t;
  }
  return f;
}

template <typename T, int kMaxT, int NW>
__device__ __forceinline__ void factor_body(const SubDesc *__restrict__ subs, const int *__restrict__ order,
                                            int slot, const double *__restrict__ coef,
                                            const double *__restrict__ scal, T *__restrict__ Lg,
                                            T *__restrict__ Dg, DevStatus *st, int ldb, unsigned char *smem_raw,
                                            int &tile_ctr) {
  const int sub = order[slot];
  const SubDesc &D = subs[sub];
  const int N = D.N, b = D.b, n0 = D.n0, bp1 = b + 1;
  const int W = max(b, kNB) + kNB;
  T *S = reinterpret_cast<T *>(smem_raw);
  // X = L11^{-1} of the current and of the next panel (alternating buffers)
  T *Xbuf = S + (size_t)W * ldb;
  // spare entries for the diagonal factorisation's masked-out writes
  T *junk = Xbuf + 2 * kNB * kNB;
  // NW waves; tiles per wave in the L21 phase, and per batch of the
  // trailing update
  constexpr int NTH = 64 * NW;
  constexpr int kNBA = (kMaxT + NW) / NW;
  constexpr int kNB1 = 3;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *cf = coef + 4 * D.cell_off;
  const double *sc = scal + D.cell_off;
  T *L = Lg + D.L_off;
  T *Dinv = Dg + D.D_off;
  const int nT = (b + 15) >> 4;
  // band offsets of the four coefficient kinds: diagonal, +ax0, +ax1, +ax2
  const int pos[4] = {0, 1, n0, b};
  // entering-column work of threads 0..63: column jj = tid/4, kind tid%4
  const int ejj = (tid >> 2) & 15, ekind = tid & 3, et = pos[ekind];
  bool efirst = true;
  for (int q = 0; q < ekind; ++q) efirst = efirst && (pos[q] != et);
  int bad = 0;

  // the whole window starts at zero: padding beyond offset b stays zero
  for (int e = tid; e < W * ldb; e += NTH) S[e] = T(0);
  if (tid == 0) tile_ctr = 0;
  __syncthreads();
  // prologue: the first W columns, then panel 0
  {
    const int ncol = min(N, W);
    const int ne = ncol * bp1;
    // eight entries per thread at a time, their loads all issued (at clamped
    // addresses) before any is used, so the memory latency is paid once per
    // batch rather than once per entry
    constexpr int kPB = 8;
    for (int e0 = tid; e0 < ne; e0 += kPB * NTH) {
      double c[kPB][4], s1[kPB], s2[kPB];
#pragma unroll
      for (int q = 0; q < kPB; ++q) {
        const int e = e0 + q * NTH;
        const int j = e / bp1, t = e % bp1;
        const bool ok = e < ne && j + t < N;
        const int jj = ok ? j : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) c[q][u] = cf[4 * jj + u];
        s1[q] = sc[jj];
        s2[q] = sc[ok ? j + t : 0];
      }
#pragma unroll
      for (int q = 0; q < kPB; ++q) {
        const int e = e0 + q * NTH;
        if (e < ne) {
          const int j = e / bp1, t = e % bp1;
          double v = 0.0;
          if (j + t < N) {
            if (t == 0) v += c[q][0];
            if (t == 1) v -= c[q][1];
            if (t == n0) v -= c[q][2];
            if (t == b) v -= c[q][3];
            if (v != 0.0) v *= s1[q] * s2[q];
          }
          S[j * ldb + t] = T(v);
        }
      }
    }
  }
  ColFetch cur{0.0, 0.0, 0.0, 0.0, 1.0, 1.0, -1};
  if (tid < 64) cur = fetch_column_entry(cf, sc, W + ejj, et, efirst, N, n0, b);
  __syncthreads();
  if (wave == 0) bad |= factor_diag<T>(S, Xbuf, junk, ldb, 0, min(kNB, N), b, W, lane);
  __syncthreads();
  if (wave < nT)
    panel_l21_tiles<T, kNBA>(S, Xbuf, ldb, 0, min(kNB, N), b, W, lane, 1 + wave, NW, (nT - wave + NW - 1) / NW);
  __syncthreads();

  for (int k = 0; k < N; k += kNB) {
    const bool more = k + kNB < N;
    const int sk = k % W;
    const int kb = min(kNB, N - k);
    const int kb1 = min(kNB, N - k - kNB);
    const T *Xc = Xbuf + ((k / kNB) & 1) * (kNB * kNB);
    T *Xn = Xbuf + (((k / kNB) + 1) & 1) * (kNB * kNB);
    // coefficients of the columns entering at the end of the next iteration
    ColFetch nxt{0.0, 0.0, 0.0, 0.0, 1.0, 1.0, -1};
    if (tid < 64) nxt = fetch_column_entry(cf, sc, k + kNB + W + ejj, et, efirst, N, n0, b);
    int colA[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) colA[q] = wrap(sk + 4 * q + (lane >> 4), W) * ldb;
    // -- P1: wave 0 applies panel k to the next panel's diagonal block (tile
    // (0, 0)) and factors it; the other waves -- and wave 0 once done -- take
    // the remaining tiles of the update and the copies of panel k to global
    // memory from a shared counter
    if (wave == 0 && more) {
      // the critical path: wave 0 takes issue priority over the tile waves
      // that share its SIMD and the LDS while it runs
      __builtin_amdgcn_s_setprio(3);
      const int z[1] = {0};
      factor_tiles<T, 1>(S, ldb, b, W, sk, lane, z, z, 1, colA);
      bad |= factor_diag<T>(S, Xn, junk, ldb, k + kNB, kb1, b, W, lane);
      __builtin_amdgcn_s_setprio(0);
    }
    // With eight waves, wave 4 shares wave 0's SIMD: it takes no MFMA work in
    // this phase (the tile waves' MFMAs would hold up wave 0's chain) but the
    // copies to global memory.  With four waves the copies go round the
    // shared counter with the tiles.
    constexpr int kCopyWave = NW == 8 ? 4 : -1;
    if (wave == (kCopyWave >= 0 ? kCopyWave : NW - 1)) {
      // inverse diagonal block of panel k
      T *dst = Dinv + (size_t)(k / kNB) * (kNB * kNB);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q;
        dst[e] = ((e >> 4) < kb && (e & 15) < kb) ? Xc[e] : T(0);
      }
    }
    {
      // tiles by column: tp = 0 holds ti = 1 .. nT-1, tp >= 1 holds
      // ti = tp .. nT-1
      const int n_tiles = more ? (nT - 1) + nT * (nT - 1) / 2 : 0;
      const int n_batch = (n_tiles + kNB1 - 1) / kNB1;
      const int n_items = n_batch + (kCopyWave >= 0 ? 0 : kb);
      if (wave == kCopyWave) {
        // columns k .. k + kb - 1 of the factor to global memory
        for (int jj = 0; jj < kb; ++jj) {
          const T *col = S + wrap(sk + jj, W) * ldb;
          T *dst = L + (size_t)(k + jj) * bp1;
          for (int t = lane; t <= b; t += 64) dst[t] = col[t];
        }
      }
      for (; wave != kCopyWave;) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(&tile_ctr, 1);
        idx = __builtin_amdgcn_readfirstlane(idx);
        if (idx >= n_items) break;
        if (idx < n_batch) {
          const int f0 = idx * kNB1;
          int cp = 0, ci = f0;
          while (ci >= nT - max(cp, 1)) {
            ci -= nT - max(cp, 1);
            ++cp;
          }
          ci += max(cp, 1);
          const int ti0 = ci, tp0 = cp;
          int ti[kNB1], tp[kNB1];
#pragma unroll
          for (int t = 0; t < kNB1; ++t) {
            const bool valid = f0 + t < n_tiles;
            ti[t] = valid ? ci : ti0;
            tp[t] = valid ? cp : tp0;
            if (++ci >= nT) {
              ++cp;
              ci = cp;
            }
          }
          factor_tiles<T, kNB1>(S, ldb, b, W, sk, lane, ti, tp, min(kNB1, n_tiles - f0), colA);
        } else {
          // column k + jj of the factor to global memory
          const int jj = idx - n_batch;
          const T *col = S + wrap(sk + jj, W) * ldb;
          T *dst = L + (size_t)(k + jj) * bp1;
          for (int t = lane; t <= b; t += 64) dst[t] = col[t];
        }
      }
    }
    __syncthreads();
    // -- P2: the next panel's L21 on all waves; columns k+W .. k+W+15 take
    // the slots of panel k
    if (more && wave < nT)
      panel_l21_tiles<T, kNBA>(S, Xn, ldb, k + kNB, kb1, b, W, lane, 1 + wave, NW, (nT - wave + NW - 1) / NW);
    {
      const int j0 = k + W;
      if (j0 < N) {
        const int ncol = min(kNB, N - j0);
        constexpr int TPC = NTH / kNB;  // threads per entering column
        const int jj = tid / TPC;
        if (jj < ncol) {
          T *col = S + wrap(sk + jj, W) * ldb;
          for (int t = tid % TPC; t <= b; t += TPC) {
            if (t != 0 && t != 1 && t != n0 && t != b) col[t] = T(0);
          }
        }
        if (tid < 64 && ejj < ncol) {
          T *col = S + wrap(sk + ejj, W) * ldb;
          if (cur.slot >= 0) {
            col[cur.slot] = T((cur.c0 - cur.c1 - cur.c2 - cur.c3) * (cur.s1 * cur.s2));
          } else if (j0 + ejj + et >= N) {
            col[et] = T(0);  // entries beyond the matrix at the special offsets
          }
        }
      }
    }
    if (tid == 0) tile_ctr = 0;
    __syncthreads();
    cur = nxt;
  }
  if (bad && tid == 0) set_status(st, -3, sub, 0.0);
}

// One workgroup per subdomain.  The FP64 ring fills most of the LDS (one
// workgroup per CU), so the FP64 kernel runs eight waves: wave 0's diagonal
// block (VALU) shares its SIMD with a wave issuing MFMA tiles.  The FP32
// kernel runs four waves, held to two waves per SIMD so that two workgroups
// share a CU.
template <int kMaxT>
__global__ __launch_bounds__(512, 1) void k_factor64(const SubDesc *__restrict__ subs,
                                                     const int *__restrict__ order,
                                                     const double *__restrict__ coef,
                                                     const double *__restrict__ scal,
                                                     double *__restrict__ Lg, double *__restrict__ Dg,
                                                     DevStatus *st, int ldb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int tile_ctr;
  factor_body<double, kMaxT, 8>(subs, order, blockIdx.x, coef, scal, Lg, Dg, st, ldb, smem_raw, tile_ctr);
}
template <int kMaxT>
__global__ __launch_bounds__(256, 2) void k_factor32(const SubDesc *__restrict__ subs,
                                                     const int *__restrict__ order,
                                                     const double *__restrict__ coef,
                                                     const double *__restrict__ scal,
                                                     float *__restrict__ Lg, float *__restrict__ Dg,
                                                     DevStatus *st, int ldb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int tile_ctr;
  factor_body<float, kMaxT, 4>(subs, order, blockIdx.x, coef, scal, Lg, Dg, st, ldb, smem_raw, tile_ctr);
}

// ---------------------------------------------------------------------------
// Persistent form of a ragged launch: a fixed grid of resident workgroups
// takes the items from a device work queue, one atomic counter per XCD
// (workgroup i runs on XCD i mod 8 and takes the items 8 k + i mod 8, as the
// plain launch would place them), until the counter passes the item count.
// No workgroup waits on another; every one exits once its XCD's queue is
// empty.  The caller zeroes the eight counters on the stream first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int queue_next(int *queue, int n) {
  __shared__ int item;
  const int xcd = blockIdx.x & 7;
  __syncthreads();  // the previous item is done by every thread
  if (threadIdx.x == 0) {
    const int k = atomicAdd(queue + xcd, 1);
    item = 8 * k + xcd;
  }
  __syncthreads();
  return item < n ? item : -1;
}

__global__ void k_zero_queue(int *queue) {
  if (threadIdx.x < 8) queue[threadIdx.x] = 0;
}

template <int kMaxT>
__global__ __launch_bounds__(512, 1) void k_factor64_q(const SubDesc *__restrict__ subs,
                                                       const int *__restrict__ order, int n, int *queue,
                                                       const double *__restrict__ coef,
                                                       const double *__restrict__ scal,
                                                       double *__restrict__ Lg, double *__restrict__ Dg,
                                                       DevStatus *st, int ldb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int tile_ctr;
  for (int it = queue_next(queue, n); it >= 0; it = queue_next(queue, n))
    factor_body<double, kMaxT, 8>(subs, order, it, coef, scal, Lg, Dg, st, ldb, smem_raw, tile_ctr);
}
template <int kMaxT>
__global__ __launch_bounds__(256, 2) void k_factor32_q(const SubDesc *__restrict__ subs,
                                                       const int *__restrict__ order, int n, int *queue,
                                                       const double *__restrict__ coef,
                                                       const double *__restrict__ scal,
                                                       float *__restrict__ Lg, float *__restrict__ Dg,
                                                       DevStatus *st, int ldb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int tile_ctr;
  for (int it = queue_next(queue, n); it >= 0; it = queue_next(queue, n))
    factor_body<float, kMaxT, 4>(subs, order, it, coef, scal, Lg, Dg, st, ldb, smem_raw, tile_ctr);
}

// ---------------------------------------------------------------------------
// Multi-right-hand-side band solve with the stored factor, for one column
// chunk [c0, c1) of one subdomain per workgroup.
//   mode 0: B holds R; on exit X = s.(L L^T)^{-1}(s.R), and B holds the
//           forward-sweep values (X may be B itself);
//   mode 1: B holds a residual; X += s.(L L^T)^{-1}(s.B), B is clobbered.
// s is 1/sqrt(diag) when `scaled` (the factor is of the Jacobi-scaled matrix
// D^-1/2 A D^-1/2, which keeps the 16x16 diagonal blocks -- applied through
// their explicit inverses -- well scaled under strong permeability contrast)
// and 1 otherwise.
//
// Column-split form.  A workgroup of three waves; wave w < nct owns the
// 16-column tile w of the chunk and runs both sweeps on it alone, holding its
// band window in MFMA accumulators from panel to panel.  An accumulator tile
// is the B operand of the next product as it stands: at k-step s lane l
// supplies register s, which holds row crow(s, l) of the tile, so the A
// operand (read from LDS) is taken at that same k index and no lane exchange
// is needed.  Per 16-row panel:
//   forward:  Y1 = inv(L11) R1 from the window's first tile; R2 -= L21 Y1 on
//             the NRT tiles below it; the window moves down one tile and the
//             next rows of the right-hand sides (fetched a panel ahead)
//             enter at its end;
//   backward: Z = Y1 - L21^T X2 over the NRT solved tiles below the panel,
//             X1 = inv(L11)^T Z, and X1 enters the window.
// A chunk of 16t + 1 columns gives its last column to wave nct, which runs
// the same sweeps for that column on the vector ALUs with its window spread
// over the lanes.  The waves share only the panels of L and of the
// diagonal-block inverses, fetched into registers a panel ahead and staged
// through two LDS buffers: one barrier per panel.
// ---------------------------------------------------------------------------
constexpr int kBsWaves = 3;
constexpr int kBsThreads = 64 * kBsWaves;
constexpr int kMaxChunk = 16 * kBsWaves;
constexpr int kDStride = kNB + 1;  // LDS row stride of an inverse diagonal block (bank spread)

// R(:, c0..c1) = R0 - A^H_l X(:, c0..c1) for one work item, R0 holding the
// right-hand sides (R0 may be R itself for a single sweep): the FP64 residual
// of a refinement sweep, formed by the workgroup that then solves for the
// correction.  Matrix-free from the coefficients, kPB entries per thread at
// a time with all their loads issued first (kPB = 4 in the FP32 kernel,
// whose register budget at three workgroups per CU does not hold eight).
template <int kPB, int NT>
__device__ __forceinline__ void item_residual(const Geom &g, const int4 item, const double *__restrict__ coef,
                                              const double *Xg, const double *R0g, double *Rg) {
  const SubDesc &S = g.sub[item.x];
  const int c0 = item.y, cw = item.z - item.y;
  const int N = S.N, m = S.m, n0 = S.n0, b = S.b;
  const double *cf = coef + 4 * S.cell_off;
  const double *X = Xg + S.X_off;
  const double *R0 = R0g + S.X_off;
  double *R = Rg + S.X_off;
  const int ne = N * cw;
  for (int e0 = threadIdx.x; e0 < ne; e0 += kPB * NT) {
    double ax[kPB], rv[kPB];
#pragma unroll
    for (int q = 0; q < kPB; ++q) {
      const int e = min(e0 + q * NT, ne - 1);
      const int r = e / cw, c = c0 + e % cw;
      const size_t o = (size_t)r * m + c;
      const int rp1 = min(r + 1, N - 1), rm1 = max(r - 1, 0);
      const int rpn = min(r + n0, N - 1), rmn = max(r - n0, 0);
      const int rpb = min(r + b, N - 1), rmb = max(r - b, 0);
      double a = cf[4 * r] * X[o];
      const double t1 = cf[4 * r + 1] * X[(size_t)rp1 * m + c];
      const double t2 = cf[4 * rm1 + 1] * X[(size_t)rm1 * m + c];
      const double t3 = cf[4 * r + 2] * X[(size_t)rpn * m + c];
      const double t4 = cf[4 * rmn + 2] * X[(size_t)rmn * m + c];
      const double t5 = cf[4 * r + 3] * X[(size_t)rpb * m + c];
      const double t6 = cf[4 * rmb + 3] * X[(size_t)rmb * m + c];
      if (r + 1 < N) a -= t1;
      if (r >= 1) a -= t2;
      if (r + n0 < N) a -= t3;
      if (r >= n0) a -= t4;
      if (r + b < N) a -= t5;
      if (r >= b) a -= t6;
      ax[q] = a;
      rv[q] = R0[o];
    }
#pragma unroll
    for (int q = 0; q < kPB; ++q) {
      const int e = e0 + q * NT;
      if (e < ne) R[(size_t)(e / cw) * m + c0 + e % cw] = rv[q] - ax[q];
    }
  }
}

// NRT: most 16-row tiles of the band below a panel (b <= 16 NRT).  coef
// non-null (corrections only): form the item's FP64 residual into Bg first,
// from the right-hand sides in rhs0 (or in Bg itself when rhs0 is null).
template <typename T, int mode, int NRT>
__device__ __forceinline__ void solve_item(const Geom &g, const int4 item, const double *__restrict__ scal,
                                           const T *__restrict__ Lg, const T *__restrict__ Dg, double *Bg,
                                           double *Xg, int scaled, const double *__restrict__ coef,
                                           const double *rhs0, unsigned char *smem_raw) {
  using M = Mma<T>;
  using v4 = typename M::v4;
  // a staged panel of L is read by column: kPThr threads per column, each
  // taking rows prow + kPThr j, j < kLPer
  constexpr int kPThr = kBsThreads / kNB;
  constexpr int kLPer = (16 * NRT + 1 + kPThr - 1) / kPThr;
  // LDS column length of a staged panel: every offset a product reads,
  // 1 .. 16 NRT + 15, lies inside the column, and those past b hold zeros,
  // so that the A operands are read without masks
  constexpr int kLdl = 16 * (NRT + 1);
  constexpr int kLBuf = kNB * kLdl;
  constexpr int kWF = 16 * (NRT + 1) / 64;      // vector column: forward window rows per lane
  constexpr int kWB = (16 * NRT + 63) / 64;     // backward window rows per lane
  static_assert(16 * (NRT + 1) % 64 == 0, "the forward window spans whole waves");
  if (item.x < 0) return;
  if constexpr ((mode & 1) != 0) {
    if (coef) {
      item_residual<4, kBsThreads>(g, item, coef, Xg, rhs0 ? rhs0 : Bg, Bg);
      __syncthreads();
    }
  }
  const SubDesc &D = g.sub[item.x];
  const int c0 = item.y, cw = item.z - item.y;
  const int N = D.N, b = D.b, m = D.m, bp1 = b + 1;
  const bool vcol = (cw & 15) == 1;
  const int nct = vcol ? (cw >> 4) : ((cw + 15) >> 4);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15;
  const bool mwave = wave < nct;            // an MFMA column tile
  const bool vwave = vcol && wave == nct;   // the vector column
  const int lcol = 16 * wave + lr;          // an MFMA lane's column in the chunk
  const bool colok = mwave && lcol < cw;
  const int lsz = kNB * bp1;                // entries of one panel of L
  T *Lb = reinterpret_cast<T *>(smem_raw);  // [2][16][kLdl]: panels, column-major, zero past b
  T *Db = Lb + 2 * kLBuf;                   // [2][16][kDStride]
  const T *L = Lg + D.L_off;
  const T *Dinv = Dg + D.D_off;
  double *B = Bg + D.X_off;
  double *Xo = Xg + D.X_off;
  const double *sc = scal + D.cell_off;
  const int nP = (N + kNB - 1) / kNB;
  double *Bc = B + c0 + (colok ? lcol : 0);  // this lane's column (row stride m)
  double *Bv = B + c0 + (vwave ? 16 * nct : 0);
  double *Xc = Xo + c0 + (colok ? lcol : 0);
  double *Xv = Xo + c0 + (vwave ? 16 * nct : 0);

  // the next panel of L and of the inverses, loaded without arithmetic or
  // branches on the loaded values (masks are applied when they are stored);
  // this thread's entries are rows prow + kPThr j of column pcol, so that
  // their LDS positions follow from one base
  T lreg[kLPer], dreg[2];
  unsigned lok = 0u;
  const int pcol = tid / kPThr, prow = tid - pcol * kPThr;
  const int lsrc0 = pcol * bp1 + prow, ldst0 = pcol * kLdl + prow;
  for (int e = tid; e < 2 * kLBuf; e += kBsThreads) Lb[e] = T(0);
  auto fetch_panel = [&](int p) {
    const T *src = L + (size_t)p * lsz;
    const bool colv = pcol < N - p * kNB;  // columns past the last row stay zero
    lok = 0u;
#pragma unroll
    for (int j = 0; j < kLPer; ++j) {
      const bool ok = colv && prow + kPThr * j < bp1;
      lreg[j] = src[ok ? lsrc0 + kPThr * j : 0];
      lok |= ok ? (1u << j) : 0u;
    }
    const T *dsrc = Dinv + (size_t)p * kNB * kNB;
    dreg[0] = dsrc[tid];
    dreg[1] = dsrc[min(tid + kBsThreads, kNB * kNB - 1)];
  };
  auto store_panel = [&](int buf) {
    T *lp = Lb + buf * kLBuf;
#pragma unroll
    for (int j = 0; j < kLPer; ++j) {
      if (prow + kPThr * j < bp1) lp[ldst0 + kPThr * j] = ((lok >> j) & 1u) ? lreg[j] : T(0);
    }
    T *dp = Db + buf * (kNB * kDStride);
    // the thread index made opaque, so that the two positions are formed
    // here rather than held (and spilled) across the sweep
    int t0 = tid;
    asm volatile("" : "+v"(t0));
    dp[(t0 >> 4) * kDStride + (t0 & 15)] = dreg[0];
    const int e1 = t0 + kBsThreads;
    if (e1 < kNB * kNB) dp[(e1 >> 4) * kDStride + (e1 & 15)] = dreg[1];
  };

  // ------------------------------ forward ------------------------------
  // MFMA waves: R[0] the panel's rows, R[1 + ti] the tiles below; rows
  // 16 s + crow(v, lane) of the window in R[s][v]
  v4 R[NRT + 1];
  double nraw[4], nsc[4];
  unsigned nok = 0u;
  auto fetch_rows = [&](int r0) {
    nok = 0u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = r0 + M::crow(v, lane);
      const bool ok = colok && r < N;
      nraw[v] = Bc[(size_t)(ok ? r : 0) * m];
      nsc[v] = sc[ok ? r : 0];
      nok |= ok ? (1u << v) : 0u;
    }
  };
  auto rows_tile = [&]() {
    v4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = ((nok >> v) & 1u) ? T((scaled ? nsc[v] : 1.0) * nraw[v]) : T(0);
    return t;
  };
  // vector wave: window row lane + 64 j in vw[j]; vnew the next 16 rows
  T vw[kWF > kWB ? kWF : kWB];
  double vraw = 0.0, vscl = 1.0;
  bool vok = false;
  auto fetch_vrow = [&](int r) {  // lanes 0-15: row r + lane
    vok = lane < kNB && r + lane < N;
    vraw = Bv[(size_t)(vok ? r + lane : 0) * m];
    vscl = sc[vok ? r + lane : 0];
  };
  if (mwave) {
#pragma unroll
    for (int s = 0; s <= NRT; ++s) {
      fetch_rows(16 * s);
      R[s] = rows_tile();
    }
    fetch_rows(16 * (NRT + 1));
  }
  if (vwave) {
#pragma unroll
    for (int j = 0; j < kWF; ++j) {
      const int r = lane + 64 * j;
      vw[j] = r < N ? T((scaled ? sc[r] : 1.0) * Bv[(size_t)r * m]) : T(0);
    }
    fetch_vrow(16 * (NRT + 1));
  }
  fetch_panel(0);
  __syncthreads();  // zeroed buffers
  store_panel(0);
  for (int p = 0; p < nP; ++p) {
    const int k = p * kNB, kb = min(kNB, N - k);
    const T *lp = Lb + (p & 1) * kLBuf;
    const T *dp = Db + (p & 1) * (kNB * kDStride);
    const bool has_next = p + 1 < nP;
    __syncthreads();  // panel p staged; panel p - 1's buffer free
    // the next panel (the last panel loads itself again, unused): no branch,
    // so that the counts of loads in flight stay known to the compiler and
    // a wait for an older load does not wait for these
    fetch_panel(has_next ? p + 1 : p);
    if (mwave) {
      // Y1 = inv(L11) R1 (two chains)
      v4 ya = {T(0), T(0), T(0), T(0)}, yb = ya;
#pragma unroll
      for (int s = 0; s < 4; s += 2) {
        ya = M::mma(dp[lr * kDStride + M::crow(s, lane)], R[0][s], ya);
        yb = M::mma(dp[lr * kDStride + M::crow(s + 1, lane)], R[0][s + 1], yb);
      }
      v4 y = ya + yb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = M::crow(v, lane);
        y[v] = row < kb ? y[v] : T(0);
        if (colok && row < kb) Bc[(size_t)(k + row) * m] = (double)y[v];
      }
      // R2 -= L21 Y1: tile ti, k-step s: A = L21[16 ti + lr][crow(s, lane)].
      // Every tile of the window, without branches (tiles past the band and
      // the last panel's update, which reaches only rows past N, add zeros or
      // unused values): a branch per tile would copy the accumulator array.
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = M::crow(s, lane);
        T a[NRT];
#pragma unroll
        for (int ti = 0; ti < NRT; ++ti) {
          a[ti] = lp[kk * kLdl + 16 + 16 * ti + lr - kk];
        }
#pragma unroll
        for (int ti = 0; ti < NRT; ++ti) R[ti + 1] = M::mma(-a[ti], y[s], R[ti + 1]);
      }
      // the window moves down one tile
#pragma unroll
      for (int i = 0; i < NRT; ++i) R[i] = R[i + 1];
      R[NRT] = rows_tile();
    }
    if (vwave) {
      const int i = lane & 15;
      T y = T(0);
#pragma unroll 4
      for (int j = 0; j < kNB; ++j) y += dp[i * kDStride + j] * __shfl(vw[0], j, 64);
      if (i >= kb) y = T(0);
      if (lane < kb) Bv[(size_t)(k + lane) * m] = (double)y;
#pragma unroll 4
      for (int jj = 0; jj < kNB; ++jj) {
        const T yj = __shfl(y, jj, 64);
#pragma unroll
        for (int j = 0; j < kWF; ++j) {
          const int ii = lane + 64 * j - 16;  // row below the panel
          const int off = 16 + ii - jj;
          const T a = ii >= 0 ? lp[jj * kLdl + max(off, 0)] : T(0);
          vw[j] -= a * yj;
        }
      }
      // the window moves down 16 rows: row w takes row w + 16
      const T vnew = vok ? T((scaled ? vscl : 1.0) * vraw) : T(0);
      const int src = (lane + 16) & 63;
      T sh[kWF];
#pragma unroll
      for (int j = 0; j < kWF; ++j) sh[j] = __shfl(vw[j], src, 64);
      const T nv = __shfl(vnew, src, 64);
#pragma unroll
      for (int j = 0; j < kWF; ++j) vw[j] = lane < 48 ? sh[j] : (j + 1 < kWF ? sh[j + 1] : nv);
    }
    // The rows entering after the next panel, loaded by every wave at every
    // panel (past the end or outside the wave's columns the addresses clamp
    // and the values go unused): outside any branch, the loads stay in flight
    // across the next panel instead of being waited on where branches join.
    fetch_rows(k + kNB + 16 * (NRT + 1));
    fetch_vrow(k + kNB + 16 * (NRT + 1));
    if (has_next) store_panel((p + 1) & 1);
  }

  // ------------------------------ backward ------------------------------
  // The last panel is still staged in its buffer.  MFMA waves: X[ti] the
  // solved tile ti below the panel (rows k + 16 + 16 ti + crow(v, lane)).
  v4 X[NRT];
#pragma unroll
  for (int i = 0; i < NRT; ++i) X[i] = (v4){T(0), T(0), T(0), T(0)};
  // the forward values of a panel, loaded a panel ahead; the rows' scaling,
  // loaded at the start of the panel that stores them, so that no store
  // waits on a load (a correction adds to X with atomic adds, which return
  // nothing: one lane owns each entry, so the sum is X + s x as written)
  double yraw[4], scur[4];
  unsigned yok = 0u;
  auto fetch_y = [&](int p) {
    yok = 0u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = p * kNB + M::crow(v, lane);
      const bool ok = colok && r < N;
      yraw[v] = Bc[(size_t)(ok ? r : 0) * m];
      yok |= ok ? (1u << v) : 0u;
    }
  };
  auto fetch_sx = [&](int p) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = p * kNB + M::crow(v, lane);
      scur[v] = sc[colok && r < N ? r : 0];
    }
  };
  // vector wave: window row (below the panel) lane + 64 j in vw[j]
#pragma unroll
  for (int j = 0; j < (kWF > kWB ? kWF : kWB); ++j) vw[j] = T(0);
  double vyraw = 0.0, vscur = 1.0;
  bool vyok = false;
  auto fetch_vy = [&](int p) {
    vyok = lane < kNB && p * kNB + lane < N;
    vyraw = Bv[(size_t)(vyok ? p * kNB + lane : 0) * m];
  };
  auto fetch_vsx = [&](int p) { vscur = sc[lane < kNB && p * kNB + lane < N ? p * kNB + lane : 0]; };
  fetch_y(nP - 1);
  fetch_vy(nP - 1);
  for (int p = nP - 1; p >= 0; --p) {
    const int k = p * kNB, kb = min(kNB, N - k);
    const T *lp = Lb + (p & 1) * kLBuf;
    const T *dp = Db + (p & 1) * (kNB * kDStride);
    const bool has_prev = p > 0;
    if (p < nP - 1) __syncthreads();  // panel p staged
    fetch_panel(has_prev ? p - 1 : p);
    // this panel's forward values (prefetched), then, by every wave outside
    // any branch, the next panel's (panel 0 loads itself again at the end,
    // unused) and this panel's scaling
    v4 z0, z1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int v = 0; v < 4; ++v) z0[v] = ((yok >> v) & 1u) ? T(yraw[v]) : T(0);
    const T vycur = vyok ? T(vyraw) : T(0);
    fetch_y(max(p - 1, 0));
    fetch_vy(max(p - 1, 0));
    fetch_sx(p);
    fetch_vsx(p);
    if (mwave) {
      // Z = Y1 - L21^T X2: tile ti, k-step s: A = L[k + 16 + 16 ti + crow(s, lane)][k + lr]
#pragma unroll
      for (int ti = 0; ti < NRT; ++ti) {
        T a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          a[s] = lp[lr * kLdl + 16 + 16 * ti + M::crow(s, lane) - lr];
        }
        z0 = M::mma(-a[0], X[ti][0], z0);
        z1 = M::mma(-a[1], X[ti][1], z1);
        z0 = M::mma(-a[2], X[ti][2], z0);
        z1 = M::mma(-a[3], X[ti][3], z1);
      }
      const v4 z = z0 + z1;
      // X1 = inv(L11)^T Z (two chains)
      v4 xa = {T(0), T(0), T(0), T(0)}, xb = xa;
#pragma unroll
      for (int s = 0; s < 4; s += 2) {
        xa = M::mma(dp[M::crow(s, lane) * kDStride + lr], z[s], xa);
        xb = M::mma(dp[M::crow(s + 1, lane) * kDStride + lr], z[s + 1], xb);
      }
      v4 x = xa + xb;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = M::crow(v, lane);
        x[v] = row < kb ? x[v] : T(0);
        if (colok && row < kb) {
          const double s = scaled ? scur[v] : 1.0;
          double *dst = Xc + (size_t)(k + row) * m;
          if ((mode & 1) == 0) *dst = s * (double)x[v];
          else atomicAdd(dst, s * (double)x[v]);
        }
      }
#pragma unroll
      for (int i = NRT - 1; i > 0; --i) X[i] = X[i - 1];
      X[0] = x;
    }
    if (vwave) {
      const T ycur = vycur;
      // lanes (i, g): sum over the window rows t = g + 4 q of L[k+16+t][k+i] X2[t]
      const int i = lane & 15, gq = lane >> 4;
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < kWB; ++j) {
#pragma unroll 4
        for (int q = 0; q < 16; ++q) {
          const int tl = gq + 4 * q, t = 64 * j + tl;
          const T xt = __shfl(vw[j], tl, 64);
          // slots t >= 16 NRT lie past the window: the clamp reads a zero
          acc += lp[i * kLdl + min(16 + t - i, kLdl - 1)] * xt;
        }
      }
      acc += __shfl_xor(acc, 16, 64);
      acc += __shfl_xor(acc, 32, 64);
      const T z = ycur - acc;  // lanes 0-15
      T x = T(0);
#pragma unroll 4
      for (int j = 0; j < kNB; ++j) x += dp[j * kDStride + i] * __shfl(z, j, 64);
      if (i >= kb) x = T(0);
      if (lane < kb) {
        const double s = scaled ? vscur : 1.0;
        double *dst = Xv + (size_t)(k + lane) * m;
        if ((mode & 1) == 0) *dst = s * (double)x;
        else atomicAdd(dst, s * (double)x);
      }
      // the new rows enter at the start of the window: row t takes row t - 16
      const int src = (lane - 16) & 63;
      T sh[kWB];
#pragma unroll
      for (int j = 0; j < kWB; ++j) sh[j] = __shfl(vw[j], src, 64);
#pragma unroll
      for (int j = 0; j < kWB; ++j) vw[j] = lane >= 16 ? sh[j] : (j == 0 ? x : sh[j - 1]);
    }
    if (has_prev) store_panel((p - 1) & 1);
  }
}

// Three waves per SIMD (four workgroups per CU).
template <typename T, int mode, int NRT>
__global__ __launch_bounds__(kBsThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_solve(
    Geom g, const int4 *__restrict__ work, const double *__restrict__ scal, const T *__restrict__ Lg,
    const T *__restrict__ Dg, double *Bg, double *Xg, int scaled, const double *__restrict__ coef,
    const double *rhs0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  solve_item<T, mode, NRT>(g, work[blockIdx.x], scal, Lg, Dg, Bg, Xg, scaled, coef, rhs0, smem_raw);
}

// The same over the persistent work queue (queue_next).
template <typename T, int mode, int NRT>
__global__ __launch_bounds__(kBsThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_solve_q(
    Geom g, const int4 *__restrict__ work, int n, int *queue, const double *__restrict__ scal,
    const T *__restrict__ Lg, const T *__restrict__ Dg, double *Bg, double *Xg, int scaled,
    const double *__restrict__ coef, const double *rhs0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  for (int it = queue_next(queue, n); it >= 0; it = queue_next(queue, n))
    solve_item<T, mode, NRT>(g, work[it], scal, Lg, Dg, Bg, Xg, scaled, coef, rhs0, smem_raw);
}

// ---------------------------------------------------------------------------
// FP64 residual of all right-hand sides, Rb = R - A^H_l X, matrix-free from
// the coefficients.  Unless norms is null (a fixed number of refinement
// sweeps needs none) it accumulates per column, at norms[3 col + 0..2],
// ||Rb||^2, ||R||^2 and ||s||^2 with s_r = |R_r| + sum of |a_rj X_j| over the
// row's stencil: the componentwise bound on the rounding of Rb itself is
// gamma_8 s_r (eight terms summed), gamma_8 = 8u / (1 - 8u) with the unit
// roundoff u = 2^-53.
// ---------------------------------------------------------------------------
// Rbuf null: the norms only (a check whose next sweep forms its own residual).
// Thread t of a workgroup takes column t mod m of rows t / m, t / m + T, ...
// (T = 256 / m threads per column, the rest idle), so that its norms
// accumulate in registers and only T partial sums per column meet in LDS;
// consecutive threads read consecutive entries of a row.  The tile of the
// right-hand sides and the column sums take (kRowsPB + 3) m doubles of dynamic
// LDS, sized to the launch's largest m.
__global__ __launch_bounds__(256) void k_residual(Geom g, const double *__restrict__ coef,
                                                  const double *__restrict__ r0,
                                                  const double *__restrict__ Xg,
                                                  double *__restrict__ Rbuf,
                                                  double *__restrict__ norms, int ntile, int n_sub,
                                                  const int *__restrict__ subs) {
  extern __shared__ double tile[];
  // XCD-aware order: workgroups go round-robin to the eight XCDs, so XCD x
  // gets subdomains x, x + 8, ... with all their row tiles in sequence, and
  // the stencil's neighbour rows come from that XCD's L2
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int isub = xcd + 8 * (slot / ntile);
  if (isub >= n_sub) return;
  const SubDesc &S = g.sub[subs ? subs[isub] : isub];
  const int m = S.m, N = S.N;
  const int rbase = (slot % ntile) * kRowsPB;
  if (rbase >= N) return;
  double *red = tile + kRowsPB * m;
  const bool acc_norms = norms != nullptr;
  if (acc_norms)
    for (int i = threadIdx.x; i < 3 * m; i += blockDim.x) red[i] = 0.0;
  rhs_tile(g, S, r0, rbase, tile);
  const double *cf = coef + 4 * S.cell_off;
  const double *X = Xg + S.X_off;
  const int n0 = S.n0, b = S.b;
  const int rows = min(kRowsPB, N - rbase);
  const int tpc = blockDim.x / m, c = threadIdx.x % m, j0 = threadIdx.x / m;
  double nr = 0.0, nR = 0.0, ns = 0.0;
  if (j0 < tpc) {
    for (int j = j0; j < rows; j += tpc) {
      const int r = rbase + j;
      double t = cf[4 * r] * X[(size_t)r * m + c];
      double ax = t, ab = fabs(t);
      auto sub = [&](double v) {
        ax -= v;
        ab += fabs(v);
      };
      if (r + 1 < N) sub(cf[4 * r + 1] * X[(size_t)(r + 1) * m + c]);
      if (r >= 1) sub(cf[4 * (r - 1) + 1] * X[(size_t)(r - 1) * m + c]);
      if (r + n0 < N) sub(cf[4 * r + 2] * X[(size_t)(r + n0) * m + c]);
      if (r >= n0) sub(cf[4 * (r - n0) + 2] * X[(size_t)(r - n0) * m + c]);
      if (r + b < N) sub(cf[4 * r + 3] * X[(size_t)(r + b) * m + c]);
      if (r >= b) sub(cf[4 * (r - b) + 3] * X[(size_t)(r - b) * m + c]);
      const double rhs = tile[j * m + c];
      const double res = rhs - ax;
      if (Rbuf) Rbuf[S.X_off + (size_t)r * m + c] = res;
      ab += fabs(rhs);
      nr += res * res;
      nR += rhs * rhs;
      ns += ab * ab;
    }
  }
  if (!acc_norms) return;
  if (j0 < tpc) {
    atomicAdd(&red[3 * c], nr);
    atomicAdd(&red[3 * c + 1], nR);
    atomicAdd(&red[3 * c + 2], ns);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * m; i += blockDim.x) {
    if (red[i] != 0.0) atomicAdd(&norms[3 * (long long)S.col_off + i], red[i]);
  }
}

// Largest relative column residual sqrt(||Rb||^2 / ||R||^2) (a zero
// right-hand side counts its absolute residual): out[0] over the columns
// whose residual is above its own rounding floor, ||Rb|| > 8u ||s||
// (refinement can still reduce those), out[1] over all columns.  One
// workgroup.
__global__ __launch_bounds__(256) void k_ir_check(const double *__restrict__ norms, int ncols,
                                                  double *__restrict__ out) {
  __shared__ double red[2][256];
  constexpr double kFloor = 8.0 * 0x1.0p-53;  // gamma_8 / eps64 = 8, unit roundoff 2^-53
  double mx = 0.0, ma = 0.0;
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) {
    const double rr = norms[3 * i], RR = norms[3 * i + 1], ss = norms[3 * i + 2];
    const double v = RR > 0.0 ? sqrt(rr / RR) : sqrt(rr);
    // a non-finite residual counts as infinite, and never as at its floor
    const bool fin = v <= 1.7976931348623157e308;
    const double vv = fin ? v : INFINITY;
    ma = fmax(ma, vv);
    if (!fin || !(rr <= kFloor * kFloor * ss)) mx = fmax(mx, vv);
  }
  red[0][threadIdx.x] = mx;
  red[1][threadIdx.x] = ma;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
  }
}

// ---------------------------------------------------------------------------
// Gamma-flux blocks of one subdomain (one workgroup per subdomain):
//   F[i,col] = sum_{f in i} Q_f,  Fb[i,col] = sum_{f in i} beta_f Q_f,
//   Q_f = T_f (X[c_f, col] - G_f[col]),  SAb[i] = sum_{f in i} A_f beta_f.
// Each (patch, column) pair is reduced by one thread in a fixed order, so the
// result does not depend on scheduling.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_flux(Geom g, const double *__restrict__ Xg,
                                              double *__restrict__ F, double *__restrict__ Fb,
                                              double *__restrict__ SAb) {
  const SubDesc &S = g.sub[blockIdx.x];
  const int n = S.npatch, m = S.m;
  const double *X = Xg + S.X_off;
  for (int e = threadIdx.x; e < n * m; e += blockDim.x) {
    const int lp = e / m, c = e % m;
    int f = 0;
    for (int ff = 0; ff < 6; ++ff) {
      const int fi = S.face_if[ff];
      if (fi < 0) continue;
      const IfaceDesc &I = g.ifc[fi];
      if (lp >= S.face_p0[ff] && lp < S.face_p0[ff] + I.na * I.nb) f = ff;
    }
    const IfaceDesc &I = g.ifc[S.face_if[f]];
    const int w = lp - S.face_p0[f];
    const int pa = w % I.na, pb = w / I.na;
    const int a0 = split_start(pa, I.la, I.na), a1 = split_start(pa + 1, I.la, I.na);
    const int b0 = split_start(pb, I.lb, I.nb), b1 = split_start(pb + 1, I.lb, I.nb);
    const int d = f >> 1;
    const int sigma = (f & 1) ? 1 : -1;
    const double hd = hdir(g, d), A = adir(g, d);
    const double *kd_arr = kdir(g, d);
    const int xd = sigma < 0 ? S.lo[d] : S.lo[d] + S.ext[d] - 1;
    double sf = 0.0, sb = 0.0, sab = 0.0;
    for (int tb = b0; tb < b1; ++tb) {
      for (int ta = a0; ta < a1; ++ta) {
        I3 x{0, 0, 0};
        x.set(I.a, S.lo[I.a] + ta);
        x.set(I.b, S.lo[I.b] + tb);
        x.set(d, xd);
        const double kd = kd_arr[cell_index(g, x)];
        const double beta = robin_beta(g, S, x, f, kd);
        const double T = A / (hd / (2.0 * kd) + beta);
        const double G = (c == 1 + lp) ? 1.0 : ((c == 1 + n + lp) ? -sigma * beta : 0.0);
        const double Q = T * (X[(size_t)local_row(S, x) * m + c] - G);
        sf += Q;
        sb += beta * Q;
        sab += A * beta;
      }
    }
    F[S.F_off + (size_t)lp * m + c] = sf;
    Fb[S.F_off + (size_t)lp * m + c] = sb;
    if (c == 0) SAb[S.patch_off + lp] = sab;
  }
}

// ---------------------------------------------------------------------------
// Reconstruction by solving the local problems again (the second option the
// paper gives after the combination (2.23)): one right-hand side per
// subdomain, the particular data plus T_f G_f(pi) on every Robin face with
// G_f = pi^p - sigma beta_f pi^u, solved with the kept band factors.  The
// vectors are per subdomain, N_l rows at the subdomain's cell offset.
// ---------------------------------------------------------------------------
__global__ void k_resolve_rhs(Geom g, const double *__restrict__ r0, const double *__restrict__ pi, int nv,
                              double *__restrict__ B) {
  const SubDesc &S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.N) return;
  double v = r0[S.cell_off + r];  // zero on the pinned row
  if (r != S.pin_local) {
    const I3 x = local_to_global(S, r);
    const long long c = cell_index(g, x);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const int sigma = (f & 1) ? 1 : -1;
      const int xn = x[d] + sigma;
      if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) continue;
      int lp;
      double T, beta;
      if (gamma_face(g, S, x, f, kdir(g, d)[c], lp, T, beta)) {
        const int patch = g.ifc[S.face_if[f]].p0 + (lp - S.face_p0[f]);
        v += T * (pi[patch] - sigma * beta * pi[nv + patch]);
      }
    }
  }
  B[S.cell_off + r] = v;
}

// R = B - A X for one column per subdomain, A from the stored coefficients
// (diagonal, and the transmissibilities to the +ax0, +ax1, +ax2 neighbours,
// whose negatives are the off-diagonal entries on both sides).
__global__ void k_resolve_residual(Geom g, const double *__restrict__ coef, const double *__restrict__ B,
                                   const double *__restrict__ X, double *__restrict__ R) {
  const SubDesc &S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = S.N;
  if (r >= N) return;
  const double *cf = coef + 4 * S.cell_off;
  const double *x = X + S.cell_off;
  const int st[3] = {1, S.n0, S.b};
  double acc = cf[4 * r] * x[r];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (r + st[k] < N) acc -= cf[4 * r + 1 + k] * x[r + st[k]];
    if (r - st[k] >= 0) acc -= cf[4 * (r - st[k]) + 1 + k] * x[r - st[k]];
  }
  R[S.cell_off + r] = B[S.cell_off + r] - acc;
}

// p at the global cells from the per-subdomain solution vectors.
__global__ void k_resolve_scatter(Geom g, const double *__restrict__ X, double *__restrict__ p) {
  const SubDesc &S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.N) return;
  p[cell_index(g, local_to_global(S, r))] = X[S.cell_off + r];
}

// ---------------------------------------------------------------------------
// "Mean" post-processing of the multiscale velocity (Sec. 6, eq.
// (locprob_submean)): one Neumann problem per subdomain with a unique normal
// velocity on Gamma, the mean of the two sides' values.  Outward from cell c
// across face f towards cell n the unique value is (U[f][c] - U[f^1][n]) / 2;
// on the walls the multiscale velocity U[f][c] itself is the data.  The
// subdomain's lowest-corner cell (local row 0) is fixed at zero: its row is
// the identity, its column is removed, its neighbours keep their diagonals.
// ---------------------------------------------------------------------------
__global__ void k_mean_coef(Geom g, const double *__restrict__ U, double *__restrict__ coef,
                            double *__restrict__ B, double *__restrict__ X, double *__restrict__ scal) {
  const SubDesc &S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.N) return;
  const long long N = (long long)g.nx * g.ny * g.nz;
  const I3 x = local_to_global(S, r);
  const long long c = cell_index(g, x);
  const double kc0 = g.k[0][c], kc1 = g.k[1][c], kc2 = g.k[2][c];
  const int a0 = S.ax[0], a1 = S.ax[1];
  double diag = 0.0, rhs = g.q[c];
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const double kd = d == 0 ? kc0 : (d == 1 ? kc1 : kc2);
    const int xn = x[d] + side;
    const double hd = hdir(g, d), ad = adir(g, d);
    I3 y = x;
    y.set(d, xn);
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) {
      const double kn = kdir(g, d)[cell_index(g, y)];
      const double T = ad * (2.0 * kd * kn / (kd + kn)) / hd;
      diag += T;
      if (side > 0) {
        const int p = (d == a0) ? 0 : ((d == a1) ? 1 : 2);
        t0 = (p == 0) ? T : t0;
        t1 = (p == 1) ? T : t1;
        t2 = (p == 2) ? T : t2;
      }
    } else if (xn >= 0 && xn < ndir(g, d)) {
      rhs -= ad * 0.5 * (U[f * N + c] - U[(f ^ 1) * N + cell_index(g, y)]);
    } else {
      rhs -= ad * U[f * N + c];
    }
  }
  if (r == 0) {
    diag = 1.0;
    t0 = t1 = t2 = 0.0;
    rhs = 0.0;
  }
  const long long o = S.cell_off + r;
  coef[4 * o + 0] = diag;
  coef[4 * o + 1] = t0;
  coef[4 * o + 2] = t1;
  coef[4 * o + 3] = t2;
  B[o] = rhs;
  X[o] = rhs;
  scal[o] = 1.0 / sqrt(diag);
}

// The post-processed pressure pt and velocity Ut per global cell: faces
// inside the cell's subdomain from the Neumann solution P (per subdomain, at
// its cell offset), Gamma faces from the two sides' mean, walls from U.
__global__ void k_mean_velocity(Geom g, const double *__restrict__ U, const double *__restrict__ P,
                                double *__restrict__ pt, double *__restrict__ Ut) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  I3 x;
  x.v0 = (int)(c % g.nx);
  x.v1 = (int)((c / g.nx) % g.ny);
  x.v2 = (int)(c / ((long long)g.nx * g.ny));
  const int l = g.sub_of[0][x.v0] + g.nd[0] * (g.sub_of[1][x.v1] + g.nd[1] * g.sub_of[2][x.v2]);
  const SubDesc &S = g.sub[l];
  const double *Pl = P + S.cell_off;
  const double pc = Pl[local_row(S, x)];
  pt[c] = pc;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const int xn = x[d] + side;
    I3 y = x;
    y.set(d, xn);
    double u;
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) {
      const double *karr = kdir(g, d);
      const double kd = karr[c], kn = karr[cell_index(g, y)];
      u = (2.0 * kd * kn / (kd + kn)) * (pc - Pl[local_row(S, y)]) / hdir(g, d);
    } else if (xn >= 0 && xn < ndir(g, d)) {
      u = 0.5 * (U[f * N + c] - U[(f ^ 1) * N + cell_index(g, y)]);
    } else {
      u = U[f * N + c];
    }
    Ut[f * N + c] = u;
  }
}

}  // namespace mrcm

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace mrcm {

__global__ void k_reset_status(DevStatus *st) {
  if (threadIdx.x == 0) {
    st->code = 0;
    st->where = 0;
    st->value = 0.0;
  }
}

hipError_t launch_reset_status(DevStatus *st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_status, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_check_perm(const double *kx, const double *ky, const double *kz, long long n,
                             DevStatus *st, hipStream_t s) {
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_check_perm, dim3((unsigned)blocks), dim3(256), 0, s, kx, ky, kz, n, st);
  return hipGetLastError();
}

hipError_t launch_coef(const Geom &g, int n_sub, int max_cells, double *coef, double *r0,
                       double *scal, hipStream_t s) {
  dim3 grid((max_cells + 255) / 256, n_sub);
  hipLaunchKernelGGL(k_coef, grid, dim3(256), 0, s, g, coef, r0, scal);
  return hipGetLastError();
}

// Column stride of the factor's LDS ring: room for offsets up to 16*(nT+1)
// (nT = ceil(b/16) tiles), odd to spread LDS banks.
// Ring column stride: at least 16*(nT+1) entries, and chosen so that the
// MFMA operand and accumulator accesses of a trailing-update tile spread over
// the LDS banks (the offsets were picked by counting bank collisions).
int factor_ldb(int fp32, int bmax) { return 16 * ((bmax + 15) / 16) + (fp32 ? 26 : 19); }

size_t factor_lds_bytes(int fp32, int bmax) {
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  return ((size_t)(std::max(bmax, kNB) + kNB) * factor_ldb(fp32, bmax) + 2 * kNB * kNB + kNB) * es;
}

// Column stride of the solve's panel buffers: operand offsets reach b + 31.
size_t solve_lds_bytes(int fp32, int bmax, int mmax) {
  (void)mmax;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  const int nrt = bmax <= 112 ? 7 : (kMaxBand32 + 15) / 16;
  return (2 * (size_t)kNB * 16 * (nrt + 1) + 2 * (size_t)kNB * kDStride) * es;
}

int solve_chunk_max() { return kMaxChunk; }

// Compute units of the current device (the persistent grids' size).
static int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess)
    return 0;
  return n;
}

// Resident workgroups of a kernel on one CU at the given LDS.
static int blocks_per_cu(const void *k, int threads, size_t lds) {
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, threads, lds) != hipSuccess) return 0;
  return nb;
}

// A persistent grid: every CU full, a multiple of 8 workgroups (one queue per
// XCD), and no more workgroups than items (rounded up to a multiple of 8).
static int persistent_grid(const void *k, int threads, size_t lds, int n_items) {
  const int g = device_cus() * std::max(1, blocks_per_cu(k, threads, lds));
  return std::max(8, std::min(g, ((n_items + 7) / 8) * 8) / 8 * 8);
}

// kMaxT: most tiles in one tile column of the trailing update, nT - 1
template <typename T, typename K, typename KQ>
static hipError_t launch_factor_t(K kern, KQ kern_q, int threads, const SubDesc *subs, const int *order, int n_sub,
                                  const double *coef, const double *scal, T *L, T *Dg,
                                  DevStatus *st, int bmax, hipStream_t s, int *queue) {
  const int fp32 = sizeof(T) == 4;
  const size_t lds = factor_lds_bytes(fp32, bmax);
  if (n_sub <= 0) return hipSuccess;
  if (queue) {
    hipError_t e = hipFuncSetAttribute((const void *)kern_q, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, queue);
    const int grid = persistent_grid((const void *)kern_q, threads, lds, n_sub);
    hipLaunchKernelGGL(kern_q, dim3(grid), dim3(threads), lds, s, subs, order, n_sub, queue, coef, scal, L, Dg, st,
                       factor_ldb(fp32, bmax));
    return hipGetLastError();
  }
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_sub), dim3(threads), lds, s, subs, order, coef, scal, L, Dg, st,
                     factor_ldb(fp32, bmax));
  return hipGetLastError();
}

hipError_t launch_factor(int fp32, const SubDesc *subs, const int *order, int n_sub,
                         const double *coef, const double *scal, void *L, void *Dg, DevStatus *st,
                         int bmax, hipStream_t s, int *queue) {
  const int nT = (bmax + 15) / 16;
  if (fp32) {
    if (nT <= 7)
      return launch_factor_t(k_factor32<6>, k_factor32_q<6>, 256, subs, order, n_sub, coef, scal, (float *)L,
                             (float *)Dg, st, bmax, s, queue);
    return launch_factor_t(k_factor32<(kMaxBand32 + 15) / 16 - 1>, k_factor32_q<(kMaxBand32 + 15) / 16 - 1>, 256,
                           subs, order, n_sub, coef, scal, (float *)L, (float *)Dg, st, bmax, s, queue);
  }
  return launch_factor_t(k_factor64<(kMaxBand64 + 15) / 16 - 1>, k_factor64_q<(kMaxBand64 + 15) / 16 - 1>, 512,
                         subs, order, n_sub, coef, scal, (double *)L, (double *)Dg, st, bmax, s, queue);
}

template <typename T, int mode, int NRT>
static hipError_t launch_solve_t(const Geom &g, const int4 *work, int n_work, const double *scal,
                                 const T *L, const T *Dg, double *B, double *X, int bmax, int scaled,
                                 hipStream_t s, const double *coef, const double *rhs0, int *queue) {
  const size_t lds = solve_lds_bytes(sizeof(T) == 4, bmax, 0);
  if (n_work <= 0) return hipSuccess;
  if (queue) {
    const void *kq = (const void *)k_solve_q<T, mode, NRT>;
    hipError_t e = hipFuncSetAttribute(kq, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, s, queue);
    const int grid = persistent_grid(kq, kBsThreads, lds, n_work);
    hipLaunchKernelGGL((k_solve_q<T, mode, NRT>), dim3(grid), dim3(kBsThreads), lds, s, g, work, n_work, queue,
                       scal, L, Dg, B, X, scaled, coef, rhs0);
    return hipGetLastError();
  }
  hipError_t e = hipFuncSetAttribute((const void *)k_solve<T, mode, NRT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve<T, mode, NRT>), dim3(n_work), dim3(kBsThreads), lds, s, g, work, scal, L, Dg, B,
                     X, scaled, coef, rhs0);
  return hipGetLastError();
}

// NRT = 7 serves bands up to 112 (FP64, and FP32 up to there); FP32 takes
// bands up to 176 with NRT = 11.
template <typename T, int mode>
static hipError_t launch_solve_m(const Geom &g, const int4 *work, int n_work, const double *scal,
                                 const T *L, const T *Dg, double *B, double *X, int bmax, hipStream_t s,
                                 const double *coef, const double *rhs0, int *queue) {
  if (bmax <= 112)
    return launch_solve_t<T, mode, 7>(g, work, n_work, scal, L, Dg, B, X, bmax, 1, s, coef, rhs0, queue);
  if constexpr (sizeof(T) == 4)
    return launch_solve_t<T, mode, (kMaxBand32 + 15) / 16>(g, work, n_work, scal, L, Dg, B, X, bmax, 1, s, coef,
                                                             rhs0, queue);
  return hipErrorInvalidValue;
}

hipError_t launch_solve(int fp32, const Geom &g, const int4 *work, int n_work, const double *scal,
                        const void *L, const void *Dg, double *B, double *X, int mode, int bmax,
                        hipStream_t s, const double *coef, const double *rhs0, int *queue) {
  // Separate instantiations per mode, so that profiles tell them apart: bit 0
  // set for a correction (X += ...), bit 1 set for the second group of work
  // items when the first solve is split.
  if (fp32) {
    const float *Lf = (const float *)L, *Df = (const float *)Dg;
    switch (mode) {
      case 0: return launch_solve_m<float, 0>(g, work, n_work, scal, Lf, Df, B, X, bmax, s, coef, rhs0, queue);
      case 1: return launch_solve_m<float, 1>(g, work, n_work, scal, Lf, Df, B, X, bmax, s, coef, rhs0, queue);
      case 2: return launch_solve_m<float, 2>(g, work, n_work, scal, Lf, Df, B, X, bmax, s, coef, rhs0, queue);
      default: return launch_solve_m<float, 3>(g, work, n_work, scal, Lf, Df, B, X, bmax, s, coef, rhs0, queue);
    }
  }
  const double *Ld = (const double *)L, *Dd = (const double *)Dg;
  switch (mode) {
    case 0: return launch_solve_m<double, 0>(g, work, n_work, scal, Ld, Dd, B, X, bmax, s, coef, rhs0, queue);
    case 1: return launch_solve_m<double, 1>(g, work, n_work, scal, Ld, Dd, B, X, bmax, s, coef, rhs0, queue);
    case 2: return launch_solve_m<double, 2>(g, work, n_work, scal, Ld, Dd, B, X, bmax, s, coef, rhs0, queue);
    default: return launch_solve_m<double, 3>(g, work, n_work, scal, Ld, Dd, B, X, bmax, s, coef, rhs0, queue);
  }
}

// Workgroups of the FP64 factorisation that one CU holds at once.
int factor64_blocks_per_cu(int bmax) {
  const size_t lds = factor_lds_bytes(0, bmax);
  const void *k = (const void *)k_factor64<(kMaxBand64 + 15) / 16 - 1>;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 512, lds) != hipSuccess) return 0;
  return nb;
}

// Workgroups of the FP32 factorisation that one CU holds at once.
int factor32_blocks_per_cu(int bmax) {
  const size_t lds = factor_lds_bytes(1, bmax);
  const void *k = ((bmax + 15) / 16 <= 7) ? (const void *)k_factor32<6>
                                           : (const void *)k_factor32<(kMaxBand32 + 15) / 16 - 1>;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, lds) != hipSuccess) return 0;
  return nb;
}

// Workgroups of the solve that one CU holds at once.
int solve_blocks_per_cu(int fp32, int bmax) {
  const size_t lds = solve_lds_bytes(fp32, bmax, 0);
  const void *k = fp32 ? (bmax <= 112 ? (const void *)k_solve<float, 0, 7>
                                      : (const void *)k_solve<float, 0, (kMaxBand32 + 15) / 16>)
                       : (const void *)k_solve<double, 0, 7>;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBsThreads, lds) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_rhs(const Geom &g, int n_sub, int max_cells, int mmax, const double *r0, double *B,
                      hipStream_t s, double *B2) {
  dim3 grid((unsigned)((max_cells + kRowsPB - 1) / kRowsPB), n_sub);
  const size_t lds = (size_t)kRowsPB * mmax * sizeof(double);
  hipLaunchKernelGGL(k_rhs, grid, dim3(256), lds, s, g, r0, B, B2);
  return hipGetLastError();
}

hipError_t launch_residual(const Geom &g, int n_sub, int max_cells, int mmax, const double *coef,
                           const double *r0, const double *X, double *R, double *norms,
                           hipStream_t s, const int *subs) {
  const int ntile = (max_cells + kRowsPB - 1) / kRowsPB;
  const long long nblk = 8LL * ntile * ((n_sub + 7) / 8);
  const size_t lds = (size_t)(kRowsPB + 3) * mmax * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_residual, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)nblk), dim3(256), lds, s, g, coef, r0, X, R, norms, ntile, n_sub,
                     subs);
  return hipGetLastError();
}

hipError_t launch_ir_check(const double *norms, int ncols, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(256), 0, s, norms, ncols, out);
  return hipGetLastError();
}

hipError_t launch_flux(const Geom &g, int n_sub, const double *X, double *F, double *Fb,
                       double *SAb, hipStream_t s) {
  hipLaunchKernelGGL(k_flux, dim3(n_sub), dim3(256), 0, s, g, X, F, Fb, SAb);
  return hipGetLastError();
}

hipError_t launch_resolve_rhs(const Geom &g, int n_sub, int max_cells, const double *r0, const double *pi, int nv,
                              double *B, hipStream_t s) {
  dim3 grid((max_cells + 255) / 256, n_sub);
  hipLaunchKernelGGL(k_resolve_rhs, grid, dim3(256), 0, s, g, r0, pi, nv, B);
  return hipGetLastError();
}

hipError_t launch_resolve_residual(const Geom &g, int n_sub, int max_cells, const double *coef, const double *B,
                                   const double *X, double *R, hipStream_t s) {
  dim3 grid((max_cells + 255) / 256, n_sub);
  hipLaunchKernelGGL(k_resolve_residual, grid, dim3(256), 0, s, g, coef, B, X, R);
  return hipGetLastError();
}

hipError_t launch_resolve_scatter(const Geom &g, int n_sub, int max_cells, const double *X, double *p,
                                  hipStream_t s) {
  dim3 grid((max_cells + 255) / 256, n_sub);
  hipLaunchKernelGGL(k_resolve_scatter, grid, dim3(256), 0, s, g, X, p);
  return hipGetLastError();
}

hipError_t launch_mean_coef(const Geom &g, int n_sub, int max_cells, const double *U, double *coef, double *B,
                            double *X, double *scal, hipStream_t s) {
  dim3 grid((max_cells + 255) / 256, n_sub);
  hipLaunchKernelGGL(k_mean_coef, grid, dim3(256), 0, s, g, U, coef, B, X, scal);
  return hipGetLastError();
}

hipError_t launch_mean_velocity(const Geom &g, const double *U, const double *P, double *pt, double *Ut,
                                hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_mean_velocity, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, U, P, pt, Ut);
  return hipGetLastError();
}

}  // namespace mrcm
