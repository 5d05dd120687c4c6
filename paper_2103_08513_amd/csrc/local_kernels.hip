// Loop 1 of the MRCM (Algorithm 2) on gfx950: per-subdomain coefficients,
// band Cholesky of the local matrix A^H_l, the 2|I^l|+1 band solves of
// (2.25)/(2.26), the FP64 residual used by mixed-precision refinement, and
// the reduction of the MBF fluxes over each patch.
//
// One workgroup (256 lanes, four wave64s) owns one subdomain.  The local rows
// are ordered with the box's shortest axis fastest, so the lower bandwidth is
// b = n0*n1 and the factor of a 20x20x5 block has b = 100.
#include <hip/hip_runtime.h>

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
  const SubDesc S = g.sub[blockIdx.y];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= S.N) return;
  int x[3];
  local_to_global(S, r, x);
  const long long c = cell_index(g, x);
  const double kc[3] = {g.k[0][c], g.k[1][c], g.k[2][c]};
  int pos[3];
  pos[S.ax[0]] = 0;
  pos[S.ax[1]] = 1;
  pos[S.ax[2]] = 2;
  const int n[3] = {g.nx, g.ny, g.nz};
  double diag = 0.0, rhs = g.q[c];
  double toff[3] = {0.0, 0.0, 0.0};
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int side = (f & 1) ? 1 : -1;
    const int xn = x[d] + side;
    if (xn >= S.lo[d] && xn < S.lo[d] + S.ext[d]) {
      int y[3] = {x[0], x[1], x[2]};
      y[d] = xn;
      const long long cn = cell_index(g, y);
      const double kn = g.k[d][cn];
      const double T = g.area[d] * (2.0 * kc[d] * kn / (kc[d] + kn)) / g.h[d];
      diag += T;
      if (side > 0) toff[pos[d]] = (cn == g.pin) ? 0.0 : T;
    } else if (xn >= 0 && xn < n[d]) {
      const double beta = g.alpha * (S.ext[d] * g.h[d]) / kc[d];
      diag += g.area[d] / (g.h[d] / (2.0 * kc[d]) + beta);
    } else {
      const int wt = g.wall_type[f];
      if (wt != 0) {
        const int a = (d == 0) ? 1 : 0;
        const int b = (d == 2) ? 1 : 2;
        const double gv = g.wall_value[f] ? g.wall_value[f][x[a] + (long long)n[a] * x[b]] : 0.0;
        if (wt == 1) {
          const double T = g.area[d] * 2.0 * kc[d] / g.h[d];
          diag += T;
          rhs += T * gv;
        } else {
          rhs -= g.area[d] * gv;
        }
      }
    }
  }
  if (c == g.pin) {
    diag = 1.0;
    toff[0] = toff[1] = toff[2] = 0.0;
    rhs = 0.0;
  }
  const long long o = S.cell_off + r;
  coef[4 * o + 0] = diag;
  coef[4 * o + 1] = toff[0];
  coef[4 * o + 2] = toff[1];
  coef[4 * o + 3] = toff[2];
  r0[o] = rhs;
  scal[o] = 1.0 / sqrt(diag);
}

// ---------------------------------------------------------------------------
// Band Cholesky.  The active part of the band -- the current panel of kNB
// columns and the b columns it updates -- lives in LDS as a ring of
// W = b + kNB column slots, each holding the b+1 entries L[j..j+b][j].
// Columns are assembled straight from the coefficients when they enter the
// ring, so A^H_l never exists in global memory.
//   panel:    wave 0 keeps the panel's rows in registers (row k+lane+64q in
//             lane `lane`), factors it with lane broadcasts instead of
//             workgroup barriers, and forms the inverse of the 16x16
//             diagonal block.
//   update:   all four waves subtract L21 L21^T from the b x b lower
//             triangle that follows the panel, in 16x16 MFMA tiles.
// The factor is written by column, (b+1) entries per column; the inverses of
// its 16x16 diagonal blocks (what the solves use) go to a separate array.
// ---------------------------------------------------------------------------
template <typename T, int RPL>
__device__ __forceinline__ void factor_panel(T *S, T *L, T *Dinv, int ldb, int k, int kb, int N, int b,
                                             int W, int lane, DevStatus *st, int sub) {
  T v[RPL][kNB];
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int ri = lane + 64 * q;
#pragma unroll
    for (int jj = 0; jj < kNB; ++jj) {
      const int t = ri - jj;
      v[q][jj] = (jj < kb && t >= 0 && t <= b && k + ri < N) ? S[((k + jj) % W) * ldb + t] : T(0);
    }
  }
#pragma unroll
  for (int jj = 0; jj < kNB; ++jj) {
    if (jj < kb) {
      T d2 = lane_bcast(v[0][jj], jj);
      if (!(d2 > T(0))) {
        if (lane == 0) set_status(st, -3, sub, (double)d2);
        d2 = T(1);
      }
      const T d = sqrt(d2);
      const T inv = T(1) / d;
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int ri = lane + 64 * q;
        if (ri > jj) v[q][jj] *= inv;
        else if (ri == jj) v[q][jj] = d;
      }
#pragma unroll
      for (int pp = jj + 1; pp < kNB; ++pp) {
        if (pp < kb) {
          const T lpj = lane_bcast(v[0][jj], pp);
#pragma unroll
          for (int q = 0; q < RPL; ++q) {
            const int ri = lane + 64 * q;
            if (ri >= pp) v[q][pp] -= v[q][jj] * lpj;
          }
        }
      }
    }
  }
  // Inverse of the diagonal block: lane r < kb ends with row r of L11^{-1}.
  T xi[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) xi[c] = (c == lane) ? T(1) : T(0);
#pragma unroll
  for (int p = 0; p < kNB; ++p) {
    if (p < kb) {
      if (lane == p) {
        const T dinv = T(1) / v[0][p];
#pragma unroll
        for (int c = 0; c <= p; ++c) xi[c] *= dinv;
      }
#pragma unroll
      for (int c = 0; c <= p; ++c) {
        const T xpc = lane_bcast(xi[c], p);
        if (lane > p) xi[c] -= v[0][p] * xpc;
      }
    }
  }
  if (lane < kNB) {
    T *dst = Dinv + (size_t)(k / kNB) * (kNB * kNB) + lane * kNB;
#pragma unroll
    for (int c = 0; c < kNB; ++c) dst[c] = (lane < kb && c < kb) ? xi[c] : T(0);
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int ri = lane + 64 * q;
#pragma unroll
    for (int jj = 0; jj < kNB; ++jj) {
      const int t = ri - jj;
      if (jj < kb && t >= 0 && t <= b) {
        const T val = (k + ri < N) ? v[q][jj] : T(0);
        L[(size_t)(k + jj) * (b + 1) + t] = val;
        if (ri >= kb) S[((k + jj) % W) * ldb + t] = val;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void factor_update(T *S, int ldb, int k, int kb, int N, int b, int W,
                                              int lane, int wave) {
  using M = Mma<T>;
  const int nT = (b + 15) >> 4;
  const int lr = lane & 15, lk = lane >> 4;
  const int base = k + kb;
  int tile = 0;
  for (int ti = 0; ti < nT; ++ti) {
    for (int tp = 0; tp <= ti; ++tp, ++tile) {
      if ((tile & 3) != wave) continue;
      typename M::v4 c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = ti * 16 + M::crow(v, lane), pp = tp * 16 + lr;
        const bool ok = ii >= pp && ii < b && base + ii < N;
        c[v] = ok ? S[((base + pp) % W) * ldb + (ii - pp)] : T(0);
      }
#pragma unroll
      for (int s = 0; s < kNB / 4; ++s) {
        const int jj = 4 * s + lk;
        const int ia = ti * 16 + lr, ib = tp * 16 + lr;
        const int ta = kb + ia - jj, tb = kb + ib - jj;
        const T a = (jj < kb && ta <= b && base + ia < N) ? S[((k + jj) % W) * ldb + ta] : T(0);
        const T bb = (jj < kb && tb <= b && base + ib < N) ? S[((k + jj) % W) * ldb + tb] : T(0);
        c = M::mma(-a, bb, c);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ii = ti * 16 + M::crow(v, lane), pp = tp * 16 + lr;
        if (ii >= pp && ii < b && base + ii < N) S[((base + pp) % W) * ldb + (ii - pp)] = c[v];
      }
    }
  }
}

template <typename T, int RPL>
__global__ __launch_bounds__(256) void k_factor(const SubDesc *__restrict__ subs,
                                                const int *__restrict__ order,
                                                const double *__restrict__ coef,
                                                const double *__restrict__ scal,
                                                T *__restrict__ Lg, T *__restrict__ Dg,
                                                DevStatus *st, int ldb, int scaled) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *S = reinterpret_cast<T *>(smem_raw);
  const int sub = order[blockIdx.x];
  const SubDesc D = subs[sub];
  const int N = D.N, b = D.b, n0 = D.n0, W = b + kNB, bp1 = b + 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double *cf = coef + 4 * D.cell_off;
  const double *sc = scal + D.cell_off;
  T *L = Lg + D.L_off;
  T *Dinv = Dg + D.D_off;

  auto load_cols = [&](int j0, int j1) {
    const int cnt = (j1 - j0) * bp1;
    for (int e = tid; e < cnt; e += 256) {
      const int j = j0 + e / bp1, t = e % bp1;
      double v = 0.0;
      if (j + t < N) {
        if (t == 0) v += cf[4 * j];
        if (t == 1) v -= cf[4 * j + 1];
        if (t == n0) v -= cf[4 * j + 2];
        if (t == b) v -= cf[4 * j + 3];
        if (scaled && v != 0.0) v *= sc[j] * sc[j + t];
      }
      S[(j % W) * ldb + t] = T(v);
    }
  };

  load_cols(0, min(N, W));
  __syncthreads();
  for (int k = 0; k < N; k += kNB) {
    const int kb = min(kNB, N - k);
    if (wave == 0) factor_panel<T, RPL>(S, L, Dinv, ldb, k, kb, N, b, W, lane, st, sub);
    __syncthreads();
    if (k + kb < N) factor_update<T>(S, ldb, k, kb, N, b, W, lane, wave);
    __syncthreads();
    const int j0 = k + W;
    if (j0 < N) load_cols(j0, min(N, j0 + kb));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Right-hand sides of one local row (mode 0): column 0 the particular problem,
// column 1+j the P-type MBF of local patch j (G = 1 on the patch), column
// 1+n+j the U-type MBF (G = -sigma beta_f); entry = T_f G_f per Robin face.
// Calls emit(col, value) for each nonzero of the row; the pinned row is zero.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ void rhs_row_faces(const Geom &g, const SubDesc &S, int r, F emit) {
  if (r == S.pin_local) return;
  int x[3];
  local_to_global(S, r, x);
  const long long c = cell_index(g, x);
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1;
    const int sigma = (f & 1) ? 1 : -1;
    int lp;
    double T, beta;
    if (gamma_face(g, S, x, f, g.k[d][c], lp, T, beta)) {
      emit(1 + lp, T);
      emit(1 + S.npatch + lp, -sigma * beta * T);
    }
  }
}

// ---------------------------------------------------------------------------
// Multi-right-hand-side band solve with the stored factor.
//   mode 0: right-hand sides built on the fly; X = s.(L L^T)^{-1}(s.R).
//   mode 1: right-hand sides read from Rbuf (an FP64 residual);
//           X += s.(L L^T)^{-1}(s.Rbuf).  Rbuf is overwritten.
// s is 1/sqrt(diag) when `scaled` (the FP32 factor is of the Jacobi-scaled
// matrix) and 1 otherwise.  Forward sweep: a ring of W = b + kNB rows of the
// m (padded to MP) columns in LDS; per panel Y1 = inv(L11) R1 and
// R2 -= L21 Y1 as MFMA tiles.  Backward sweep: X1 = inv(L11)^T (Y1 - L21^T X2).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_solve(Geom g, const int *__restrict__ order,
                                               const double *__restrict__ r0,
                                               const double *__restrict__ scal,
                                               const T *__restrict__ Lg, const T *__restrict__ Dg,
                                               double *__restrict__ Xg,
                                               double *__restrict__ Rbuf, int mode, int scaled,
                                               int ldb, int wmax, int mpmax) {
  using M = Mma<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const SubDesc D = g.sub[order[blockIdx.x]];
  const int N = D.N, b = D.b, m = D.m, W = b + kNB, bp1 = b + 1;
  const int MP = (m + 15) & ~15;
  const int nct = MP >> 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  T *Lp = reinterpret_cast<T *>(smem_raw);  // [kNB][ldb]
  T *Dp = Lp + kNB * ldb;                    // [kNB][kNB] inverse of the diagonal block
  T *Y = Dp + kNB * kNB;                     // [wmax][mpmax] ring (stride MP)
  T *Zs = Y + (size_t)wmax * mpmax;          // [16][mpmax]
  const T *L = Lg + D.L_off;
  const T *Dinv = Dg + D.D_off;
  double *X = Xg + D.X_off;
  double *Rb = Rbuf ? Rbuf + D.X_off : nullptr;
  double *Ybuf = (mode == 0) ? X : Rb;
  const double *sc = scal + D.cell_off;

  auto slot = [&](int r) { return (r % W) * MP; };

  auto build_rows = [&](int ra, int rb) {
    const int cnt = (rb - ra) * MP;
    for (int e = tid; e < cnt; e += 256) Y[slot(ra + e / MP) + e % MP] = T(0);
    __syncthreads();
    if (mode == 0) {
      for (int e = tid; e < (rb - ra) * 2; e += 256) {
        const int r = ra + (e >> 1);
        if (r >= N) continue;
        const double s = scaled ? sc[r] : 1.0;
        T *row = Y + slot(r);
        if ((e & 1) == 0) {
          row[0] = T(s * r0[D.cell_off + r]);
        } else {
          rhs_row_faces(g, D, r, [&](int col, double v) { row[col] = T(s * v); });
        }
      }
    } else {
      const int cnt2 = (rb - ra) * m;
      for (int e = tid; e < cnt2; e += 256) {
        const int r = ra + e / m, c = e % m;
        if (r >= N) continue;
        const double s = scaled ? sc[r] : 1.0;
        Y[slot(r) + c] = T(s * Rb[(size_t)r * m + c]);
      }
    }
    __syncthreads();
  };

  auto load_panel = [&](int k, int kb) {
    for (int e = tid; e < kNB * bp1; e += 256) {
      const int jj = e / bp1, t = e % bp1;
      Lp[jj * ldb + t] = (jj < kb) ? L[(size_t)(k + jj) * bp1 + t] : T(0);
    }
    Dp[tid] = Dinv[(size_t)(k / kNB) * (kNB * kNB) + tid];
  };

  // ------------------------------ forward ------------------------------
  build_rows(0, min(N, W));
  for (int k = 0; k < N; k += kNB) {
    const int kb = min(kNB, N - k);
    load_panel(k, kb);
    __syncthreads();
    typename M::v4 acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ct = wave + 4 * i;
      acc[i] = typename M::v4{0, 0, 0, 0};
      if (ct < nct) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int jj = 4 * s + lk;
          const T a = Dp[lr * kNB + jj];
          const T bb = (jj < kb) ? Y[slot(k + jj) + ct * 16 + lr] : T(0);
          acc[i] = M::mma(a, bb, acc[i]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ct = wave + 4 * i;
      if (ct < nct) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = M::crow(v, lane), col = ct * 16 + lr;
          if (row < kb) {
            Y[slot(k + row) + col] = acc[i][v];
            if (col < m) Ybuf[(size_t)(k + row) * m + col] = (double)acc[i][v];
          }
        }
      }
    }
    __syncthreads();
    if (k + kb < N) {
      const int nrt = (b + 15) >> 4;
      for (int tile = wave; tile < nrt * nct; tile += 4) {
        const int ti = tile / nct, ct = tile % nct;
        typename M::v4 c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = ti * 16 + M::crow(v, lane);
          const bool ok = ii < b && k + kb + ii < N;
          c[v] = ok ? Y[slot(k + kb + ii) + ct * 16 + lr] : T(0);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int jj = 4 * s + lk;
          const int ia = ti * 16 + lr;
          const int ta = kb + ia - jj;
          const T a = (jj < kb && ta <= b && k + kb + ia < N) ? Lp[jj * ldb + ta] : T(0);
          const T bb = (jj < kb) ? Y[slot(k + jj) + ct * 16 + lr] : T(0);
          c = M::mma(-a, bb, c);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = ti * 16 + M::crow(v, lane);
          if (ii < b && k + kb + ii < N) Y[slot(k + kb + ii) + ct * 16 + lr] = c[v];
        }
      }
    }
    __syncthreads();
    if (k + W < N) build_rows(k + W, min(N, k + W + kb));
  }

  // ------------------------------ backward ------------------------------
  for (int e = tid; e < W * MP; e += 256) Y[e] = T(0);
  __syncthreads();
  const int klast = ((N - 1) / kNB) * kNB;
  for (int k = klast; k >= 0; k -= kNB) {
    const int kb = min(kNB, N - k);
    load_panel(k, kb);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ct = wave + 4 * i;
      if (ct < nct) {
        typename M::v4 c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = M::crow(v, lane), col = ct * 16 + lr;
          c[v] = (row < kb && col < m) ? T(Ybuf[(size_t)(k + row) * m + col]) : T(0);
        }
        const int ks = (b + 3) >> 2;
        for (int s = 0; s < ks; ++s) {
          const int t = 4 * s + lk;
          const int ta = kb + t - lr;
          const T a = (lr < kb && t < b && ta <= b && k + kb + t < N) ? Lp[lr * ldb + ta] : T(0);
          const T bb = (t < b) ? Y[slot(k + kb + t) + ct * 16 + lr] : T(0);
          c = M::mma(-a, bb, c);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = M::crow(v, lane), col = ct * 16 + lr;
          Zs[row * MP + col] = c[v];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ct = wave + 4 * i;
      if (ct < nct) {
        typename M::v4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int jj = 4 * s + lk;
          const T a = Dp[jj * kNB + lr];
          const T bb = Zs[jj * MP + ct * 16 + lr];
          acc = M::mma(a, bb, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = M::crow(v, lane), col = ct * 16 + lr;
          if (row < kb) {
            Y[slot(k + row) + col] = acc[v];
            if (col < m) {
              const double s = scaled ? sc[k + row] : 1.0;
              const double xv = s * (double)acc[v];
              double *dst = X + (size_t)(k + row) * m + col;
              if (mode == 0) *dst = xv;
              else *dst += xv;
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// FP64 residual of all right-hand sides, Rb = R - A^H_l X, matrix-free from
// the coefficients; accumulates per-column ||Rb||^2 and ||R||^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_residual(Geom g, const double *__restrict__ coef,
                                                  const double *__restrict__ r0,
                                                  const double *__restrict__ Xg,
                                                  double *__restrict__ Rbuf,
                                                  double *__restrict__ norms) {
  __shared__ double red[2 * kMaxRhs];
  const SubDesc S = g.sub[blockIdx.y];
  const int m = S.m, N = S.N;
  for (int i = threadIdx.x; i < 2 * m; i += blockDim.x) red[i] = 0.0;
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long long)N * m) {
    const int r = (int)(e / m), c = (int)(e % m);
    const double *cf = coef + 4 * S.cell_off;
    const double *X = Xg + S.X_off;
    const int n0 = S.n0, b = S.b;
    double ax = cf[4 * r] * X[(size_t)r * m + c];
    if (r + 1 < N) ax -= cf[4 * r + 1] * X[(size_t)(r + 1) * m + c];
    if (r >= 1) ax -= cf[4 * (r - 1) + 1] * X[(size_t)(r - 1) * m + c];
    if (r + n0 < N) ax -= cf[4 * r + 2] * X[(size_t)(r + n0) * m + c];
    if (r >= n0) ax -= cf[4 * (r - n0) + 2] * X[(size_t)(r - n0) * m + c];
    if (r + b < N) ax -= cf[4 * r + 3] * X[(size_t)(r + b) * m + c];
    if (r >= b) ax -= cf[4 * (r - b) + 3] * X[(size_t)(r - b) * m + c];
    double rhs = 0.0;
    if (c == 0) {
      rhs = r0[S.cell_off + r];
    } else {
      rhs_row_faces(g, S, r, [&](int col, double v) {
        if (col == c) rhs = v;
      });
    }
    const double res = rhs - ax;
    Rbuf[S.X_off + (size_t)r * m + c] = res;
    atomicAdd(&red[2 * c], res * res);
    atomicAdd(&red[2 * c + 1], rhs * rhs);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * m; i += blockDim.x) {
    if (red[i] != 0.0) atomicAdd(&norms[2 * (long long)S.col_off + i], red[i]);
  }
}

// Largest relative column residual sqrt(||Rb||^2 / ||R||^2) over all columns
// (a zero right-hand side counts its absolute residual).  One workgroup.
__global__ __launch_bounds__(256) void k_ir_check(const double *__restrict__ norms, int ncols,
                                                  double *__restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) {
    const double rr = norms[2 * i], RR = norms[2 * i + 1];
    const double v = RR > 0.0 ? sqrt(rr / RR) : sqrt(rr);
    mx = fmax(mx, v);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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
  const SubDesc S = g.sub[blockIdx.x];
  const int n = S.npatch, m = S.m;
  const double *X = Xg + S.X_off;
  for (int e = threadIdx.x; e < n * m; e += blockDim.x) {
    const int lp = e / m, c = e % m;
    int f = 0;
    for (int ff = 0; ff < 6; ++ff) {
      if (S.face_if[ff] < 0) continue;
      const IfaceDesc I = g.ifc[S.face_if[ff]];
      if (lp >= S.face_p0[ff] && lp < S.face_p0[ff] + I.na * I.nb) f = ff;
    }
    const IfaceDesc I = g.ifc[S.face_if[f]];
    const int w = lp - S.face_p0[f];
    const int pa = w % I.na, pb = w / I.na;
    const int a0 = split_start(pa, I.la, I.na), a1 = split_start(pa + 1, I.la, I.na);
    const int b0 = split_start(pb, I.lb, I.nb), b1 = split_start(pb + 1, I.lb, I.nb);
    const int d = f >> 1;
    const int sigma = (f & 1) ? 1 : -1;
    const double H = S.ext[d] * g.h[d], A = g.area[d], hd = g.h[d];
    double sf = 0.0, sb = 0.0, sab = 0.0;
    for (int tb = b0; tb < b1; ++tb) {
      for (int ta = a0; ta < a1; ++ta) {
        int x[3];
        x[I.a] = S.lo[I.a] + ta;
        x[I.b] = S.lo[I.b] + tb;
        x[d] = sigma < 0 ? S.lo[d] : S.lo[d] + S.ext[d] - 1;
        const double kd = g.k[d][cell_index(g, x)];
        const double beta = g.alpha * H / kd;
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

size_t factor_lds_bytes(int fp32, int bmax) {
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  return (size_t)(bmax + kNB) * (bmax + 1) * es;
}

size_t solve_lds_bytes(int fp32, int bmax, int mmax) {
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  const size_t mp = (size_t)((mmax + 15) & ~15);
  return ((size_t)kNB * (bmax + 1) + kNB * kNB + (size_t)(bmax + kNB) * mp + 16 * mp) * es;
}

template <typename T, int RPL>
static hipError_t launch_factor_t(const SubDesc *subs, const int *order, int n_sub,
                                  const double *coef, const double *scal, T *L, T *Dg,
                                  DevStatus *st, int bmax, int scaled, hipStream_t s) {
  const size_t lds = factor_lds_bytes(sizeof(T) == 4, bmax);
  hipError_t e = hipFuncSetAttribute((const void *)k_factor<T, RPL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor<T, RPL>), dim3(n_sub), dim3(256), lds, s, subs, order, coef, scal, L,
                     Dg, st, bmax + 1, scaled);
  return hipGetLastError();
}

hipError_t launch_factor(int fp32, const SubDesc *subs, const int *order, int n_sub,
                         const double *coef, const double *scal, void *L, void *Dg, DevStatus *st,
                         int bmax, hipStream_t s) {
  const int W = bmax + kNB;
  if (fp32) {
    if (W <= 128)
      return launch_factor_t<float, 2>(subs, order, n_sub, coef, scal, (float *)L, (float *)Dg, st,
                                       bmax, 1, s);
    return launch_factor_t<float, 3>(subs, order, n_sub, coef, scal, (float *)L, (float *)Dg, st,
                                     bmax, 1, s);
  }
  if (W <= 128)
    return launch_factor_t<double, 2>(subs, order, n_sub, coef, scal, (double *)L, (double *)Dg, st,
                                      bmax, 0, s);
  return launch_factor_t<double, 3>(subs, order, n_sub, coef, scal, (double *)L, (double *)Dg, st,
                                    bmax, 0, s);
}

template <typename T>
static hipError_t launch_solve_t(const Geom &g, const int *order, int n_sub, const double *r0,
                                 const double *scal, const T *L, const T *Dg, double *X, double *R,
                                 int mode, int bmax, int mmax, int scaled, hipStream_t s) {
  const size_t lds = solve_lds_bytes(sizeof(T) == 4, bmax, mmax);
  hipError_t e = hipFuncSetAttribute((const void *)k_solve<T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int mpmax = (mmax + 15) & ~15;
  hipLaunchKernelGGL(k_solve<T>, dim3(n_sub), dim3(256), lds, s, g, order, r0, scal, L, Dg, X, R,
                     mode, scaled, bmax + 1, bmax + kNB, mpmax);
  return hipGetLastError();
}

hipError_t launch_solve(int fp32, const Geom &g, const int *order, int n_sub, const double *r0,
                        const double *scal, const void *L, const void *Dg, double *X, double *R,
                        int mode, int bmax, int mmax, hipStream_t s) {
  if (fp32)
    return launch_solve_t<float>(g, order, n_sub, r0, scal, (const float *)L, (const float *)Dg, X,
                                 R, mode, bmax, mmax, 1, s);
  return launch_solve_t<double>(g, order, n_sub, r0, scal, (const double *)L, (const double *)Dg, X,
                                R, mode, bmax, mmax, 0, s);
}

hipError_t launch_residual(const Geom &g, int n_sub, long long max_nm, const double *coef,
                           const double *r0, const double *X, double *R, double *norms,
                           hipStream_t s) {
  dim3 grid((unsigned)((max_nm + 255) / 256), n_sub);
  hipLaunchKernelGGL(k_residual, grid, dim3(256), 0, s, g, coef, r0, X, R, norms);
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

}  // namespace mrcm
