// Iterative form of loop 1 of the MRCM (Algorithm 2): every right-hand side
// of (2.25)/(2.26) solved by a preconditioned conjugate-gradient method
// instead of the band factorisation, with the band Cholesky kept as the
// fallback for columns that do not converge.
//
// One workgroup (256 lanes) owns one column of one subdomain and runs the
// whole solve out of registers and LDS:
//  * outer loop in FP64: r = b - A^H_l x from the coefficients, stop when
//    ||r|| <= tol ||b||;
//  * inner loop in FP32: conjugate gradients on the symmetrically Jacobi-
//    scaled matrix D^-1/2 A D^-1/2 (unit diagonal, which is Jacobi
//    preconditioning), for the normalised scaled residual, until its own
//    residual has dropped by kInnerTol; x += D^-1/2 y in FP64.
// The budget max_iter counts inner iterations (matrix-vector products) over
// all outer steps.  A starting guess whose residual exceeds ||b|| is replaced
// by zero.  The starting guess X0 may be X itself: a workgroup reads
// its column of X0 before it writes that column of X.  Thread t owns local rows t + 256 i, i < CPT; the search
// direction is exchanged through LDS for the 7-point product, and every
// branch depends only on workgroup sums that all lanes read alike.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "launch.h"

namespace mrcm {
namespace {

constexpr float kInnerTol = 1e-3f;
// zero rows on both sides of the LDS vectors: every neighbour offset of a
// row (+-1, +-n0, +-b with b <= kMaxBand64) stays inside the array
constexpr int kPad = 128;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// FP32 sums over a wave by DPP moves (no LDS traffic): prefix sums within
// rows of 16 lanes (row_shr 1, 2, 4, 8), then the row totals carried into
// rows 1 and 3 (row_bcast 15) and 2 and 3 (row_bcast 31); lane 63 ends with
// the total, which every lane reads.
template <int ctrl, int row_mask>
__device__ __forceinline__ float dpp_add(float v) {
  const int x = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, row_mask, 0xf, false);
  return v + __builtin_bit_cast(float, x);
}

// Two such sums at once: the steps of the two chains alternate, so that each
// DPP move's wait states are filled by the other chain.
__device__ __forceinline__ void wave_sum2_dpp(float &a, float &b) {
  a = dpp_add<0x111, 0xf>(a);
  b = dpp_add<0x111, 0xf>(b);
  a = dpp_add<0x112, 0xf>(a);
  b = dpp_add<0x112, 0xf>(b);
  a = dpp_add<0x114, 0xf>(a);
  b = dpp_add<0x114, 0xf>(b);
  a = dpp_add<0x118, 0xf>(a);
  b = dpp_add<0x118, 0xf>(b);
  a = dpp_add<0x142, 0xa>(a);
  b = dpp_add<0x142, 0xa>(b);
  a = dpp_add<0x143, 0xc>(a);
  b = dpp_add<0x143, 0xc>(b);
  a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a), 63));
  b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, b), 63));
}

// Sum over the workgroup's NW waves; every lane returns the same bits.  A
// slot of red must not be reused before a later barrier.
template <int NW, typename T>
__device__ __forceinline__ T block_sum(T v, T *red, int wave, int lane) {
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) s += red[k];
  return s;
}

// Keeps the compiler from hoisting per-row address arithmetic out of loops
// (which would hold six addresses per row in registers for the whole kernel).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <int NT, int CPT>
__global__ __launch_bounds__(NT) void k_pcg(Geom g, const int *__restrict__ col_sub, int ncols,
                                            const double *__restrict__ coef, const double *__restrict__ scal,
                                            const double *__restrict__ Bg, const double *X0g, double *Xg,
                                            int max_iter, double tol,
                                            int *__restrict__ iters, int *__restrict__ conv) {
  constexpr int NW = NT / 64;
  constexpr int LEN = NT * CPT + 2 * kPad;
  __shared__ float ps[LEN];
  __shared__ double xs[LEN];
  __shared__ float redf[2][NW];
  __shared__ double redd[2][NW];
  // columns in contiguous ranges per XCD (workgroup i runs on XCD i mod 8),
  // so that the columns of one subdomain share that XCD's L2
  const int per = (ncols + 7) >> 3;
  const int col = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (col >= ncols) return;
  const SubDesc &S = g.sub[col_sub[col]];
  const int N = S.N, m = S.m, n0 = S.n0, b = S.b;
  const int c = col - S.col_off;
  const double *cf = coef + 4 * S.cell_off;
  const double *sc = scal + S.cell_off;
  const double *B = Bg + S.X_off;
  double *X = Xg + S.X_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = tid; k < LEN; k += NT) {
    ps[k] = 0.0f;
    xs[k] = 0.0;
  }
  float *pr = ps + kPad + tid;   // row tid + NT i at pr[NT i]
  double *xr = xs + kPad + tid;

  // Scaled off-diagonal weights s_r t s_n (the matrix entries are their
  // negatives): the + side from the row's own coefficients and the
  // neighbour's scale, the - side copied from the neighbour's + side through
  // LDS, so that the FP32 matrix is exactly symmetric.  Rows outside the box
  // read zero rows of the padded vectors.
  float w[6][CPT];
  double bsq = 0.0;
  __syncthreads();  // zeroed vectors
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    if (r < N) xr[NT * i] = sc[r];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    const int rc = min(r, N - 1);
    const double *cr = cf + 4 * rc;
    const double *sn = xr + NT * i;
    const double sr = sn[0];
    w[0][i] = (float)(sr * cr[1] * sn[1]);
    w[2][i] = (float)(sr * cr[2] * sn[n0]);
    w[4][i] = (float)(sr * cr[3] * sn[b]);
    const double bv = B[(size_t)rc * m + c];
    bsq += r < N ? bv * bv : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int off = k == 0 ? 1 : (k == 1 ? n0 : b);
#pragma unroll
    for (int i = 0; i < CPT; ++i)
      if (tid + NT * i < N) pr[NT * i] = w[2 * k][i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) w[2 * k + 1][i] = tid + NT * i < N ? pr[NT * i - off] : 0.0f;
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    if (r < N) {
      pr[NT * i] = 0.0f;
      xr[NT * i] = X0g ? X0g[S.X_off + (size_t)r * m + c] : 0.0;
    }
  }
  const double bn2 = block_sum<NW>(bsq, redd[0], wave, lane);
  const double tol2 = tol * tol * bn2;
  int it = 0;
  bool ok = bn2 == 0.0;
  if (ok) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) xr[NT * i] = 0.0;
  }
  // (A x)_r in FP64 from the coefficients, x in xs (row rc, clamped);
  // neighbours outside the box carry zero coefficients or read zero rows
  const auto apply_a = [&](int rc) {
    const int m1 = max(rc - 1, 0), mn = max(rc - n0, 0), mb = max(rc - b, 0);
    const double *xc = xs + kPad + rc;
    double a = cf[4 * rc] * xc[0];
    a -= cf[4 * rc + 1] * xc[1];
    a -= cf[4 * m1 + 1] * xc[-1];
    a -= cf[4 * rc + 2] * xc[n0];
    a -= cf[4 * mn + 2] * xc[-n0];
    a -= cf[4 * rc + 3] * xc[b];
    a -= cf[4 * mb + 3] * xc[-b];
    return a;
  };
  // a starting guess is kept only if its residual is no larger than that of
  // the zero start (the stopping test is relative to ||b||, and a guess close
  // in the A-norm can still carry a large high-frequency residual)
  bool check_start = X0g != nullptr;
  while (!ok) {
    // FP64 residual r = b - A x from the coefficients (x in xs)
    double res[CPT];
    double rsq = 0.0, nsq = 0.0;
    const int t = opaque(tid);
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int r = t + NT * i;
      const int rc = min(r, N - 1);
      const double a = apply_a(rc);
      const double rv = r < N ? B[(size_t)rc * m + c] - a : 0.0;
      const double sv = sc[rc] * rv;
      res[i] = sv;
      rsq += rv * rv;
      nsq += sv * sv;
      __builtin_amdgcn_sched_barrier(0);
    }
    const double rn2 = block_sum<NW>(rsq, redd[1], wave, lane);
    if (rn2 <= tol2) {
      ok = true;
      break;
    }
    if (check_start) {
      check_start = false;
      if (!(rn2 <= bn2)) {
#pragma unroll
        for (int i = 0; i < CPT; ++i)
          if (tid + NT * i < N) xr[NT * i] = 0.0;
        __syncthreads();
        continue;
      }
    }
    if (it >= max_iter || !isfinite(rn2)) break;
    const double sn2 = block_sum<NW>(nsq, redd[0], wave, lane);
    const double sn = sqrt(sn2), inv_sn = 1.0 / sn;
    // Inner solve of (D^-1/2 A D^-1/2) y = D^-1/2 r / ||D^-1/2 r|| by the
    // conjugate-gradient recurrences of Chronopoulos and Gear (1989): both
    // dot products of an iteration, (r, r) and (A r, r), are reduced
    // together, so an iteration takes two barriers (the exchange of r for
    // the product, the reduction).  Vectors: r residual, w = A r, p
    // direction, s = A p.
    float y[CPT], rv[CPT], wv[CPT], sv[CPT], p[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      rv[i] = (float)(res[i] * inv_sn);
      y[i] = sv[i] = p[i] = 0.0f;
    }
    const float eta2 = kInnerTol * kInnerTol;
    float gam_prev = 1.0f, alpha_prev = 1.0f;
    for (int k = 0;; ++k) {
#pragma unroll
      for (int i = 0; i < CPT; ++i)
        if (tid + NT * i < N) pr[NT * i] = rv[i];
      __syncthreads();
      float gp = 0.0f, dp = 0.0f;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const float *q = pr + NT * i;
        float a = rv[i];
        a = fmaf(-w[0][i], q[1], a);
        a = fmaf(-w[1][i], q[-1], a);
        a = fmaf(-w[2][i], q[n0], a);
        a = fmaf(-w[3][i], q[-n0], a);
        a = fmaf(-w[4][i], q[b], a);
        a = fmaf(-w[5][i], q[-b], a);
        wv[i] = a;
        gp = fmaf(rv[i], rv[i], gp);
        dp = fmaf(a, rv[i], dp);
      }
      wave_sum2_dpp(gp, dp);
      if (lane == 0) {
        redf[0][wave] = gp;
        redf[1][wave] = dp;
      }
      __syncthreads();
      float gam = redf[0][0], del = redf[1][0];
#pragma unroll
      for (int j = 1; j < NW; ++j) {
        gam += redf[0][j];
        del += redf[1][j];
      }
      // the product above is counted once the step is taken
      if (gam <= eta2 || it >= max_iter) break;
      ++it;
      // the step lengths by hardware reciprocals: their relative error
      // (about 1e-7) is that of the FP32 iteration itself
      const float beta = k == 0 ? 0.0f : gam * __builtin_amdgcn_rcpf(gam_prev);
      const float den = k == 0 ? del : del - beta * gam * __builtin_amdgcn_rcpf(alpha_prev);
      const float alpha = gam * __builtin_amdgcn_rcpf(den);
      // a non-positive or non-finite step (rounding): keep y and restart
      // from the true residual
      if (!(alpha > 0.0f) || !isfinite(alpha)) break;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        p[i] = fmaf(beta, p[i], rv[i]);
        sv[i] = fmaf(beta, sv[i], wv[i]);
        y[i] = fmaf(alpha, p[i], y[i]);
        rv[i] = fmaf(-alpha, sv[i], rv[i]);
      }
      gam_prev = gam;
      alpha_prev = alpha;
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int r = tid + NT * i;
      if (r < N) xr[NT * i] += sn * sc[r] * (double)y[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    if (r < N) X[(size_t)r * m + c] = xr[NT * i];
  }
  if (tid == 0) {
    iters[col] = it;
    conv[col] = ok ? 1 : 0;
  }
}

// Galerkin scaling of a starting guess, one workgroup per column as k_pcg:
// X = c V with c = (V, b) / (V, A V), the multiple of V closest to the
// solution in the A-norm (zero when V is zero).  X may alias V only if every
// column is read before it is written, which holds per workgroup.
template <int NT, int CPT>
__global__ __launch_bounds__(NT) void k_pcg_scale(Geom g, const int *__restrict__ col_sub, int ncols,
                                                  const double *__restrict__ coef, const double *__restrict__ Bg,
                                                  const double *V0, double *Xg) {
  constexpr int NW = NT / 64;
  constexpr int LEN = NT * CPT + 2 * kPad;
  __shared__ double xs[LEN];
  __shared__ double redd[2][NW];
  const int per = (ncols + 7) >> 3;
  const int col = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (col >= ncols) return;
  const SubDesc &S = g.sub[col_sub[col]];
  const int N = S.N, m = S.m, n0 = S.n0, b = S.b;
  const int c = col - S.col_off;
  const double *cf = coef + 4 * S.cell_off;
  const double *B = Bg + S.X_off;
  const double *V = V0 + S.X_off;
  double *X = Xg + S.X_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = tid; k < LEN; k += NT) xs[k] = 0.0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    if (r < N) xs[kPad + r] = V[(size_t)r * m + c];
  }
  __syncthreads();
  double vb = 0.0, vav = 0.0;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    const int rc = min(r, N - 1);
    const int m1 = max(rc - 1, 0), mn = max(rc - n0, 0), mb = max(rc - b, 0);
    const double *xc = xs + kPad + rc;
    double a = cf[4 * rc] * xc[0];
    a -= cf[4 * rc + 1] * xc[1];
    a -= cf[4 * m1 + 1] * xc[-1];
    a -= cf[4 * rc + 2] * xc[n0];
    a -= cf[4 * mn + 2] * xc[-n0];
    a -= cf[4 * rc + 3] * xc[b];
    a -= cf[4 * mb + 3] * xc[-b];
    vb += r < N ? xc[0] * B[(size_t)rc * m + c] : 0.0;
    vav += r < N ? xc[0] * a : 0.0;
  }
  const double sb = block_sum<NW>(vb, redd[0], wave, lane);
  const double sa = block_sum<NW>(vav, redd[1], wave, lane);
  const double cs = sa > 0.0 ? sb / sa : 0.0;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int r = tid + NT * i;
    if (r < N) X[(size_t)r * m + c] = cs * xs[kPad + r];
  }
}

template <int NT, int CPT>
hipError_t launch_pcg_t(const Geom &g, const int *col_sub, int ncols, const double *coef, const double *scal,
                        const double *B, const double *X0, double *X, int max_iter, double tol, int x0_scale,
                        int *iters, int *conv, hipStream_t s) {
  const int per = (ncols + 7) / 8;
  if (X0 && x0_scale) {
    hipLaunchKernelGGL((k_pcg_scale<NT, CPT>), dim3(8 * per), dim3(NT), 0, s, g, col_sub, ncols, coef, B, X0, X);
    X0 = X;
  }
  hipLaunchKernelGGL((k_pcg<NT, CPT>), dim3(8 * per), dim3(NT), 0, s, g, col_sub, ncols, coef, scal, B, X0, X,
                     max_iter, tol, iters, conv);
  return hipGetLastError();
}

}  // namespace

int pcg_max_cells() { return 512 * 4; }

hipError_t launch_pcg(const Geom &g, const int *col_sub, int ncols, int max_cells, const double *coef,
                      const double *scal, const double *B, const double *X0, double *X, int max_iter, double tol,
                      int x0_scale, int *iters, int *conv, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  if (max_cells <= 512)
    return launch_pcg_t<256, 2>(g, col_sub, ncols, coef, scal, B, X0, X, max_iter, tol, x0_scale, iters, conv, s);
  if (max_cells <= 1024)
    return launch_pcg_t<512, 2>(g, col_sub, ncols, coef, scal, B, X0, X, max_iter, tol, x0_scale, iters, conv, s);
  if (max_cells <= 2048)
    return launch_pcg_t<512, 4>(g, col_sub, ncols, coef, scal, B, X0, X, max_iter, tol, x0_scale, iters, conv, s);
  return hipErrorInvalidValue;
}

}  // namespace mrcm
