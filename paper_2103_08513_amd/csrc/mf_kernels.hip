// Multifrontal LDL^T of the interface system on gfx950, over the nested-
// dissection tree of nd_plan.cpp (InterfaceSolver of Algorithm 2).
//
// With s = -1 on the pressure rows and +1 on the velocity rows, M = diag(s) A
// is symmetric quasi-definite (eqs. (2.19)-(2.22)); any symmetric order admits
// LDL^T without pivoting.  Every tree node owns a dense f x f column-major
// front: its separator's sp unknowns (the separator rounded up to a multiple
// of 16 with identity pad rows), then its r boundary unknowns, which its
// ancestors eliminate.  Its lower triangle receives the assembled entries of
// the separator's rows and columns and the children's update matrices; the
// partial factorisation of the separator columns then leaves
//   the 16x16 diagonal blocks: L below, D on the diagonal, U = D L^T above,
//     with L11^{-1} and 1/D per block in `inv` (272 doubles);
//   W = A21 L11^{-T} of each block (the unscaled L21 = W D^{-1}) stored
//     transposed above the diagonal: W[i][c] at column i, row k0 + c;
//   the update matrix (Schur complement) in the trailing r x r block.
// Levels are processed bottom-up, each as one extend-add per child slot, the
// factorisation of every node's first block, then panel by panel (up to
// kMfPanelMax blocks of 16 columns): one launch per block over the row tiles below it,
// which forms W and updates the rest of the panel only, and the trailing
// update past the panel, with W read back from its transposed store,
// deferred over kMfDefer panels: a narrow launch brings the next panel's
// columns up to date, and one launch per group of panels updates the tiles
// past it.  The trailing matrix is thus read and written once per 128
// columns rather than once per 16.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "launch.h"
#include "ldl16.h"
#include "nd_plan.h"

namespace mrcm {

// ---------------------------------------------------------------------------
// One row pair of the assembled interface system (P-row and U-row of patch
// a), as assemble_interface defines it: each entry is the sum over the (at
// most two) subdomains holding both patches, of
//   P-row: F^s[i, P_j], F^s[i, U_j];  U-row: sigma Fb^s[i, P_j],
//   sigma Fb^s[i, U_j] - [i = j] SAb^s[i],
// taken as fl(lower side + upper side), the order in which the front
// scatter's two atomic additions onto zero round.  visit(b, cPP, cPU, cUP, cUU)
// receives each column patch once; bP, bU the right-hand side.
// ---------------------------------------------------------------------------
template <typename Visit>
__device__ __forceinline__ void iface_rows(const Geom &g, const int *__restrict__ patches, const double *__restrict__ F,
                                           const double *__restrict__ Fb, const double *__restrict__ SAb, int a,
                                           const int4 pinfo, double &bP, double &bU, Visit visit) {
  const IfaceDesc &I = g.ifc[pinfo.x];
  const SubDesc &S1 = g.sub[I.lo_sub];
  const SubDesc &S2 = g.sub[I.hi_sub];
  const int li1 = pinfo.y, li2 = pinfo.z;
  const int n1 = S1.npatch, m1 = S1.m, n2 = S2.npatch, m2 = S2.m;
  const double *f1 = F + S1.F_off + (size_t)li1 * m1;
  const double *b1 = Fb + S1.F_off + (size_t)li1 * m1;
  const double *f2 = F + S2.F_off + (size_t)li2 * m2;
  const double *b2 = Fb + S2.F_off + (size_t)li2 * m2;
  const int np = I.na * I.nb;
  const int j2base = S2.face_p0[2 * I.d];
  for (int j = 0; j < n1; ++j) {
    const int bq = patches[S1.patch_off + j];
    double cPP = f1[1 + j], cPU = f1[1 + n1 + j], cUP = b1[1 + j];
    double cUU = b1[1 + n1 + j] - (j == li1 ? SAb[S1.patch_off + li1] : 0.0);
    if (bq >= I.p0 && bq < I.p0 + np) {
      // a patch of the shared interface: the upper side adds its part
      const int j2 = j2base + (bq - I.p0);
      cPP = cPP + f2[1 + j2];
      cPU = cPU + f2[1 + n2 + j2];
      cUP = cUP + (-b2[1 + j2]);
      cUU = cUU + (-b2[1 + n2 + j2] - (j2 == li2 ? SAb[S2.patch_off + li2] : 0.0));
    }
    visit(bq, cPP, cPU, cUP, cUU);
  }
  for (int j = 0; j < n2; ++j) {
    const int bq = patches[S2.patch_off + j];
    if (bq >= I.p0 && bq < I.p0 + np) continue;
    visit(bq, f2[1 + j], f2[1 + n2 + j], -b2[1 + j], -b2[1 + n2 + j]);
  }
  bP = (-f1[0]) + (-f2[0]);
  bU = (-b1[0]) + b2[0];
}

// r = b - A x (unflipped, interleaved unknowns 2p, 2p+1), one thread per patch.
__global__ __launch_bounds__(256) void k_mf_residual(Geom g, const int *__restrict__ patches,
                                                     const double *__restrict__ F, const double *__restrict__ Fb,
                                                     const double *__restrict__ SAb, const int4 *__restrict__ pinfo,
                                                     int nv, const double *__restrict__ x, double *__restrict__ r,
                                                     double *__restrict__ b) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nv) return;
  double rP = 0.0, rU = 0.0, bP, bU;
  iface_rows(g, patches, F, Fb, SAb, a, pinfo[a], bP, bU,
             [&](int bq, double cPP, double cPU, double cUP, double cUU) {
               if (!x) return;  // x = 0: r = b
               const double xp = x[2 * bq], xu = x[2 * bq + 1];
               rP = fma(cPP, xp, fma(cPU, xu, rP));
               rU = fma(cUP, xp, fma(cUU, xu, rU));
             });
  r[2 * a] = bP - rP;
  r[2 * a + 1] = bU - rU;
  if (b) {
    b[2 * a] = bP;
    b[2 * a + 1] = bU;
  }
}

// Dense rows of A (natural order: P-row of patch a at a, U-row at nv + a),
// for inspection.  One thread per patch; the rows must be zero beforehand.
__global__ __launch_bounds__(256) void k_mf_dense(Geom g, const int *__restrict__ patches,
                                                  const double *__restrict__ F, const double *__restrict__ Fb,
                                                  const double *__restrict__ SAb, const int4 *__restrict__ pinfo,
                                                  int nv, double *__restrict__ A, double *__restrict__ b) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nv) return;
  const size_t n = 2 * (size_t)nv;
  double *rowP = A + (size_t)a * n, *rowU = A + (size_t)(nv + a) * n;
  double bP, bU;
  iface_rows(g, patches, F, Fb, SAb, a, pinfo[a], bP, bU,
             [&](int bq, double cPP, double cPU, double cUP, double cUU) {
               rowP[bq] = cPP;
               rowP[nv + bq] = cPU;
               rowU[bq] = cUP;
               rowU[nv + bq] = cUU;
             });
  b[a] = bP;
  b[nv + a] = bU;
}

// Scatter of the assembled entries into the fronts: one workgroup per
// subdomain, one thread per (row patch, column patch) pair.  The sign flip
// negates the pressure rows.  An entry receives one contribution per
// subdomain holding both patches -- at most two -- so the atomic sums onto
// zero do not depend on their order.  Pairs above the diagonal are skipped:
// their transposes are below it.
__global__ __launch_bounds__(256) void k_mf_scatter(Geom g, const int *__restrict__ patches,
                                                    const double *__restrict__ F, const double *__restrict__ Fb,
                                                    const double *__restrict__ SAb,
                                                    const int64_t *__restrict__ sub_pair_off,
                                                    const int64_t *__restrict__ pair_off,
                                                    const int *__restrict__ pair_ld, double *__restrict__ fronts) {
  const SubDesc &S = g.sub[blockIdx.x];
  const int n = S.npatch, m = S.m;
  const double *Fs = F + S.F_off;
  const double *Fbs = Fb + S.F_off;
  const int64_t e0 = sub_pair_off[blockIdx.x];
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int64_t off = pair_off[e0 + e];
    if (off < 0) continue;
    const int ld = pair_ld[e0 + e];
    const int li = e / n, lj = e % n;
    int fi = 0;
    for (int ff = 0; ff < 6; ++ff) {
      const int ii = S.face_if[ff];
      if (ii < 0) continue;
      const IfaceDesc &I = g.ifc[ii];
      if (li >= S.face_p0[ff] && li < S.face_p0[ff] + I.na * I.nb) fi = ff;
    }
    const double sig = (fi & 1) ? 1.0 : -1.0;
    const double *fr = Fs + (size_t)li * m;
    const double *br = Fbs + (size_t)li * m;
    double uu = sig * br[1 + n + lj];
    if (li == lj) uu -= SAb[S.patch_off + li];
    atomicAdd(&fronts[off], -fr[1 + lj]);           // (P_a, P_b), flipped row
    atomicAdd(&fronts[off + 1], sig * br[1 + lj]);  // (U_a, P_b)
    if (li != lj) atomicAdd(&fronts[off + ld], -fr[1 + n + lj]);  // (P_a, U_b), flipped row
    atomicAdd(&fronts[off + ld + 1], uu);           // (U_a, U_b)
  }
}

// Identity on the pad rows of every separator.
__global__ void k_mf_pad(const MfNode *__restrict__ nodes, int nn, double *__restrict__ fronts) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const MfNode nd = nodes[k];
  for (int p = nd.s; p < nd.sp; ++p) fronts[nd.off + (int64_t)p * nd.f + p] = 1.0;
}

// Extend-add of one child slot: the update matrix of child `slot` of each of
// the level's nodes into the node's front, through the child's map.
// grid = (nodes of the level, groups of 16 child columns).
__global__ __launch_bounds__(256) void k_mf_extend(const MfNode *__restrict__ nodes, const int *__restrict__ list,
                                                   const int *__restrict__ map, int slot,
                                                   double *__restrict__ fronts) {
  const MfNode P = nodes[list[blockIdx.x]];
  const int c = slot ? P.child1 : P.child0;
  if (c < 0) return;
  const MfNode C = nodes[c];
  const int j0 = 16 * blockIdx.y;
  if (j0 >= C.r) return;
  const int *cm = map + C.map_off;
  const double *src = fronts + C.off;
  double *dst = fronts + P.off;
  const int nj = min(C.r, j0 + 16) - j0;
  // the block's 16 columns: the parent column offsets once, then each thread
  // takes a row i and adds its entries of all the columns j <= i (sixteen
  // independent updates in flight, each parent entry written by one thread)
  __shared__ int64_t pcol[16];
  if ((int)threadIdx.x < nj) pcol[threadIdx.x] = (int64_t)cm[j0 + threadIdx.x] * P.f;
  __syncthreads();
  const double *col0 = src + (int64_t)(C.sp + j0) * C.f + C.sp;
  for (int i = j0 + threadIdx.x; i < C.r; i += blockDim.x) {
    const int pi = cm[i];
    const int jn = min(nj, i - j0 + 1);
    if (jn == 16) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) dst[pcol[jj] + pi] += col0[(int64_t)jj * C.f + i];
    } else {
      for (int jj = 0; jj < jn; ++jj) dst[pcol[jj] + pi] += col0[(int64_t)jj * C.f + i];
    }
  }
}

// LDL^T of the first 16x16 block of every node of a level (one wave each).
__global__ __launch_bounds__(64) void k_mf_first(const MfNode *__restrict__ nodes, const int *__restrict__ list,
                                                 double *__restrict__ fronts, double *__restrict__ inv,
                                                 DevStatus *st) {
  __shared__ double blk[2 * kLB * (kLB + 1)];
  __shared__ double T[kInvStride];
  const int k = list[blockIdx.x];
  const MfNode nd = nodes[k];
  const int lane = threadIdx.x;
  double *A = fronts + nd.off;
  for (int e = lane; e < kLB * kLB; e += 64) {
    const int r = e / kLB, c = e % kLB;
    blk[r * (kLB + 1) + c] = (c <= r) ? A[(int64_t)c * nd.f + r] : 0.0;
  }
  __syncthreads();
  const int f = nd.f;
  auto store = [&](int t, int i, double v) { A[(int64_t)t * f + i] = v; };
  if (ldl_diag16(blk, kLB, lane, store, inv + nd.inv_off, blk, T) && lane == 0)
    set_status(st, kStatusSingular, k, 0.0);
}

// LDL^T of diagonal block t of every node listed (one wave each): the first
// block of a panel, once the trailing update has reached it.
__global__ __launch_bounds__(64) void k_mf_diag(const MfNode *__restrict__ nodes, const int2 *__restrict__ blocks,
                                                int t, double *__restrict__ fronts, double *__restrict__ inv,
                                                DevStatus *st) {
  __shared__ double blk[2 * kLB * (kLB + 1)];
  __shared__ double T[kInvStride];
  const int k = blocks[blockIdx.x].x;
  const MfNode nd = nodes[k];
  const int lane = threadIdx.x, f = nd.f, k0 = kLB * t;
  double *A = fronts + nd.off;
  for (int e = lane; e < kLB * kLB; e += 64) {
    const int r = e / kLB, c = e % kLB;
    blk[r * (kLB + 1) + c] = (c <= r) ? A[(int64_t)(k0 + c) * f + k0 + r] : 0.0;
  }
  __syncthreads();
  auto store = [&](int tt, int i, double v) { A[(int64_t)(k0 + tt) * f + k0 + i] = v; };
  if (ldl_diag16(blk, kLB, lane, store, inv + nd.inv_off + (int64_t)t * kInvStride, blk, T) && lane == 0)
    set_status(st, kStatusSingular, k, 0.0);
}

// Step t of the partial factorisation, for every node of a level with a
// block t: the rows r0 = 16 (t + 1) .. f - 1 in 64-row tiles, one workgroup
// (four waves of 16 rows) per tile.  Each tile forms W = A21 L11^{-T} for its
// rows and stores W^T above the diagonal (column i, rows 16 t .. 16 t + 15),
// and applies C -= W D^{-1} W^T to the columns r0 .. pe - 1 that remain in
// the block's panel (pe its end); the columns past the panel receive the
// panel's blocks together in k_mf_trailing.  A fifth wave, in the first tile
// of a node whose next block lies in the same panel, factors that block while
// the other waves finish.  The A21 entries below the diagonal are left as
// they are, so every tile reads the same A21 whatever the order of the tiles.
constexpr int kMfStepThreads = 320;

__global__ __launch_bounds__(kMfStepThreads) void k_mf_step(const MfNode *__restrict__ nodes,
                                                            const int2 *__restrict__ blocks, int t, int panel,
                                                            double *__restrict__ fronts, double *__restrict__ inv,
                                                            DevStatus *st) {
  using M = Mma<double>;
  __shared__ double Wi[64 * (kLB + 1)];
  __shared__ double Wj[64 * (kLB + 1)];
  __shared__ double Dn[2 * kLB * (kLB + 1)];
  __shared__ double Ts[kInvStride];
  const int2 bt = blocks[blockIdx.x];
  const MfNode nd = nodes[bt.x];
  const int f = nd.f;
  double *A = fronts + nd.off;
  const double *inv_k = inv + nd.inv_off + (int64_t)t * kInvStride;
  const int k0 = kLB * t;
  const int r0 = k0 + kLB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int ti = bt.y, tj = 0;
  const int pe = kLB * min(t - t % panel + panel, nd.sp / kLB);  // end of the panel
  const int i0 = r0 + 64 * ti, j0 = r0;
  auto a21 = [&](int i, int c) -> double { return i < f ? A[(int64_t)(k0 + c) * f + i] : 0.0; };
  const bool rows = wave < 4;
  double ai[4] = {0.0, 0.0, 0.0, 0.0}, aj[4] = {0.0, 0.0, 0.0, 0.0};
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
#pragma unroll
    for (int tc = 0; tc < 4; ++tc) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * wave + M::crow(v, lane), j = j0 + 16 * tc + lr;
        const bool ok = i < f && j < pe && i >= j;
        c[tc][v] = ok ? A[(int64_t)j * f + i] : 0.0;
      }
    }
  }
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
  const bool has_next = ti == 0 && r0 < pe;
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
      Dn[(i - r0) * (kLB + 1) + (j - r0)] = (i >= j) ? c[0][v] : 0.0;
    }
  }
  __syncthreads();
  if (has_next && wave == 4) {
    auto store = [&](int tt, int i, double v) { A[(int64_t)(r0 + tt) * f + r0 + i] = v; };
    if (ldl_diag16(Dn, kLB, lane, store, inv + nd.inv_off + (int64_t)(t + 1) * kInvStride, Dn, Ts) && lane == 0)
      set_status(st, kStatusSingular, bt.x, 0.0);
  } else if (rows && !(has_next && wave == 0)) {
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
          if (i < f && j < pe && i >= j) A[(int64_t)j * f + i] = c[tc][v];
        }
      }
    };
    // column tiles of the panel past r0 (at most three)
    const int lim = (pe - r0) / 16;
    const int ntc = ti == 0 ? min(wave + 1, lim) : lim;
    if (ntc == 3)
      update_cols(std::integral_constant<int, 3>{});
    else if (ntc == 2)
      update_cols(std::integral_constant<int, 2>{});
    else if (ntc == 1)
      update_cols(std::integral_constant<int, 1>{});
  }
  if (rows) {
    for (int e = tid; e < 64 * kLB; e += 256) {
      const int rr = e / kLB, cc = e % kLB;
      const int i = i0 + rr;
      if (i < f) A[(int64_t)i * f + (k0 + cc)] = Wi[rr * (kLB + 1) + cc];
    }
  }
}

// Trailing update past the blocks t0 .. t0 + nb - 1 (nb = min(nb_max, the
// node's blocks from t0): one panel, or a group of deferred panels):
// C -= W D^{-1} W^T on the lower 64x64 tiles of the rows and columns
// R0 = 16 (t0 + nb) .. f - 1, K = 16 nb; with jend > 0 only the columns
// below block min(jend, the separator's end) are written (the deferred
// update of the next panel's columns).  The tile stays in accumulators
// while W of its rows i and columns j comes block by block (16 columns of K)
// from its transposed store (column i, rows 16 t .. 16 t + 15, contiguous)
// through 17 KB of LDS, so that eight workgroups fit on a CU; 1/D comes from
// the blocks' inverses.  Each wave computes C^T for 16 columns j by the
// tile's 64 rows i, so that the lanes of the accumulator layout run along i,
// contiguous in the column-major front.
constexpr int kMfTrailThreads = 256;
constexpr int kMfTrailStride = kLB + 1;

__global__ __launch_bounds__(kMfTrailThreads) void k_mf_trailing(const MfNode *__restrict__ nodes,
                                                                 const int2 *__restrict__ blocks, int t0, int nb_max,
                                                                 int jend, double *__restrict__ fronts,
                                                                 const double *__restrict__ inv) {
  using M = Mma<double>;
  constexpr int LS = kMfTrailStride;
  __shared__ double Wi[64 * LS];  // W D^{-1} of rows i0 .. i0 + 63, one block
  __shared__ double Wj[64 * LS];  // W of rows j0 .. j0 + 63, one block
  const int2 bt = blocks[blockIdx.x];
  const MfNode nd = nodes[bt.x];
  const int f = nd.f;
  const int nb = min(nb_max, nd.sp / kLB - t0);
  const int R0 = kLB * (t0 + nb);
  const int jmax = jend > 0 ? kLB * min(jend, nd.sp / kLB) : f;
  int ti = 0, tj = bt.y;
  while (tj > ti) {
    tj -= ti + 1;
    ++ti;
  }
  const int i0 = R0 + 64 * ti, j0 = R0 + 64 * tj;
  double *A = fronts + nd.off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
  typename M::v4 c[4];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + 16 * wave + M::crow(v, lane), i = i0 + 16 * tc + lr;
      c[tc][v] = (i < f && j < f && i >= j) ? A[(int64_t)j * f + i] : 0.0;
    }
  }
  for (int b = 0; b < nb; ++b) {
    const int kb0 = kLB * (t0 + b);
    const double *iv = inv + nd.inv_off + (int64_t)(t0 + b) * kInvStride + kLB * kLB;
    if (b > 0) __syncthreads();  // the previous block's operands are consumed
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kMfTrailThreads * q, r = e >> 4, cc = e & 15;
      const int ii = i0 + r, jj = j0 + r;
      Wi[r * LS + cc] = ii < f ? A[(int64_t)ii * f + kb0 + cc] * iv[cc] : 0.0;
      Wj[r * LS + cc] = jj < f ? A[(int64_t)jj * f + kb0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double a = Wj[(16 * wave + lr) * LS + 4 * s + lk];
#pragma unroll
      for (int tc = 0; tc < 4; ++tc) c[tc] = M::mma(-a, Wi[(16 * tc + lr) * LS + 4 * s + lk], c[tc]);
    }
  }
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + 16 * wave + M::crow(v, lane), i = i0 + 16 * tc + lr;
      if (i < f && j < jmax && i >= j) A[(int64_t)j * f + i] = c[tc][v];
    }
  }
}

// Wave-wide sum (every lane receives it).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int kMfSweepThreads = 1024;
// the forward sweep gives one wave to each row of a 16-row block
static_assert(kMfSweepThreads / 64 == kLB, "one wave per block row");

// Forward sweep L z = diag(s) rhs of one level, one workgroup per node:
// the node's right-hand side (its separator's entries of rhs, sign-flipped on
// the pressure rows) plus its children's boundary parts; then block by block
// y_k = L11^{-1} (z_k - sum_{j<k} W_kj D_j^{-1} y_j) with one wave per row of
// the block.  The node's vector (y on the separator, the boundary part before
// z_b -= W_b D^{-1} y, which k_mf_fwd_bnd applies) goes to zbuf.
__global__ __launch_bounds__(kMfSweepThreads) void k_mf_fwd(const MfNode *__restrict__ nodes,
                                                            const int *__restrict__ list, const int *__restrict__ idx,
                                                            const int *__restrict__ map,
                                                            const double *__restrict__ fronts,
                                                            const double *__restrict__ inv,
                                                            const double *__restrict__ rhs,
                                                            double *__restrict__ zbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double zk[kLB];
  const int k = list[blockIdx.x];
  const MfNode nd = nodes[k];
  const int f = nd.f, sp = nd.sp;
  double *z = reinterpret_cast<double *>(smem_raw);  // f entries
  double *u = z + f;                                 // sp entries: D^{-1} y
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int *id = idx + nd.idx_off;
  for (int p = tid; p < f; p += kMfSweepThreads) {
    const int q = id[p];
    double v = 0.0;
    if (p < sp && q >= 0) v = (q & 1) ? rhs[q] : -rhs[q];
    z[p] = v;
  }
  __syncthreads();
  for (int slot = 0; slot < 2; ++slot) {
    const int c = slot ? nd.child1 : nd.child0;
    if (c < 0) continue;
    const MfNode C = nodes[c];
    const double *zc = zbuf + C.z_off + C.sp;
    for (int i = tid; i < C.r; i += kMfSweepThreads) z[map[C.map_off + i]] += zc[i];
    __syncthreads();
  }
  const double *A = fronts + nd.off;
  const double *iv0 = inv + nd.inv_off;
  for (int k0 = 0; k0 < sp; k0 += kLB) {
    {
      // wave w: row k0 + w of the block against the solved prefix
      const double *row = A + (int64_t)(k0 + wave) * f;
      // eight independent partial sums, so that eight loads of the row are
      // in flight per lane (the large top separators stream their triangle
      // through one workgroup)
      double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int cidx = lane;
      for (; cidx + 7 * 64 < k0; cidx += 8 * 64) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = fma(row[cidx + 64 * q], u[cidx + 64 * q], a[q]);
      }
      for (; cidx < k0; cidx += 64) a[0] = fma(row[cidx], u[cidx], a[0]);
      double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
      acc = wave_sum(acc);
      if (lane == 0) zk[wave] = z[k0 + wave] - acc;
    }
    __syncthreads();
    if (tid < kLB) {
      const double *iv = iv0 + (int64_t)(k0 / kLB) * kInvStride;
      double y = 0.0;
#pragma unroll
      for (int cc = 0; cc < kLB; ++cc) y = fma(iv[tid * kLB + cc], zk[cc], y);
      z[k0 + tid] = y;
      u[k0 + tid] = y * iv[kLB * kLB + tid];
    }
    __syncthreads();
  }
  double *zo = zbuf + nd.z_off;
  for (int p = tid; p < f; p += kMfSweepThreads) zo[p] = z[p];
}

// The forward sweep's boundary rows, kMfFwdRows of one node per workgroup:
// z_b -= W_b D^{-1} y, with y from zbuf and W_b^T read from the upper part of
// the front (column i, rows 0 .. sp - 1, contiguous).  Each wave takes 16
// rows, four at a time.
constexpr int kMfBndThreads = 256;

__global__ __launch_bounds__(kMfBndThreads) void k_mf_fwd_bnd(const MfNode *__restrict__ nodes,
                                                              const int2 *__restrict__ list,
                                                              const double *__restrict__ fronts,
                                                              const double *__restrict__ inv,
                                                              double *__restrict__ zbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *u = reinterpret_cast<double *>(smem_raw);  // sp entries: D^{-1} y
  const int2 e = list[blockIdx.x];
  const MfNode nd = nodes[e.x];
  const int f = nd.f, sp = nd.sp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *zo = zbuf + nd.z_off;
  const double *iv = inv + nd.inv_off;
  for (int c = tid; c < sp; c += kMfBndThreads) u[c] = zo[c] * iv[(int64_t)(c >> 4) * kInvStride + kLB * kLB + (c & 15)];
  __syncthreads();
  const double *A = fronts + nd.off;
  const int ib = sp + kMfFwdRows * e.y + 16 * wave;
  for (int q = 0; q < 16; q += 4) {
    const int i0 = ib + q;
    const double *r0 = A + (int64_t)min(i0, f - 1) * f;
    const double *r1 = A + (int64_t)min(i0 + 1, f - 1) * f;
    const double *r2 = A + (int64_t)min(i0 + 2, f - 1) * f;
    const double *r3 = A + (int64_t)min(i0 + 3, f - 1) * f;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int c = lane; c < sp; c += 64) {
      const double uc = u[c];
      a0 = fma(r0[c], uc, a0);
      a1 = fma(r1[c], uc, a1);
      a2 = fma(r2[c], uc, a2);
      a3 = fma(r3[c], uc, a3);
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    a3 = wave_sum(a3);
    if (lane == 0) {
      if (i0 < f) zo[i0] -= a0;
      if (i0 + 1 < f) zo[i0 + 1] -= a1;
      if (i0 + 2 < f) zo[i0 + 2] -= a2;
      if (i0 + 3 < f) zo[i0 + 3] -= a3;
    }
  }
}

// The backward sweep's boundary product in pieces of kMfBwdCols separator
// columns by kMfBwdRows boundary rows, one piece per workgroup: the partial
// sums of W_b^T x_b over the piece's rows, for k_mf_bwd to subtract.
__global__ __launch_bounds__(kMfBwdCols) void k_mf_bwd_part(const MfNode *__restrict__ nodes,
                                                            const int2 *__restrict__ list,
                                                            const int *__restrict__ idx,
                                                            const double *__restrict__ fronts,
                                                            const double *__restrict__ x,
                                                            double *__restrict__ pbuf) {
  __shared__ double xs[kMfBwdRows];
  const int2 e = list[blockIdx.x];
  const MfNode nd = nodes[e.x];
  const int f = nd.f, sp = nd.sp;
  const int ncc = (sp + kMfBwdCols - 1) / kMfBwdCols;
  const int cc = e.y % ncc, rc = e.y / ncc;
  const int i0 = sp + kMfBwdRows * rc, i1 = min(f, i0 + kMfBwdRows);
  const int *id = idx + nd.idx_off;
  for (int q = threadIdx.x; q < i1 - i0; q += kMfBwdCols) xs[q] = x[id[i0 + q]];
  __syncthreads();
  const int cidx = kMfBwdCols * cc + threadIdx.x;
  if (cidx >= sp) return;
  const double *A = fronts + nd.off + cidx;
  double a0 = 0.0, a1 = 0.0;
  int i = i0;
  for (; i + 1 < i1; i += 2) {
    a0 = fma(A[(int64_t)i * f], xs[i - i0], a0);
    a1 = fma(A[(int64_t)(i + 1) * f], xs[i + 1 - i0], a1);
  }
  if (i < i1) a0 = fma(A[(int64_t)i * f], xs[i - i0], a0);
  pbuf[nd.part_off + (int64_t)rc * sp + cidx] = a0 + a1;
}

// Backward sweep of one level (top-down), one workgroup per node: with the
// boundary unknowns x_b solved by the ancestors, t = y - W_b^T x_b (the
// product summed from k_mf_bwd_part's pieces in order); then from
// the last block down, x_k = L11^{-T} D_k^{-1} t_k and t_j -= W_kj^T x_k for
// the earlier blocks.  The separator's unknowns go to x.
// Levels whose separators hold at most kMfSmallSp unknowns take one
// wavefront per node in the sweeps (the bottom of the tree has tens of
// thousands of small fronts, each of which would otherwise hold a 1024-lane
// workgroup).
constexpr int kMfSmallSp = 64;

// The forward sweep of k_mf_fwd with one wavefront per node: the block's 16
// row products one after another, each the same lane products and wave sum.
__global__ __launch_bounds__(64) void k_mf_fwd_small(const MfNode *__restrict__ nodes,
                                                     const int *__restrict__ list, const int *__restrict__ idx,
                                                     const int *__restrict__ map,
                                                     const double *__restrict__ fronts,
                                                     const double *__restrict__ inv,
                                                     const double *__restrict__ rhs,
                                                     double *__restrict__ zbuf) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double zk[kLB];
  const int k = list[blockIdx.x];
  const MfNode nd = nodes[k];
  const int f = nd.f, sp = nd.sp;
  double *z = reinterpret_cast<double *>(smem_raw);  // f entries
  double *u = z + f;                                 // sp entries: D^{-1} y
  const int lane = threadIdx.x;
  const int *id = idx + nd.idx_off;
  for (int p = lane; p < f; p += 64) {
    const int q = id[p];
    double v = 0.0;
    if (p < sp && q >= 0) v = (q & 1) ? rhs[q] : -rhs[q];
    z[p] = v;
  }
  __syncthreads();
  for (int slot = 0; slot < 2; ++slot) {
    const int c = slot ? nd.child1 : nd.child0;
    if (c < 0) continue;
    const MfNode C = nodes[c];
    const double *zc = zbuf + C.z_off + C.sp;
    for (int i = lane; i < C.r; i += 64) z[map[C.map_off + i]] += zc[i];
    __syncthreads();
  }
  const double *A = fronts + nd.off;
  const double *iv0 = inv + nd.inv_off;
  for (int k0 = 0; k0 < sp; k0 += kLB) {
    for (int w = 0; w < kLB; ++w) {
      // row k0 + w of the block against the solved prefix (k0 < 64: one term a lane)
      const double *row = A + (int64_t)(k0 + w) * f;
      double acc = lane < k0 ? fma(row[lane], u[lane], 0.0) : 0.0;
      acc = wave_sum(acc);
      if (lane == 0) zk[w] = z[k0 + w] - acc;
    }
    __syncthreads();
    if (lane < kLB) {
      const double *iv = iv0 + (int64_t)(k0 / kLB) * kInvStride;
      double y = 0.0;
#pragma unroll
      for (int cc = 0; cc < kLB; ++cc) y = fma(iv[lane * kLB + cc], zk[cc], y);
      z[k0 + lane] = y;
      u[k0 + lane] = y * iv[kLB * kLB + lane];
    }
    __syncthreads();
  }
  double *zo = zbuf + nd.z_off;
  for (int p = lane; p < f; p += 64) zo[p] = z[p];
}

// NT threads: kMfSweepThreads, or one wavefront for the levels whose
// separators hold at most kMfSmallSp unknowns (the many small fronts at the
// bottom of the tree); the arithmetic does not depend on NT.
template <int NT>
__global__ __launch_bounds__(NT) void k_mf_bwd(const MfNode *__restrict__ nodes, const int *__restrict__ list,
                                               const int *__restrict__ idx, const double *__restrict__ fronts,
                                               const double *__restrict__ inv, const double *__restrict__ zbuf,
                                               const double *__restrict__ pbuf, double *__restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int k = list[blockIdx.x];
  const MfNode nd = nodes[k];
  const int f = nd.f, sp = nd.sp;
  double *xs = reinterpret_cast<double *>(smem_raw);  // f entries
  double *tv = xs + f;                                // sp entries
  const int tid = threadIdx.x;
  const int *id = idx + nd.idx_off;
  const double *A = fronts + nd.off;
  const double *zo = zbuf + nd.z_off;
  const int nrc = (nd.r + kMfBwdRows - 1) / kMfBwdRows;
  const double *pp = pbuf + nd.part_off;
  for (int cidx = tid; cidx < sp; cidx += NT) {
    double acc = zo[cidx];
    for (int rc = 0; rc < nrc; ++rc) acc -= pp[(int64_t)rc * sp + cidx];
    tv[cidx] = acc;
  }
  __syncthreads();
  const double *iv0 = inv + nd.inv_off;
  for (int k0 = sp - kLB; k0 >= 0; k0 -= kLB) {
    if (tid < kLB) {
      const double *iv = iv0 + (int64_t)(k0 / kLB) * kInvStride;
      double v = 0.0;
#pragma unroll
      for (int cc = 0; cc < kLB; ++cc) v = fma(iv[cc * kLB + tid], iv[kLB * kLB + cc] * tv[k0 + cc], v);
      xs[k0 + tid] = v;
    }
    __syncthreads();
    for (int cidx = tid; cidx < k0; cidx += NT) {
      double acc = tv[cidx];
#pragma unroll
      for (int r = 0; r < kLB; ++r) acc = fma(-A[(int64_t)(k0 + r) * f + cidx], xs[k0 + r], acc);
      tv[cidx] = acc;
    }
    __syncthreads();
  }
  for (int p = tid; p < sp; p += NT) {
    const int q = id[p];
    if (q >= 0) x[q] = xs[p];
  }
}

__global__ void k_mf_deinterleave(const double *__restrict__ x, int nv, double *__restrict__ X) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nv) return;
  X[p] = x[2 * p];
  X[nv + p] = x[2 * p + 1];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_mf_assemble(const Geom &g, int n_sub, const int *patches, const double *F, const double *Fb,
                              const double *SAb, const MfDevPlan &dp, double *fronts, hipStream_t s) {
  hipError_t e = launch_fill(fronts, dp.front_doubles, 0.0, s);
  if (e != hipSuccess) return e;
  if (n_sub > 0)
    hipLaunchKernelGGL(k_mf_scatter, dim3(n_sub), dim3(256), 0, s, g, patches, F, Fb, SAb, dp.sub_pair_off,
                       dp.pair_off, dp.pair_ld, fronts);
  if (dp.n_nodes > 0)
    hipLaunchKernelGGL(k_mf_pad, dim3((dp.n_nodes + 255) / 256), dim3(256), 0, s, dp.nodes, dp.n_nodes, fronts);
  return hipGetLastError();
}

hipError_t launch_mf_factor(const NdPlan &plan, const MfDevPlan &dp, double *fronts, double *inv, DevStatus *st,
                            hipStream_t s) {
  const int H = (int)plan.level_off.size() - 1;
  size_t si = 0;
  for (int h = 0; h < H; ++h) {
    const int n0 = plan.level_off[h], nn = plan.level_off[h + 1] - n0;
    if (nn <= 0) continue;
    const int *list = dp.level_nodes + n0;
    if (plan.level_child_rmax[h] > 0) {
      const unsigned gy = (unsigned)((plan.level_child_rmax[h] + 15) / 16);
      hipLaunchKernelGGL(k_mf_extend, dim3(nn, gy), dim3(256), 0, s, dp.nodes, list, dp.map, 0, fronts);
      hipLaunchKernelGGL(k_mf_extend, dim3(nn, gy), dim3(256), 0, s, dp.nodes, list, dp.map, 1, fronts);
    }
    hipLaunchKernelGGL(k_mf_first, dim3(nn), dim3(64), 0, s, dp.nodes, list, fronts, inv, st);
    for (; si < plan.steps.size() && plan.steps[si].level == h; ++si) {
      const MfStepLaunch &L = plan.steps[si];
      const int2 *bl = dp.step_blocks + L.blk_off;
      if (L.kind == kMfPanelStep)
        hipLaunchKernelGGL(k_mf_step, dim3(L.n_blocks), dim3(kMfStepThreads), 0, s, dp.nodes, bl, L.t, plan.panel,
                           fronts, inv, st);
      else if (L.kind == kMfTrailing)
        hipLaunchKernelGGL(k_mf_trailing, dim3(L.n_blocks), dim3(kMfTrailThreads), 0, s, dp.nodes, bl, L.t, L.nb,
                           L.jend, fronts, inv);
      else
        hipLaunchKernelGGL(k_mf_diag, dim3(L.n_blocks), dim3(64), 0, s, dp.nodes, bl, L.t, fronts, inv, st);
    }
  }
  return hipGetLastError();
}

hipError_t launch_mf_solve(const NdPlan &plan, const MfDevPlan &dp, const double *fronts, const double *inv,
                           double *zbuf, double *pbuf, const double *rhs, double *x, hipStream_t s) {
  const int H = (int)plan.level_off.size() - 1;
  // the plan keeps every level's (f + sp) within kMfSweepLdsMax, which
  // mf_init_kernels has allowed
  for (int h = 0; h < H; ++h) {
    const int n0 = plan.level_off[h], nn = plan.level_off[h + 1] - n0;
    const size_t lds = (size_t)plan.level_lds[h] * sizeof(double);
    if (plan.level_spmax[h] <= kMfSmallSp)
      hipLaunchKernelGGL(k_mf_fwd_small, dim3(nn), dim3(64), lds, s, dp.nodes, dp.level_nodes + n0, dp.idx, dp.map,
                         fronts, inv, rhs, zbuf);
    else
      hipLaunchKernelGGL(k_mf_fwd, dim3(nn), dim3(kMfSweepThreads), lds, s, dp.nodes, dp.level_nodes + n0, dp.idx,
                         dp.map, fronts, inv, rhs, zbuf);
    const int nfb = plan.level_fb_off[h + 1] - plan.level_fb_off[h];
    if (nfb > 0)
      hipLaunchKernelGGL(k_mf_fwd_bnd, dim3(nfb), dim3(kMfBndThreads), (size_t)plan.level_spmax[h] * sizeof(double),
                         s, dp.nodes, dp.fwd_bnd + plan.level_fb_off[h], fronts, inv, zbuf);
  }
  for (int h = H - 1; h >= 0; --h) {
    const int n0 = plan.level_off[h], nn = plan.level_off[h + 1] - n0;
    const size_t lds = (size_t)plan.level_lds[h] * sizeof(double);
    const int nbb = plan.level_bb_off[h + 1] - plan.level_bb_off[h];
    if (nbb > 0)
      hipLaunchKernelGGL(k_mf_bwd_part, dim3(nbb), dim3(kMfBwdCols), 0, s, dp.nodes, dp.bwd_bnd + plan.level_bb_off[h],
                         dp.idx, fronts, x, pbuf);
    if (plan.level_spmax[h] <= kMfSmallSp)
      hipLaunchKernelGGL((k_mf_bwd<64>), dim3(nn), dim3(64), lds, s, dp.nodes, dp.level_nodes + n0, dp.idx, fronts,
                         inv, zbuf, pbuf, x);
    else
      hipLaunchKernelGGL((k_mf_bwd<kMfSweepThreads>), dim3(nn), dim3(kMfSweepThreads), lds, s, dp.nodes,
                         dp.level_nodes + n0, dp.idx, fronts, inv, zbuf, pbuf, x);
  }
  return hipGetLastError();
}

hipError_t mf_init_kernels() {
  hipError_t e = hipFuncSetAttribute((const void *)k_mf_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kMfSweepLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_mf_bwd<kMfSweepThreads>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMfSweepLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_mf_bwd<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMfSweepLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_mf_fwd_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMfSweepLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)k_mf_fwd_bnd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kMfSweepLdsMax);
  return e;
}

hipError_t launch_mf_residual(const Geom &g, const int *patches, const double *F, const double *Fb,
                              const double *SAb, const int4 *pinfo, int nv, const double *x, double *r, double *b,
                              hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_residual, dim3((nv + 255) / 256), dim3(256), 0, s, g, patches, F, Fb, SAb, pinfo, nv, x, r,
                     b);
  return hipGetLastError();
}

hipError_t launch_mf_dense(const Geom &g, const int *patches, const double *F, const double *Fb, const double *SAb,
                           const int4 *pinfo, int nv, double *A, double *b, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipError_t e = launch_fill(A, 4LL * nv * nv, 0.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mf_dense, dim3((nv + 255) / 256), dim3(256), 0, s, g, patches, F, Fb, SAb, pinfo, nv, A, b);
  return hipGetLastError();
}

hipError_t launch_mf_deinterleave(const double *x, int nv, double *X, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mf_deinterleave, dim3((nv + 255) / 256), dim3(256), 0, s, x, nv, X);
  return hipGetLastError();
}

}  // namespace mrcm
