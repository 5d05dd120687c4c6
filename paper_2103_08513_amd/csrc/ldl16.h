// LDL^T of a 16x16 diagonal block on one wave, shared by the band and the
// multifrontal factorisations of the interface system.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace mrcm {

constexpr int kLB = 16;
constexpr int kInvStride = kLB * kLB + kLB;

// 16x16 LDL^T of a diagonal block of size kb <= 16 whose lower triangle is
// given row-major in blk (stride 17, the upper part zero); rows and columns
// past kb act as the identity.  Runs on one wave; hands L (below the
// diagonal), D (on it) and U = D L^T (above it) to store(t, i, value) for
// entry (row i, column t), and writes L11^{-1} (row-major), 1/D into inv, both staged
// through the LDS buffers S (544 doubles, may start at blk: blk is read
// first) and T (272 doubles), so that the global stores are contiguous runs.
// The wave's LDS accesses complete in order, so its reads see its writes.  Returns nonzero on a zero or
// non-finite pivot.
template <typename Store>
__device__ __attribute__((always_inline)) int ldl_diag16(const double *blk, int kb, int lane, Store store,
                                                         double *__restrict__ inv, double *S, double *T) {
  int r = lane & 15;
  // opaque to the optimiser, as in the local factor: lane-derived constants
  // are recomputed rather than held across the caller's loop
  asm volatile("" : "+v"(r));
  double v[kLB], x[kLB];
#pragma unroll
  for (int c = 0; c < kLB; ++c) {
    const double a = blk[r * (kLB + 1) + c];
    v[c] = (c < kb && r < kb) ? a : ((r == c) ? 1.0 : 0.0);
    x[c] = (r == c) ? 1.0 : 0.0;
  }
  double ok = 1.0;
  // 1/d from the hardware estimate q (relative error near 2^-24) by one
  // third-order step: with e = 1 - d q, 1/d = q (1 + e + e^2 + ...), and the
  // truncation leaves an error of order e^3.  A zero or non-finite pivot is
  // flagged beside the chain, not on it.
  auto recip = [&](double d) -> double {
    ok = (d != 0.0 && isfinite(d)) ? ok : 0.0;
    const double q = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, q, 1.0);
    return fma(q, fma(e, e, e), q);
  };
  // Software-pipelined: pivot jj finishes row jj + 1 first and starts the
  // reciprocal of the next pivot; the updates of the remaining rows are
  // issued between the dependent steps of that reciprocal, whose latency they
  // cover (the scheduling barriers keep this interleaving, which the
  // compiler would otherwise undo by grouping the dependent chain).
  double dcur = row_bcast(v[0], 0);
  double q = recip(dcur);
#pragma unroll
  for (int jj = 0; jj < kLB; ++jj) {
    double dn = 0.0;
    const double wv = v[jj] * q;
    const double xq = x[jj] * q;
    // Results of pivot jj, final from here on, go to LDS off the chain, at
    // lane-based addresses with constant offsets.  S[t * 17 + i] = entry
    // (i, t) of the factored block: lane r > jj holds L[r][jj] = wv (written
    // to the lower half of S) and U[jj][r] = v[jj] (the upper half of S + 272);
    // D_jj is the pivot dcur.  Lanes r < jj write to the other half of
    // each, which is never read.  Lane r's x is column r of L11^{-1}, whose
    // entry jj is final too.
    S[jj * (kLB + 1) + r] = (r == jj) ? dcur : wv;
    S[kLB * (kLB + 1) + r * (kLB + 1) + jj] = (r == jj) ? dcur : v[jj];
    T[jj * kLB + r] = x[jj];
    T[kLB * kLB + jj] = q;
    auto upd = [&](int i) {
      if (i < kLB) {
        const double a = row_bcast(v[jj], i);
        v[i] -= wv * a;
        x[i] -= a * xq;
      }
    };
    if (jj + 1 < kLB) {
      // The next pivot, d = A'[jj+1][jj+1] - a^2 / D with a = A'[jj+1][jj],
      // formed in every lane from values final before this pivot, so that
      // only one FMA after 1/D sits on the chain; it is also the D stored for
      // that pivot (lane jj+1's own update of v[jj+1] agrees up to rounding).
      const double a = row_bcast(v[jj], jj + 1);
      const double vd = row_bcast(v[jj + 1], jj + 1);
      const double d = fma(-q, a * a, vd);
      dn = d;
      v[jj + 1] -= wv * a;
      x[jj + 1] -= a * xq;
      ok = (d != 0.0 && isfinite(d)) ? ok : 0.0;
      const double q0 = __builtin_amdgcn_rcp(d);
      upd(jj + 2);
      upd(jj + 3);
      __builtin_amdgcn_sched_barrier(0);
      const double e = fma(-d, q0, 1.0);
      upd(jj + 4);
      upd(jj + 5);
      __builtin_amdgcn_sched_barrier(0);
      const double t = fma(e, e, e);
      upd(jj + 6);
      upd(jj + 7);
      __builtin_amdgcn_sched_barrier(0);
      q = fma(q0, t, q0);
#pragma unroll
      for (int i = jj + 8; i < kLB; ++i) upd(i);
    }
    dcur = dn;
    __builtin_amdgcn_sched_barrier(0);
  }
  // column t of the block, rows 0 .. 15: sixteen entries per column, which the
  // caller's store places (contiguously in both storage forms used)
#pragma unroll
  for (int e = lane; e < kLB * kLB; e += 64) {
    const int t = e >> 4, i = e & 15;
    const double val = S[(i < t ? kLB * (kLB + 1) : 0) + t * (kLB + 1) + i];
    if (t < kb && i < kb) store(t, i, val);
  }
#pragma unroll
  for (int e = lane; e < kInvStride; e += 64) inv[e] = T[e];
  return ok == 1.0 ? 0 : 1;
}


}  // namespace mrcm
