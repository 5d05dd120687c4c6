// C ABI of the MRCM library: argument validation, subdomain / interface
// descriptors, reverse Cuthill-McKee ordering of the interface unknowns,
// device memory plan, and the enqueueing of the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "../../include/mrcm.h"
#include "../../include/mrcm_nn.h"
#include "internal.h"
#include "launch.h"
#include "nd_plan.h"

using namespace mrcm;

namespace {

thread_local std::string g_last_error;

mrcm_status fail(mrcm_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(MRCM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));       \
  } while (0)

template <typename T>
hipError_t dev_alloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void **)p, n * sizeof(T));
}

template <typename T>
hipError_t upload(T **p, const std::vector<T> &v) {
  hipError_t e = dev_alloc(p, v.size());
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Host description of the geometry: everything that does not depend on the
// coefficient arrays.
struct HostGeom {
  int n[3];
  double h[3];
  double alpha;
  int beta_mode = 0;
  uint32_t keep = 0;
  int precision;
  int wall_type[6];
  int64_t pin;
  std::vector<int> cuts[3];
  std::vector<int> split;  // 2 per interface (resolved, never 0)
  std::vector<SubDesc> subs;
  std::vector<IfaceDesc> ifcs;
  std::vector<int> patches;  // concatenated I^l
  std::vector<int> order;    // launch order, most expensive first
  std::vector<int4> work;    // solve work items (subdomain, first column, end column)
  std::vector<int> col_sub;  // per right-hand-side column: its subdomain
  std::vector<int> sub_of[3];
  int n_patch = 0;
  int solve_tiles = 0;   // 16-column tiles per solve work item (0: the largest chunk)
  int solve_group = 0;   // FP64 pipeline: solve group 0's size (0: occupancy rule, -1: none)
  int iface_panel = kMfPanelMax;  // blocks per panel of the multifrontal interface factorisation
  int launch_mode = MRCM_LAUNCH_GRID;  // ragged launches: grid, or persistent over a work queue
  int bmax = 0, mmax = 0, max_cells = 0;
  long long max_nm = 0;
  int64_t totL = 0, totD = 0, totX = 0, totF = 0, totCells = 0;
  int totCols = 0;
  int64_t n_mbfs = 0, n_rhs = 0;
  double factor_flops = 0.0, solve_flops = 0.0;
};

// The raw inputs that determine a handle's geometry, compared before any
// rebuild so that a rebuild in place skips the host-side geometry work.
struct ConfigKey {
  int32_t n[3] = {0, 0, 0};
  double h[3] = {0.0, 0.0, 0.0};
  int32_t wall_type[6] = {0, 0, 0, 0, 0, 0};
  int64_t pin = 0;
  double alpha = 0.0;
  int32_t beta_mode = 0;
  uint32_t keep = 0;
  int32_t precision = 0;
  int32_t solve_tiles = 0, solve_group = 0, iface_panel = 0, launch_mode = 0;
  std::vector<int32_t> cuts[3];
  int32_t us[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  std::vector<int32_t> split;
  bool operator==(const ConfigKey &o) const {
    for (int d = 0; d < 3; ++d)
      if (n[d] != o.n[d] || h[d] != o.h[d] || cuts[d] != o.cuts[d] || us[d][0] != o.us[d][0] ||
          us[d][1] != o.us[d][1])
        return false;
    for (int f = 0; f < 6; ++f)
      if (wall_type[f] != o.wall_type[f]) return false;
    return pin == o.pin && alpha == o.alpha && beta_mode == o.beta_mode && keep == o.keep && precision == o.precision &&
           split == o.split && solve_tiles == o.solve_tiles && solve_group == o.solve_group &&
           iface_panel == o.iface_panel && launch_mode == o.launch_mode;
  }
};

// false when an input is missing or malformed: the full check then reports it
bool make_key(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
              const mrcm_options *opt, ConfigKey &k) {
  if (!pb || !part || !ifs || !opt) return false;
  k.n[0] = pb->nx;
  k.n[1] = pb->ny;
  k.n[2] = pb->nz;
  k.h[0] = pb->hx;
  k.h[1] = pb->hy;
  k.h[2] = pb->hz;
  for (int f = 0; f < 6; ++f) k.wall_type[f] = pb->wall_type[f];
  k.pin = pb->pin_cell;
  k.alpha = opt->alpha;
  k.beta_mode = opt->beta_mode;
  k.keep = opt->keep;
  k.precision = opt->precision;
  k.solve_tiles = opt->solve_tiles;
  k.solve_group = opt->solve_group;
  k.iface_panel = opt->iface_panel;
  k.launch_mode = opt->launch_mode;
  const int nd[3] = {part->ndx, part->ndy, part->ndz};
  const int32_t *cut_in[3] = {part->cut_x, part->cut_y, part->cut_z};
  for (int d = 0; d < 3; ++d) {
    if (nd[d] < 1 || nd[d] > (1 << 20) || !cut_in[d]) return false;
    k.cuts[d].assign(cut_in[d], cut_in[d] + nd[d] + 1);
    k.us[d][0] = ifs->uniform_split[d][0];
    k.us[d][1] = ifs->uniform_split[d][1];
  }
  if (ifs->split) {
    const int64_t ni = (int64_t)(nd[0] - 1) * nd[1] * nd[2] + (int64_t)nd[0] * (nd[1] - 1) * nd[2] +
                       (int64_t)nd[0] * nd[1] * (nd[2] - 1);
    k.split.assign(ifs->split, ifs->split + 2 * ni);
  }
  return true;
}

bool same_config(const HostGeom &a, const HostGeom &b) {
  for (int d = 0; d < 3; ++d)
    if (a.n[d] != b.n[d] || a.h[d] != b.h[d] || a.cuts[d] != b.cuts[d]) return false;
  for (int f = 0; f < 6; ++f)
    if (a.wall_type[f] != b.wall_type[f]) return false;
  return a.alpha == b.alpha && a.beta_mode == b.beta_mode && a.keep == b.keep && a.precision == b.precision &&
         a.pin == b.pin &&
         a.split == b.split && a.solve_tiles == b.solve_tiles && a.solve_group == b.solve_group;
}

mrcm_status build_host_geom(const mrcm_problem *pb, const mrcm_partition *part,
                            const mrcm_iface_space *ifs, const mrcm_options *opt, HostGeom &G) {
  if (!pb || !part || !ifs || !opt) return fail(MRCM_EINVAL, "null argument");
  G.n[0] = pb->nx;
  G.n[1] = pb->ny;
  G.n[2] = pb->nz;
  G.h[0] = pb->hx;
  G.h[1] = pb->hy;
  G.h[2] = pb->hz;
  for (int d = 0; d < 3; ++d) {
    if (G.n[d] < 1) return fail(MRCM_EINVAL, "grid dimensions must be positive");
    if (!(G.h[d] > 0.0) || !std::isfinite(G.h[d])) return fail(MRCM_EINVAL, "cell sizes must be positive");
  }
  if (!pb->kx || !pb->ky || !pb->kz || !pb->q) return fail(MRCM_EINVAL, "kx, ky, kz and q are required");
  const int64_t N = (int64_t)G.n[0] * G.n[1] * G.n[2];
  if (N > (int64_t)1 << 31) return fail(MRCM_EUNSUPPORTED, "more than 2^31 cells");
  bool dirichlet = false;
  for (int f = 0; f < 6; ++f) {
    G.wall_type[f] = pb->wall_type[f];
    if (G.wall_type[f] < 0 || G.wall_type[f] > 2) return fail(MRCM_EINVAL, "wall type must be 0, 1 or 2");
    if (G.wall_type[f] == MRCM_WALL_DIRICHLET) dirichlet = true;
  }
  G.pin = pb->pin_cell;
  if (G.pin < -1 || G.pin >= N) return fail(MRCM_EINVAL, "pin_cell out of range");
  if (G.pin < 0 && !dirichlet)
    return fail(MRCM_EINVAL, "a pinned cell or a Dirichlet wall is needed to fix the pressure");
  G.alpha = opt->alpha;
  if (!(G.alpha > 0.0) || !std::isfinite(G.alpha)) return fail(MRCM_EINVAL, "alpha must be positive");
  G.beta_mode = opt->beta_mode;
  if (G.beta_mode != MRCM_BETA_PER_SIDE && G.beta_mode != MRCM_BETA_FACE)
    return fail(MRCM_EINVAL, "beta_mode must be MRCM_BETA_PER_SIDE or MRCM_BETA_FACE");
  G.precision = opt->precision;
  if (opt->solve_tiles < 0 || opt->solve_tiles > solve_chunk_max() / 16)
    return fail(MRCM_EINVAL, "solve_tiles must be in [0, " + std::to_string(solve_chunk_max() / 16) + "]");
  if (opt->solve_group < -1) return fail(MRCM_EINVAL, "solve_group must be -1, 0 or a positive count");
  G.solve_tiles = opt->solve_tiles;
  G.solve_group = opt->solve_group;
  if (opt->iface_panel < 0 || opt->iface_panel > kMfPanelMax)
    return fail(MRCM_EINVAL, "iface_panel must be in [0, " + std::to_string(kMfPanelMax) + "]");
  G.iface_panel = opt->iface_panel > 0 ? opt->iface_panel : kMfPanelMax;
  if (opt->launch_mode != MRCM_LAUNCH_GRID && opt->launch_mode != MRCM_LAUNCH_QUEUE)
    return fail(MRCM_EINVAL, "launch_mode must be MRCM_LAUNCH_GRID or MRCM_LAUNCH_QUEUE");
  G.launch_mode = opt->launch_mode;
  if (G.precision != MRCM_FP64 && G.precision != MRCM_FP32_IR && G.precision != MRCM_PCG)
    return fail(MRCM_EINVAL, "precision must be MRCM_FP64, MRCM_FP32_IR or MRCM_PCG");
  G.keep = opt->keep ? opt->keep : (MRCM_KEEP_FACTORS | MRCM_KEEP_MBFS);
  if (G.keep & ~(uint32_t)(MRCM_KEEP_FACTORS | MRCM_KEEP_MBFS)) return fail(MRCM_EINVAL, "unknown keep bits");
  if (!(G.keep & MRCM_KEEP_MBFS) && !(G.keep & MRCM_KEEP_FACTORS))
    return fail(MRCM_EINVAL, "reconstruction needs the MBFs or the factors: keep one of them");
  if (!(G.keep & MRCM_KEEP_MBFS) && G.precision == MRCM_PCG)
    return fail(MRCM_EINVAL, "the conjugate-gradient form keeps no factors: reconstruction needs the MBFs");

  const int nd[3] = {part->ndx, part->ndy, part->ndz};
  const int32_t *cut_in[3] = {part->cut_x, part->cut_y, part->cut_z};
  for (int d = 0; d < 3; ++d) {
    if (nd[d] < 1 || nd[d] > G.n[d]) return fail(MRCM_EINVAL, "subdomain counts must be in [1, n]");
    G.cuts[d].resize(nd[d] + 1);
    for (int s = 0; s <= nd[d]; ++s)
      G.cuts[d][s] = cut_in[d] ? cut_in[d][s] : (int)(((int64_t)s * G.n[d]) / nd[d]);
    if (G.cuts[d][0] != 0 || G.cuts[d][nd[d]] != G.n[d])
      return fail(MRCM_EINVAL, "cuts must start at 0 and end at n");
    for (int s = 0; s < nd[d]; ++s)
      if (G.cuts[d][s + 1] <= G.cuts[d][s]) return fail(MRCM_EINVAL, "cuts must increase strictly");
    G.sub_of[d].resize(G.n[d]);
    for (int s = 0; s < nd[d]; ++s)
      for (int x = G.cuts[d][s]; x < G.cuts[d][s + 1]; ++x) G.sub_of[d][x] = s;
  }
  const int n_sub = nd[0] * nd[1] * nd[2];
  G.subs.assign(n_sub, SubDesc{});
  auto sid = [&](int sx, int sy, int sz) { return sx + nd[0] * (sy + nd[1] * sz); };
  for (int sz = 0; sz < nd[2]; ++sz)
    for (int sy = 0; sy < nd[1]; ++sy)
      for (int sx = 0; sx < nd[0]; ++sx) {
        SubDesc &S = G.subs[sid(sx, sy, sz)];
        const int s[3] = {sx, sy, sz};
        for (int d = 0; d < 3; ++d) {
          S.lo[d] = G.cuts[d][s[d]];
          S.ext[d] = G.cuts[d][s[d] + 1] - G.cuts[d][s[d]];
        }
        // shortest axis fastest, ties by lower axis id
        int ax[3] = {0, 1, 2};
        std::stable_sort(ax, ax + 3, [&](int a, int b) { return S.ext[a] < S.ext[b]; });
        for (int k = 0; k < 3; ++k) S.ax[k] = ax[k];
        S.n0 = S.ext[ax[0]];
        S.n1 = S.ext[ax[1]];
        S.n2 = S.ext[ax[2]];
        S.N = S.n0 * S.n1 * S.n2;
        S.b = S.n0 * S.n1;
        for (int f = 0; f < 6; ++f) {
          S.face_if[f] = -1;
          S.face_p0[f] = 0;
        }
        S.pin_local = -1;
      }
  // interfaces: x-normal, then y, then z, each by increasing lower id
  G.ifcs.clear();
  int p0 = 0;
  int t = 0;
  int n_if = 0;
  for (int d = 0; d < 3; ++d) {
    int c = 1;
    for (int e = 0; e < 3; ++e) c *= (e == d) ? nd[e] - 1 : nd[e];
    n_if += c;
  }
  G.split.assign(2 * (size_t)n_if, 0);
  for (int d = 0; d < 3; ++d) {
    const int a = (d == 0) ? 1 : 0;
    const int b = (d == 2) ? 1 : 2;
    for (int l = 0; l < n_sub; ++l) {
      const int s[3] = {l % nd[0], (l / nd[0]) % nd[1], l / (nd[0] * nd[1])};
      if (s[d] + 1 >= nd[d]) continue;
      int s2[3] = {s[0], s[1], s[2]};
      s2[d] += 1;
      const int l2 = sid(s2[0], s2[1], s2[2]);
      IfaceDesc I;
      I.d = d;
      I.lo_sub = l;
      I.hi_sub = l2;
      I.a = a;
      I.b = b;
      I.la = G.subs[l].ext[a];
      I.lb = G.subs[l].ext[b];
      int na = ifs->split ? ifs->split[2 * t] : ifs->uniform_split[d][0];
      int nb = ifs->split ? ifs->split[2 * t + 1] : ifs->uniform_split[d][1];
      if (na == 0 && nb == 0) {
        na = I.la;
        nb = I.lb;
      }
      if (na < 1 || nb < 1 || na > I.la || nb > I.lb)
        return fail(MRCM_EINVAL, "interface split " + std::to_string(t) + " does not fit its face");
      I.na = na;
      I.nb = nb;
      I.p0 = p0;
      G.split[2 * t] = na;
      G.split[2 * t + 1] = nb;
      p0 += na * nb;
      G.ifcs.push_back(I);
      G.subs[l].face_if[2 * d + 1] = t;
      G.subs[l2].face_if[2 * d] = t;
      ++t;
    }
  }
  G.n_patch = p0;
  // per-subdomain patch lists (faces -x..+z, i.e. increasing global id) and offsets
  G.patches.clear();
  G.bmax = G.mmax = G.max_cells = 0;
  G.max_nm = 0;
  G.totL = G.totD = G.totX = G.totF = G.totCells = 0;
  G.totCols = 0;
  G.n_mbfs = G.n_rhs = 0;
  G.factor_flops = G.solve_flops = 0.0;
  for (int l = 0; l < n_sub; ++l) {
    SubDesc &S = G.subs[l];
    S.patch_off = (int)G.patches.size();
    int np = 0;
    for (int f = 0; f < 6; ++f) {
      if (S.face_if[f] < 0) continue;
      const IfaceDesc &I = G.ifcs[S.face_if[f]];
      S.face_p0[f] = np;
      for (int k = 0; k < I.na * I.nb; ++k) G.patches.push_back(I.p0 + k);
      np += I.na * I.nb;
    }
    S.npatch = np;
    S.m = 2 * np + 1;
    S.cell_off = G.totCells;
    S.L_off = G.totL;
    S.D_off = G.totD;
    S.X_off = G.totX;
    S.F_off = G.totF;
    S.col_off = G.totCols;
    G.totCells += S.N;
    G.totL += (int64_t)S.N * (S.b + 1);
    G.totD += (int64_t)((S.N + kNB - 1) / kNB) * kNB * kNB;
    G.totX += (int64_t)S.N * S.m;
    G.totF += (int64_t)S.npatch * S.m;
    G.totCols += S.m;
    G.bmax = std::max(G.bmax, S.b);
    G.mmax = std::max(G.mmax, S.m);
    G.max_cells = std::max(G.max_cells, S.N);
    G.max_nm = std::max(G.max_nm, (long long)S.N * S.m);
    G.n_mbfs += 2 * np;
    G.n_rhs += S.m;
    for (int k = 0; k < S.N; ++k) {
      const double bk = std::min(S.b, S.N - 1 - k);
      G.factor_flops += bk * bk + 2.0 * bk + 1.0;
    }
    G.solve_flops += 4.0 * S.N * (double)S.b * S.m;
    if (G.pin >= 0) {
      const int x[3] = {(int)(G.pin % G.n[0]), (int)((G.pin / G.n[0]) % G.n[1]),
                        (int)(G.pin / ((int64_t)G.n[0] * G.n[1]))};
      bool inside = true;
      for (int d = 0; d < 3; ++d) inside = inside && x[d] >= S.lo[d] && x[d] < S.lo[d] + S.ext[d];
      if (inside) {
        const int t0 = x[S.ax[0]] - S.lo[S.ax[0]], t1 = x[S.ax[1]] - S.lo[S.ax[1]],
                  t2 = x[S.ax[2]] - S.lo[S.ax[2]];
        S.pin_local = t0 + S.n0 * (t1 + S.n1 * t2);
      }
    }
  }
  const int bcap = G.precision == MRCM_FP32_IR ? kMaxBand32 : kMaxBand64;
  if (G.bmax > bcap)
    return fail(MRCM_EUNSUPPORTED, "local bandwidth " + std::to_string(G.bmax) + " exceeds " +
                                       std::to_string(bcap) + " for this precision");
  if (G.mmax > kMaxRhs)
    return fail(MRCM_EUNSUPPORTED, "a subdomain has " + std::to_string(G.mmax) +
                                       " right-hand sides; the limit is " + std::to_string(kMaxRhs));
  if (G.precision == MRCM_PCG && G.max_cells > pcg_max_cells())
    return fail(MRCM_EUNSUPPORTED, "a subdomain has " + std::to_string(G.max_cells) +
                                       " cells; the conjugate-gradient kernel holds at most " +
                                       std::to_string(pcg_max_cells()));
  G.col_sub.resize(G.totCols);
  for (int l = 0; l < n_sub; ++l)
    for (int c = 0; c < G.subs[l].m; ++c) G.col_sub[G.subs[l].col_off + c] = l;
  const int fp32 = G.precision == MRCM_FP32_IR;
  // the factor kernel also holds a few bytes of static LDS
  if (solve_lds_bytes(fp32, G.bmax, G.mmax) > 160 * 1024 || factor_lds_bytes(fp32, G.bmax) > 160 * 1024 - 64)
    return fail(MRCM_EUNSUPPORTED, "band and right-hand-side window exceed the 160 KiB LDS");
  // launch order: most expensive subdomain first (N b^2 + N b m)
  G.order.resize(n_sub);
  for (int l = 0; l < n_sub; ++l) G.order[l] = l;
  std::stable_sort(G.order.begin(), G.order.end(), [&](int a, int b) {
    const SubDesc &A = G.subs[a], &B = G.subs[b];
    const double ca = (double)A.N * A.b * (A.b + 4.0 * A.m);
    const double cb = (double)B.N * B.b * (B.b + 4.0 * B.m);
    return ca > cb;
  });
  // Solve work items: column chunks of whole 16-column tiles, at most
  // solve_chunk_max() columns, balanced.  Chunks of one subdomain go to the
  // same XCD (workgroup i runs on XCD i mod 8) so they share its L2 when they
  // read the subdomain's factor; consecutive subdomains rotate over XCDs.
  {
    const int kXcd = 8;
    std::vector<std::vector<int4>> per(kXcd);
    const int maxt = G.solve_tiles > 0 ? G.solve_tiles : solve_chunk_max() / 16;
    for (int idx = 0; idx < n_sub; ++idx) {
      const int l = G.order[idx];
      const SubDesc &S = G.subs[l];
      const int nt = (S.m + 15) / 16;
      const int nch = (nt + maxt - 1) / maxt;
      for (int ch = 0; ch < nch; ++ch) {
        const int t0 = split_start(ch, nt, nch), t1 = split_start(ch + 1, nt, nch);
        per[idx % kXcd].push_back(make_int4(l, 16 * t0, std::min(S.m, 16 * t1), 0));
      }
    }
    size_t kmax = 0;
    for (auto &v : per) kmax = std::max(kmax, v.size());
    G.work.assign(kXcd * kmax, make_int4(-1, 0, 0, 0));
    for (int x = 0; x < kXcd; ++x)
      for (size_t k = 0; k < per[x].size(); ++k) G.work[kXcd * k + x] = per[x][k];
  }
  return MRCM_OK;
}

// Reverse Cuthill-McKee ordering of the patch graph (patches adjacent when a
// subdomain contains both); returns pos[patch] and the resulting bandwidth of
// the interleaved (pi^p, pi^u) unknowns.
void rcm_order(const HostGeom &G, std::vector<int> &pos, int &w) {
  const int nv = G.n_patch;
  std::vector<std::vector<int>> adj(nv);
  for (const SubDesc &S : G.subs) {
    for (int i = 0; i < S.npatch; ++i)
      for (int j = 0; j < S.npatch; ++j)
        if (i != j) adj[G.patches[S.patch_off + i]].push_back(G.patches[S.patch_off + j]);
  }
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  std::vector<int> deg(nv);
  for (int i = 0; i < nv; ++i) deg[i] = (int)adj[i].size();
  std::vector<int> perm;
  perm.reserve(nv);
  std::vector<char> seen(nv, 0);
  auto bfs = [&](int start, std::vector<int> &out, std::vector<int> &level) {
    out.clear();
    std::vector<int> lev(nv, -1);
    std::deque<int> qu;
    qu.push_back(start);
    lev[start] = 0;
    while (!qu.empty()) {
      const int u = qu.front();
      qu.pop_front();
      out.push_back(u);
      std::vector<int> nb;
      for (int v : adj[u])
        if (lev[v] < 0 && !seen[v]) nb.push_back(v);
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); });
      for (int v : nb) {
        lev[v] = lev[u] + 1;
        qu.push_back(v);
      }
    }
    level = lev;
  };
  for (int s0 = 0; s0 < nv; ++s0) {
    if (seen[s0]) continue;
    // pseudo-peripheral start: repeat BFS from the farthest, lowest-degree node
    int start = s0;
    std::vector<int> comp, lev;
    int ecc = -1;
    for (int it = 0; it < 4; ++it) {
      bfs(start, comp, lev);
      int far = start, best = -1;
      for (int u : comp)
        if (lev[u] > best || (lev[u] == best && deg[u] < deg[far])) {
          best = lev[u];
          far = u;
        }
      if (best <= ecc) break;
      ecc = best;
      start = far;
    }
    bfs(start, comp, lev);
    for (int u : comp) {
      seen[u] = 1;
      perm.push_back(u);
    }
  }
  std::reverse(perm.begin(), perm.end());
  pos.assign(nv, 0);
  for (int i = 0; i < nv; ++i) pos[perm[i]] = i;
  int bw = 1;
  for (int u = 0; u < nv; ++u)
    for (int v : adj[u]) bw = std::max(bw, 2 * std::abs(pos[u] - pos[v]) + 1);
  w = bw;
}

// Stage profiling: event pairs recorded on the caller's stream, resolved
// after the call's own synchronisation.
struct Profile {
  bool on = false;
  double ms[16] = {};
  int64_t count[16] = {};
  struct Pending {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
};
Profile g_prof;
// set while mrcm_graph_capture records a step: every call then only
// enqueues work (no status reads, synchronisations or profiling events)
thread_local bool g_capturing = false;

struct Stage {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Stage(int st, hipStream_t str) : stage(st), s(str) {
    if (!g_prof.on || g_capturing) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
  }
  ~Stage() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    g_prof.pending.push_back({stage, a, b});
  }
};

void profile_flush() {
  if (g_capturing) return;
  for (auto &p : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_prof.ms[p.stage] += ms;
      g_prof.count[p.stage] += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_prof.pending.clear();
}

}  // namespace

struct mrcm_mbfs {
  ConfigKey key;  // raw configuration inputs of the build that created the handle
  HostGeom G;
  Geom g{};
  int n_sub = 0;
  SubDesc *d_sub = nullptr;
  IfaceDesc *d_ifc = nullptr;
  int *d_order = nullptr;
  int4 *d_work = nullptr;
  int *d_queue = nullptr;  // work-queue counters: eight per stream (slot 0 the caller's, 1 the second)
  // FP64 path: when the solve work exceeds one round of resident workgroups,
  // the first n_first items form group 0 and the rest group 1 (whole
  // subdomains each); group 0's refinement overlaps group 1's first solve on
  // a second stream
  int n_first = 0;
  std::vector<int> solve_group;  // per subdomain
  int *d_grp_subs[2] = {nullptr, nullptr};
  int *d_order_split = nullptr;  // group 0's subdomains, then group 1's
  int n_fac_main = 0;            // subdomains factored before the fork (whole factor rounds)
  int n_grp_subs[2] = {0, 0};
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // PCG form: column -> subdomain, per-column iteration counts and
  // convergence flags, and the fallback's factor order and solve items
  int *d_colsub = nullptr, *d_iters = nullptr, *d_conv = nullptr;
  int *d_fb_order = nullptr;
  int4 *d_fb_work = nullptr;
  int pcg_max = 50;
  const double *pcg_x0 = nullptr;
  int pcg_x0_scale = 0;
  int pcg_fallback = 0;
  int64_t pcg_iters = 0;
  std::vector<int> fb_order;   // host copies kept until the next build
  std::vector<int4> fb_work;
  // network samples: selected subdomains and their first sample index
  int *d_nn_sel = nullptr, *d_nn_s0 = nullptr;
  bool nn_rhs_ready = false;  // R holds the current build's right-hand sides
  std::vector<int> nn_sel, nn_s0;
  int *d_patches = nullptr;
  int *d_subof[3] = {nullptr, nullptr, nullptr};
  // reconstruction by re-solve (keep without MRCM_KEEP_MBFS): descriptors of
  // one right-hand side per subdomain, its work list and vectors
  uint32_t keep = MRCM_KEEP_FACTORS | MRCM_KEEP_MBFS;
  SubDesc *d_sub_rs = nullptr;
  int4 *d_work_rs = nullptr;
  double *Brs = nullptr, *Xrs = nullptr, *Rrs = nullptr;
  // Mean post-processing, set up on its first use: descriptors of one column
  // per subdomain whose factor offsets are relative to the start of their
  // chunk, the factor order cut into chunks that fit the factor scratch
  // (mean_chunk holds the boundaries), the Neumann coefficients and vectors
  SubDesc *d_sub_mean = nullptr;
  int *d_order_mean = nullptr;
  int4 *d_work_mean = nullptr;
  std::vector<int> mean_chunk;
  double *mcoef = nullptr, *mscal = nullptr, *mB = nullptr, *mX = nullptr, *mR = nullptr, *mfac = nullptr;
  double *coef = nullptr, *r0 = nullptr, *scal = nullptr;
  void *L = nullptr, *Dinv = nullptr;
  double *X = nullptr, *R = nullptr;
  double *R0 = nullptr;  // FP32 pipeline: the right-hand sides, kept for every sweep's own residual
  double *F = nullptr, *Fb = nullptr, *SAb = nullptr;
  double *norms = nullptr, *scalar = nullptr;
  DevStatus *st = nullptr;
  hipStream_t stream = nullptr;
  int ir_iters = 0;
  double ir_res = 0.0;
  double ir_tol = 1e-13;
  int ir_max = 30;
  int refine64 = 0;
  int64_t bytes = 0;
};

struct mrcm_interface {
  const mrcm_mbfs *mb = nullptr;
  int nv = 0, n = 0;
  // multifrontal form (nested dissection of the patch graph), always built
  NdPlan plan;
  MfDevPlan dp;
  double *fronts = nullptr, *minv = nullptr, *zbuf = nullptr, *pbuf = nullptr;
  double *xv = nullptr, *rv = nullptr, *bv = nullptr, *dv = nullptr;
  bool fronts_fresh = false;  // fronts hold the assembled entries (not yet factored)
  // band form, built on its first use
  int w = -1;
  std::vector<int> pos;
  int *d_pos = nullptr;
  double *AB = nullptr, *AB0 = nullptr;
  double *b = nullptr, *b0 = nullptr;
  double *inv = nullptr, *r = nullptr, *y = nullptr;
  double *scalar = nullptr;
  DevStatus *st = nullptr;
  hipStream_t stream = nullptr;
  int64_t bytes = 0;
  int last_method = 0, last_iters = 0;
  double last_residual = -1.0;
};

namespace {

void free_mbfs(mrcm_mbfs *h) {
  if (!h) return;
  void *ptrs[] = {h->d_sub, h->d_ifc, h->d_order, h->d_work, h->d_patches, h->d_subof[0], h->d_subof[1],
                  h->d_subof[2], h->coef, h->r0, h->scal, h->L, h->Dinv, h->X, h->R, h->R0, h->F, h->Fb, h->SAb,
                  h->norms, h->scalar, h->st, h->d_grp_subs[0], h->d_grp_subs[1], h->d_order_split,
                  h->d_colsub, h->d_iters, h->d_conv, h->d_fb_order, h->d_fb_work, h->d_nn_sel, h->d_nn_s0,
                  h->d_sub_rs, h->d_work_rs, h->Brs, h->Xrs, h->Rrs, h->d_queue, h->d_sub_mean,
                  h->d_order_mean, h->d_work_mean, h->mcoef, h->mscal, h->mB, h->mX, h->mR, h->mfac};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->s2) (void)hipStreamDestroy(h->s2);
  delete h;
}

void free_iface(mrcm_interface *h) {
  if (!h) return;
  void *ptrs[] = {h->d_pos, h->AB, h->AB0, h->b, h->b0, h->inv, h->r, h->y, h->scalar, h->st,
                  h->fronts, h->minv, h->zbuf, h->pbuf, h->xv, h->rv, h->bv, h->dv,
                  h->dp.nodes, h->dp.idx, h->dp.map, h->dp.level_nodes, h->dp.step_blocks, h->dp.fwd_bnd,
                  h->dp.bwd_bnd, h->dp.pair_off,
                  h->dp.sub_pair_off, h->dp.pair_ld, h->dp.pinfo};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete h;
}

// The multifrontal plan of the handle's interface system, its device copy and
// the fronts, factor and vector storage.
mrcm_status init_mf(mrcm_interface *h) {
  const mrcm_mbfs *mb = h->mb;
  const HostGeom &G = mb->G;
  const int nd[3] = {(int)G.cuts[0].size() - 1, (int)G.cuts[1].size() - 1, (int)G.cuts[2].size() - 1};
  const std::string err = build_nd_plan(nd, G.subs, G.ifcs, G.patches, G.n_patch, G.iface_panel, h->plan);
  if (!err.empty()) return fail(MRCM_EUNSUPPORTED, err);
  const NdPlan &P = h->plan;
  std::vector<int4> pinfo(G.n_patch);
  for (const IfaceDesc &I : G.ifcs)
    for (int k = 0; k < I.na * I.nb; ++k)
      pinfo[I.p0 + k] = make_int4((int)(&I - G.ifcs.data()), G.subs[I.lo_sub].face_p0[2 * I.d + 1] + k,
                                  G.subs[I.hi_sub].face_p0[2 * I.d] + k, 0);
  HIP_TRY(mf_init_kernels());
  MfDevPlan &dp = h->dp;
  dp.n_nodes = (int)P.nodes.size();
  dp.front_doubles = P.front_doubles;
  HIP_TRY(upload(&dp.nodes, P.nodes));
  HIP_TRY(upload(&dp.idx, P.idx));
  HIP_TRY(upload(&dp.map, P.map));
  HIP_TRY(upload(&dp.level_nodes, P.level_nodes));
  HIP_TRY(upload(&dp.step_blocks, P.step_blocks));
  HIP_TRY(upload(&dp.fwd_bnd, P.fwd_bnd));
  HIP_TRY(upload(&dp.bwd_bnd, P.bwd_bnd));
  HIP_TRY(upload(&dp.pair_off, P.pair_off));
  HIP_TRY(upload(&dp.sub_pair_off, P.sub_pair_off));
  HIP_TRY(upload(&dp.pair_ld, P.pair_ld));
  HIP_TRY(upload(&dp.pinfo, pinfo));
  const bool ok = dev_alloc(&h->fronts, (size_t)P.front_doubles) == hipSuccess &&
                  dev_alloc(&h->minv, (size_t)P.inv_doubles) == hipSuccess &&
                  dev_alloc(&h->zbuf, (size_t)P.z_doubles) == hipSuccess &&
                  dev_alloc(&h->pbuf, (size_t)P.part_doubles) == hipSuccess && dev_alloc(&h->xv, h->n) == hipSuccess &&
                  dev_alloc(&h->rv, h->n) == hipSuccess && dev_alloc(&h->bv, h->n) == hipSuccess &&
                  dev_alloc(&h->dv, h->n) == hipSuccess;
  if (!ok) return fail(MRCM_ENOMEM, "device allocation of the interface fronts failed");
  h->bytes += 8 * (P.front_doubles + P.inv_doubles + P.z_doubles + P.part_doubles + 4LL * h->n) +
              (int64_t)sizeof(MfNode) * P.nodes.size() + 4LL * (P.idx.size() + P.map.size()) +
              12LL * (int64_t)P.pair_off.size() +
              8LL * (int64_t)(P.step_blocks.size() + P.fwd_bnd.size() + P.bwd_bnd.size());
  return MRCM_OK;
}

// The band form: reverse Cuthill-McKee order, band storage and work vectors.
mrcm_status init_band(mrcm_interface *h) {
  rcm_order(h->mb->G, h->pos, h->w);
  const int64_t band = (int64_t)h->n * (2 * h->w + 1);
  const bool ok = upload(&h->d_pos, h->pos) == hipSuccess && dev_alloc(&h->AB, band) == hipSuccess &&
                  dev_alloc(&h->AB0, band) == hipSuccess && dev_alloc(&h->b, h->n) == hipSuccess &&
                  dev_alloc(&h->b0, h->n) == hipSuccess &&
                  dev_alloc(&h->inv, (int64_t)ldl_inv_size(h->n)) == hipSuccess &&
                  dev_alloc(&h->y, h->n) == hipSuccess && dev_alloc(&h->r, h->n) == hipSuccess;
  if (!ok) return fail(MRCM_ENOMEM, "device allocation of the interface band failed");
  h->bytes += 2 * band * 8 + 4 * (int64_t)h->n * 8 + (int64_t)ldl_inv_size(h->n) * 8;
  return MRCM_OK;
}

mrcm_status alloc_mbfs(mrcm_mbfs *h) {
  const HostGeom &G = h->G;
  h->n_sub = (int)G.subs.size();
  std::vector<int> subof[3] = {G.sub_of[0], G.sub_of[1], G.sub_of[2]};
  const size_t es = G.precision == MRCM_FP32_IR ? sizeof(float) : sizeof(double);
  int64_t bytes = 0;
#define ALLOC(p, n, T)                                                                \
  do {                                                                                \
    if (dev_alloc(&p, (size_t)(n)) != hipSuccess)                                     \
      return fail(MRCM_ENOMEM, "device allocation of " #p " failed");                 \
    bytes += (int64_t)(n) * (int64_t)sizeof(T);                                       \
  } while (0)
  HIP_TRY(upload(&h->d_sub, G.subs));
  HIP_TRY(upload(&h->d_ifc, G.ifcs));
  HIP_TRY(upload(&h->d_order, G.order));
  HIP_TRY(upload(&h->d_work, G.work));
  HIP_TRY(upload(&h->d_queue, std::vector<int>(16, 0)));
  HIP_TRY(upload(&h->d_patches, G.patches));
  for (int d = 0; d < 3; ++d) HIP_TRY(upload(&h->d_subof[d], subof[d]));
  ALLOC(h->coef, 4 * G.totCells, double);
  ALLOC(h->r0, G.totCells, double);
  ALLOC(h->scal, G.totCells, double);
  {
    char *p = nullptr;
    if (hipMalloc((void **)&p, (size_t)G.totL * es) != hipSuccess)
      return fail(MRCM_ENOMEM, "device allocation of the band factors failed");
    h->L = p;
    bytes += G.totL * (int64_t)es;
    if (hipMalloc((void **)&p, (size_t)G.totD * es) != hipSuccess)
      return fail(MRCM_ENOMEM, "device allocation of the diagonal-block inverses failed");
    h->Dinv = p;
    bytes += G.totD * (int64_t)es;
  }
  ALLOC(h->X, G.totX, double);
  if (G.precision != MRCM_FP64) ALLOC(h->R, G.totX, double);
  if (G.precision == MRCM_PCG) {
    HIP_TRY(upload(&h->d_colsub, G.col_sub));
    ALLOC(h->d_iters, G.totCols, int);
    ALLOC(h->d_conv, G.totCols, int);
    ALLOC(h->d_fb_order, G.subs.size(), int);
    ALLOC(h->d_fb_work, G.work.size(), int4);
  }
  ALLOC(h->F, std::max<int64_t>(1, G.totF), double);
  ALLOC(h->Fb, std::max<int64_t>(1, G.totF), double);
  ALLOC(h->SAb, std::max<int64_t>(1, (int64_t)G.patches.size()), double);
  ALLOC(h->norms, 3 * (int64_t)G.totCols, double);
  ALLOC(h->scalar, 4, double);
  {
    DevStatus *p = nullptr;
    HIP_TRY(hipMalloc((void **)&p, sizeof(DevStatus)));
    h->st = p;
  }
#undef ALLOC
  // the split of the solve work into resident rounds (FP64 path)
  h->solve_group.assign(G.subs.size(), 0);
  if (G.precision == MRCM_FP64 || G.precision == MRCM_FP32_IR) {
    const int f32 = G.precision == MRCM_FP32_IR;
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // The factorisation runs whole rounds of resident workgroups and a last,
    // partial round (the tail).  Group 0 is what the solve can hold beside
    // the tail: its first solve starts when the whole rounds are factored,
    // on the CUs the tail leaves free.  A multiple of 8 keeps every item on
    // its XCD (workgroup i runs on XCD i mod 8).
    const int fpc = std::max(1, f32 ? factor32_blocks_per_cu(G.bmax) : factor64_blocks_per_cu(G.bmax));
    const int spc = solve_blocks_per_cu(f32, G.bmax);
    const int n_sub_all = (int)G.subs.size();
    const int tail = n_sub_all % (ncu * fpc);
    const int tail_cus = (tail + fpc - 1) / fpc;
    size_t slots = (size_t)std::max(0, ncu - tail_cus) * spc;
    slots = std::min(slots, (size_t)(n_sub_all - tail));
    if (G.solve_group > 0) slots = std::min((size_t)G.solve_group, (size_t)(n_sub_all - tail));
    if (G.solve_group < 0) slots = 0;
    slots = (slots / 8) * 8;
    // the factor's whole rounds must cover group 0: true when every work
    // item is one whole subdomain taken in factor order, checked below
    bool in_order = G.work.size() >= (size_t)n_sub_all;
    for (size_t i = 0; in_order && i < (size_t)n_sub_all; ++i) in_order = G.work[i].x == G.order[i];
    if (in_order && slots > 0 && slots < G.work.size()) {
      std::vector<int> grp(G.subs.size(), -1);
      bool whole = true;
      for (size_t i = 0; i < G.work.size(); ++i) {
        const int l = G.work[i].x;
        if (l < 0) continue;
        const int gi = i < slots ? 0 : 1;
        if (grp[l] >= 0 && grp[l] != gi) whole = false;
        grp[l] = gi;
      }
      if (whole) {
        std::vector<int> lists[2];
        for (size_t i = 0; i < G.work.size(); ++i) {
          const int l = G.work[i].x;
          if (l >= 0 && (lists[grp[l]].empty() || lists[grp[l]].back() != l)) lists[grp[l]].push_back(l);
        }
        for (int gi = 0; gi < 2; ++gi) {
          HIP_TRY(upload(&h->d_grp_subs[gi], lists[gi]));
          h->n_grp_subs[gi] = (int)lists[gi].size();
        }
        std::vector<int> ord(lists[0]);
        ord.insert(ord.end(), lists[1].begin(), lists[1].end());
        HIP_TRY(upload(&h->d_order_split, ord));
        h->n_fac_main = n_sub_all - tail;
        for (size_t l = 0; l < grp.size(); ++l) h->solve_group[l] = std::max(0, grp[l]);
        HIP_TRY(hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        h->n_first = (int)slots;
      }
    }
  }
  h->bytes = bytes;
  Geom &g = h->g;
  g.nx = G.n[0];
  g.ny = G.n[1];
  g.nz = G.n[2];
  const double V = G.h[0] * G.h[1] * G.h[2];
  for (int d = 0; d < 3; ++d) {
    g.h[d] = G.h[d];
    g.area[d] = V / G.h[d];
    g.sub_of[d] = h->d_subof[d];
    g.nd[d] = (int)G.cuts[d].size() - 1;
  }
  g.alpha = G.alpha;
  g.beta_mode = G.beta_mode;
  for (int f = 0; f < 6; ++f) g.wall_type[f] = G.wall_type[f];
  g.pin = G.pin;
  g.sub = h->d_sub;
  g.ifc = h->d_ifc;
  return MRCM_OK;
}

mrcm_status read_status(DevStatus *st, hipStream_t s, const char *what) {
  if (g_capturing) return MRCM_OK;  // read after a replay by mrcm_graph_check
  DevStatus hs;
  HIP_TRY(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hs.code == 0) return MRCM_OK;
  char buf[256];
  if (hs.code == MRCM_ENOTSPD)
    snprintf(buf, sizeof buf, "%s: non-positive pivot %.6g in subdomain %d", what, hs.value, hs.where);
  else if (hs.code == MRCM_EINVAL)
    snprintf(buf, sizeof buf, "%s: permeability %.6g at cell %d is not positive and finite", what,
             hs.value, hs.where);
  else if (hs.code == MRCM_ESINGULAR)
    snprintf(buf, sizeof buf, "%s: zero pivot in the interface factorisation (block or node %d)", what, hs.where);
  else
    snprintf(buf, sizeof buf, "%s: device status %d", what, hs.code);
  return fail((mrcm_status)hs.code, buf);
}

}  // namespace

extern "C" {

const char *mrcm_status_string(mrcm_status s) {
  switch (s) {
    case MRCM_OK: return "ok";
    case MRCM_EINVAL: return "invalid argument";
    case MRCM_ENOMEM: return "out of device memory";
    case MRCM_ENOTSPD: return "local matrix not positive definite";
    case MRCM_ENOCONV: return "iterative refinement did not converge";
    case MRCM_ESINGULAR: return "interface matrix singular";
    case MRCM_EHIP: return "HIP runtime error";
    case MRCM_EUNSUPPORTED: return "unsupported by this build";
  }
  return "unknown status";
}

const char *mrcm_last_error(void) { return g_last_error.c_str(); }

mrcm_status mrcm_build_mbfs(const mrcm_problem *pb, const mrcm_partition *part,
                            const mrcm_iface_space *ifs, const mrcm_options *opt, void *stream,
                            mrcm_mbfs **out) {
  if (!out) return fail(MRCM_EINVAL, "out is null");
  mrcm_mbfs *h = *out;
  mrcm_status st = MRCM_OK;
  ConfigKey key;
  const bool have_key = make_key(pb, part, ifs, opt, key);
  // a rebuild in place with the same configuration skips the host geometry
  const bool same = h && have_key && key == h->key && pb->kx && pb->ky && pb->kz && pb->q;
  HostGeom G;
  if (!same) {
    st = build_host_geom(pb, part, ifs, opt, G);
    if (st != MRCM_OK) return st;
  }
  bool created = false;
  if (h && !same && !same_config(h->G, G))
    return fail(MRCM_EINVAL, "handle was built for a different configuration");
  if (!h) {
    h = new mrcm_mbfs();
    h->key = key;
    h->G = std::move(G);
    st = alloc_mbfs(h);
    if (st != MRCM_OK) {
      free_mbfs(h);
      return st;
    }
    created = true;
  }
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  h->nn_rhs_ready = false;
  h->ir_tol = opt->ir_tol > 0.0 ? opt->ir_tol : (opt->precision == MRCM_PCG ? 1e-10 : 1e-13);
  h->pcg_max = opt->pcg_max_iter > 0 ? opt->pcg_max_iter : 50;
  h->pcg_x0 = opt->pcg_x0;
  h->pcg_x0_scale = opt->pcg_x0_scale;
  h->ir_max = opt->ir_max_iter > 0 ? opt->ir_max_iter : 30;
  if (opt->fp64_refine < 0 || opt->fp64_refine > 10) return fail(MRCM_EINVAL, "fp64_refine must be in [0, 10]");
  h->refine64 = opt->fp64_refine;
  Geom &g = h->g;
  g.k[0] = pb->kx;
  g.k[1] = pb->ky;
  g.k[2] = pb->kz;
  g.q = pb->q;
  for (int f = 0; f < 6; ++f) g.wall_value[f] = pb->wall_value[f];
  const HostGeom &H = h->G;
  const int fp32 = H.precision == MRCM_FP32_IR;
  auto bail = [&](mrcm_status e) {
    if (created) free_mbfs(h);
    return e;
  };
#define ENQ(expr)                                                                   \
  do {                                                                              \
    hipError_t _e = (expr);                                                         \
    if (_e != hipSuccess) return bail(fail(MRCM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e))); \
  } while (0)
  const long long N = (long long)H.n[0] * H.n[1] * H.n[2];
  ENQ(launch_reset_status(h->st, s));
  // an invalid permeability is reported by the status read at the end of the
  // call (the first status set wins), not by a synchronisation here
  ENQ(launch_check_perm(pb->kx, pb->ky, pb->kz, N, h->st, s));
  {
    Stage t(MRCM_STAGE_COEF, s);
    ENQ(launch_coef(g, h->n_sub, H.max_cells, h->coef, h->r0, h->scal, s));
  }
  const bool pcg = H.precision == MRCM_PCG;
  // the two-stream pipeline: the FP64 form with refinement, and the FP32
  // form, whose first min(3, ir_max) sweeps run in it before the first
  // convergence check (three reach 1e-13 on the channelised workloads)
  const bool split = !pcg && h->n_first > 0 && (fp32 || h->refine64 > 0);
  const int nsweep = fp32 ? std::min(3, h->ir_max) : h->refine64;
  const int n_work = (int)H.work.size();
  // the work-queue counters of a stream (slot 0: the caller's, 1: the
  // second), or null for the plain grid launches
  auto queue = [&](int slot) -> int * { return H.launch_mode == MRCM_LAUNCH_QUEUE ? h->d_queue + 8 * slot : nullptr; };
  h->ir_iters = 0;
  h->ir_res = 0.0;
  h->pcg_fallback = 0;
  h->pcg_iters = 0;
  if (!fp32 && !pcg && h->refine64 > 0 && !h->R) {
    if (dev_alloc(&h->R, (size_t)H.totX) != hipSuccess)
      return bail(fail(MRCM_ENOMEM, "device allocation of the refinement buffer failed"));
    h->bytes += H.totX * 8;
  }
  // Pipelined sweeps: each correction workgroup forms its own residual from
  // a copy of the right-hand sides.  One FP64 sweep keeps the copy in R (the
  // correction overwrites it); the FP32 form's several sweeps keep it in R0.
  const bool own_res = split && (fp32 || h->refine64 == 1);
  if (own_res && fp32 && !h->R0) {
    if (dev_alloc(&h->R0, (size_t)H.totX) != hipSuccess)
      return bail(fail(MRCM_ENOMEM, "device allocation of the right-hand-side copy failed"));
    h->bytes += H.totX * 8;
  }
  const double *rhs0 = own_res && fp32 ? h->R0 : nullptr;
  {
    Stage t(MRCM_STAGE_RHS, s);
    ENQ(launch_rhs(g, h->n_sub, H.max_cells, H.mmax, h->r0, pcg ? h->R : h->X, s,
                   own_res ? (fp32 ? h->R0 : h->R) : nullptr));
  }
  if (pcg) {
    // Conjugate gradients for every column (right-hand sides in R), then the
    // band Cholesky and direct solves for every subdomain with a column that
    // did not converge, which overwrite all of that subdomain's columns.
    std::vector<int> conv(H.totCols), its(H.totCols);
    {
      Stage t(MRCM_STAGE_PCG, s);
      ENQ(launch_pcg(g, h->d_colsub, H.totCols, H.max_cells, h->coef, h->scal, h->R, h->pcg_x0, h->X, h->pcg_max,
                     h->ir_tol, h->pcg_x0_scale, h->d_iters, h->d_conv, s));
      ENQ(hipMemcpyAsync(conv.data(), h->d_conv, conv.size() * sizeof(int), hipMemcpyDeviceToHost, s));
      ENQ(hipMemcpyAsync(its.data(), h->d_iters, its.size() * sizeof(int), hipMemcpyDeviceToHost, s));
      ENQ(hipStreamSynchronize(s));
    }
    std::vector<char> bad(h->n_sub, 0);
    for (int c = 0; c < H.totCols; ++c) {
      h->pcg_iters += its[c];
      if (!conv[c]) bad[H.col_sub[c]] = 1;
    }
    h->fb_order.clear();
    h->fb_work.clear();
    for (int l : H.order)
      if (bad[l]) h->fb_order.push_back(l);
    for (const int4 &w : H.work)
      if (w.x >= 0 && bad[w.x]) h->fb_work.push_back(w);
    h->pcg_fallback = (int)h->fb_order.size();
    if (!h->fb_order.empty()) {
      Stage t(MRCM_STAGE_FALLBACK, s);
      ENQ(hipMemcpyAsync(h->d_fb_order, h->fb_order.data(), h->fb_order.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
      ENQ(hipMemcpyAsync(h->d_fb_work, h->fb_work.data(), h->fb_work.size() * sizeof(int4), hipMemcpyHostToDevice,
                         s));
      ENQ(launch_factor(0, h->d_sub, h->d_fb_order, h->pcg_fallback, h->coef, h->scal, h->L, h->Dinv, h->st,
                        H.bmax, s));
      ENQ(launch_solve(0, g, h->d_fb_work, (int)h->fb_work.size(), h->scal, h->L, h->Dinv, h->R, h->X, 0, H.bmax,
                       s));
      // the FP64 refinement sweeps of the direct form, on the same subdomains
      for (int it = 0; it < h->refine64; ++it) {
        ENQ(launch_residual(g, h->pcg_fallback, H.max_cells, H.mmax, h->coef, h->r0, h->X, h->R, nullptr, s,
                            h->d_fb_order));
        ENQ(launch_solve(0, g, h->d_fb_work, (int)h->fb_work.size(), h->scal, h->L, h->Dinv, h->R, h->X, 1,
                         H.bmax, s));
      }
    }
  } else if (split) {
    // Per-subdomain pipeline over two streams.  The whole rounds of the
    // factorisation go first; group 0's first solve, residuals and
    // corrections then run on the second stream while the caller's stream
    // factors the last, partial round and solves and refines group 1 (the
    // rest of the subdomains).  The streams join before the fluxes.  The
    // groups hold disjoint subdomains, so they touch disjoint parts of L,
    // Dinv, X and R; group 0 lies inside the whole rounds.
    const int n0 = h->n_grp_subs[0], n1s = h->n_grp_subs[1];
    {
      Stage t(MRCM_STAGE_FACTOR, s);
      const int nm = h->n_fac_main;
      ENQ(launch_factor(fp32, h->d_sub, h->d_order_split, nm, h->coef, h->scal, h->L, h->Dinv, h->st,
                        H.bmax, s, queue(0)));
      ENQ(hipEventRecord(h->ev_fork, s));
      if (h->n_sub > nm)
        ENQ(launch_factor(fp32, h->d_sub, h->d_order_split + nm, h->n_sub - nm, h->coef, h->scal, h->L, h->Dinv,
                          h->st, H.bmax, s, queue(0)));
    }
    ENQ(hipStreamWaitEvent(h->s2, h->ev_fork, 0));
    {
      Stage t(MRCM_STAGE_SOLVE, h->s2);
      ENQ(launch_solve(fp32, g, h->d_work, h->n_first, h->scal, h->L, h->Dinv, h->X, h->X, 0, H.bmax, h->s2,
                       nullptr, nullptr, queue(1)));
    }
    for (int it = 0; it < nsweep; ++it) {
      if (!own_res)
        ENQ(launch_residual(g, n0, H.max_cells, H.mmax, h->coef, h->r0, h->X, h->R, nullptr, h->s2, h->d_grp_subs[0]));
      ENQ(launch_solve(fp32, g, h->d_work, h->n_first, h->scal, h->L, h->Dinv, h->R, h->X, 1, H.bmax, h->s2,
                       own_res ? h->coef : nullptr, rhs0, queue(1)));
    }
    ENQ(hipEventRecord(h->ev_join, h->s2));
    Stage t(MRCM_STAGE_REFINE, s);
    const int4 *w1 = h->d_work + h->n_first;
    const int n1 = n_work - h->n_first;
    {
      Stage t1(MRCM_STAGE_SOLVE_REST, s);
      ENQ(launch_solve(fp32, g, w1, n1, h->scal, h->L, h->Dinv, h->X, h->X, 2, H.bmax, s, nullptr, nullptr,
                       queue(0)));
    }
    for (int it = 0; it < nsweep; ++it) {
      if (!own_res)
        ENQ(launch_residual(g, n1s, H.max_cells, H.mmax, h->coef, h->r0, h->X, h->R, nullptr, s, h->d_grp_subs[1]));
      ENQ(launch_solve(fp32, g, w1, n1, h->scal, h->L, h->Dinv, h->R, h->X, 3, H.bmax, s,
                       own_res ? h->coef : nullptr, rhs0, queue(0)));
    }
    ENQ(hipStreamWaitEvent(s, h->ev_join, 0));
    h->ir_iters = nsweep;
  } else {
    {
      Stage t(MRCM_STAGE_FACTOR, s);
      ENQ(launch_factor(fp32, h->d_sub, h->d_order, h->n_sub, h->coef, h->scal, h->L, h->Dinv, h->st,
                        H.bmax, s, queue(0)));
    }
    {
      Stage t(MRCM_STAGE_SOLVE, s);
      ENQ(launch_solve(fp32, g, h->d_work, n_work, h->scal, h->L, h->Dinv, h->X, h->X, 0, H.bmax, s, nullptr,
                       nullptr, queue(0)));
    }
  }
  if (split || pcg) {
    // refinement done in the pipeline above, or none (PCG)
  } else if (!fp32 && h->refine64 > 0) {
    for (int it = 0; it < h->refine64; ++it) {
      {
        Stage t(MRCM_STAGE_RESIDUAL, s);
        ENQ(launch_residual(g, h->n_sub, H.max_cells, H.mmax, h->coef, h->r0, h->X, h->R, nullptr, s));
      }
      Stage t(MRCM_STAGE_REFINE, s);
      ENQ(launch_solve(fp32, g, h->d_work, (int)H.work.size(), h->scal, h->L, h->Dinv, h->R, h->X,
                       1, H.bmax, s, nullptr, nullptr, queue(0)));
    }
    h->ir_iters = h->refine64;
  }
  if (fp32) {
    // CG-IR fallback: when the sweeps stop short of the tolerance, the
    // conjugate-gradient kernel (FP64 residual, FP32 inner iterations) polishes
    // every column from the current X, once
    const bool cg_ok = H.bmax <= kMaxBand64 && H.max_cells <= pcg_max_cells();
    bool polished = false;
    for (int it = split ? nsweep : 0;; ++it) {
      {
        Stage t(MRCM_STAGE_RESIDUAL, s);
        ENQ(launch_fill(h->norms, 3LL * H.totCols, 0.0, s));
        // with the pipelined sweeps a further sweep forms its own residual
        // from the kept right-hand sides, so the check writes no residual
        ENQ(launch_residual(g, h->n_sub, H.max_cells, H.mmax, h->coef, h->r0, h->X, own_res ? nullptr : h->R,
                            h->norms, s));
        ENQ(launch_ir_check(h->norms, H.totCols, h->scalar, s));
      }
      // res: the largest relative residual of the columns still above the
      // rounding floor of their own residual (those that a sweep can still
      // improve); the reported residual is the largest of all columns
      double rv[2] = {0.0, 0.0};
      ENQ(hipMemcpyAsync(rv, h->scalar, sizeof(rv), hipMemcpyDeviceToHost, s));
      ENQ(hipStreamSynchronize(s));
      const double res = rv[0];
      h->ir_res = rv[1];
      h->ir_iters = it;
      if (res <= h->ir_tol) break;
      if ((it >= h->ir_max || !std::isfinite(res)) && !polished && cg_ok && std::isfinite(res)) {
        polished = true;
        if (!h->d_colsub) {
          if (upload(&h->d_colsub, H.col_sub) != hipSuccess || dev_alloc(&h->d_iters, (size_t)H.totCols) != hipSuccess ||
              dev_alloc(&h->d_conv, (size_t)H.totCols) != hipSuccess)
            return bail(fail(MRCM_ENOMEM, "device allocation of the CG buffers failed"));
        }
        std::vector<int> its(H.totCols);
        {
          Stage t(MRCM_STAGE_PCG, s);
          ENQ(launch_rhs(g, h->n_sub, H.max_cells, H.mmax, h->r0, h->R, s));
          ENQ(launch_pcg(g, h->d_colsub, H.totCols, H.max_cells, h->coef, h->scal, h->R, h->X, h->X, 1000,
                         h->ir_tol, 0, h->d_iters, h->d_conv, s));
          ENQ(hipMemcpyAsync(its.data(), h->d_iters, its.size() * sizeof(int), hipMemcpyDeviceToHost, s));
          ENQ(hipStreamSynchronize(s));
        }
        h->pcg_iters = 0;
        for (int v : its) h->pcg_iters += v;
        continue;  // the residual check above decides
      }
      if (it >= h->ir_max || !std::isfinite(res)) {
        st = read_status(h->st, s, "mrcm_build_mbfs");
        if (st != MRCM_OK) return bail(st);
        char buf[160];
        snprintf(buf, sizeof buf, "refinement stopped at relative residual %.3g after %d sweeps", res, it);
        return bail(fail(MRCM_ENOCONV, buf));
      }
      {
        Stage t(MRCM_STAGE_REFINE, s);
        ENQ(launch_solve(fp32, g, h->d_work, (int)H.work.size(), h->scal, h->L, h->Dinv, h->R, h->X,
                         1, H.bmax, s, own_res ? h->coef : nullptr, own_res ? h->R0 : nullptr));
      }
    }
  }
  {
    Stage t(MRCM_STAGE_FLUX, s);
    ENQ(launch_flux(g, h->n_sub, h->X, h->F, h->Fb, h->SAb, s));
  }
  st = read_status(h->st, s, "mrcm_build_mbfs");
  profile_flush();
  if (st != MRCM_OK) return bail(st);
#undef ENQ
  *out = h;
  return MRCM_OK;
}

mrcm_status mrcm_assemble_interface(const mrcm_mbfs *mb, void *stream, mrcm_interface **out) {
  if (!mb || !out) return fail(MRCM_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  mrcm_interface *h = *out;
  bool created = false;
  if (h && h->mb != mb) return fail(MRCM_EINVAL, "interface handle belongs to another mbfs handle");
  if (!h) {
    h = new mrcm_interface();
    created = true;
    h->mb = mb;
    h->nv = mb->G.n_patch;
    h->n = 2 * h->nv;
    mrcm_status st = MRCM_OK;
    if (dev_alloc(&h->scalar, 4) != hipSuccess || hipMalloc((void **)&h->st, sizeof(DevStatus)) != hipSuccess)
      st = fail(MRCM_ENOMEM, "device allocation of the interface status failed");
    if (st == MRCM_OK && h->nv > 0) st = init_mf(h);
    if (st != MRCM_OK) {
      free_iface(h);
      return st;
    }
  }
  h->stream = s;
  auto bail = [&](mrcm_status e) {
    if (created) free_iface(h);
    return e;
  };
  hipError_t e = hipSuccess;
  if (h->nv > 0) {
    Stage t(MRCM_STAGE_ASSEMBLE, s);
    e = launch_mf_assemble(mb->g, mb->n_sub, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp, h->fronts, s);
    if (e == hipSuccess)
      e = launch_mf_residual(mb->g, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp.pinfo, h->nv, nullptr, h->bv,
                             nullptr, s);
    h->fronts_fresh = true;
  }
  if (e == hipSuccess && !g_capturing) e = hipStreamSynchronize(s);
  profile_flush();
  if (e != hipSuccess) return bail(fail(MRCM_EHIP, std::string("interface assembly: ") + hipGetErrorString(e)));
  *out = h;
  return MRCM_OK;
}

namespace {

// relative residual ||r|| / ||b|| from two device vectors (synchronises)
mrcm_status rel_norm(mrcm_interface *h, const double *r, const double *b, hipStream_t s, double &out) {
  HIP_TRY(launch_norm2(r, h->n, h->scalar, s));
  HIP_TRY(launch_norm2(b, h->n, h->scalar + 1, s));
  double v[2];
  HIP_TRY(hipMemcpyAsync(v, h->scalar, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out = v[1] > 0.0 ? std::sqrt(v[0] / v[1]) : std::sqrt(v[0]);
  return MRCM_OK;
}

mrcm_status solve_mf(mrcm_interface *h, double rtol, int max_refine, hipStream_t s, double *X, int &iters,
                     double *rel_residual) {
  const mrcm_mbfs *mb = h->mb;
  HIP_TRY(launch_reset_status(h->st, s));
  {
    Stage t(MRCM_STAGE_LU, s);
    // the fronts are consumed by the factorisation: a second solve of the
    // same assembly scatters the entries again
    if (!h->fronts_fresh)
      HIP_TRY(launch_mf_assemble(mb->g, mb->n_sub, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp, h->fronts, s));
    HIP_TRY(launch_mf_factor(h->plan, h->dp, h->fronts, h->minv, h->st, s));
    h->fronts_fresh = false;
  }
  iters = 0;
  {
    Stage t(MRCM_STAGE_SWEEP, s);
    HIP_TRY(launch_mf_solve(h->plan, h->dp, h->fronts, h->minv, h->zbuf, h->pbuf, h->bv, h->xv, s));
    for (; iters < max_refine; ++iters) {
      HIP_TRY(launch_mf_residual(mb->g, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp.pinfo, h->nv, h->xv, h->rv,
                                 nullptr, s));
      if (rtol > 0.0 && !g_capturing) {
        double rel = 0.0;
        mrcm_status st = rel_norm(h, h->rv, h->bv, s, rel);
        if (st != MRCM_OK) return st;
        if (rel <= rtol) break;
      }
      HIP_TRY(launch_mf_solve(h->plan, h->dp, h->fronts, h->minv, h->zbuf, h->pbuf, h->rv, h->dv, s));
      HIP_TRY(launch_axpy(h->xv, h->dv, h->n, s));
    }
    HIP_TRY(launch_mf_deinterleave(h->xv, h->nv, X, s));
  }
  mrcm_status st = read_status(h->st, s, "mrcm_solve_interface");
  profile_flush();
  if (st != MRCM_OK) return st;
  if (rel_residual) {
    HIP_TRY(launch_mf_residual(mb->g, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp.pinfo, h->nv, h->xv, h->rv,
                               nullptr, s));
    st = rel_norm(h, h->rv, h->bv, s, *rel_residual);
  }
  return st;
}

mrcm_status solve_band(mrcm_interface *h, double rtol, int max_refine, hipStream_t s, double *X, int &iters,
                       double *rel_residual) {
  const mrcm_mbfs *mb = h->mb;
  if (h->w < 0) {
    if (g_capturing) return fail(MRCM_EUNSUPPORTED, "the band form allocates on its first use: not under capture");
    mrcm_status st = init_band(h);
    if (st != MRCM_OK) return st;
  }
  const int64_t band = (int64_t)h->n * (2 * h->w + 1);
  HIP_TRY(launch_reset_status(h->st, s));
  {
    Stage t(MRCM_STAGE_ASSEMBLE, s);
    HIP_TRY(launch_fill(h->AB0, band, 0.0, s));
    HIP_TRY(launch_fill(h->b0, h->n, 0.0, s));
    HIP_TRY(launch_iface_scatter(mb->g, mb->n_sub, mb->d_patches, h->d_pos, mb->F, mb->Fb, mb->SAb, h->AB0, h->w,
                                 h->b0, s));
  }
  {
    // factor a sign-flipped copy of the assembled system (the assembled one
    // stays for refinement and the residual); the factorisation also carries
    // out the forward substitution into y
    Stage t(MRCM_STAGE_LU, s);
    HIP_TRY(launch_band_ldl(h->AB0, h->AB, h->b0, h->b, h->y, h->n, h->w, h->inv, h->st, s));
  }
  iters = 0;
  {
    Stage t(MRCM_STAGE_SWEEP, s);
    HIP_TRY(launch_lu_sweep(h->AB, h->inv, h->n, h->w, h->y, 1, s));
    for (; iters < max_refine; ++iters) {
      HIP_TRY(launch_band_residual(h->AB0, h->n, h->w, h->y, h->b0, h->r, 1, s));
      if (rtol > 0.0 && !g_capturing) {
        double rel = 0.0;
        mrcm_status st = rel_norm(h, h->r, h->b0, s, rel);
        if (st != MRCM_OK) return st;
        if (rel <= rtol) break;
      }
      HIP_TRY(launch_lu_sweep(h->AB, h->inv, h->n, h->w, h->r, 0, s));
      HIP_TRY(launch_lu_sweep(h->AB, h->inv, h->n, h->w, h->r, 1, s));
      HIP_TRY(launch_axpy(h->y, h->r, h->n, s));
    }
    HIP_TRY(launch_perm(h->y, h->d_pos, h->nv, X, 1, s));
  }
  mrcm_status st = read_status(h->st, s, "mrcm_solve_interface");
  profile_flush();
  if (st != MRCM_OK) return st;
  if (rel_residual) {
    HIP_TRY(launch_band_residual(h->AB0, h->n, h->w, h->y, h->b0, h->r, 0, s));
    st = rel_norm(h, h->r, h->b0, s, *rel_residual);
  }
  return st;
}

}  // namespace

mrcm_status mrcm_solve_interface(mrcm_interface *h, int32_t method, double rtol, int32_t max_refine, void *stream,
                                 double *X, int32_t *iters, double *rel_residual) {
  if (!h) return fail(MRCM_EINVAL, "null interface handle");
  if (h->n > 0 && !X) return fail(MRCM_EINVAL, "X is null");
  if (method < MRCM_IFACE_AUTO || method > MRCM_IFACE_MULTIFRONTAL)
    return fail(MRCM_EINVAL, "method must be MRCM_IFACE_AUTO, MRCM_IFACE_BAND or MRCM_IFACE_MULTIFRONTAL");
  if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(MRCM_EINVAL, "rtol must be finite and non-negative");
  if (max_refine < 0 || max_refine > 20) return fail(MRCM_EINVAL, "max_refine must be in [0, 20]");
  hipStream_t s = (hipStream_t)stream;
  h->stream = s;
  const int m = method == MRCM_IFACE_AUTO ? MRCM_IFACE_MULTIFRONTAL : method;
  int it = 0;
  double res = -1.0;
  mrcm_status st = MRCM_OK;
  if (h->n > 0) {
    st = (m == MRCM_IFACE_BAND) ? solve_band(h, rtol, max_refine, s, X, it, rel_residual ? &res : nullptr)
                                : solve_mf(h, rtol, max_refine, s, X, it, rel_residual ? &res : nullptr);
  } else {
    res = 0.0;
  }
  if (st != MRCM_OK) return st;
  h->last_method = m;
  h->last_iters = it;
  if (iters) *iters = it;
  if (rel_residual) {
    *rel_residual = res;
    h->last_residual = res;
  }
  return MRCM_OK;
}

mrcm_status mrcm_interface_query(const mrcm_interface *h, mrcm_interface_info *info) {
  if (!h || !info) return fail(MRCM_EINVAL, "null argument");
  const NdPlan &P = h->plan;
  info->n = h->n;
  info->nodes = (int32_t)P.nodes.size();
  info->levels = P.level_off.empty() ? 0 : (int32_t)P.level_off.size() - 1;
  info->max_front = P.max_f;
  info->front_bytes = 8 * P.front_doubles;
  info->factor_flops = P.flops;
  info->factor_launches = (int32_t)P.steps.size();
  info->bandwidth = h->w;
  info->device_bytes = h->bytes;
  info->method = h->last_method;
  info->refine_iters = h->last_iters;
  info->rel_residual = h->last_residual;
  return MRCM_OK;
}

namespace {

// The second reconstruction option: every local problem solved again with
// the particular data and G(pi) on Gamma, by the kept band factors, then
// the FP64 refinement sweeps of the build's form.
mrcm_status reconstruct_resolve(const mrcm_mbfs *cmb, const double *X, hipStream_t s, double *p) {
  mrcm_mbfs *mb = const_cast<mrcm_mbfs *>(cmb);  // lazily allocated re-solve buffers
  const HostGeom &G = mb->G;
  if (!mb->d_sub_rs) {
    if (g_capturing) return fail(MRCM_EUNSUPPORTED, "the re-solve allocates on its first use: not under capture");
    std::vector<SubDesc> rs(G.subs);
    std::vector<int4> work;
    for (SubDesc &S : rs) {
      S.m = 1;
      S.X_off = S.cell_off;
    }
    for (int l : G.order) work.push_back(make_int4(l, 0, 1, 0));
    HIP_TRY(upload(&mb->d_sub_rs, rs));
    HIP_TRY(upload(&mb->d_work_rs, work));
    if (dev_alloc(&mb->Brs, (size_t)G.totCells) != hipSuccess || dev_alloc(&mb->Xrs, (size_t)G.totCells) != hipSuccess ||
        dev_alloc(&mb->Rrs, (size_t)G.totCells) != hipSuccess)
      return fail(MRCM_ENOMEM, "device allocation of the re-solve vectors failed");
    mb->bytes += 24 * G.totCells;
  }
  Geom g1 = mb->g;
  g1.sub = mb->d_sub_rs;
  const int fp32 = G.precision == MRCM_FP32_IR;
  const int n = mb->n_sub;
  HIP_TRY(launch_resolve_rhs(g1, n, G.max_cells, mb->r0, X, G.n_patch, mb->Brs, s));
  // the band solve overwrites its right-hand side with the forward sweep's
  // result: solve a copy in place and keep Brs for the residuals
  HIP_TRY(launch_copy(mb->Brs, mb->Xrs, G.totCells, s));
  HIP_TRY(launch_solve(fp32, g1, mb->d_work_rs, n, mb->scal, mb->L, mb->Dinv, mb->Xrs, mb->Xrs, 0, G.bmax, s));
  const int sweeps = fp32 ? std::max(3, mb->ir_iters) : mb->refine64;
  for (int it = 0; it < sweeps; ++it) {
    HIP_TRY(launch_resolve_residual(g1, n, G.max_cells, mb->coef, mb->Brs, mb->Xrs, mb->Rrs, s));
    HIP_TRY(launch_solve(fp32, g1, mb->d_work_rs, n, mb->scal, mb->L, mb->Dinv, mb->Rrs, mb->Xrs, 1, G.bmax, s));
  }
  HIP_TRY(launch_resolve_scatter(g1, n, G.max_cells, mb->Xrs, p, s));
  return MRCM_OK;
}

// Largest factor scratch of the Mean post-processing: the subdomains are
// factored in chunks whose factors fit it.
constexpr int64_t kMeanScratchBytes = 8LL << 30;

int64_t round_up256(int64_t v) { return (v + 255) & ~(int64_t)255; }

mrcm_status init_mean(mrcm_mbfs *mb) {
  const HostGeom &G = mb->G;
  std::vector<SubDesc> ms(G.subs);
  int64_t total = 0, largest = 0;
  auto need = [](const SubDesc &S) {
    return round_up256((int64_t)S.N * (S.b + 1)) + round_up256((int64_t)((S.N + kNB - 1) / kNB) * kNB * kNB);
  };
  for (const SubDesc &S : ms) {
    total += need(S);
    largest = std::max(largest, need(S));
  }
  // the scratch: the whole factor when it is small, else the cap (the
  // environment's MRCM_MEAN_SCRATCH_BYTES when set), halved while the
  // allocation fails, down to one subdomain's factor
  int64_t cap_bytes = kMeanScratchBytes;
  if (const char *e = getenv("MRCM_MEAN_SCRATCH_BYTES")) {
    const long long v = atoll(e);
    if (v > 0) cap_bytes = std::min<int64_t>(v, kMeanScratchBytes);
  }
  int64_t cap = std::max(largest, std::min(total, cap_bytes / 8));
  while (dev_alloc(&mb->mfac, (size_t)cap) != hipSuccess) {
    (void)hipGetLastError();
    if (cap == largest) return fail(MRCM_ENOMEM, "device allocation of the Mean factor scratch failed");
    cap = std::max(largest, cap / 2);
  }
  std::vector<int> order;
  std::vector<int4> work;
  mb->mean_chunk.assign(1, 0);
  int64_t off = 0;
  for (int l : G.order) {
    SubDesc &S = ms[l];
    if (off + need(S) > cap) {
      mb->mean_chunk.push_back((int)order.size());
      off = 0;
    }
    S.m = 1;
    S.X_off = S.cell_off;
    S.pin_local = 0;
    S.L_off = off;
    S.D_off = off + round_up256((int64_t)S.N * (S.b + 1));
    off += need(S);
    order.push_back(l);
    work.push_back(make_int4(l, 0, 1, 0));
  }
  mb->mean_chunk.push_back((int)order.size());
  HIP_TRY(upload(&mb->d_sub_mean, ms));
  HIP_TRY(upload(&mb->d_order_mean, order));
  HIP_TRY(upload(&mb->d_work_mean, work));
  const int64_t n = G.totCells;
  if (dev_alloc(&mb->mcoef, (size_t)(4 * n)) != hipSuccess || dev_alloc(&mb->mscal, (size_t)n) != hipSuccess ||
      dev_alloc(&mb->mB, (size_t)n) != hipSuccess || dev_alloc(&mb->mX, (size_t)n) != hipSuccess ||
      dev_alloc(&mb->mR, (size_t)n) != hipSuccess)
    return fail(MRCM_ENOMEM, "device allocation of the Mean coefficients failed");
  mb->bytes += 8 * (8 * n + cap) + (int64_t)(sizeof(SubDesc) + 4 + sizeof(int4)) * (int64_t)ms.size();
  return MRCM_OK;
}

}  // namespace

namespace {

mrcm_status twophase_grid(const mrcm_twophase *tp, TwoPhaseGrid &t) {
  if (!tp) return fail(MRCM_EINVAL, "null two-phase descriptor");
  if (tp->nx <= 0 || tp->ny <= 0 || tp->nz <= 0) return fail(MRCM_EINVAL, "grid dimensions must be positive");
  const double v[5] = {tp->hx, tp->hy, tp->hz, tp->mu_w, tp->mu_o};
  for (double x : v)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(MRCM_EINVAL, "cell sizes and viscosities must be positive and finite");
  t = TwoPhaseGrid{tp->nx, tp->ny, tp->nz, tp->hx, tp->hy, tp->hz, tp->mu_w, tp->mu_o};
  return MRCM_OK;
}

}  // namespace

mrcm_status mrcm_transport_step(const mrcm_twophase *tp, const double *U, const double *q, const double *S,
                                const double *dt, void *stream, double *S_out) {
  TwoPhaseGrid t;
  const mrcm_status st = twophase_grid(tp, t);
  if (st != MRCM_OK) return st;
  if (!U || !S || !dt || !S_out) return fail(MRCM_EINVAL, "null argument");
  if (S_out == S) return fail(MRCM_EINVAL, "S_out must not overlap S");
  HIP_TRY(launch_transport(t, U, q, S, dt, S_out, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_transport_advance(const mrcm_twophase *tp, const double *U, const double *q, const void *marks,
                                   const double *S, const double *dt, double cfl, double dt_max, void *stream,
                                   double *S_out, double *dt_next) {
  TwoPhaseGrid t;
  const mrcm_status st = twophase_grid(tp, t);
  if (st != MRCM_OK) return st;
  if (!U || !S || !dt || !S_out || !dt_next) return fail(MRCM_EINVAL, "null argument");
  if (S_out == S) return fail(MRCM_EINVAL, "S_out must not overlap S");
  if (dt_next == dt) return fail(MRCM_EINVAL, "dt_next must not be dt");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(MRCM_EINVAL, "cfl must be positive and finite");
  if (!(dt_max > 0.0)) return fail(MRCM_EINVAL, "dt_max must be positive (or +inf)");
  const hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_speed_clear(dt_next, s));
  {
    Stage st(MRCM_STAGE_TRANSPORT, s);
    HIP_TRY(launch_transport_fused(t, U, q, S, dt, S_out, dt_next, s, static_cast<const unsigned char *>(marks)));
  }
  HIP_TRY(launch_speed_finish(t, cfl, dt_max, dt_next, s));
  return MRCM_OK;
}

int64_t mrcm_transport_marks_bytes(const mrcm_twophase *tp) {
  TwoPhaseGrid t;
  if (twophase_grid(tp, t) != MRCM_OK) return 0;
  return transport_tile_count(t);
}

mrcm_status mrcm_transport_mark_sources(const mrcm_twophase *tp, const double *q, void *stream, void *marks) {
  TwoPhaseGrid t;
  const mrcm_status st = twophase_grid(tp, t);
  if (st != MRCM_OK) return st;
  if (!q || !marks) return fail(MRCM_EINVAL, "null argument");
  HIP_TRY(launch_source_tiles(t, q, static_cast<unsigned char *>(marks), (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_transport_dt(const mrcm_twophase *tp, const double *U, const double *S, double cfl, double dt_max,
                              void *stream, double *dt) {
  TwoPhaseGrid t;
  const mrcm_status st = twophase_grid(tp, t);
  if (st != MRCM_OK) return st;
  if (!U || !S || !dt) return fail(MRCM_EINVAL, "null argument");
  if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(MRCM_EINVAL, "cfl must be positive and finite");
  if (!(dt_max > 0.0)) return fail(MRCM_EINVAL, "dt_max must be positive (or +inf)");
  HIP_TRY(launch_transport_dt(t, U, S, cfl, dt_max, dt, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_mobility_scale(const mrcm_twophase *tp, const double *S, const double *kx, const double *ky,
                                const double *kz, void *stream, double *kx_out, double *ky_out, double *kz_out) {
  TwoPhaseGrid t;
  const mrcm_status st = twophase_grid(tp, t);
  if (st != MRCM_OK) return st;
  if (!S || !kx || !ky || !kz || !kx_out || !ky_out || !kz_out) return fail(MRCM_EINVAL, "null argument");
  HIP_TRY(launch_mobility(t, S, kx, ky, kz, kx_out, ky_out, kz_out, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_postprocess_mean(const mrcm_mbfs *cmb, const double *U, void *stream, double *pt, double *Ut) {
  if (!cmb || !U || !pt || !Ut) return fail(MRCM_EINVAL, "null argument");
  mrcm_mbfs *mb = const_cast<mrcm_mbfs *>(cmb);  // lazily allocated Mean buffers
  const HostGeom &G = mb->G;
  if (G.bmax > kMaxBand64)
    return fail(MRCM_EUNSUPPORTED, "the Mean post-processing factors in FP64, whose band limit is 112");
  hipStream_t s = (hipStream_t)stream;
  if (!mb->d_sub_mean) {
    if (g_capturing) return fail(MRCM_EUNSUPPORTED, "the Mean post-processing allocates on its first use: not under capture");
    const mrcm_status st = init_mean(mb);
    if (st != MRCM_OK) return st;
  }
  Geom gm = mb->g;
  gm.sub = mb->d_sub_mean;
  {
    Stage t(MRCM_STAGE_MEAN, s);
    HIP_TRY(launch_reset_status(mb->st, s));
    HIP_TRY(launch_mean_coef(gm, mb->n_sub, G.max_cells, U, mb->mcoef, mb->mB, mb->mX, mb->mscal, s));
    for (size_t k = 0; k + 1 < mb->mean_chunk.size(); ++k) {
      const int c0 = mb->mean_chunk[k], nc = mb->mean_chunk[k + 1] - c0;
      HIP_TRY(launch_factor(0, mb->d_sub_mean, mb->d_order_mean + c0, nc, mb->mcoef, mb->mscal, mb->mfac, mb->mfac,
                            mb->st, G.bmax, s));
      HIP_TRY(launch_solve(0, gm, mb->d_work_mean + c0, nc, mb->mscal, mb->mfac, mb->mfac, mb->mX, mb->mX, 0, G.bmax,
                           s));
      // one FP64 refinement sweep: residual from the kept right-hand side,
      // then the correction
      HIP_TRY(launch_solve(0, gm, mb->d_work_mean + c0, nc, mb->mscal, mb->mfac, mb->mfac, mb->mR, mb->mX, 1,
                           G.bmax, s, mb->mcoef, mb->mB));
    }
    HIP_TRY(launch_mean_velocity(gm, U, mb->mX, pt, Ut, s));
  }
  if (g_prof.on && !g_capturing) {
    HIP_TRY(hipStreamSynchronize(s));
    profile_flush();
  }
  return read_status(mb->st, s, "mrcm_postprocess_mean");
}

namespace {

// Device buffers, events and handles of one IMPES run, released on every
// return path.
struct ImpesState {
  std::vector<double *> bufs;
  std::vector<hipEvent_t> ev;
  mrcm_mbfs *mb = nullptr;
  mrcm_interface *ih = nullptr;
  double *host = nullptr;  // pinned: the batch's step sizes read back
  ~ImpesState() {
    if (host) (void)hipHostFree(host);
    if (ih) mrcm_interface_destroy(ih);
    if (mb) mrcm_mbfs_destroy(mb);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (double *p : bufs) (void)hipFree(p);
  }
  hipError_t alloc(double **p, size_t n) {
    hipError_t e = dev_alloc(p, n);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  }
};

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.0f;
}

}  // namespace

mrcm_status mrcm_impes_run(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
                           const mrcm_options *opt, const mrcm_twophase *tp, const mrcm_impes_options *io,
                           void *stream, double *S, mrcm_impes_stats *stats) {
  if (!pb || !part || !ifs || !opt || !io || !S) return fail(MRCM_EINVAL, "null argument");
  TwoPhaseGrid tg;
  mrcm_status st = twophase_grid(tp, tg);
  if (st != MRCM_OK) return st;
  if (tp->nx != pb->nx || tp->ny != pb->ny || tp->nz != pb->nz || tp->hx != pb->hx || tp->hy != pb->hy ||
      tp->hz != pb->hz)
    return fail(MRCM_EINVAL, "the two-phase grid differs from the problem's");
  if (!pb->kx || !pb->ky || !pb->kz || !pb->q) return fail(MRCM_EINVAL, "null permeability or sources");
  if (io->skip < 1) return fail(MRCM_EINVAL, "skip must be at least 1");
  if (io->max_steps < 0) return fail(MRCM_EINVAL, "max_steps must be non-negative");
  if (std::isnan(io->t_end) || (io->max_steps == 0 && !std::isfinite(io->t_end)))
    return fail(MRCM_EINVAL, "the loop needs a finite t_end or a step cap");
  if (!(io->cfl > 0.0) || !std::isfinite(io->cfl)) return fail(MRCM_EINVAL, "cfl must be positive and finite");
  if (!(io->dt_max > 0.0)) return fail(MRCM_EINVAL, "dt_max must be positive (or +inf)");
  if (io->refine < 0 || io->refine > 20) return fail(MRCM_EINVAL, "refine must be within 0 .. 20");
  hipStream_t s = (hipStream_t)stream;
  const size_t N = (size_t)pb->nx * pb->ny * pb->nz;
  ImpesState W;
  double *ke, *pr, *U, *Ut, *pt, *S2, *dts, *X = nullptr;
  HIP_TRY(W.alloc(&ke, 3 * N));
  HIP_TRY(W.alloc(&pr, N));
  HIP_TRY(W.alloc(&U, 6 * N));
  HIP_TRY(W.alloc(&Ut, 6 * N));
  HIP_TRY(W.alloc(&pt, N));
  HIP_TRY(W.alloc(&S2, N));
  HIP_TRY(W.alloc(&dts, 2));
  // q holds through the run: the step reads it only in the tiles it marks
  double *marks = nullptr;
  HIP_TRY(W.alloc(&marks, (size_t)(transport_tile_count(tg) + 7) / 8));
  unsigned char *src_tiles = reinterpret_cast<unsigned char *>(marks);
  HIP_TRY(launch_source_tiles(tg, pb->q, src_tiles, s));
  W.ev.resize(5);
  for (auto &e : W.ev) HIP_TRY(hipEventCreate(&e));
  mrcm_problem pe = *pb;  // the Darcy problem of each solve: K lambda(S)
  pe.kx = ke;
  pe.ky = ke + N;
  pe.kz = ke + 2 * N;
  double t = 0.0, ms_d = 0.0, ms_d1 = 0.0, ms_m = 0.0, ms_t = 0.0;
  int32_t ns = 0, nd = 0;
  double *Scur = S, *Snext = S2, *dcur = dts, *dnext = dts + 1;
  auto finish = [&](mrcm_status code) -> mrcm_status {
    // the caller's S holds the last finite state
    if (Scur != S) {
      if (hipMemcpyAsync(S, Scur, N * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(MRCM_EHIP, "impes: copy of the final saturation failed");
    }
    if (stats) *stats = mrcm_impes_stats{nd, ns, t, ms_d, ms_d1, ms_m, ms_t};
    return code;
  };
  // Saturation steps go in batches of up to kImpesBatch (never past the next
  // Darcy solve or the step cap), each step's dt logged on the device; one
  // read-back per batch replays t on the host.  If the run ends inside a
  // batch (t passes t_end, or a step is not finite), the batch's starting
  // state is restored and exactly the steps that count are taken again: the
  // kernels are deterministic, so the result is that of stepping one by one.
  constexpr int kImpesBatch = 64;
  double *Sa, *dlog;
  HIP_TRY(W.alloc(&Sa, N));
  HIP_TRY(W.alloc(&dlog, kImpesBatch));
  HIP_TRY(hipHostMalloc((void **)&W.host, kImpesBatch * sizeof(double), hipHostMallocDefault));
  auto step = [&]() -> mrcm_status {
    HIP_TRY(launch_speed_clear(dnext, s));
    {
      Stage stg(MRCM_STAGE_TRANSPORT, s);
      HIP_TRY(launch_transport_fused(tg, Ut, pb->q, Scur, dcur, Snext, dnext, s, src_tiles));
    }
    HIP_TRY(launch_speed_finish(tg, io->cfl, io->dt_max, dnext, s));
    std::swap(Scur, Snext);
    std::swap(dcur, dnext);
    return MRCM_OK;
  };
  while (t <= io->t_end && (io->max_steps == 0 || ns < io->max_steps)) {
    const bool darcy = ns % io->skip == 0;
    if (darcy) {
      HIP_TRY(hipEventRecord(W.ev[0], s));
      HIP_TRY(launch_mobility(tg, Scur, pb->kx, pb->ky, pb->kz, ke, ke + N, ke + 2 * N, s));
      if ((st = mrcm_build_mbfs(&pe, part, ifs, opt, stream, &W.mb)) != MRCM_OK) return st;
      if (!X) HIP_TRY(W.alloc(&X, 2 * (size_t)W.mb->G.n_patch));
      if ((st = mrcm_assemble_interface(W.mb, stream, &W.ih)) != MRCM_OK) return st;
      if ((st = mrcm_solve_interface(W.ih, MRCM_IFACE_AUTO, 0.0, io->refine, stream, X, nullptr, nullptr)) !=
          MRCM_OK)
        return st;
      if ((st = mrcm_reconstruct(W.mb, X, stream, pr, U)) != MRCM_OK) return st;
      HIP_TRY(hipEventRecord(W.ev[1], s));
      if ((st = mrcm_postprocess_mean(W.mb, U, stream, pt, Ut)) != MRCM_OK) return st;
      HIP_TRY(launch_transport_dt(tg, Ut, Scur, io->cfl, io->dt_max, dcur, s));
      HIP_TRY(hipEventRecord(W.ev[2], s));
      ++nd;
    }
    int kmax = std::min(kImpesBatch, io->skip - ns % io->skip);
    if (io->max_steps > 0) kmax = std::min(kmax, io->max_steps - ns);
    HIP_TRY(hipMemcpyAsync(Sa, Scur, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipEventRecord(W.ev[3], s));
    for (int j = 0; j < kmax; ++j) {
      HIP_TRY(hipMemcpyAsync(dlog + j, dcur, sizeof(double), hipMemcpyDeviceToDevice, s));
      if ((st = step()) != MRCM_OK) return st;
    }
    HIP_TRY(hipEventRecord(W.ev[4], s));
    HIP_TRY(hipMemcpyAsync(W.host, dlog, kmax * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (darcy) {
      if (nd == 1) ms_d1 = elapsed_ms(W.ev[0], W.ev[1]);
      ms_d += elapsed_ms(W.ev[0], W.ev[1]);
      ms_m += elapsed_ms(W.ev[1], W.ev[2]);
    }
    ms_t += elapsed_ms(W.ev[3], W.ev[4]);
    // the loop head of each step, replayed: t <= t_end, then the step
    int taken = 0;
    bool bad = false;
    while (taken < kmax && t <= io->t_end) {
      if (!std::isfinite(W.host[taken])) {
        bad = true;
        break;
      }
      t += W.host[taken];
      ++taken;
    }
    ns += taken;
    if (taken < kmax) {
      HIP_TRY(hipMemcpyAsync(S, Sa, N * sizeof(double), hipMemcpyDeviceToDevice, s));
      Scur = S;
      Snext = S2;
      dcur = dts;
      dnext = dts + 1;
      HIP_TRY(hipMemcpyAsync(dcur, dlog, sizeof(double), hipMemcpyDeviceToDevice, s));
      for (int j = 0; j < taken; ++j)
        if ((st = step()) != MRCM_OK) return st;
      HIP_TRY(hipStreamSynchronize(s));
      if (bad)
        return finish(fail(MRCM_EINVAL, "impes: the step is not finite (nothing moves under the CFL bound and "
                                        "dt_max is infinite)"));
      break;
    }
  }
  return finish(MRCM_OK);
}

mrcm_status mrcm_reconstruct(const mrcm_mbfs *mb, const double *X, void *stream, double *p,
                             double *U) {
  if (!mb || !p || !U) return fail(MRCM_EINVAL, "null argument");
  if (mb->G.n_patch > 0 && !X) return fail(MRCM_EINVAL, "X is null");
  hipStream_t s = (hipStream_t)stream;
  {
    Stage t(MRCM_STAGE_RECONSTRUCT, s);
    if (mb->G.keep & MRCM_KEEP_MBFS) {
      HIP_TRY(launch_recon_p(mb->g, mb->n_sub, mb->d_patches, mb->X, X, mb->G.n_patch, p, s));
    } else {
      mrcm_status st = reconstruct_resolve(mb, X, s, p);
      if (st != MRCM_OK) return st;
    }
    HIP_TRY(launch_recon_u(mb->g, p, X, mb->G.n_patch, U, s));
  }
  if (g_prof.on && !g_capturing) {
    HIP_TRY(hipStreamSynchronize(s));
    profile_flush();
  }
  return MRCM_OK;
}

mrcm_status mrcm_query(const mrcm_mbfs *mb, mrcm_info *info) {
  if (!mb || !info) return fail(MRCM_EINVAL, "null argument");
  const HostGeom &G = mb->G;
  info->n_sub = (int32_t)G.subs.size();
  info->n_patch = G.n_patch;
  info->n_cells = G.totCells;
  info->n_mbfs = G.n_mbfs;
  info->n_rhs = G.n_rhs;
  info->max_band = G.bmax;
  info->max_rhs = G.mmax;
  info->precision = G.precision;
  info->ir_iters = mb->ir_iters;
  info->ir_residual = mb->ir_res;
  info->factor_flops = G.factor_flops;
  info->solve_flops = G.solve_flops;
  info->device_bytes = mb->bytes;
  info->pcg_fallback = mb->pcg_fallback;
  info->pcg_iters = mb->pcg_iters;
  return MRCM_OK;
}

mrcm_status mrcm_get_subdomain(const mrcm_mbfs *mb, int32_t l, mrcm_subdomain_info *info) {
  if (!mb || !info) return fail(MRCM_EINVAL, "null argument");
  if (l < 0 || l >= (int32_t)mb->G.subs.size()) return fail(MRCM_EINVAL, "subdomain out of range");
  const SubDesc &S = mb->G.subs[l];
  for (int d = 0; d < 3; ++d) {
    info->lo[d] = S.lo[d];
    info->ext[d] = S.ext[d];
    info->ax[d] = S.ax[d];
  }
  info->n_cells = S.N;
  info->band = S.b;
  info->n_rhs = S.m;
  info->n_patch = S.npatch;
  info->pin_local = S.pin_local;
  info->solve_group = mb->solve_group.empty() ? 0 : mb->solve_group[l];
  return MRCM_OK;
}

mrcm_status mrcm_copy_mbfs(const mrcm_mbfs *mb, int32_t l, double *X) {
  if (!mb || !X) return fail(MRCM_EINVAL, "null argument");
  if (!(mb->G.keep & MRCM_KEEP_MBFS)) return fail(MRCM_EINVAL, "the handle does not keep its MBFs");
  if (l < 0 || l >= (int32_t)mb->G.subs.size()) return fail(MRCM_EINVAL, "subdomain out of range");
  const SubDesc &S = mb->G.subs[l];
  HIP_TRY(hipStreamSynchronize(mb->stream));
  HIP_TRY(hipMemcpy(X, mb->X + S.X_off, (size_t)S.N * S.m * sizeof(double), hipMemcpyDeviceToHost));
  return MRCM_OK;
}

mrcm_status mrcm_copy_flux(const mrcm_mbfs *mb, int32_t l, double *F, double *Fb, double *SAb) {
  if (!mb || !F || !Fb || !SAb) return fail(MRCM_EINVAL, "null argument");
  if (l < 0 || l >= (int32_t)mb->G.subs.size()) return fail(MRCM_EINVAL, "subdomain out of range");
  const SubDesc &S = mb->G.subs[l];
  HIP_TRY(hipStreamSynchronize(mb->stream));
  const size_t nb = (size_t)S.npatch * S.m * sizeof(double);
  HIP_TRY(hipMemcpy(F, mb->F + S.F_off, nb, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(Fb, mb->Fb + S.F_off, nb, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(SAb, mb->SAb + S.patch_off, (size_t)S.npatch * sizeof(double), hipMemcpyDeviceToHost));
  return MRCM_OK;
}

mrcm_status mrcm_copy_factor(const mrcm_mbfs *mb, int32_t l, double *Lband) {
  if (!mb || !Lband) return fail(MRCM_EINVAL, "null argument");
  if (l < 0 || l >= (int32_t)mb->G.subs.size()) return fail(MRCM_EINVAL, "subdomain out of range");
  const SubDesc &S = mb->G.subs[l];
  const size_t cnt = (size_t)S.N * (S.b + 1);
  HIP_TRY(hipStreamSynchronize(mb->stream));
  if (mb->G.precision == MRCM_FP32_IR) {
    std::vector<float> tmp(cnt);
    HIP_TRY(hipMemcpy(tmp.data(), (const float *)mb->L + S.L_off, cnt * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < cnt; ++i) Lband[i] = tmp[i];
  } else {
    HIP_TRY(hipMemcpy(Lband, (const double *)mb->L + S.L_off, cnt * sizeof(double), hipMemcpyDeviceToHost));
  }
  return MRCM_OK;
}

mrcm_status mrcm_interface_dims(const mrcm_interface *h, int32_t *n, int32_t *bandwidth) {
  if (!h || !n || !bandwidth) return fail(MRCM_EINVAL, "null argument");
  *n = h->n;
  *bandwidth = h->w;
  return MRCM_OK;
}

mrcm_status mrcm_copy_interface(const mrcm_interface *h, double *A, double *b) {
  if (!h || !A || !b) return fail(MRCM_EINVAL, "null argument");
  const int n = h->n, nv = h->nv;
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (n == 0) return MRCM_OK;
  const mrcm_mbfs *mb = h->mb;
  double *dA = nullptr, *db = nullptr;
  if (dev_alloc(&dA, (size_t)n * n) != hipSuccess || dev_alloc(&db, (size_t)n) != hipSuccess) {
    if (dA) (void)hipFree(dA);
    return fail(MRCM_ENOMEM, "device allocation of the dense copy failed");
  }
  hipError_t e = launch_mf_dense(mb->g, mb->d_patches, mb->F, mb->Fb, mb->SAb, h->dp.pinfo, nv, dA, db, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(A, dA, (size_t)n * n * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(b, db, (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(dA);
  (void)hipFree(db);
  if (e != hipSuccess) return fail(MRCM_EHIP, std::string("mrcm_copy_interface: ") + hipGetErrorString(e));
  return MRCM_OK;
}

void mrcm_profile_enable(int32_t on) {
  profile_flush();
  g_prof.on = on != 0;
}

void mrcm_profile_reset(void) {
  profile_flush();
  for (int i = 0; i < 16; ++i) {
    g_prof.ms[i] = 0.0;
    g_prof.count[i] = 0;
  }
}

mrcm_status mrcm_profile_get(mrcm_profile *out) {
  if (!out) return fail(MRCM_EINVAL, "null argument");
  profile_flush();
  for (int i = 0; i < 16; ++i) {
    out->ms[i] = g_prof.ms[i];
    out->count[i] = g_prof.count[i];
  }
  return MRCM_OK;
}

mrcm_status mrcm_autotune(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
                          const mrcm_options *base, void *stream, mrcm_options *best, double *best_ms,
                          double *rule_ms) {
  if (!pb || !part || !ifs || !base || !best) return fail(MRCM_EINVAL, "null argument");
  // one handle per candidate: an untimed build, then the fastest of three
  auto time_opts = [&](const mrcm_options &o, double &ms, int *n_first) -> mrcm_status {
    mrcm_mbfs *h = nullptr;
    mrcm_status st = mrcm_build_mbfs(pb, part, ifs, &o, stream, &h);
    if (st != MRCM_OK) return st;
    if (n_first) *n_first = h->n_first;
    ms = 1e300;
    for (int r = 0; r < 3 && st == MRCM_OK; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      st = mrcm_build_mbfs(pb, part, ifs, &o, stream, &h);  // returns after synchronising
      const auto t1 = std::chrono::steady_clock::now();
      ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    mrcm_mbfs_destroy(h);
    return st;
  };
  mrcm_options cur = *base;
  double t_rule = 0.0;
  int nf = 0;
  mrcm_status st = time_opts(cur, t_rule, &nf);
  if (st != MRCM_OK) return st;
  mrcm_options win = cur;
  double t_best = t_rule;
  auto consider = [&](int tiles, int group, int lm) -> mrcm_status {
    if (tiles == cur.solve_tiles && group == cur.solve_group && lm == cur.launch_mode) return MRCM_OK;
    mrcm_options o = cur;
    o.solve_tiles = tiles;
    o.solve_group = group;
    o.launch_mode = lm;
    double t = 0.0;
    mrcm_status e = time_opts(o, t, nullptr);
    if (e != MRCM_OK) return e;
    // a candidate must beat the current choice by 2%, more than the
    // run-to-run spread of the timings, so that near-ties keep the default
    if (t < 0.98 * t_best) {
      t_best = t;
      win = o;
    }
    return MRCM_OK;
  };
  const int tmax = solve_chunk_max() / 16;
  for (int tiles = 0; tiles <= tmax && st == MRCM_OK; ++tiles) {
    st = consider(tiles, 0, cur.launch_mode);
    if (st == MRCM_OK && base->precision == MRCM_FP64) st = consider(tiles, -1, cur.launch_mode);
  }
  // the size of the pipeline's first group around the occupancy rule's
  if (st == MRCM_OK && nf > 0)
    for (int dg : {-128, -64, 64, 128})
      if (st == MRCM_OK && nf + dg > 0) st = consider(win.solve_tiles, nf + dg, cur.launch_mode);
  // the persistent work-queue form of the ragged launches, with the winners
  if (st == MRCM_OK && base->precision != MRCM_PCG)
    st = consider(win.solve_tiles, win.solve_group, 1 - cur.launch_mode);
  if (st != MRCM_OK) return st;
  // the interface factorisation's panel width, on assembly and solve with
  // the winning build: one interface handle per candidate, one untimed and
  // three timed runs, the fastest counted, the same 2% rule
  {
    mrcm_mbfs *h = nullptr;
    st = mrcm_build_mbfs(pb, part, ifs, &win, stream, &h);
    if (st != MRCM_OK) return st;
    const int nv = h->G.n_patch;
    double *X = nullptr;
    if (nv > 0 && hipMalloc((void **)&X, 2 * (size_t)nv * sizeof(double)) != hipSuccess) {
      mrcm_mbfs_destroy(h);
      return fail(MRCM_ENOMEM, "autotune: allocation of the interface vector failed");
    }
    const int p0 = win.iface_panel > 0 ? win.iface_panel : kMfPanelMax;
    double t_p0 = 0.0, t_pbest = 0.0;
    int p_best = p0;
    for (int P : {p0, 4, 2, 1}) {
      if (nv == 0 || st != MRCM_OK) break;
      if (P == p0 && t_p0 > 0.0) continue;
      h->G.iface_panel = P;  // the plan of a new interface handle takes it
      mrcm_interface *ih = nullptr;
      double ms = 1e300;
      for (int r = 0; r < 4 && st == MRCM_OK; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        st = mrcm_assemble_interface(h, stream, &ih);
        if (st == MRCM_OK) st = mrcm_solve_interface(ih, MRCM_IFACE_AUTO, 0.0, 0, stream, X, nullptr, nullptr);
        if (st == MRCM_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
          st = fail(MRCM_EHIP, "autotune: stream synchronisation failed");
        const auto t1 = std::chrono::steady_clock::now();
        if (r > 0) ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
      }
      if (ih) mrcm_interface_destroy(ih);
      if (st != MRCM_OK) break;
      if (t_p0 == 0.0) {
        t_p0 = t_pbest = ms;
      } else if (ms < 0.98 * t_pbest) {
        t_pbest = ms;
        p_best = P;
      }
    }
    if (X) (void)hipFree(X);
    mrcm_mbfs_destroy(h);
    if (st != MRCM_OK) return st;
    win.iface_panel = nv > 0 ? p_best : win.iface_panel;
  }
  *best = win;
  if (best_ms) *best_ms = t_best;
  if (rule_ms) *rule_ms = t_rule;
  return MRCM_OK;
}

namespace {
// What the tuned values depend on, as text: the shapes of the problem and of
// its partition and interface spaces, the form, and the device.
std::string tune_signature(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
                           const mrcm_options *base, const ConfigKey &k) {
  std::string sig = "n";
  for (int d = 0; d < 3; ++d) sig += " " + std::to_string(k.n[d]);
  char buf[64];
  for (int d = 0; d < 3; ++d) {
    std::snprintf(buf, sizeof buf, " %.17g", k.h[d]);
    sig += buf;
  }
  for (int d = 0; d < 3; ++d) {
    sig += "|c";
    for (int c : k.cuts[d]) sig += " " + std::to_string(c);
    sig += "|u " + std::to_string(k.us[d][0]) + " " + std::to_string(k.us[d][1]);
  }
  sig += "|s";
  for (int v : k.split) sig += " " + std::to_string(v);
  sig += "|w";
  for (int f = 0; f < 6; ++f) sig += " " + std::to_string(k.wall_type[f]);
  sig += "|p " + std::to_string(base->precision) + " b " + std::to_string(base->beta_mode) + " k " +
         std::to_string(base->keep);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    sig += std::string("|d ") + prop.gcnArchName + " " + std::to_string(prop.multiProcessorCount);
  (void)pb;
  (void)part;
  (void)ifs;
  return sig;
}

uint64_t fnv1a64(const std::string &s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}
}  // namespace

mrcm_status mrcm_autotune_cached(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
                                 const mrcm_options *base, void *stream, const char *cache_path, mrcm_options *best,
                                 double *best_ms, double *rule_ms, int32_t *from_cache) {
  if (!pb || !part || !ifs || !base || !best || !cache_path) return fail(MRCM_EINVAL, "null argument");
  if (from_cache) *from_cache = 0;
  ConfigKey k;
  if (!make_key(pb, part, ifs, base, k))  // malformed input: the full check reports it
    return mrcm_autotune(pb, part, ifs, base, stream, best, best_ms, rule_ms);
  char key[32];
  std::snprintf(key, sizeof key, "%016llx", (unsigned long long)fnv1a64(tune_signature(pb, part, ifs, base, k)));
  if (FILE *f = std::fopen(cache_path, "r")) {
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
      char tag[32], kk[32];
      int tiles = 0, group = 0, panel = 0, lm = 0;
      double bm = 0.0, rm = 0.0;
      if (std::sscanf(line, "%31s %31s %d %d %d %d %lf %lf", tag, kk, &tiles, &group, &panel, &lm, &bm, &rm) != 8)
        continue;
      if (std::strcmp(tag, "mrcm-tune-2") != 0 || std::strcmp(kk, key) != 0) continue;
      if (tiles < 0 || tiles > solve_chunk_max() / 16 || group < -1 || panel < 0 || panel > kMfPanelMax ||
          (lm != MRCM_LAUNCH_GRID && lm != MRCM_LAUNCH_QUEUE))
        continue;
      std::fclose(f);
      *best = *base;
      best->solve_tiles = tiles;
      best->solve_group = group;
      best->iface_panel = panel;
      best->launch_mode = lm;
      if (best_ms) *best_ms = bm;
      if (rule_ms) *rule_ms = rm;
      if (from_cache) *from_cache = 1;
      return MRCM_OK;
    }
    std::fclose(f);
  }
  double bm = 0.0, rm = 0.0;
  const mrcm_status st = mrcm_autotune(pb, part, ifs, base, stream, best, &bm, &rm);
  if (st != MRCM_OK) return st;
  if (best_ms) *best_ms = bm;
  if (rule_ms) *rule_ms = rm;
  FILE *f = std::fopen(cache_path, "a");
  if (!f) return fail(MRCM_EINVAL, std::string("autotune cache not writable: ") + cache_path);
  const int ok = std::fprintf(f, "mrcm-tune-2 %s %d %d %d %d %.6f %.6f\n", key, best->solve_tiles,
                              best->solve_group, best->iface_panel, best->launch_mode, bm, rm);
  const int closed = std::fclose(f);
  if (ok < 0 || closed != 0) return fail(MRCM_EINVAL, std::string("autotune cache not writable: ") + cache_path);
  return MRCM_OK;
}

struct mrcm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mrcm_mbfs *mb = nullptr;
  mrcm_interface *ifc = nullptr;
};

mrcm_status mrcm_graph_capture(const mrcm_problem *pb, const mrcm_partition *part, const mrcm_iface_space *ifs,
                               const mrcm_options *opt, mrcm_mbfs *mb, mrcm_interface *ifc, int32_t refine,
                               double *X, double *p, double *U, void *stream, mrcm_graph **out) {
  if (!pb || !part || !ifs || !opt || !mb || !ifc || !p || !U || !out) return fail(MRCM_EINVAL, "null argument");
  if (ifc->mb != mb) return fail(MRCM_EINVAL, "interface handle belongs to another mbfs handle");
  if (opt->precision != MRCM_FP64 || mb->G.precision != MRCM_FP64)
    return fail(MRCM_EUNSUPPORTED, "only the FP64 form can be captured");
  if (!stream) return fail(MRCM_EINVAL, "capture needs a stream other than the null stream");
  if (mb->G.n_patch > 0 && !X) return fail(MRCM_EINVAL, "X is null");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  g_capturing = true;
  mrcm_mbfs *h = mb;
  mrcm_interface *hi = ifc;
  mrcm_status st = mrcm_build_mbfs(pb, part, ifs, opt, stream, &h);
  if (st == MRCM_OK && h != mb) st = fail(MRCM_EINVAL, "the options or problem differ from the handle's");
  if (st == MRCM_OK) st = mrcm_assemble_interface(mb, stream, &hi);
  if (st == MRCM_OK) st = mrcm_solve_interface(ifc, MRCM_IFACE_AUTO, 0.0, refine, stream, X, nullptr, nullptr);
  if (st == MRCM_OK) st = mrcm_reconstruct(mb, X, stream, p, U);
  g_capturing = false;
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != MRCM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(MRCM_EHIP, std::string("stream capture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(MRCM_EHIP, std::string("graph instantiation: ") + hipGetErrorString(e2));
  }
  mrcm_graph *gr = new mrcm_graph();
  gr->graph = graph;
  gr->exec = exec;
  gr->mb = mb;
  gr->ifc = ifc;
  *out = gr;
  return MRCM_OK;
}

mrcm_status mrcm_graph_launch(mrcm_graph *gr, void *stream) {
  if (!gr) return fail(MRCM_EINVAL, "null graph");
  HIP_TRY(hipGraphLaunch(gr->exec, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_graph_check(mrcm_graph *gr, void *stream) {
  if (!gr) return fail(MRCM_EINVAL, "null graph");
  hipStream_t s = (hipStream_t)stream;
  mrcm_status st = read_status(gr->mb->st, s, "mrcm_build_mbfs (graph)");
  if (st != MRCM_OK) return st;
  if (gr->ifc->n > 0) return read_status(gr->ifc->st, s, "mrcm_solve_interface (graph)");
  return MRCM_OK;
}

void mrcm_graph_destroy(mrcm_graph *gr) {
  if (!gr) return;
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
}

int32_t mrcm_conv3d_max_channels(void) { return conv3d_max_channels(); }

namespace {
mrcm_status check_conv(const void *x, const void *w, const void *y, int32_t batch, int32_t cin, int32_t cout,
                       int32_t d, int32_t h, int32_t wd) {
  if (!x || !w || !y) return fail(MRCM_EINVAL, "null tensor");
  if (batch <= 0 || cin <= 0 || cout <= 0 || d <= 0 || h <= 0 || wd <= 0)
    return fail(MRCM_EINVAL, "sizes must be positive");
  if (cin > conv3d_max_channels() || cout > conv3d_max_channels())
    return fail(MRCM_EINVAL, "at most " + std::to_string(conv3d_max_channels()) + " channels");
  if ((long long)batch * d * h * wd * std::max(cin, cout) >= (1LL << 40)) return fail(MRCM_EUNSUPPORTED, "tensor too large");
  return MRCM_OK;
}

// Uploads the selection (subdomains with the same grid) and each one's first
// sample; returns the sample size V and the largest column count.
mrcm_status nn_select(mrcm_mbfs *h, const int32_t *subs, int32_t n, hipStream_t s, int &V, int &mmax) {
  if (!h || !subs || n <= 0) return fail(MRCM_EINVAL, "null handle or empty subdomain list");
  const HostGeom &G = h->G;
  const int n_sub = (int)G.subs.size();
  // the previous selection's upload may still be in flight from these host
  // arrays: let the stream pass it before they change
  if (h->d_nn_sel) HIP_TRY(hipStreamSynchronize(s));
  h->nn_sel.assign(subs, subs + n);
  h->nn_s0.resize(n);
  int s0 = 0;
  mmax = 0;
  V = -1;
  int shape[3] = {0, 0, 0};
  for (int k = 0; k < n; ++k) {
    const int l = subs[k];
    if (l < 0 || l >= n_sub) return fail(MRCM_EINVAL, "subdomain out of range");
    const SubDesc &S = G.subs[l];
    if (k == 0) {
      shape[0] = S.n0;
      shape[1] = S.n1;
      shape[2] = S.n2;
      V = S.N;
    } else if (S.n0 != shape[0] || S.n1 != shape[1] || S.n2 != shape[2]) {
      return fail(MRCM_EINVAL, "the listed subdomains must share one grid");
    }
    h->nn_s0[k] = s0;
    s0 += S.m;
    mmax = std::max(mmax, S.m);
  }
  if (!h->d_nn_sel) {
    if (dev_alloc(&h->d_nn_sel, (size_t)n_sub) != hipSuccess || dev_alloc(&h->d_nn_s0, (size_t)n_sub) != hipSuccess)
      return fail(MRCM_ENOMEM, "device allocation of the sample lists failed");
  }
  if (n > n_sub) return fail(MRCM_EINVAL, "more subdomains listed than the handle has");
  HIP_TRY(hipMemcpyAsync(h->d_nn_sel, h->nn_sel.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->d_nn_s0, h->nn_s0.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  return MRCM_OK;
}
}  // namespace

mrcm_status mrcm_conv3d_forward(const float *x, const float *weights, const float *bias, float *y,
                                const float *mask, int32_t batch, int32_t cin, int32_t cout, int32_t d,
                                int32_t h, int32_t w, int32_t dilation, int32_t relu, void *stream) {
  mrcm_status st = check_conv(x, weights, y, batch, cin, cout, d, h, w);
  if (st != MRCM_OK) return st;
  if (dilation < 1) return fail(MRCM_EINVAL, "dilation must be at least 1");
  HIP_TRY(launch_conv3d(x, weights, bias, y, mask, batch, cin, cout, d, h, w, dilation, relu, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_conv3d_backward(const float *x, const float *weights, const float *dy, float *dx, float *dw,
                                 float *db, float *wt, const float *dx_mask, int32_t batch, int32_t cin,
                                 int32_t cout, int32_t d, int32_t h, int32_t w, int32_t dilation, void *stream) {
  mrcm_status st = check_conv(x, weights, dy, batch, cin, cout, d, h, w);
  if (st != MRCM_OK) return st;
  if (dilation < 1) return fail(MRCM_EINVAL, "dilation must be at least 1");
  if (!dw) return fail(MRCM_EINVAL, "dw is required");
  if (dx && !wt) return fail(MRCM_EINVAL, "dx needs the workspace wt");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_conv3d_wgrad(x, dy, dw, db, batch, cin, cout, d, h, w, dilation, s));
  if (dx) {
    HIP_TRY(launch_conv3d_flip(weights, wt, cin, cout, s));
    HIP_TRY(launch_conv3d(dy, wt, nullptr, dx, dx_mask, batch, cout, cin, d, h, w, dilation, 0, s));
  }
  return MRCM_OK;
}

mrcm_status mrcm_mse(const float *y, const float *t, float *dy, double *loss, double *workspace, int64_t n,
                     void *stream) {
  if (!y || !t || !dy || !loss || !workspace) return fail(MRCM_EINVAL, "null argument");
  if (n <= 0) return fail(MRCM_EINVAL, "n must be positive");
  HIP_TRY(launch_mse(y, t, dy, workspace, loss, n, (hipStream_t)stream));
  return MRCM_OK;
}

int32_t mrcm_unet_max_channels(void) { return unet_max_channels(); }
int32_t mrcm_unet_padded(int32_t c) { return unet_pad16(c); }

namespace {
mrcm_status check_unet(int32_t batch, int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout) {
  if (batch <= 0 || d <= 0 || h <= 0 || w <= 0 || cin <= 0 || cout <= 0)
    return fail(MRCM_EINVAL, "sizes must be positive");
  if (cin > unet_max_channels() || cout > unet_max_channels())
    return fail(MRCM_EINVAL, "at most " + std::to_string(unet_max_channels()) + " channels");
  if ((long long)batch * d * h * w >= (1LL << 31)) return fail(MRCM_EUNSUPPORTED, "more than 2^31 voxels");
  return MRCM_OK;
}
}  // namespace

mrcm_status mrcm_unet_pack(const float *w, uint16_t *wf, uint16_t *wt, int32_t cin, int32_t cout, void *stream) {
  if (!w || !wf || !wt) return fail(MRCM_EINVAL, "null argument");
  mrcm_status st = check_unet(1, 1, 1, 1, cin, cout);
  if (st != MRCM_OK) return st;
  HIP_TRY(launch_unet_pack(w, wf, wt, cin, cout, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_unet_conv(const float *x, const uint16_t *wf, const float *bias, float *y, const float *mask,
                           int32_t batch, int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t relu,
                           void *stream) {
  if (!x || !wf || !y) return fail(MRCM_EINVAL, "null tensor");
  mrcm_status st = check_unet(batch, d, h, w, cin, cout);
  if (st != MRCM_OK) return st;
  HIP_TRY(launch_unet_conv(x, wf, bias, y, mask, batch, d, h, w, cin, cout, relu, (hipStream_t)stream));
  return MRCM_OK;
}

int64_t mrcm_unet_wgrad_workspace(int32_t batch, int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout) {
  if (check_unet(batch, d, h, w, cin, cout) != MRCM_OK) return -1;
  return unet_wgrad_workspace((long long)batch * d * h * w, cin, cout);
}

mrcm_status mrcm_unet_wgrad(const float *x, const float *dy, float *dw, float *db, float *workspace, int32_t batch,
                            int32_t d, int32_t h, int32_t w, int32_t cin, int32_t cout, void *stream) {
  if (!x || !dy || !dw || !workspace) return fail(MRCM_EINVAL, "null tensor");
  mrcm_status st = check_unet(batch, d, h, w, cin, cout);
  if (st != MRCM_OK) return st;
  HIP_TRY(launch_unet_wgrad(x, dy, dw, db, workspace, batch, d, h, w, cin, cout, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_unet_pool(const float *x, float *y, int32_t batch, int32_t d, int32_t h, int32_t w, int32_t c,
                           int32_t backward, void *stream) {
  if (!x || !y) return fail(MRCM_EINVAL, "null tensor");
  mrcm_status st = check_unet(batch, d, h, w, c, c);
  if (st != MRCM_OK) return st;
  if (d % 2 || h % 2) return fail(MRCM_EINVAL, "pooling needs even d and h");
  HIP_TRY(launch_unet_pool(x, y, batch, d, h, w, c, backward, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_unet_upsample(const float *x, float *y, int32_t batch, int32_t d, int32_t h, int32_t w, int32_t c,
                               int32_t backward, void *stream) {
  if (!x || !y) return fail(MRCM_EINVAL, "null tensor");
  mrcm_status st = check_unet(batch, 2 * d, 2 * h, w, c, c);
  if (st != MRCM_OK) return st;
  HIP_TRY(launch_unet_up(x, y, batch, d, h, w, c, backward, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_unet_relu_mask(float *g, const float *out, int64_t n, void *stream) {
  if (!g || !out) return fail(MRCM_EINVAL, "null tensor");
  if (n <= 0) return fail(MRCM_EINVAL, "n must be positive");
  HIP_TRY(launch_unet_relu_mask(g, out, n, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_nn_channels_last(const float *in, float *out, int32_t batch, int32_t c, int64_t voxels, void *stream) {
  if (!in || !out) return fail(MRCM_EINVAL, "null tensor");
  if (batch <= 0 || c <= 0 || voxels <= 0) return fail(MRCM_EINVAL, "sizes must be positive");
  HIP_TRY(launch_channels_last(in, out, batch, c, voxels, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_mse_noalloc(const float *y, const float *t, float *dy, double *loss, int64_t n, void *stream) {
  if (!y || !t || !dy || !loss) return fail(MRCM_EINVAL, "null argument");
  if (n <= 0) return fail(MRCM_EINVAL, "n must be positive");
  if (n > MRCM_MSE_NOALLOC_MAX_N)
    return fail(MRCM_EINVAL, "n exceeds " + std::to_string(MRCM_MSE_NOALLOC_MAX_N) +
                                 ", the largest this entry point takes");
  HIP_TRY(launch_mse_static(y, t, dy, loss, n, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_adam_step(float *p, const float *g, float *m, float *v, int32_t n, int32_t t, float lr,
                           float b1, float b2, float eps, void *stream) {
  if (!p || !g || !m || !v) return fail(MRCM_EINVAL, "null argument");
  if (n <= 0 || t < 1) return fail(MRCM_EINVAL, "n must be positive and t at least 1");
  HIP_TRY(launch_adam(p, g, m, v, n, t, lr, b1, b2, eps, (hipStream_t)stream));
  return MRCM_OK;
}

mrcm_status mrcm_nn_features(mrcm_mbfs *h, const int32_t *subs, int32_t n_subs, float *inp, float *tgt,
                             void *stream) {
  if (!inp) return fail(MRCM_EINVAL, "null input tensor");
  hipStream_t s = (hipStream_t)stream;
  int V = 0, mmax = 0;
  mrcm_status st = nn_select(h, subs, n_subs, s, V, mmax);
  if (st != MRCM_OK) return st;
  const HostGeom &H = h->G;
  if (!h->R) {
    if (dev_alloc(&h->R, (size_t)H.totX) != hipSuccess)
      return fail(MRCM_ENOMEM, "device allocation of the right-hand-side buffer failed");
    h->bytes += H.totX * 8;
  }
  // the right-hand sides of the current build, formed once for all calls
  if (!h->nn_rhs_ready) {
    HIP_TRY(launch_rhs(h->g, h->n_sub, H.max_cells, H.mmax, h->r0, h->R, s));
    h->nn_rhs_ready = true;
  }
  HIP_TRY(launch_nn_features(h->g, h->d_nn_sel, h->d_nn_s0, n_subs, mmax, h->R, h->X, V, inp, tgt, s));
  return MRCM_OK;
}

mrcm_status mrcm_nn_scatter(mrcm_mbfs *h, const int32_t *subs, int32_t n_subs, const float *out, double *x0,
                            void *stream) {
  if (!out || !x0) return fail(MRCM_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  int V = 0, mmax = 0;
  mrcm_status st = nn_select(h, subs, n_subs, s, V, mmax);
  if (st != MRCM_OK) return st;
  HIP_TRY(launch_nn_scatter(h->g, h->d_nn_sel, h->d_nn_s0, n_subs, mmax, out, V, x0, s));
  return MRCM_OK;
}

void mrcm_mbfs_destroy(mrcm_mbfs *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  free_mbfs(h);
}

void mrcm_interface_destroy(mrcm_interface *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  free_iface(h);
}

}  // extern "C"
