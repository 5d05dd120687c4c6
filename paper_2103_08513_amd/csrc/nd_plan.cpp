// Nested-dissection plan of the interface system (host side): the tree of
// separators, the frontal matrices' index lists and storage, the scatter map
// of the assembled entries and the launch tables of the factorisation.
#include "nd_plan.h"

#include <algorithm>
#include <functional>

namespace mrcm {

namespace {

struct TmpNode {
  int lo[3], hi[3];
  std::vector<int> front;  // unknowns (2*patch + t) or -1 (pad)
  int s = 0, sp = 0;
  int parent = -1, child[2] = {-1, -1};
  int height = 1;
  std::vector<int> map;    // boundary position -> position in the parent's front
};

}  // namespace

std::string build_nd_plan(const int nd[3], const std::vector<SubDesc> &subs, const std::vector<IfaceDesc> &ifcs,
                          const std::vector<int> &patches, int n_patch, int panel, NdPlan &plan) {
  if (panel < 1 || panel > kMfPanelMax)
    return "the interface panel must hold 1 to " + std::to_string(kMfPanelMax) + " blocks";
  plan.panel = panel;
  plan = NdPlan();
  plan.n_unknowns = 2 * n_patch;
  if (n_patch == 0) return "";
  // patch -> interface
  std::vector<int> if_of(n_patch, -1);
  for (size_t t = 0; t < ifcs.size(); ++t)
    for (int k = 0; k < ifcs[t].na * ifcs[t].nb; ++k) if_of[ifcs[t].p0 + k] = (int)t;
  auto coord = [&](int l, int d) {
    return d == 0 ? l % nd[0] : (d == 1 ? (l / nd[0]) % nd[1] : l / (nd[0] * nd[1]));
  };
  auto inside = [&](int l, const int lo[3], const int hi[3]) {
    for (int d = 0; d < 3; ++d) {
      const int c = coord(l, d);
      if (c < lo[d] || c >= hi[d]) return false;
    }
    return true;
  };
  auto sid = [&](int x, int y, int z) { return x + nd[0] * (y + nd[1] * z); };

  std::vector<TmpNode> tn;
  std::vector<int> node_of_patch(n_patch, -1);
  // recursive dissection; returns the node id (preorder) or -1 for a single subdomain
  std::function<int(const int *, const int *, const std::vector<int> &, int)> rec =
      [&](const int *lo, const int *hi, const std::vector<int> &pfront, int parent) -> int {
    int ext[3];
    long long cnt = 1;
    for (int d = 0; d < 3; ++d) {
      ext[d] = hi[d] - lo[d];
      cnt *= ext[d];
    }
    if (cnt <= 1) return -1;
    // the cut plane with the fewest separator patches (ties: the longer
    // extent, then the lower axis), through the middle of the box
    int best_a = -1, best_m = 0;
    long long best_cnt = -1;
    for (int a = 0; a < 3; ++a) {
      if (ext[a] < 2) continue;
      const int m = lo[a] + ext[a] / 2;
      long long c = 0;
      int s[3];
      for (s[2] = lo[2]; s[2] < hi[2]; ++s[2])
        for (s[1] = lo[1]; s[1] < hi[1]; ++s[1])
          for (s[0] = lo[0]; s[0] < hi[0]; ++s[0]) {
            if (s[a] != m - 1) continue;
            const int t = subs[sid(s[0], s[1], s[2])].face_if[2 * a + 1];
            c += ifcs[t].na * ifcs[t].nb;
          }
      if (best_cnt < 0 || c < best_cnt || (c == best_cnt && ext[a] > ext[best_a])) {
        best_cnt = c;
        best_a = a;
        best_m = m;
      }
    }
    const int id = (int)tn.size();
    tn.emplace_back();
    {
      TmpNode &N = tn[id];
      for (int d = 0; d < 3; ++d) {
        N.lo[d] = lo[d];
        N.hi[d] = hi[d];
      }
      N.parent = parent;
      int s[3];
      const int a = best_a;
      for (s[2] = lo[2]; s[2] < hi[2]; ++s[2])
        for (s[1] = lo[1]; s[1] < hi[1]; ++s[1])
          for (s[0] = lo[0]; s[0] < hi[0]; ++s[0]) {
            if (s[a] != best_m - 1) continue;
            const IfaceDesc &I = ifcs[subs[sid(s[0], s[1], s[2])].face_if[2 * a + 1]];
            for (int k = 0; k < I.na * I.nb; ++k) {
              const int p = I.p0 + k;
              node_of_patch[p] = id;
              N.front.push_back(2 * p);
              N.front.push_back(2 * p + 1);
            }
          }
      N.s = (int)N.front.size();
      N.sp = (N.s + kNB - 1) / kNB * kNB;
      N.front.resize(N.sp, -1);
      // boundary: the unknowns of the parent's front whose interface has one
      // side inside this box, in the parent's order
      for (size_t q = 0; q < pfront.size(); ++q) {
        const int u = pfront[q];
        if (u < 0) continue;
        const IfaceDesc &I = ifcs[if_of[u >> 1]];
        if (inside(I.lo_sub, lo, hi) != inside(I.hi_sub, lo, hi)) {
          N.front.push_back(u);
          N.map.push_back((int)q);
        }
      }
    }
    const std::vector<int> myfront = tn[id].front;  // recursion may reallocate tn
    int h1[3] = {hi[0], hi[1], hi[2]}, l2[3] = {lo[0], lo[1], lo[2]};
    h1[best_a] = best_m;
    l2[best_a] = best_m;
    const int c0 = rec(lo, h1, myfront, id);
    const int c1 = rec(l2, hi, myfront, id);
    TmpNode &N = tn[id];
    N.child[0] = c0;
    N.child[1] = c1;
    int h = 0;
    for (int c : {c0, c1})
      if (c >= 0) h = std::max(h, tn[c].height);
    N.height = h + 1;
    return id;
  };
  const int root_lo[3] = {0, 0, 0};
  const int root_hi[3] = {nd[0], nd[1], nd[2]};
  rec(root_lo, root_hi, std::vector<int>(), -1);
  for (int p = 0; p < n_patch; ++p)
    if (node_of_patch[p] < 0) return "nested dissection left patch " + std::to_string(p) + " without a separator";

  // elimination order: postorder (children first)
  const int nn = (int)tn.size();
  std::vector<int> post(nn, -1), order;
  order.reserve(nn);
  std::function<void(int)> visit = [&](int v) {
    for (int c : tn[v].child)
      if (c >= 0) visit(c);
    post[v] = (int)order.size();
    order.push_back(v);
  };
  visit(0);
  plan.nodes.resize(nn);
  int64_t off = 0, ioff = 0, zoff = 0, poff = 0;
  for (int k = 0; k < nn; ++k) {
    const TmpNode &T = tn[order[k]];
    MfNode &M = plan.nodes[k];
    M.f = (int)T.front.size();
    M.sp = T.sp;
    M.s = T.s;
    M.r = M.f - M.sp;
    M.off = off;
    M.inv_off = ioff;
    M.z_off = zoff;
    M.part_off = poff;
    M.idx_off = (int)plan.idx.size();
    M.map_off = (int)plan.map.size();
    M.child0 = T.child[0] >= 0 ? post[T.child[0]] : -1;
    M.child1 = T.child[1] >= 0 ? post[T.child[1]] : -1;
    plan.idx.insert(plan.idx.end(), T.front.begin(), T.front.end());
    plan.map.insert(plan.map.end(), T.map.begin(), T.map.end());
    off += (int64_t)M.f * M.f;
    ioff += (int64_t)(M.sp / kNB) * (kNB * kNB + kNB);
    zoff += M.f;
    poff += (int64_t)((M.r + kMfBwdRows - 1) / kMfBwdRows) * M.sp;
    plan.max_f = std::max(plan.max_f, M.f);
    for (int k2 = 0; k2 < M.s; ++k2) {
      const double t = M.f - 1 - k2;
      plan.flops += t * t;
    }
  }
  plan.front_doubles = off;
  plan.inv_doubles = ioff;
  plan.z_doubles = zoff;
  plan.part_doubles = poff;
  if (plan.idx.size() > (size_t)INT32_MAX || plan.map.size() > (size_t)INT32_MAX)
    return "nested-dissection index lists exceed 2^31 entries";

  // levels by height, bottom-up
  int H = 0;
  for (const TmpNode &T : tn) H = std::max(H, T.height);
  plan.level_off.assign(H + 1, 0);
  std::vector<std::vector<int>> lv(H);
  for (int k = 0; k < nn; ++k) lv[tn[order[k]].height - 1].push_back(k);
  plan.level_fmax.assign(H, 0);
  plan.level_rmax.assign(H, 0);
  plan.level_child_rmax.assign(H, 0);
  plan.level_lds.assign(H, 0);
  plan.level_spmax.assign(H, 0);
  for (int h = 0; h < H; ++h) {
    plan.level_off[h] = (int)plan.level_nodes.size();
    for (int k : lv[h]) {
      plan.level_nodes.push_back(k);
      const MfNode &M = plan.nodes[k];
      plan.level_fmax[h] = std::max(plan.level_fmax[h], M.f);
      plan.level_rmax[h] = std::max(plan.level_rmax[h], M.r);
      plan.level_lds[h] = std::max(plan.level_lds[h], M.f + M.sp);
      plan.level_spmax[h] = std::max(plan.level_spmax[h], M.sp);
      for (int c : {M.child0, M.child1})
        if (c >= 0) plan.level_child_rmax[h] = std::max(plan.level_child_rmax[h], plan.nodes[c].r);
    }
  }
  plan.level_off[H] = (int)plan.level_nodes.size();
  for (int h = 0; h < H; ++h)
    if ((size_t)plan.level_lds[h] * sizeof(double) > kMfSweepLdsMax)
      return "an interface front of " + std::to_string(plan.level_fmax[h]) +
             " unknowns exceeds the sweep kernels' LDS";

  // pieces of the sweeps' boundary products, level by level
  plan.level_fb_off.assign(H + 1, 0);
  plan.level_bb_off.assign(H + 1, 0);
  for (int h = 0; h < H; ++h) {
    plan.level_fb_off[h] = (int)plan.fwd_bnd.size();
    plan.level_bb_off[h] = (int)plan.bwd_bnd.size();
    for (int k : lv[h]) {
      const MfNode &M = plan.nodes[k];
      if (M.r <= 0 || M.sp <= 0) continue;
      for (int c = 0; c < (M.r + kMfFwdRows - 1) / kMfFwdRows; ++c) plan.fwd_bnd.push_back(make_int2(k, c));
      const int nq = ((M.r + kMfBwdRows - 1) / kMfBwdRows) * ((M.sp + kMfBwdCols - 1) / kMfBwdCols);
      for (int q = 0; q < nq; ++q) plan.bwd_bnd.push_back(make_int2(k, q));
    }
  }
  plan.level_fb_off[H] = (int)plan.fwd_bnd.size();
  plan.level_bb_off[H] = (int)plan.bwd_bnd.size();

  // factorisation launches, per level, per panel of plan.panel blocks starting
  // at block t0: the LDL^T of block t0 (t0 > 0; block 0 is factored by the
  // level's first launch), then per block t of the panel its step over the
  // row tiles below it, then the trailing update past the panel
  for (int h = 0; h < H; ++h) {
    int tmax = 0;
    for (int k : lv[h]) tmax = std::max(tmax, plan.nodes[k].sp / kNB);
    // one launch over the level's nodes, tiles(node) workgroups each with
    // tile ids id(q); returns the launch, or null when it has no workgroup
    auto push_ids = [&](int kind, int t, auto tiles, auto id) -> MfStepLaunch * {
      MfStepLaunch L;
      L.level = h;
      L.kind = kind;
      L.t = t;
      L.blk_off = (int64_t)plan.step_blocks.size();
      for (int k : lv[h]) {
        const int n = tiles(plan.nodes[k]);
        for (int q = 0; q < n; ++q) plan.step_blocks.push_back(make_int2(k, id(q)));
      }
      L.n_blocks = (int)(plan.step_blocks.size() - L.blk_off);
      if (L.n_blocks == 0) return nullptr;
      plan.steps.push_back(L);
      return &plan.steps.back();
    };
    auto push = [&](int kind, int t, auto tiles) { return push_ids(kind, t, tiles, [](int q) { return q; }); };
    const int P = plan.panel;
    for (int t0 = 0; t0 < tmax; t0 += P) {
      if (t0 > 0) push(kMfDiag, t0, [&](const MfNode &M) { return M.sp / kNB > t0 ? 1 : 0; });
      for (int t = t0; t < t0 + P; ++t)
        push(kMfPanelStep, t, [&](const MfNode &M) {
          if (M.sp / kNB <= t) return 0;
          const int nr = M.f - kNB * (t + 1);
          return nr > 0 ? (nr + 63) / 64 : 0;
        });
      // the group of panels g .. t0 whose trailing update is deferred
      const int g = t0 - ((t0 / P) % kMfDefer) * P;
      const int nb = t0 + P - g;
      const bool last = (t0 / P) % kMfDefer == kMfDefer - 1 || t0 + P >= tmax;
      if (!last) {
        // the next panel's columns, for the nodes whose separator goes on past
        // this panel: tile column 0, whose tile (ti, 0) has the id
        // ti (ti + 1) / 2 in the triangular numbering of the trailing tiles
        MfStepLaunch *L = push_ids(
            kMfTrailing, g,
            [&](const MfNode &M) {
              if (M.sp / kNB <= t0 + P) return 0;
              const int nr = M.f - kNB * (t0 + P);
              return nr > 0 ? (nr + 63) / 64 : 0;
            },
            [](int ti) { return ti * (ti + 1) / 2; });
        if (L) {
          L->nb = nb;
          L->jend = t0 + 2 * P;
        }
      } else {
        MfStepLaunch *L = push(kMfTrailing, g, [&](const MfNode &M) {
          if (M.sp / kNB <= g) return 0;
          const int nr = M.f - kNB * std::min(g + nb, M.sp / kNB);
          const int tt = nr > 0 ? (nr + 63) / 64 : 0;
          return tt * (tt + 1) / 2;
        });
        if (L) L->nb = nb;
      }
    }
  }

  // scatter map of the assembled entries, pair by pair within each subdomain
  std::vector<int> own_pos(n_patch, -1);  // position of 2p in its own node's front
  for (int k = 0; k < nn; ++k) {
    const MfNode &M = plan.nodes[k];
    for (int q = 0; q < M.s; q += 2) own_pos[plan.idx[M.idx_off + q] >> 1] = q;
  }
  std::vector<int> node_post(n_patch);
  for (int p = 0; p < n_patch; ++p) node_post[p] = post[node_of_patch[p]];
  // per node: its boundary unknowns sorted, for the position lookups
  std::vector<std::vector<std::pair<int, int>>> bsorted(nn);
  auto pos_in = [&](int k, int u) -> int {
    auto &v = bsorted[k];
    if (v.empty() && plan.nodes[k].r > 0) {
      const MfNode &M = plan.nodes[k];
      for (int q = M.sp; q < M.f; ++q) v.emplace_back(plan.idx[M.idx_off + q], q);
      std::sort(v.begin(), v.end());
    }
    auto it = std::lower_bound(v.begin(), v.end(), std::make_pair(u, -1));
    return (it != v.end() && it->first == u) ? it->second : -1;
  };
  plan.sub_pair_off.resize(subs.size() + 1);
  int64_t npairs = 0;
  for (size_t l = 0; l < subs.size(); ++l) {
    plan.sub_pair_off[l] = npairs;
    npairs += (int64_t)subs[l].npatch * subs[l].npatch;
  }
  plan.sub_pair_off[subs.size()] = npairs;
  plan.pair_off.assign(npairs, -1);
  plan.pair_ld.assign(npairs, 0);
  for (size_t l = 0; l < subs.size(); ++l) {
    const SubDesc &S = subs[l];
    const int n = S.npatch;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const int a = patches[S.patch_off + i], b = patches[S.patch_off + j];
        const int X = std::min(node_post[a], node_post[b]);
        const int ra = node_post[a] == X ? own_pos[a] : pos_in(X, 2 * a);
        const int cb = node_post[b] == X ? own_pos[b] : pos_in(X, 2 * b);
        if (ra < 0 || cb < 0) return "nested-dissection front is missing a coupled unknown";
        if (ra < cb) continue;  // above the diagonal: the pair (b, a) carries it
        const MfNode &M = plan.nodes[X];
        const int64_t e = plan.sub_pair_off[l] + (int64_t)i * n + j;
        plan.pair_off[e] = M.off + (int64_t)cb * M.f + ra;
        plan.pair_ld[e] = M.f;
      }
  }
  return "";
}

}  // namespace mrcm
