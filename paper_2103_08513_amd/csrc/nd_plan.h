// Nested-dissection plan of the interface system for its multifrontal LDL^T
// (host side).  The patch graph -- patches adjacent when one subdomain holds
// both -- inherits the tensor structure of the partition, so the dissection
// is geometric: a box of subdomains is cut by a plane of interfaces into two
// halves, recursively, and each plane's patches form one separator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "internal.h"

namespace mrcm {

// Device view of one tree node (one separator and its frontal matrix).
struct MfNode {
  int64_t off;      // offset (doubles) of the f x f column-major front
  int64_t inv_off;  // offset (doubles) of the per-16-block L11^{-1}, 1/D (272 each)
  int64_t z_off;    // offset (doubles) of the node's f-entry vector of the sweeps
  int64_t part_off; // offset (doubles) of the backward sweep's partial boundary sums
                    // [ceil(r / kMfBwdRows)][sp]
  int32_t f;        // front size: sp + r
  int32_t sp;       // separator unknowns rounded up to 16 (pad rows are identity)
  int32_t s;        // separator unknowns (two per patch: pi^p, pi^u)
  int32_t r;        // boundary unknowns (eliminated by ancestors)
  int32_t idx_off;  // offset of idx[f]: front position -> unknown 2*patch + {0,1}, -1 for pad
  int32_t map_off;  // offset of map[r]: boundary position -> position in the parent's front
  int32_t child0, child1;  // child nodes or -1
};

// The factorisation proceeds per level in panels of `panel` 16-column blocks
// (1 .. kMfPanelMax; a panel of one block is the plain right-looking step).
// One launch of it: the nodes of one level that have the block or panel
// concerned, one workgroup per (node, tile) entry of the table.
constexpr int kMfPanelMax = 4;
enum MfLaunchKind {
  kMfPanelStep = 0,  // block t: W of every row below it, the update of the panel's later columns
  kMfTrailing = 1,   // the panel starting at block t: rank-(16 panel) update of the trailing tiles
  kMfDiag = 2,       // LDL^T of the diagonal block t (the first block of a panel)
};
// The trailing update of a panel is deferred over kMfDefer panels: after
// each panel but the group's last, a narrow launch brings the next panel's
// columns (one tile column, up to the separator's end) up to date with the
// group's panels so far; after the group's last panel one launch applies
// all of them to the tiles past it, which are read and written once per
// group rather than once per panel.  Each entry of the trailing matrix sees
// the same updates in the same order as with no deferral.
constexpr int kMfDefer = 4;
struct MfStepLaunch {
  int level;
  int kind;          // MfLaunchKind
  int t;             // block index within each node's separator
  int64_t blk_off;   // offset of this launch's (node, tile) table
  int n_blocks;      // workgroups
  int nb = 0;        // kMfTrailing: blocks t .. t + nb - 1 applied
  int jend = 0;      // kMfTrailing: columns limited to blocks below jend (0: none)
};

// The sweeps' boundary products W_b^T and W_b, (f - sp) x sp per node, run
// beside the sequential triangular part over many workgroups: forward in
// chunks of kMfFwdRows boundary rows, backward in pieces of kMfBwdCols
// separator columns by kMfBwdRows boundary rows whose partial sums the
// triangular part adds in a fixed order.
constexpr int kMfFwdRows = 64;
constexpr int kMfBwdRows = 512;
constexpr int kMfBwdCols = 256;

struct NdPlan {
  int n_unknowns = 0;                 // 2 * patches
  int panel = kMfPanelMax;            // 16-column blocks per panel of the factorisation
  std::vector<MfNode> nodes;          // in elimination order (children first)
  std::vector<int> idx, map;          // concatenated per node
  std::vector<int> level_off;         // nodes of level h: [level_off[h], level_off[h+1]) (levels bottom-up)
  std::vector<int> level_nodes;       // node ids sorted by level
  std::vector<int> level_fmax;        // largest f per level
  std::vector<int> level_rmax;        // largest r per level
  std::vector<int> level_child_rmax;  // largest r of the children of the level's nodes
  std::vector<MfStepLaunch> steps;    // factorisation launches in order
  std::vector<int2> step_blocks;      // (node, tile) per workgroup of each step launch
  // original entries: per subdomain patch pair (a at row, b at column) in the
  // subdomain's local patch order, the front offset of the (P_a, P_b) entry
  // and the front's leading dimension; off = -1 when the pair lies above the
  // diagonal (its transpose carries it)
  std::vector<int64_t> pair_off;      // [sum_l npatch_l^2]
  std::vector<int> pair_ld;
  std::vector<int64_t> sub_pair_off;  // per subdomain: offset of its pairs
  std::vector<int> level_lds;         // largest (f + sp) per level: the sweeps' LDS doubles
  std::vector<int> level_spmax;       // largest sp per level
  std::vector<int2> fwd_bnd, bwd_bnd; // (node, piece) of the sweeps' boundary launches, level by level
  std::vector<int> level_fb_off, level_bb_off;  // [H + 1] offsets into fwd_bnd, bwd_bnd
  int64_t part_doubles = 0;
  int64_t front_doubles = 0, inv_doubles = 0, z_doubles = 0;
  double flops = 0.0;                 // sum over nodes of the partial LDL^T flops
  int max_f = 0;
};

// Device copies of a plan's arrays.
struct MfDevPlan {
  MfNode *nodes = nullptr;
  int n_nodes = 0;
  int *idx = nullptr, *map = nullptr, *level_nodes = nullptr;
  int2 *step_blocks = nullptr;
  int2 *fwd_bnd = nullptr, *bwd_bnd = nullptr;
  int64_t *pair_off = nullptr, *sub_pair_off = nullptr;
  int *pair_ld = nullptr;
  int4 *pinfo = nullptr;  // per patch: interface, local index on its lower and upper side
  int64_t front_doubles = 0;
};

// Largest (f + sp) * 8 bytes of LDS the sweep kernels may take.
constexpr size_t kMfSweepLdsMax = 150 * 1024;

// Builds the plan for the subdomain grid nd[3] with the given subdomain and
// interface descriptors and concatenated patch lists.  Returns an empty
// string on success, else a message.
std::string build_nd_plan(const int nd[3], const std::vector<SubDesc> &subs, const std::vector<IfaceDesc> &ifcs,
                          const std::vector<int> &patches, int n_patch, int panel, NdPlan &plan);

// Launchers (mf_kernels.hip).  Vectors in the interleaved unknown order
// (2p: pi^p of patch p, 2p+1: pi^u), unflipped.
//  assemble: zero the fronts, scatter the assembled entries, identity pads.
//  factor:   extend-add, first blocks and panel steps, level by level.
//  solve:    x = M^{-1} diag(s) rhs by the forward and backward sweeps.
//  residual: r = b - A x (x null: r = b), and b itself when b is non-null.
// Allows the sweep kernels their shared memory (once, before any solve).
hipError_t mf_init_kernels();
hipError_t launch_mf_assemble(const Geom &g, int n_sub, const int *patches, const double *F, const double *Fb,
                              const double *SAb, const MfDevPlan &dp, double *fronts, hipStream_t s);
hipError_t launch_mf_factor(const NdPlan &plan, const MfDevPlan &dp, double *fronts, double *inv, DevStatus *st,
                            hipStream_t s);
hipError_t launch_mf_solve(const NdPlan &plan, const MfDevPlan &dp, const double *fronts, const double *inv,
                           double *zbuf, double *pbuf, const double *rhs, double *x, hipStream_t s);
hipError_t launch_mf_residual(const Geom &g, const int *patches, const double *F, const double *Fb,
                              const double *SAb, const int4 *pinfo, int nv, const double *x, double *r, double *b,
                              hipStream_t s);
hipError_t launch_mf_dense(const Geom &g, const int *patches, const double *F, const double *Fb, const double *SAb,
                           const int4 *pinfo, int nv, double *A, double *b, hipStream_t s);
hipError_t launch_mf_deinterleave(const double *x, int nv, double *X, hipStream_t s);

}  // namespace mrcm
