// Host-side checks of the C ABI library under AddressSanitizer and
// UndefinedBehaviorSanitizer, on the CPU: the descriptor, validation and
// nested-dissection plan logic of capi.cpp and nd_plan.cpp over many
// configurations, the argument checks of the public entry points, and the
// autotuner cache's reader.  Nothing here touches a GPU: the geometry and
// the plan are host code, every public call made fails its validation before
// any HIP work, and the cache lookup is a hit.  Built by
// tests/test_host_sanitizers.py, which includes capi.cpp in this translation
// unit to reach its internal functions.
#include "../../paper_2103_08513_amd/csrc/capi.cpp"

#include <cstdlib>
#include <set>

namespace {

int g_fails = 0;
#define CHECK(c)                                                               \
  do {                                                                         \
    if (!(c)) {                                                                \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);     \
      ++g_fails;                                                               \
    }                                                                          \
  } while (0)

const double kFake[1] = {1.0};  // non-null field pointers, never dereferenced

struct Config {
  int n[3];
  int nd[3];
  int us[3][2];
  int walls[6];
  long long pin;
  bool explicit_split;
};

// interfaces in the ABI's order: x-normal, y-normal, z-normal, each
// lexicographic in the lower subdomain id
int n_interfaces(const int nd[3]) {
  return (nd[0] - 1) * nd[1] * nd[2] + nd[0] * (nd[1] - 1) * nd[2] + nd[0] * nd[1] * (nd[2] - 1);
}

void check_geometry_and_plan(const Config &c, int precision) {
  mrcm_problem pb{};
  pb.nx = c.n[0];
  pb.ny = c.n[1];
  pb.nz = c.n[2];
  pb.hx = 20.0;
  pb.hy = 10.0;
  pb.hz = 2.0;
  pb.kx = pb.ky = pb.kz = pb.q = kFake;
  for (int f = 0; f < 6; ++f) pb.wall_type[f] = c.walls[f];
  pb.pin_cell = c.pin;
  std::vector<int32_t> cuts[3];
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i <= c.nd[d]; ++i) cuts[d].push_back((int32_t)((int64_t)i * c.n[d] / c.nd[d]));
  mrcm_partition part{};
  part.ndx = c.nd[0];
  part.ndy = c.nd[1];
  part.ndz = c.nd[2];
  part.cut_x = cuts[0].data();
  part.cut_y = cuts[1].data();
  part.cut_z = cuts[2].data();
  mrcm_iface_space ifs{};
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < 2; ++t) ifs.uniform_split[d][t] = c.us[d][t];
  std::vector<int32_t> split;
  if (c.explicit_split) {
    const int ni = n_interfaces(c.nd);
    for (int i = 0; i < ni; ++i) {
      split.push_back(1 + i % 3);
      split.push_back(1 + (i / 3) % 2);
    }
    ifs.split = split.data();
  }
  mrcm_options opt{};
  opt.alpha = 1.0;
  opt.precision = precision;
  HostGeom G;
  const mrcm_status st = build_host_geom(&pb, &part, &ifs, &opt, G);
  CHECK(st == MRCM_OK);
  if (st != MRCM_OK) {
    std::fprintf(stderr, "  %s\n", mrcm_last_error());
    return;
  }
  const int64_t N = (int64_t)c.n[0] * c.n[1] * c.n[2];
  int64_t cells = 0;
  std::vector<int> sides(G.n_patch, 0);
  for (const SubDesc &S : G.subs) {
    cells += S.N;
    CHECK(S.m == 2 * S.npatch + 1);
    for (int j = 0; j < S.npatch; ++j) {
      const int p = G.patches[S.patch_off + j];
      CHECK(p >= 0 && p < G.n_patch);
      if (p >= 0 && p < G.n_patch) ++sides[p];
    }
  }
  CHECK(cells == N && G.totCells == N);
  for (int p = 0; p < G.n_patch; ++p) CHECK(sides[p] == 2);  // every patch lies between two subdomains
  const int nd[3] = {c.nd[0], c.nd[1], c.nd[2]};
  for (int panel = 1; panel <= kMfPanelMax; ++panel) {
    NdPlan plan;
    const std::string err = build_nd_plan(nd, G.subs, G.ifcs, G.patches, G.n_patch, panel, plan);
    CHECK(err.empty());
    if (!err.empty()) {
      std::fprintf(stderr, "  %s\n", err.c_str());
      return;
    }
    std::vector<int> seen(2 * (size_t)G.n_patch, 0);
    int64_t fronts = 0;
    const int nn = (int)plan.nodes.size();
    for (int k = 0; k < nn; ++k) {
      const MfNode &M = plan.nodes[k];
      CHECK(M.f == M.sp + M.r && M.sp % kNB == 0 && M.s <= M.sp && M.s % 2 == 0);
      CHECK(M.off == fronts);
      fronts += (int64_t)M.f * M.f;
      for (int q = 0; q < M.f; ++q) {
        const int u = plan.idx[M.idx_off + q];
        if (q < M.s) {
          CHECK(u >= 0 && u < 2 * G.n_patch);
          if (u >= 0 && u < 2 * G.n_patch) ++seen[u];
        } else if (q < M.sp) {
          CHECK(u == -1);  // identity pad rows
        } else {
          CHECK(u >= 0 && u < 2 * G.n_patch);
        }
      }
      for (int c2 : {M.child0, M.child1}) {
        if (c2 < 0) continue;
        CHECK(c2 < k);  // children come first
        const MfNode &C = plan.nodes[c2];
        for (int q = 0; q < C.r; ++q) {
          const int pos = plan.map[C.map_off + q];
          CHECK(pos >= 0 && pos < M.f);
          if (pos >= 0 && pos < M.f) CHECK(plan.idx[M.idx_off + pos] == plan.idx[C.idx_off + C.sp + q]);
        }
      }
    }
    CHECK(fronts == plan.front_doubles);
    for (int u = 0; u < 2 * G.n_patch; ++u) CHECK(seen[u] == 1);  // one separator per unknown
    for (size_t e = 0; e < plan.pair_off.size(); ++e) {
      const int64_t o = plan.pair_off[e];
      CHECK(o == -1 || (o >= 0 && o < plan.front_doubles));
    }
    for (const int2 &b : plan.step_blocks) CHECK(b.x >= 0 && b.x < nn && b.y >= 0);
    for (const int2 &b : plan.fwd_bnd) CHECK(b.x >= 0 && b.x < nn && plan.nodes[b.x].r > kMfFwdRows * b.y);
    for (const int2 &b : plan.bwd_bnd) CHECK(b.x >= 0 && b.x < nn && b.y >= 0);
  }
}

void check_validation() {
  mrcm_problem pb{};
  pb.nx = pb.ny = pb.nz = 8;
  pb.hx = pb.hy = pb.hz = 1.0;
  pb.kx = pb.ky = pb.kz = pb.q = kFake;
  pb.pin_cell = 0;
  int32_t cut[3] = {0, 4, 8};
  mrcm_partition part{};
  part.ndx = part.ndy = part.ndz = 2;
  part.cut_x = part.cut_y = part.cut_z = cut;
  mrcm_iface_space ifs{};
  for (int d = 0; d < 3; ++d) ifs.uniform_split[d][0] = ifs.uniform_split[d][1] = 1;
  mrcm_options opt{};
  opt.alpha = 1.0;
  mrcm_mbfs *h = nullptr;
  auto expect = [&](const char *what) {
    h = nullptr;
    const mrcm_status st = mrcm_build_mbfs(&pb, &part, &ifs, &opt, nullptr, &h);
    CHECK(st == MRCM_EINVAL || st == MRCM_EUNSUPPORTED);
    CHECK(h == nullptr);
    CHECK(std::strstr(mrcm_last_error(), what) != nullptr);
  };
  opt.alpha = -1.0;
  expect("alpha");
  opt.alpha = 1.0;
  pb.nx = 0;
  expect("grid dimensions");
  pb.nx = 8;
  int32_t bad_cut[3] = {0, 9, 8};
  part.cut_x = bad_cut;
  expect("cut");
  part.cut_x = cut;
  pb.pin_cell = 512;
  expect("pin_cell");
  pb.pin_cell = 0;
  pb.wall_type[2] = 7;
  expect("wall type");
  pb.wall_type[2] = 0;
  opt.solve_tiles = 9;
  expect("solve_tiles");
  opt.solve_tiles = 0;
  opt.iface_panel = 6;
  expect("iface_panel");
  opt.iface_panel = 0;
  opt.launch_mode = 3;
  expect("launch_mode");
  opt.launch_mode = 0;
  opt.beta_mode = 5;
  expect("beta_mode");
  opt.beta_mode = 0;
  pb.q = nullptr;
  expect("required");
  pb.q = kFake;
  CHECK(mrcm_build_mbfs(&pb, &part, &ifs, &opt, nullptr, nullptr) == MRCM_EINVAL);
  for (int code = -8; code <= 0; ++code) CHECK(mrcm_status_string((mrcm_status)code) != nullptr);
}

// The two-phase calls' and the IMPES loop's argument checks, every one of
// which returns before anything reaches the device.
void check_twophase_validation() {
  double *d = const_cast<double *>(kFake), *d2 = d + 1;
  const mrcm_twophase good{4, 3, 2, 1.0, 1.0, 1.0, 1.0, 2.0};
  auto expect = [&](mrcm_status st, const char *what) {
    CHECK(st == MRCM_EINVAL);
    CHECK(std::strstr(mrcm_last_error(), what) != nullptr);
  };
  const mrcm_twophase bad[] = {{0, 3, 2, 1.0, 1.0, 1.0, 1.0, 2.0},
                               {4, 3, 2, -1.0, 1.0, 1.0, 1.0, 2.0},
                               {4, 3, 2, 1.0, 1.0, 1.0, 0.0, 2.0},
                               {4, 3, 2, 1.0, 1.0, 1.0, 1.0, std::numeric_limits<double>::infinity()},
                               {4, 3, 2, 1.0, std::numeric_limits<double>::quiet_NaN(), 1.0, 1.0, 2.0}};
  for (const mrcm_twophase &b : bad) {
    CHECK(mrcm_transport_step(&b, d, nullptr, d, d, nullptr, d2) == MRCM_EINVAL);
    CHECK(mrcm_transport_dt(&b, d, d, 1.0, 1.0, nullptr, d) == MRCM_EINVAL);
    CHECK(mrcm_transport_advance(&b, d, nullptr, nullptr, d, d, 1.0, 1.0, nullptr, d2, d2) == MRCM_EINVAL);
    CHECK(mrcm_transport_marks_bytes(&b) == 0);
    CHECK(mrcm_transport_mark_sources(&b, d, nullptr, d2) == MRCM_EINVAL);
    CHECK(mrcm_mobility_scale(&b, d, d, d, d, nullptr, d, d, d) == MRCM_EINVAL);
  }
  expect(mrcm_transport_step(nullptr, d, nullptr, d, d, nullptr, d2), "descriptor");
  expect(mrcm_transport_step(&good, d, nullptr, d, d, nullptr, d), "overlap");
  expect(mrcm_transport_step(&good, nullptr, nullptr, d, d, nullptr, d2), "null");
  expect(mrcm_transport_dt(&good, d, d, 0.0, 1.0, nullptr, d), "cfl");
  expect(mrcm_transport_dt(&good, d, d, 1.0, -1.0, nullptr, d), "dt_max");
  expect(mrcm_transport_advance(&good, d, nullptr, nullptr, d, d, 1.0, 1.0, nullptr, d2, d), "dt_next");
  expect(mrcm_transport_advance(&good, d, nullptr, nullptr, d, d, 1.0, 1.0, nullptr, d, d2), "overlap");
  expect(mrcm_transport_mark_sources(&good, nullptr, nullptr, d2), "null");
  CHECK(mrcm_transport_marks_bytes(&good) == 1);
  expect(mrcm_mobility_scale(&good, d, nullptr, d, d, nullptr, d, d, d), "null");
  // the loop: a problem of the same grid
  mrcm_problem pb{};
  pb.nx = 4;
  pb.ny = 3;
  pb.nz = 2;
  pb.hx = pb.hy = pb.hz = 1.0;
  pb.kx = pb.ky = pb.kz = pb.q = kFake;
  pb.pin_cell = 0;
  int32_t cx[2] = {0, 4}, cy[2] = {0, 3}, cz[2] = {0, 2};
  mrcm_partition part{};
  part.ndx = part.ndy = part.ndz = 1;
  part.cut_x = cx;
  part.cut_y = cy;
  part.cut_z = cz;
  mrcm_iface_space ifs{};
  mrcm_options opt{};
  opt.alpha = 1.0;
  const mrcm_impes_options io{3, 6, 1.0, 0.5, 1.0, 1};
  mrcm_impes_stats stats{};
  auto run = [&](const mrcm_twophase *tp, mrcm_impes_options o) {
    return mrcm_impes_run(&pb, &part, &ifs, &opt, tp, &o, nullptr, d, &stats);
  };
  expect(mrcm_impes_run(&pb, &part, &ifs, &opt, &good, &io, nullptr, nullptr, &stats), "null");
  const mrcm_twophase other{4, 3, 3, 1.0, 1.0, 1.0, 1.0, 2.0};
  expect(run(&other, io), "differs");
  mrcm_impes_options o = io;
  o.skip = 0;
  expect(run(&good, o), "skip");
  o = io;
  o.max_steps = -1;
  expect(run(&good, o), "max_steps");
  o = io;
  o.max_steps = 0;
  o.t_end = std::numeric_limits<double>::infinity();
  expect(run(&good, o), "t_end");
  o = io;
  o.t_end = std::numeric_limits<double>::quiet_NaN();
  expect(run(&good, o), "t_end");
  o = io;
  o.cfl = 0.0;
  expect(run(&good, o), "cfl");
  o = io;
  o.dt_max = 0.0;
  expect(run(&good, o), "dt_max");
  o = io;
  o.refine = 21;
  expect(run(&good, o), "refine");
  pb.q = nullptr;
  expect(run(&good, io), "sources");
}

// The cache reader: malformed lines are skipped, the entry for the shapes'
// key is a hit, and its values come back.
void check_tune_cache(const char *path) {
  mrcm_problem pb{};
  pb.nx = 40;
  pb.ny = 40;
  pb.nz = 20;
  pb.hx = pb.hy = pb.hz = 1.0;
  pb.kx = pb.ky = pb.kz = pb.q = kFake;
  pb.pin_cell = 0;
  int32_t cx[5] = {0, 10, 20, 30, 40}, cz[5] = {0, 5, 10, 15, 20};
  mrcm_partition part{};
  part.ndx = part.ndy = part.ndz = 4;
  part.cut_x = part.cut_y = cx;
  part.cut_z = cz;
  mrcm_iface_space ifs{};
  for (int d = 0; d < 3; ++d) ifs.uniform_split[d][0] = ifs.uniform_split[d][1] = 1;
  mrcm_options opt{};
  opt.alpha = 1.0;
  ConfigKey k;
  CHECK(make_key(&pb, &part, &ifs, &opt, k));
  char key[32];
  std::snprintf(key, sizeof key, "%016llx", (unsigned long long)fnv1a64(tune_signature(&pb, &part, &ifs, &opt, k)));
  FILE *f = std::fopen(path, "w");
  CHECK(f != nullptr);
  if (!f) return;
  std::fprintf(f, "garbage\nmrcm-tune-2 %s 1 2\nmrcm-tune-2 %s 9 0 4 0 1.0 1.0\n", key, key);
  std::fprintf(f, "mrcm-tune-2 %s 2 -1 2 1 3.5 4.5\n", key);
  std::fclose(f);
  mrcm_options best{};
  double bm = 0.0, rm = 0.0;
  int32_t hit = 0;
  CHECK(mrcm_autotune_cached(&pb, &part, &ifs, &opt, nullptr, path, &best, &bm, &rm, &hit) == MRCM_OK);
  CHECK(hit == 1 && best.solve_tiles == 2 && best.solve_group == -1 && best.iface_panel == 2 &&
        best.launch_mode == 1 && bm == 3.5 && rm == 4.5);
  CHECK(mrcm_autotune_cached(&pb, &part, &ifs, &opt, nullptr, nullptr, &best, &bm, &rm, &hit) == MRCM_EINVAL);
}

}  // namespace

int main(int argc, char **argv) {
  const Config configs[] = {
      // the 40x40x20 and 60x220x85 workloads' partitions and patches
      {{40, 40, 20}, {4, 4, 4}, {{1, 1}, {1, 1}, {1, 1}}, {0, 0, 0, 0, 0, 0}, 31999, false},
      {{60, 220, 85}, {3, 11, 17}, {{2, 1}, {2, 1}, {2, 2}}, {0, 0, 0, 0, 0, 0}, 1121999, false},
      // ragged cuts with per-interface splits, walls, the fine trace
      {{37, 23, 11}, {3, 2, 2}, {{1, 1}, {1, 1}, {1, 1}}, {1, 0, 2, 0, 0, 1}, -1, true},
      {{6, 6, 4}, {2, 2, 1}, {{0, 0}, {0, 0}, {0, 0}}, {0, 0, 0, 0, 0, 0}, 0, false},
      {{16, 16, 4}, {4, 1, 1}, {{2, 2}, {1, 1}, {1, 1}}, {0, 0, 0, 0, 0, 0}, 5, false},
      {{8, 8, 8}, {1, 1, 1}, {{1, 1}, {1, 1}, {1, 1}}, {0, 0, 0, 0, 0, 0}, 0, false},
      {{50, 30, 26}, {5, 3, 2}, {{2, 1}, {2, 2}, {4, 2}}, {0, 0, 0, 0, 0, 0}, 17, true},
  };
  for (const Config &c : configs)
    for (int precision : {MRCM_FP64, MRCM_FP32_IR}) check_geometry_and_plan(c, precision);
  check_validation();
  check_twophase_validation();
  check_tune_cache(argc > 1 ? argv[1] : "tune_cache.txt");
  std::printf("host ABI checks: %d failures\n", g_fails);
  return g_fails == 0 ? 0 : 1;
}
