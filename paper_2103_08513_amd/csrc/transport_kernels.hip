// Saturation step of the IMPES two-phase run on gfx950: the upwind finite-
// volume Buckley-Leverett update with the divergence compensation (eqs.
// (transporte_discreto), (flux_disc_up)), the CFL time step (eq. (CFL)) and
// the total mobility that scales each Darcy solve's permeability (Sec. 5).
// All are bound by HBM: the step walks z-marching tiles, the CFL reduction
// and the mobility are plain streams over the cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "launch.h"

namespace mrcm {

namespace {

// phi(S) = M S^2 / (M S^2 + (1 - S)^2), M = mu_o / mu_w
__device__ __forceinline__ double frac_flow(double s, double M) {
  const double a = M * s * s, o = 1.0 - s;
  return a / (a + o * o);
}

__device__ __forceinline__ double frac_flow_deriv(double s, double M) {
  const double o = 1.0 - s, den = M * s * s + o * o;
  return 2.0 * M * s * o / (den * den);
}

}  // namespace

// Workgroups of 256 threads; the grids of the step and of the CFL reduction
// hold as many as are resident at once and stride over the work.
constexpr int kTile = 256;

// Largest speed of a workgroup into the bit pattern of a non-negative double
// (ordered as an unsigned integer): one atomic per workgroup.
__device__ __forceinline__ void block_max_into(double m, unsigned long long *vmax) {
  __shared__ double red[kTile / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(vmax, (unsigned long long)__double_as_longlong(m));
  }
}

// One step: S_c' = S_c - dt sum_f (phi_f - phi(S_c)) U[f][c] / h_d(f), with
// phi_f the upwind value (the cell's own on an outflow face, the neighbour's
// on an inflow face, water across a domain wall), plus dt q (1 - phi(S_c)) / V
// in an injector cell.  U face-major (U[f * N + c]), cells x fastest.  With
// kSpeed, also the largest |phi'(S'_c)| max_f |U[f][c]| of the new state (the
// next step's CFL speed under the same velocity) into vmax.
// Tiles of the step: 64 cells along x (a wavefront) by 4 rows along y (the
// workgroup's four wavefronts) by up to kZLen planes, which each thread walks
// along z, keeping S and phi(S) at z - 1, z and z + 1 in registers: S is read
// from HBM about once and phi evaluated about once per cell for the planes.
// The x-neighbours' phi come from the adjacent lanes (the wavefront's two
// edge lanes load and evaluate theirs), the y-neighbours' from the caches.
// Tiles are numbered x fastest, then y, then the z-chunk, and the resident
// workgroups take them in that order (workgroup w the tiles w, w + grid, ..):
// the whole device streams through one window of the arrays, and the rows
// on either side of a tile, read at about the same time by a workgroup on
// another XCD, come from the memory-side cache that the XCDs share.  (Giving
// each XCD its own contiguous eighth of the tiles, for its L2, measured
// slower: eight separate streams.)  A row's x-segments start on 128-byte lines of its first plane
// (an offset of up to 15 cells), so that a wavefront's loads of each array
// touch four whole lines instead of sharing one at either end with the next
// tile.  Lanes outside the grid skip the tile; the lanes next to them are on
// a wall, which does not use the neighbour's value.
constexpr int kZX = 64, kZY = kTile / 64, kZLen = 32;

struct ZTiles {
  int nxt, nyt, nzt;
};

// a[i]; with a 32-bit index type the byte offset is 32-bit as well, so that
// every array shares one offset register beside its uniform base
template <typename I>
__device__ __forceinline__ double ld(const double *__restrict__ a, I i) {
  if constexpr (sizeof(I) == 4)
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(a) + (uint32_t)(i << 3));
  else
    return a[i];
}

template <typename I>
__device__ __forceinline__ void st(double *__restrict__ a, I i, double v) {
  if constexpr (sizeof(I) == 4)
    *reinterpret_cast<double *>(reinterpret_cast<char *>(a) + (uint32_t)(i << 3)) = v;
  else
    a[i] = v;
}

// I: the cell index type, uint32_t when 8 N < 2^32, else long long.
// src_tiles: NULL, or one byte per tile, nonzero where q has a nonzero entry
// (q is read in those tiles only).
template <bool kSpeed, typename I>
__global__ __launch_bounds__(kTile) void k_transport(TwoPhaseGrid t, ZTiles zt, const double *__restrict__ U,
                                                     const double *__restrict__ q,
                                                     const unsigned char *__restrict__ src_tiles,
                                                     const double *__restrict__ S, const double *__restrict__ dtp,
                                                     double *__restrict__ Sout, unsigned long long *__restrict__ vmax) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const long long ntiles = (long long)zt.nxt * zt.nyt * zt.nzt;
  const double M = t.mu_o / t.mu_w;
  const double dt = *dtp;
  const double rx = 1.0 / t.hx, ry = 1.0 / t.hy, rz = 1.0 / t.hz, rv = rx * ry * rz;
  const I sy = (I)t.nx, sz = (I)t.nx * (I)t.ny;
  const double *Uf[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) Uf[f] = U + f * N;
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  double m = 0.0;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int xt = (int)(tile % zt.nxt);
    const long long r = tile / zt.nxt;
    const int y = (int)(r % zt.nyt) * kZY + row;
    const int z0 = (int)(r / zt.nyt) * kZLen, z1 = min(z0 + kZLen, t.nz);
    const int x = xt * kZX - (int)((sy * (I)y + sz * (I)z0) & 15) + lane;
    if (x < 0 || x >= t.nx || y >= t.ny) continue;
    const bool tq = q != nullptr && (src_tiles == nullptr || src_tiles[tile] != 0);
    I c = (I)x + sy * (I)y + sz * (I)z0;
    // phi below the chunk (unused at z = 0: a wall) and at its first plane
    double pbelow = frac_flow(ld(S, z0 > 0 ? c - sz : c), M);
    double sc = ld(S, c);
    double pc = frac_flow(sc, M);
    // the edge lanes' x-neighbour (lane 0 the one below, lane 63 the one above)
    const bool lo_edge = lane == 0;
    for (int z = z0; z < z1; ++z, c += sz) {
      const double sabove = ld(S, z + 1 < t.nz ? c + sz : c);
      const double se = ld(S, lo_edge ? (x > 0 ? c - 1 : c) : (x + 1 < t.nx ? c + 1 : c));
      const double sn2 = ld(S, y > 0 ? c - sy : c), sn3 = ld(S, y + 1 < t.ny ? c + sy : c);
      double u[6];
#pragma unroll
      for (int f = 0; f < 6; ++f) u[f] = ld(Uf[f], c);
      const double qc = tq ? ld(q, c) : 0.0;
      const double pabove = frac_flow(sabove, M);
      const double pe = frac_flow(se, M);
      const double pl = __shfl_up(pc, 1), pr = __shfl_down(pc, 1);
      // upwind phi of each face (a wall's inflow carries water)
      auto face = [&](double uf, double pn, bool wall, double rh) {
        const double pf = uf >= 0.0 ? pc : (wall ? 1.0 : pn);
        return (pf - pc) * uf * rh;
      };
      double acc = face(u[0], lo_edge ? pe : pl, x == 0, rx);
      acc += face(u[1], lane == 63 ? pe : pr, x + 1 == t.nx, rx);
      acc += face(u[2], frac_flow(sn2, M), y == 0, ry);
      acc += face(u[3], frac_flow(sn3, M), y + 1 == t.ny, ry);
      acc += face(u[4], pbelow, z == 0, rz);
      acc += face(u[5], pabove, z + 1 == t.nz, rz);
      double s = sc - dt * acc;
      if (qc > 0.0) s += dt * qc * (1.0 - pc) * rv;
      st(Sout, c, s);
      if (kSpeed) {
        double um = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) um = fmax(um, fabs(u[f]));
        m = fmax(m, fabs(frac_flow_deriv(s, M)) * um);
      }
      pbelow = pc;
      sc = sabove;
      pc = pabove;
    }
  }
  if (kSpeed) block_max_into(m, vmax);
}

// Largest |phi'(S_c)| max_f |U[f][c]| over the cells, into vmax (grid-
// stride, a few workgroups per CU, one atomic per workgroup).
__global__ __launch_bounds__(kTile) void k_transport_speed(TwoPhaseGrid t, const double *__restrict__ U,
                                                           const double *__restrict__ S,
                                                           unsigned long long *__restrict__ vmax) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const double M = t.mu_o / t.mu_w;
  double m = 0.0;
  for (long long c = (long long)blockIdx.x * kTile + threadIdx.x; c < N; c += (long long)gridDim.x * kTile) {
    double um = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) um = fmax(um, fabs(U[f * N + c]));
    m = fmax(m, fabs(frac_flow_deriv(S[c], M)) * um);
  }
  block_max_into(m, vmax);
}

// min(dt_max, cfl hmin / max speed); dt_max alone when nothing moves
__global__ void k_transport_dt(const unsigned long long *vmax, double hmin, double cfl, double dt_max, double *dt) {
  if (threadIdx.x == 0) {
    const double m = __longlong_as_double((long long)*vmax);
    *dt = m > 0.0 ? fmin(cfl * hmin / m, dt_max) : dt_max;
  }
}

__global__ void k_zero_u64(unsigned long long *p) {
  if (threadIdx.x == 0) *p = 0ull;
}

// K lambda(S) per cell, lambda(S) = S^2 / mu_w + (1 - S)^2 / mu_o.
__global__ __launch_bounds__(256) void k_mobility(TwoPhaseGrid t, const double *__restrict__ S,
                                                  const double *__restrict__ kx, const double *__restrict__ ky,
                                                  const double *__restrict__ kz, double *__restrict__ ox,
                                                  double *__restrict__ oy, double *__restrict__ oz) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double s = S[c], o = 1.0 - s;
  const double lam = s * s / t.mu_w + o * o / t.mu_o;
  ox[c] = lam * kx[c];
  oy[c] = lam * ky[c];
  oz[c] = lam * kz[c];
}

// Marks the tiles of k_transport that hold a cell with q != 0 (one thread
// per cell; every writer stores 1).  The tile of cell (x, y, z): the
// x-segment counts from the row's line offset on the tile's first plane.
__global__ __launch_bounds__(256) void k_source_tiles(TwoPhaseGrid t, ZTiles zt, const double *__restrict__ q,
                                                      unsigned char *__restrict__ flags) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N || q[c] == 0.0) return;
  const long long sy = t.nx, sz = (long long)t.nx * t.ny;
  const int x = (int)(c % t.nx), y = (int)((c / t.nx) % t.ny), z = (int)(c / sz);
  const int z0 = z / kZLen * kZLen;
  const int a = (int)((sy * y + sz * z0) & 15);
  const long long tile = (long long)((x + a) / kZX) + zt.nxt * ((long long)(y / kZY) + (long long)zt.nyt * (z / kZLen));
  flags[tile] = 1;
}

__global__ void k_fill_u8(unsigned char *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
}

namespace {

ZTiles transport_tiles(const TwoPhaseGrid &t) {
  return ZTiles{(t.nx + 15 + kZX - 1) / kZX, (t.ny + kZY - 1) / kZY, (t.nz + kZLen - 1) / kZLen};
}

// Resident workgroups of kernel k over the whole device (the kernels stride
// over their tiles, so the whole grid must be resident: a workgroup that
// starts late would hold back the end), and no more than the tiles.
// The queries run once per kernel and device (per host thread): the step is
// launched thousands of times in a run.
unsigned resident_grid(const void *k, long long ntiles) {
  struct Entry {
    const void *k;
    int dev;
    long long g;
  };
  thread_local std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = -1;
  long long g = 0;
  for (const Entry &e : cache)
    if (e.k == k && e.dev == dev) g = e.g;
  if (g == 0) {
    int cus = 0, nb = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kTile, 0) != hipSuccess)
      cus = nb = 0;
    g = std::max(8LL, (long long)cus * std::max(nb, 1));
    cache.push_back(Entry{k, dev, g});
  }
  return (unsigned)std::max(1LL, std::min(g, ntiles));
}

// the z-marching tiles' count
long long tile_count(const ZTiles &zt) { return (long long)zt.nxt * zt.nyt * zt.nzt; }

}  // namespace

hipError_t launch_transport(const TwoPhaseGrid &t, const double *U, const double *q, const double *S,
                            const double *dt, double *Sout, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  if (N == 0) return hipSuccess;
  const ZTiles zt = transport_tiles(t);
  if (8 * N < (1LL << 32)) {
    const void *k = reinterpret_cast<const void *>(&k_transport<false, uint32_t>);
    hipLaunchKernelGGL((k_transport<false, uint32_t>), dim3(resident_grid(k, tile_count(zt))), dim3(kTile), 0, s, t,
                       zt, U, q, (const unsigned char *)nullptr, S, dt, Sout, (unsigned long long *)nullptr);
  } else {
    const void *k = reinterpret_cast<const void *>(&k_transport<false, long long>);
    hipLaunchKernelGGL((k_transport<false, long long>), dim3(resident_grid(k, tile_count(zt))), dim3(kTile), 0, s, t,
                       zt, U, q, (const unsigned char *)nullptr, S, dt, Sout, (unsigned long long *)nullptr);
  }
  return hipGetLastError();
}

// The step, and the next step's CFL speed of the new state reduced into
// dt_next's eight bytes (launch_speed_clear first), which
// launch_speed_finish then turns into that step in place.
hipError_t launch_speed_clear(double *dt, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<unsigned long long *>(dt));
  return hipGetLastError();
}

hipError_t launch_transport_fused(const TwoPhaseGrid &t, const double *U, const double *q, const double *S,
                                  const double *dt, double *Sout, double *dt_next, hipStream_t s,
                                  const unsigned char *src_tiles) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  if (N == 0) return hipSuccess;
  unsigned long long *work = reinterpret_cast<unsigned long long *>(dt_next);
  const ZTiles zt = transport_tiles(t);
  if (8 * N < (1LL << 32)) {
    const void *k = reinterpret_cast<const void *>(&k_transport<true, uint32_t>);
    hipLaunchKernelGGL((k_transport<true, uint32_t>), dim3(resident_grid(k, tile_count(zt))), dim3(kTile), 0, s, t,
                       zt, U, q, src_tiles, S, dt, Sout, work);
  } else {
    const void *k = reinterpret_cast<const void *>(&k_transport<true, long long>);
    hipLaunchKernelGGL((k_transport<true, long long>), dim3(resident_grid(k, tile_count(zt))), dim3(kTile), 0, s, t,
                       zt, U, q, src_tiles, S, dt, Sout, work);
  }
  return hipGetLastError();
}

hipError_t launch_speed_finish(const TwoPhaseGrid &t, double cfl, double dt_max, double *dt, hipStream_t s) {
  const double hmin = std::fmin(t.hx, std::fmin(t.hy, t.hz));
  hipLaunchKernelGGL(k_transport_dt, dim3(1), dim3(64), 0, s, reinterpret_cast<const unsigned long long *>(dt), hmin,
                     cfl, dt_max, dt);
  return hipGetLastError();
}

// The maximum accumulates in dt's own eight bytes (as an unsigned integer)
// before the last kernel turns it into the step in place.
hipError_t launch_transport_dt(const TwoPhaseGrid &t, const double *U, const double *S, double cfl, double dt_max,
                               double *dt, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  unsigned long long *work = reinterpret_cast<unsigned long long *>(dt);
  const hipError_t e = launch_speed_clear(dt, s);
  if (e != hipSuccess) return e;
  if (N > 0)
    hipLaunchKernelGGL(k_transport_speed,
                       dim3(resident_grid(reinterpret_cast<const void *>(&k_transport_speed), (N + kTile - 1) / kTile)),
                       dim3(kTile), 0, s, t, U, S, work);
  return launch_speed_finish(t, cfl, dt_max, dt, s);
}

long long transport_tile_count(const TwoPhaseGrid &t) { return tile_count(transport_tiles(t)); }

hipError_t launch_source_tiles(const TwoPhaseGrid &t, const double *q, unsigned char *flags, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const long long nt = transport_tile_count(t);
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)std::min<long long>((nt + 255) / 256, 4096)), dim3(256), 0, s, flags,
                     nt);
  if (N > 0)
    hipLaunchKernelGGL(k_source_tiles, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, t, transport_tiles(t), q,
                       flags);
  return hipGetLastError();
}

hipError_t launch_mobility(const TwoPhaseGrid &t, const double *S, const double *kx, const double *ky,
                           const double *kz, double *ox, double *oy, double *oz, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mobility, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, t, S, kx, ky, kz, ox, oy, oz);
  return hipGetLastError();
}

}  // namespace mrcm
