// Saturation step of the IMPES two-phase run on gfx950: the upwind finite-
// volume Buckley-Leverett update with the divergence compensation (eqs.
// (transporte_discreto), (flux_disc_up)), the CFL time step (eq. (CFL)) and
// the total mobility that scales each Darcy solve's permeability (Sec. 5).
// All three are streaming stencils, one thread per cell, bound by HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

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

// One step: S_c' = S_c - dt sum_f (phi_f - phi(S_c)) U[f][c] / h_d(f), with
// phi_f the upwind value (the cell's own on an outflow face, the neighbour's
// on an inflow face, water across a domain wall), plus dt q (1 - phi(S_c)) / V
// in an injector cell.  U face-major (U[f * N + c]), cells x fastest.
__global__ __launch_bounds__(256) void k_transport(TwoPhaseGrid t, const double *__restrict__ U,
                                                   const double *__restrict__ q, const double *__restrict__ S,
                                                   const double *__restrict__ dtp, double *__restrict__ Sout) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const double M = t.mu_o / t.mu_w;
  const double dt = *dtp;
  const int x = (int)(c % t.nx);
  const int y = (int)((c / t.nx) % t.ny);
  const int z = (int)(c / ((long long)t.nx * t.ny));
  const long long sx = 1, sy = t.nx, sz = (long long)t.nx * t.ny;
  const double sc = S[c];
  const double pc = frac_flow(sc, M);
  // neighbours' saturations, loaded together (a wall reads the cell itself,
  // unused: its inflow carries water)
  const double sn0 = S[x > 0 ? c - sx : c], sn1 = S[x + 1 < t.nx ? c + sx : c];
  const double sn2 = S[y > 0 ? c - sy : c], sn3 = S[y + 1 < t.ny ? c + sy : c];
  const double sn4 = S[z > 0 ? c - sz : c], sn5 = S[z + 1 < t.nz ? c + sz : c];
  double u[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) u[f] = U[f * N + c];
  const double qc = q ? q[c] : 0.0;
  auto face = [&](double uf, double sn, bool wall, double h) {
    const double pn = wall ? 1.0 : frac_flow(sn, M);
    const double pf = uf >= 0.0 ? pc : pn;
    return (pf - pc) * uf / h;
  };
  double acc = face(u[0], sn0, x == 0, t.hx);
  acc += face(u[1], sn1, x + 1 == t.nx, t.hx);
  acc += face(u[2], sn2, y == 0, t.hy);
  acc += face(u[3], sn3, y + 1 == t.ny, t.hy);
  acc += face(u[4], sn4, z == 0, t.hz);
  acc += face(u[5], sn5, z + 1 == t.nz, t.hz);
  double s = sc - dt * acc;
  if (qc > 0.0) s += dt * qc * (1.0 - pc) / (t.hx * t.hy * t.hz);
  Sout[c] = s;
}

// Largest |phi'(S_c)| max_f |U[f][c]| over the cells, as the bit pattern of
// a non-negative double (ordered as an unsigned integer): a workgroup's
// maximum, then one atomic per workgroup.
__global__ __launch_bounds__(256) void k_transport_speed(TwoPhaseGrid t, const double *__restrict__ U,
                                                         const double *__restrict__ S,
                                                         unsigned long long *__restrict__ vmax) {
  __shared__ double red[256];
  const long long N = (long long)t.nx * t.ny * t.nz;
  const double M = t.mu_o / t.mu_w;
  double m = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
    double um = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) um = fmax(um, fabs(U[f * N + c]));
    m = fmax(m, fabs(frac_flow_deriv(S[c], M)) * um);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(vmax, (unsigned long long)__double_as_longlong(red[0]));
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

hipError_t launch_transport(const TwoPhaseGrid &t, const double *U, const double *q, const double *S,
                            const double *dt, double *Sout, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transport, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, t, U, q, S, dt, Sout);
  return hipGetLastError();
}

// The maximum accumulates in dt's own eight bytes (as an unsigned integer)
// before the last kernel turns it into the step in place.
hipError_t launch_transport_dt(const TwoPhaseGrid &t, const double *U, const double *S, double cfl, double dt_max,
                               double *dt, hipStream_t s) {
  const long long N = (long long)t.nx * t.ny * t.nz;
  unsigned long long *work = reinterpret_cast<unsigned long long *>(dt);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, work);
  if (N > 0) {
    const long long blocks = std::min<long long>((N + 255) / 256, 256LL * 64);
    hipLaunchKernelGGL(k_transport_speed, dim3((unsigned)blocks), dim3(256), 0, s, t, U, S, work);
  }
  const double hmin = std::fmin(t.hx, std::fmin(t.hy, t.hz));
  hipLaunchKernelGGL(k_transport_dt, dim3(1), dim3(64), 0, s, work, hmin, cfl, dt_max, dt);
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
