// Learned warm start for the conjugate-gradient local solves: the kernels of
// a small 3D convolutional network (forward, backward, Adam) and the
// gathering of its inputs and targets from a built MBF handle.
//
// Tensors are FP32, layout [B][C][D][H][W] with W fastest.  For a subdomain
// the grid is its local row order viewed as [n2][n1][n0], so one column of
// the MBFs is one [D][H][W] sample.  Convolutions are 3x3x3 cross-
// correlations with dilation dil (taps at offsets -dil, 0, +dil along each
// axis) and zero padding (output size = input size).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device_common.h"
#include "launch.h"

namespace mrcm {
namespace {

constexpr int kConvThreads = 256;
constexpr int kMaxCout = 16;
constexpr int kMaxCin = 16;

// y[b][co] = bias[co] + sum_ci sum_taps w[co][ci][tap] x[b][ci][shifted]
// One thread per output voxel, all output channels in registers; the weights
// sit in LDS.  relu: y = max(y, 0).  mask (optional, shaped like y): y is
// zeroed where mask <= 0, which applies the derivative of a ReLU whose output
// is mask.
__global__ __launch_bounds__(kConvThreads) void k_conv3d(const float *__restrict__ x, const float *__restrict__ w,
                                                         const float *__restrict__ bias, float *__restrict__ y,
                                                         const float *__restrict__ mask, int B, int Cin, int Cout,
                                                         int D, int H, int W, int dil, int relu) {
  __shared__ float ws[kMaxCout * kMaxCin * 27];
  const int nw = Cout * Cin * 27;
  for (int k = threadIdx.x; k < nw; k += kConvThreads) ws[k] = w[k];
  __syncthreads();
  const long long V = (long long)D * H * W;
  const long long idx = (long long)blockIdx.x * kConvThreads + threadIdx.x;
  if (idx >= (long long)B * V) return;
  const int b = (int)(idx / V);
  const int v = (int)(idx - (long long)b * V);
  const int xw = v % W, yh = (v / W) % H, zd = v / (W * H);
  float acc[kMaxCout];
#pragma unroll
  for (int co = 0; co < kMaxCout; ++co) acc[co] = (co < Cout && bias) ? bias[co] : 0.0f;
  for (int ci = 0; ci < Cin; ++ci) {
    const float *xc = x + ((long long)b * Cin + ci) * V;
    for (int kd = 0; kd < 3; ++kd) {
      const int zz = zd + (kd - 1) * dil;
      if (zz < 0 || zz >= D) continue;
      for (int kh = 0; kh < 3; ++kh) {
        const int yy = yh + (kh - 1) * dil;
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int kw = 0; kw < 3; ++kw) {
          const int xx = xw + (kw - 1) * dil;
          const bool in = xx >= 0 && xx < W;
          const float xv = in ? xc[((long long)zz * H + yy) * W + min(max(xx, 0), W - 1)] : 0.0f;
          const int tap = (kd * 3 + kh) * 3 + kw;
#pragma unroll
          for (int co = 0; co < kMaxCout; ++co)
            if (co < Cout) acc[co] = fmaf(ws[(co * Cin + ci) * 27 + tap], xv, acc[co]);
        }
      }
    }
  }
#pragma unroll
  for (int co = 0; co < kMaxCout; ++co) {
    if (co >= Cout) break;
    const long long o = ((long long)b * Cout + co) * V + v;
    float r = acc[co];
    if (relu) r = fmaxf(r, 0.0f);
    if (mask && !(mask[o] > 0.0f)) r = 0.0f;
    y[o] = r;
  }
}

// wt[ci][co][tap] = w[co][ci][26 - tap]: the weights of the transposed
// convolution, which maps dL/dy to dL/dx.
__global__ void k_conv3d_flip(const float *__restrict__ w, float *__restrict__ wt, int Cin, int Cout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Cout * Cin * 27) return;
  const int tap = k % 27, ci = (k / 27) % Cin, co = k / (27 * Cin);
  wt[(ci * Cout + co) * 27 + (26 - tap)] = w[k];
}

// dw[co][ci][tap] = sum_b sum_v dy[b][co][v] x[b][ci][v + dil (tap - 1)] and,
// from the workgroups with ci == 0, db[co] = sum_b sum_v dy[b][co][v].
// One workgroup per (co, ci); each lane sums a fixed stride of (b, v), then
// a fixed-order tree over the workgroup (deterministic).
constexpr int kWgThreads = 512;
__global__ __launch_bounds__(kWgThreads) void k_conv3d_wgrad(const float *__restrict__ x, const float *__restrict__ dy,
                                                             float *__restrict__ dw, float *__restrict__ db, int B,
                                                             int Cin, int Cout, int D, int H, int W, int dil) {
  __shared__ float red[28][kWgThreads / 64];
  const int co = blockIdx.x / Cin, ci = blockIdx.x % Cin;
  const long long V = (long long)D * H * W;
  float acc[28];
#pragma unroll
  for (int t = 0; t < 28; ++t) acc[t] = 0.0f;
  for (long long e = threadIdx.x; e < (long long)B * V; e += kWgThreads) {
    const int b = (int)(e / V);
    const int v = (int)(e - (long long)b * V);
    const int xw = v % W, yh = (v / W) % H, zd = v / (W * H);
    const float g = dy[((long long)b * Cout + co) * V + v];
    const float *xc = x + ((long long)b * Cin + ci) * V;
    acc[27] += g;
#pragma unroll
    for (int kd = 0; kd < 3; ++kd) {
      const int zz = zd + (kd - 1) * dil;
#pragma unroll
      for (int kh = 0; kh < 3; ++kh) {
        const int yy = yh + (kh - 1) * dil;
#pragma unroll
        for (int kw = 0; kw < 3; ++kw) {
          const int xx = xw + (kw - 1) * dil;
          const bool in = zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
          const long long off = ((long long)min(max(zz, 0), D - 1) * H + min(max(yy, 0), H - 1)) * W +
                                min(max(xx, 0), W - 1);
          const float xv = in ? xc[off] : 0.0f;
          acc[(kd * 3 + kh) * 3 + kw] = fmaf(g, xv, acc[(kd * 3 + kh) * 3 + kw]);
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 28; ++t) {
    float v = acc[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[t][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < 28) {
    const int t = threadIdx.x;
    float s = red[t][0];
    for (int k = 1; k < kWgThreads / 64; ++k) s += red[t][k];
    if (t < 27)
      dw[(co * Cin + ci) * 27 + t] = s;
    else if (ci == 0 && db)
      db[co] = s;
  }
}

// Mean squared error: dy = 2 (y - t) / n, and per-workgroup partial sums of
// (y - t)^2 / n, reduced by k_sum_partials.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                            float *__restrict__ dy, double *__restrict__ part, long long n) {
  __shared__ double red[4];
  double s = 0.0;
  const double inv = 1.0 / (double)n;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const float d = y[i] - t[i];
    dy[i] = (float)(2.0 * d * inv);
    s += (double)d * d * inv;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_partials(const double *__restrict__ part, int n, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] = s;
}

// Adam (Kingma and Ba, 2015) at step t (1-based), bias-corrected moments.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, int t, float lr, float b1, float b2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Network inputs and targets, one workgroup per (selected subdomain, column):
// channel 0 the subdomain's log kx minus its mean over the subdomain,
// channel 1 the column's right-hand side divided by its largest magnitude;
// target the column's solution divided by its root mean square (zero columns
// stay zero).  Rows beyond a subdomain's N are not written.
constexpr int kFeatThreads = 256;
__global__ __launch_bounds__(kFeatThreads) void k_nn_features(Geom g, const int *__restrict__ sel,
                                                              const int *__restrict__ sample0,
                                                              const double *__restrict__ R,
                                                              const double *__restrict__ X, int V,
                                                              float *__restrict__ inp, float *__restrict__ tgt) {
  __shared__ double red[3][4];
  const int l = sel[blockIdx.y];
  const SubDesc &S = g.sub[l];
  const int c = blockIdx.x;
  if (c >= S.m) return;
  const int N = S.N, m = S.m;
  const long long s = (long long)sample0[blockIdx.y] + c;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double sk = 0.0, bmax = 0.0, xx = 0.0;
  for (int r = tid; r < N; r += kFeatThreads) {
    const I3 q = local_to_global(S, r);
    sk += log(g.k[0][cell_index(g, q)]);
    bmax = fmax(bmax, fabs(R[S.X_off + (size_t)r * m + c]));
    if (tgt) {
      const double xv = X[S.X_off + (size_t)r * m + c];
      xx += xv * xv;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sk += __shfl_xor(sk, o, 64);
    bmax = fmax(bmax, __shfl_xor(bmax, o, 64));
    xx += __shfl_xor(xx, o, 64);
  }
  if (lane == 0) {
    red[0][wave] = sk;
    red[1][wave] = bmax;
    red[2][wave] = xx;
  }
  __syncthreads();
  const double mean = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) / N;
  const double bm = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
  const double ms = ((red[2][0] + red[2][1]) + (red[2][2] + red[2][3])) / N;
  const double ib = bm > 0.0 ? 1.0 / bm : 0.0;
  const double ix = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
  for (int r = tid; r < N; r += kFeatThreads) {
    const I3 q = local_to_global(S, r);
    inp[(s * 2 + 0) * V + r] = (float)(log(g.k[0][cell_index(g, q)]) - mean);
    inp[(s * 2 + 1) * V + r] = (float)(R[S.X_off + (size_t)r * m + c] * ib);
    if (tgt) tgt[s * V + r] = (float)(X[S.X_off + (size_t)r * m + c] * ix);
  }
}

// x0 in the MBF layout from the network's outputs [samples][V]: column c of
// selected subdomain k takes sample sample0[k] + c.
__global__ __launch_bounds__(256) void k_nn_scatter(Geom g, const int *__restrict__ sel,
                                                    const int *__restrict__ sample0, const float *__restrict__ out,
                                                    int V, double *__restrict__ x0) {
  const int l = sel[blockIdx.y];
  const SubDesc &S = g.sub[l];
  const int c = blockIdx.x;
  if (c >= S.m) return;
  const long long s = (long long)sample0[blockIdx.y] + c;
  for (int r = threadIdx.x; r < S.N; r += 256) x0[S.X_off + (size_t)r * S.m + c] = (double)out[s * V + r];
}

}  // namespace

int conv3d_max_channels() { return kMaxCout; }

hipError_t launch_conv3d(const float *x, const float *w, const float *bias, float *y, const float *mask, int B,
                         int Cin, int Cout, int D, int H, int W, int dil, int relu, hipStream_t s) {
  const long long n = (long long)B * D * H * W;
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + kConvThreads - 1) / kConvThreads;
  hipLaunchKernelGGL(k_conv3d, dim3((unsigned)blocks), dim3(kConvThreads), 0, s, x, w, bias, y, mask, B, Cin, Cout,
                     D, H, W, dil, relu);
  return hipGetLastError();
}

hipError_t launch_conv3d_flip(const float *w, float *wt, int Cin, int Cout, hipStream_t s) {
  const int n = Cout * Cin * 27;
  hipLaunchKernelGGL(k_conv3d_flip, dim3((n + 255) / 256), dim3(256), 0, s, w, wt, Cin, Cout);
  return hipGetLastError();
}

hipError_t launch_conv3d_wgrad(const float *x, const float *dy, float *dw, float *db, int B, int Cin, int Cout,
                               int D, int H, int W, int dil, hipStream_t s) {
  hipLaunchKernelGGL(k_conv3d_wgrad, dim3(Cout * Cin), dim3(kWgThreads), 0, s, x, dy, dw, db, B, Cin, Cout, D, H,
                     W, dil);
  return hipGetLastError();
}

int mse_partials(long long n) { return (int)std::min<long long>(kMsePartialsMax, (n + 255) / 256); }

hipError_t launch_mse(const float *y, const float *t, float *dy, double *part, double *loss, long long n,
                      hipStream_t s) {
  const int nb = mse_partials(n);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, y, t, dy, part, n);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, nb, loss);
  return hipGetLastError();
}

// Partial sums of the loss for callers that cannot allocate: one array per
// GPU, for the life of the process.  Its address on each device comes from
// hipGetSymbolAddress (the name itself is only a host-side stand-in).
static __device__ __align__(256) double scratch[kMsePartialsMax];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t launch_mse_static(const float *y, const float *t, float *dy, double *loss, long long n,
                             hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  double *part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *addr = nullptr;
      e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return e;
      g_scratch_ptr[dev] = static_cast<double *>(addr);
    }
    part = g_scratch_ptr[dev];
  }
  // every partial the sum reads is written by this call's first kernel, so
  // nothing in the array needs clearing
  return launch_mse(y, t, dy, part, loss, n, s);
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, int t, float lr, float b1, float b2,
                       float eps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, t, lr, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_nn_features(const Geom &g, const int *sel, const int *sample0, int n_sel, int mmax,
                              const double *R, const double *X, int V, float *inp, float *tgt, hipStream_t s) {
  if (n_sel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nn_features, dim3(mmax, n_sel), dim3(kFeatThreads), 0, s, g, sel, sample0, R, X, V, inp, tgt);
  return hipGetLastError();
}

hipError_t launch_nn_scatter(const Geom &g, const int *sel, const int *sample0, int n_sel, int mmax,
                             const float *out, int V, double *x0, hipStream_t s) {
  if (n_sel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nn_scatter, dim3(mmax, n_sel), dim3(256), 0, s, g, sel, sample0, out, V, x0);
  return hipGetLastError();
}

}  // namespace mrcm
