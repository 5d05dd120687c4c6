// Kernels of the encoder-decoder warm-start network: BF16 MFMA convolutions
// with FP32 accumulation, FP32 weight gradients, average pooling and
// nearest upsampling over the two long grid axes, weight packing and the
// channels-last permute of the network's inputs.
//
// Activations are FP32, channels last: [batch][D][H][W][C].  A convolution
// rounds its input and its weights to bfloat16 (round to nearest, ties to
// even) and accumulates the products in FP32 on the matrix cores: the
// implicit GEMM Y[voxel][co] = sum over (tap, ci) of X[voxel + off(tap)][ci]
// W[(tap, ci)][co], with zero padding outside the grid.  Weights are packed
// per 16-channel tile: forward wf[co][tap][ci] (co, ci padded to multiples
// of 16) and, for dL/dx, the spatially flipped transpose wt[ci][tap][co].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "launch.h"

namespace mrcm {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
  // round to nearest, ties to even, from the float's bits (finite values)
  const unsigned int u = __builtin_bit_cast(unsigned int, f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

constexpr int kConvWaves = 4;  // 16 voxels per wave, 64 per workgroup
constexpr int kMaxTiles = 8;   // up to 128 output channels

// y = conv(x, w) + bias, ReLU when relu, zeroed where mask <= 0 (mask shaped
// like y, or null).  One wave per 16 consecutive voxels (over the batch), all
// output-channel tiles in its accumulators.
template <int NT>
__global__ __launch_bounds__(64 * kConvWaves) void k_unet_conv(const float *__restrict__ x,
                                                                const unsigned short *__restrict__ wf,
                                                                const float *__restrict__ bias, float *__restrict__ y,
                                                                const float *__restrict__ mask, int nvox, int D, int H,
                                                                int W, int Cin, int CinP, int Cout, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kg = lane >> 4;
  const long long n0 = ((long long)blockIdx.x * kConvWaves + wave) * 16;
  const long long n = n0 + row;  // this lane's voxel of the A operand
  const int V = D * H * W;
  const bool vin = n < nvox;
  const long long bidx = vin ? n / V : 0;
  const int v = vin ? (int)(n - bidx * V) : 0;
  const int pw = v % W, ph = (v / W) % H, pd = v / (W * H);
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int nch = CinP >> 4;
  for (int tap = 0; tap < 27; ++tap) {
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int qd = pd + dz, qh = ph + dy, qw = pw + dx;
    const bool ok = vin && qd >= 0 && qd < D && qh >= 0 && qh < H && qw >= 0 && qw < W;
    const float *src = x + ((bidx * V + (long long)(qd * H + qh) * W + qw) * Cin);
    for (int c = 0; c < nch; ++c) {
      const int ci = 16 * c + 4 * kg;
      bf16x4 a;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float f = (ok && ci + j < Cin) ? src[ci + j] : 0.0f;
        a[j] = (short)to_bf16(f);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const unsigned short *wp = wf + ((size_t)(16 * t + row) * 27 + tap) * CinP + ci;
        const uint2 wv = *reinterpret_cast<const uint2 *>(wp);
        bf16x4 b;
        b[0] = (short)(wv.x & 0xffffu);
        b[1] = (short)(wv.x >> 16);
        b[2] = (short)(wv.y & 0xffffu);
        b[3] = (short)(wv.y >> 16);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // accumulator item j of this lane: voxel n0 + 4 kg + j, channel 16 t + row
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = 16 * t + row;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long nv = n0 + 4 * kg + j;
      if (co < Cout && nv < nvox) {
        float val = acc[t][j] + (bias ? bias[co] : 0.0f);
        if (relu) val = fmaxf(val, 0.0f);
        const long long o = nv * Cout + co;
        if (mask && !(mask[o] > 0.0f)) val = 0.0f;
        y[o] = val;
      }
    }
  }
}

// Partial weight gradients of one tap over a chunk of voxels:
// part[chunk][tap][co][ci] = sum over the chunk of dy[n][co] bf16(x)[n + off(tap)][ci],
// and for the centre tap part_b[chunk][co] = sum of dy[n][co].
constexpr int kWgVox = 32;  // voxels staged in LDS per round
constexpr int kWgMaxC = 128;

__global__ __launch_bounds__(256) void k_unet_wgrad(const float *__restrict__ x, const float *__restrict__ dy,
                                                    float *__restrict__ part, float *__restrict__ part_b, int nvox,
                                                    int D, int H, int W, int Cin, int Cout, int chunk) {
  __shared__ float gs[kWgVox][kWgMaxC + 1];
  __shared__ float xs[kWgVox][kWgMaxC + 1];
  const int tap = blockIdx.x, ck = blockIdx.y;
  const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int V = D * H * W;
  const int np = Cout * Cin;
  const int tid = threadIdx.x;
  constexpr int kPer = (kWgMaxC * kWgMaxC + 255) / 256;
  float acc[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) acc[i] = 0.0f;
  float accb = 0.0f;
  const long long nbeg = (long long)ck * chunk;
  const long long nend = std::min<long long>(nvox, nbeg + chunk);
  for (long long nb0 = nbeg; nb0 < nend; nb0 += kWgVox) {
    __syncthreads();
    for (int e = tid; e < kWgVox * (Cout + Cin); e += 256) {
      const int vv = e / (Cout + Cin), c = e % (Cout + Cin);
      const long long nn = nb0 + vv;
      if (c < Cout) {
        gs[vv][c] = nn < nend ? dy[nn * Cout + c] : 0.0f;
      } else {
        const int ci = c - Cout;
        float f = 0.0f;
        if (nn < nend) {
          const long long b = nn / V;
          const int v = (int)(nn - b * V);
          const int qw = v % W + dx, qh = (v / W) % H + dyy, qd = v / (W * H) + dz;
          if (qd >= 0 && qd < D && qh >= 0 && qh < H && qw >= 0 && qw < W)
            f = __builtin_bit_cast(float, (unsigned int)to_bf16(x[(b * V + (long long)(qd * H + qh) * W + qw) * Cin + ci]) << 16);
        }
        xs[vv][ci] = f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int p = tid + 256 * i;
      if (p < np) {
        const int co = p / Cin, ci = p % Cin;
        float s = acc[i];
        for (int vv = 0; vv < kWgVox; ++vv) s = fmaf(gs[vv][co], xs[vv][ci], s);
        acc[i] = s;
      }
    }
    if (tap == 13 && tid < Cout)
      for (int vv = 0; vv < kWgVox; ++vv) accb += gs[vv][tid];
  }
  float *out = part + ((size_t)ck * 27 + tap) * np;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int p = tid + 256 * i;
    if (p < np) out[p] = acc[i];
  }
  if (tap == 13 && tid < Cout) part_b[(size_t)ck * Cout + tid] = accb;
}

// dw[co][ci][tap] = sum over chunks (in order) of the partials; db likewise.
__global__ void k_unet_wgrad_sum(const float *__restrict__ part, const float *__restrict__ part_b, int nchunk,
                                 int Cin, int Cout, float *__restrict__ dw, float *__restrict__ db) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = Cout * Cin;
  if (e < 27 * np) {
    const int tap = e / np, p = e % np;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[((size_t)c * 27 + tap) * np + p];
    const int co = p / Cin, ci = p % Cin;
    dw[((size_t)co * Cin + ci) * 27 + tap] = s;
  }
  if (db && e < Cout) {
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part_b[(size_t)c * Cout + e];
    db[e] = s;
  }
}

// Packed BF16 weights from the FP32 master weights w[co][ci][tap].
__global__ void k_unet_pack(const float *__restrict__ w, unsigned short *__restrict__ wf,
                            unsigned short *__restrict__ wt, int Cin, int Cout, int CinP, int CoP) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= CoP * 27 * CinP) return;
  {
    // wf[co][tap][ci]
    const int ci = e % CinP, tap = (e / CinP) % 27, co = e / (CinP * 27);
    wf[e] = (co < Cout && ci < Cin) ? to_bf16(w[((size_t)co * Cin + ci) * 27 + tap]) : (unsigned short)0;
  }
  {
    // wt[ci][tap][co] = w[co][ci][26 - tap]
    const int co = e % CoP, tap = (e / CoP) % 27, ci = e / (CoP * 27);
    wt[e] = (co < Cout && ci < Cin) ? to_bf16(w[((size_t)co * Cin + ci) * 27 + (26 - tap)]) : (unsigned short)0;
  }
}

// Average of 2x2 cells over (D, H) / its adjoint (each input cell receives a
// quarter of its output cell's gradient).
__global__ void k_unet_pool(const float *__restrict__ x, float *__restrict__ y, long long nout, int D, int H, int W,
                            int C, int backward) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int Do = D / 2, Ho = H / 2;
  const int c = (int)(e % C);
  long long r = e / C;
  const int w = (int)(r % W);
  r /= W;
  const int h = (int)(r % Ho);
  r /= Ho;
  const int d = (int)(r % Do);
  const long long b = r / Do;
  auto at = [&](int dd, int hh) { return ((((b * D + dd) * H + hh) * (long long)W + w) * C + c); };
  if (!backward) {
    y[e] = 0.25f * ((x[at(2 * d, 2 * h)] + x[at(2 * d + 1, 2 * h)]) + (x[at(2 * d, 2 * h + 1)] + x[at(2 * d + 1, 2 * h + 1)]));
  } else {
    // x: gradient at the pooled output, y: gradient at the input
    const float g = 0.25f * x[e];
    y[at(2 * d, 2 * h)] = g;
    y[at(2 * d + 1, 2 * h)] = g;
    y[at(2 * d, 2 * h + 1)] = g;
    y[at(2 * d + 1, 2 * h + 1)] = g;
  }
}

// Nearest upsampling by two over (D, H) (input D x H, output 2D x 2H) / its
// adjoint (the sum of the four copies' gradients).
__global__ void k_unet_up(const float *__restrict__ x, float *__restrict__ y, long long nsmall, int D, int H, int W,
                          int C, int backward) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nsmall) return;
  const int c = (int)(e % C);
  long long r = e / C;
  const int w = (int)(r % W);
  r /= W;
  const int h = (int)(r % H);
  r /= H;
  const int d = (int)(r % D);
  const long long b = r / D;
  const int D2 = 2 * D, H2 = 2 * H;
  auto at = [&](int dd, int hh) { return ((((b * D2 + dd) * H2 + hh) * (long long)W + w) * C + c); };
  if (!backward) {
    const float v = x[e];
    y[at(2 * d, 2 * h)] = v;
    y[at(2 * d + 1, 2 * h)] = v;
    y[at(2 * d, 2 * h + 1)] = v;
    y[at(2 * d + 1, 2 * h + 1)] = v;
  } else {
    // x: gradient at the upsampled output, y: gradient at the small input
    y[e] = (x[at(2 * d, 2 * h)] + x[at(2 * d + 1, 2 * h)]) + (x[at(2 * d, 2 * h + 1)] + x[at(2 * d + 1, 2 * h + 1)]);
  }
}

// g = g where out > 0, else 0 (the ReLU's derivative).
__global__ void k_unet_relu_mask(float *__restrict__ g, const float *__restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(out[e] > 0.0f)) g[e] = 0.0f;
}

// [batch][C][V] -> [batch][V][C]
__global__ void k_channels_last(const float *__restrict__ in, float *__restrict__ out, long long total, int C,
                                long long V) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % C);
  const long long r = e / C;
  const long long v = r % V, b = r / V;
  out[e] = in[(b * C + c) * V + v];
}

unsigned blocks_for(long long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int unet_pad16(int c) { return (c + 15) & ~15; }

int unet_max_channels() { return 16 * kMaxTiles; }

hipError_t launch_unet_pack(const float *w, unsigned short *wf, unsigned short *wt, int cin, int cout, hipStream_t s) {
  const int n = unet_pad16(cout) * 27 * unet_pad16(cin);
  hipLaunchKernelGGL(k_unet_pack, dim3(blocks_for(n)), dim3(256), 0, s, w, wf, wt, cin, cout, unet_pad16(cin),
                     unet_pad16(cout));
  return hipGetLastError();
}

hipError_t launch_unet_conv(const float *x, const unsigned short *wf, const float *bias, float *y, const float *mask,
                            int batch, int d, int h, int w, int cin, int cout, int relu, hipStream_t s) {
  const long long nvox = (long long)batch * d * h * w;
  const int nt = unet_pad16(cout) / 16;
  const dim3 grid((unsigned)((nvox + 16 * kConvWaves - 1) / (16 * kConvWaves)));
  const dim3 blk(64 * kConvWaves);
  const int cinp = unet_pad16(cin);
  switch (nt) {
#define CASE(T)                                                                                              \
  case T:                                                                                                    \
    hipLaunchKernelGGL(k_unet_conv<T>, grid, blk, 0, s, x, wf, bias, y, mask, (int)nvox, d, h, w, cin, cinp, \
                       cout, relu);                                                                          \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

long long unet_wgrad_chunk(long long nvox) { return std::max<long long>(4096, (nvox + 63) / 64); }

long long unet_wgrad_workspace(long long nvox, int cin, int cout) {
  const long long ch = unet_wgrad_chunk(nvox);
  const long long nchunk = (nvox + ch - 1) / ch;
  return nchunk * 27 * (long long)cin * cout + nchunk * (long long)cout;
}

hipError_t launch_unet_wgrad(const float *x, const float *dy, float *dw, float *db, float *work, int batch, int d,
                             int h, int w, int cin, int cout, hipStream_t s) {
  const long long nvox = (long long)batch * d * h * w;
  const long long ch = unet_wgrad_chunk(nvox);
  const int nchunk = (int)((nvox + ch - 1) / ch);
  float *part_b = work + (size_t)nchunk * 27 * cin * cout;
  hipLaunchKernelGGL(k_unet_wgrad, dim3(27, nchunk), dim3(256), 0, s, x, dy, work, part_b, (int)nvox, d, h, w, cin,
                     cout, (int)ch);
  hipLaunchKernelGGL(k_unet_wgrad_sum, dim3(blocks_for(27LL * cin * cout)), dim3(256), 0, s, work, part_b, nchunk,
                     cin, cout, dw, db);
  return hipGetLastError();
}

hipError_t launch_unet_pool(const float *x, float *y, int batch, int d, int h, int w, int c, int backward,
                            hipStream_t s) {
  const long long nout = (long long)batch * (d / 2) * (h / 2) * w * c;
  hipLaunchKernelGGL(k_unet_pool, dim3(blocks_for(nout)), dim3(256), 0, s, x, y, nout, d, h, w, c, backward);
  return hipGetLastError();
}

hipError_t launch_unet_up(const float *x, float *y, int batch, int d, int h, int w, int c, int backward,
                          hipStream_t s) {
  const long long ns = (long long)batch * d * h * w * c;
  hipLaunchKernelGGL(k_unet_up, dim3(blocks_for(ns)), dim3(256), 0, s, x, y, ns, d, h, w, c, backward);
  return hipGetLastError();
}

hipError_t launch_unet_relu_mask(float *g, const float *out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_unet_relu_mask, dim3(blocks_for(n)), dim3(256), 0, s, g, out, n);
  return hipGetLastError();
}

hipError_t launch_channels_last(const float *in, float *out, int batch, int c, long long v, hipStream_t s) {
  const long long total = (long long)batch * c * v;
  hipLaunchKernelGGL(k_channels_last, dim3(blocks_for(total)), dim3(256), 0, s, in, out, total, c, v);
  return hipGetLastError();
}

}  // namespace mrcm
