// Learned coarse propagator: a 4-level convolutional encoder-decoder
// G_nn(u) = u + net(u) on an n x n grid (n divisible by 8), with BF16
// weights and FP32 accumulation, and its training kernels (backward passes,
// MSE loss, Adam).  Every reduction is a fixed-order tree, so results are
// bitwise reproducible.
//
// Layer table (must match the parameter layout of the training side):
// for each layer W[c_out][c_in][k][k] then b[c_out], in table order.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstring>
#include <mutex>
#include "ch_internal.h"

// Activations of the allocation-free forward pass (ch_nn_forward_static):
// NN_STATIC_FLOATS floats (32 MiB) in a file-scope device array.  Every GPU
// the library runs on holds its own copy, at its own address, until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): it passes the device address
// that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) float scratch[chk::NN_STATIC_FLOATS];

namespace chk {

const NNLayer kNNLayers[NN_LAYERS] = {
    // c_in, c_out, k, stride, act, cat (index of the skip layer, -1 none)
    {1, 16, 3, 1, 1, -1},   {16, 16, 3, 1, 1, -1},  {16, 32, 3, 2, 1, -1},
    {32, 32, 3, 1, 1, -1},  {32, 64, 3, 2, 1, -1},  {64, 64, 3, 1, 1, -1},
    {64, 64, 3, 2, 1, -1},  {64, 64, 3, 1, 1, -1},  {128, 64, 3, 1, 1, 5},
    {96, 32, 3, 1, 1, 3},   {48, 16, 3, 1, 1, 1},   {16, 1, 1, 1, 0, -1},
};
constexpr float kSlope = 0.1f;

int64_t nn_param_count() {
  int64_t s = 0;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const NNLayer& L = kNNLayers[l];
    s += (int64_t)L.c_out * L.c_in * L.k * L.k + L.c_out;
  }
  return s;
}
int64_t nn_param_offset(int layer) {
  int64_t s = 0;
  for (int l = 0; l < layer; ++l) {
    const NNLayer& L = kNNLayers[l];
    s += (int64_t)L.c_out * L.c_in * L.k * L.k + L.c_out;
  }
  return s;
}
// spatial size of layer l's output for input size n
static int out_size(int l, int n) {
  int s = n;
  for (int i = 0; i <= l; ++i) {
    const NNLayer& L = kNNLayers[i];
    if (L.cat >= 0) s *= 2;
    s /= L.stride;
  }
  return s;
}
static int in_size(int l, int n) {  // spatial size of the (concatenated) input of layer l
  if (l == 0) return n;
  int s = out_size(l - 1, n);
  return kNNLayers[l].cat >= 0 ? 2 * s : s;
}

// Pixel chunks of the weight-gradient GEMM over tot output pixels: at most
// 64, of at least 1024 pixels each (a multiple of 4).
static int wgrad_chunks(int64_t tot) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, (tot + 1023) / 1024));
}
static int64_t wgrad_chunk_len(int64_t tot) {
  const int nch = wgrad_chunks(tot);
  return ((tot + nch - 1) / nch + 15) / 16 * 16;
}

// Workspace layout (floats): x0 | for each layer: act | for each layer: grad | tmp | loss
// partials | weight-gradient partials
NNPlan nn_plan(int batch, int n) {
  NNPlan p;
  size_t o = 0;
  auto take = [&](size_t f) { size_t r = o; o += (f + 63) / 64 * 64; return r; };
  p.x0 = take((size_t)batch * n * n);
  size_t maxin = 0;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const int s = out_size(l, n);
    p.act[l] = take((size_t)batch * kNNLayers[l].c_out * s * s);
    const int si = in_size(l, n);
    maxin = std::max(maxin, (size_t)batch * kNNLayers[l].c_in * si * si);
  }
  for (int l = 0; l < NN_LAYERS; ++l) {
    const int s = out_size(l, n);
    p.grad[l] = take((size_t)batch * kNNLayers[l].c_out * s * s);
  }
  p.tmp = take(maxin);
  p.part = take(4096);
  size_t wp = 0;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const NNLayer& L = kNNLayers[l];
    const int64_t tot = (int64_t)batch * out_size(l, n) * out_size(l, n);
    wp = std::max(wp, (size_t)wgrad_chunks(tot) * L.c_out * (L.c_in * L.k * L.k + 1));
  }
  p.wpart = take(wp);
  p.floats = o;
  return p;
}

__device__ __forceinline__ float bf2f(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ uint16_t f2bf_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

// Input element (b, c, y, x) of a layer whose input is either A alone or the
// concatenation [A (Ca channels, full size), up2(B) (Cb channels, half size)].
__device__ __forceinline__ float in_at(const float* A, int Ca, const float* B, int Cb, int H, int b,
                                       int c, int y, int x) {
  if (y < 0 || y >= H || x < 0 || x >= H) return 0.0f;
  if (c < Ca) return A[(((int64_t)b * Ca + c) * H + y) * H + x];
  const int Hh = H >> 1;
  return B[(((int64_t)b * Cb + (c - Ca)) * Hh + (y >> 1)) * Hh + (x >> 1)];
}

// Forward convolution: one thread per output pixel, COB output channels per
// block, the block's weights staged in LDS as FP32 (from BF16).
template <int COB>
__global__ void __launch_bounds__(256)
k_conv_fwd(const float* __restrict__ A, int Ca, const float* __restrict__ B, int Cb, int H,
           const uint16_t* __restrict__ w, float* __restrict__ Y, int Co, int Ho, int k, int stride,
           int act, const int32_t* __restrict__ gate) {
  extern __shared__ float wl[];
  if (gate && !*gate) return;
  const int Ci = Ca + Cb, kk = k * k, co0 = blockIdx.y * COB, b = blockIdx.z;
  const int nw = COB * Ci * kk;
  for (int i = threadIdx.x; i < nw; i += 256) wl[i] = bf2f(w[(int64_t)co0 * Ci * kk + i]);
  const uint16_t* bias = w + (int64_t)Co * Ci * kk;
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= Ho * Ho) return;
  const int oy = p / Ho, ox = p % Ho, pad = k / 2;
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = bf2f(bias[co0 + c]);
  for (int ci = 0; ci < Ci; ++ci)
    for (int dy = 0; dy < k; ++dy)
      for (int dx = 0; dx < k; ++dx) {
        const float xv = in_at(A, Ca, B, Cb, H, b, ci, oy * stride + dy - pad, ox * stride + dx - pad);
        const float* wr = wl + (ci * k + dy) * k + dx;
#pragma unroll
        for (int c = 0; c < COB; ++c) acc[c] = fmaf(wr[c * Ci * kk], xv, acc[c]);
      }
#pragma unroll
  for (int c = 0; c < COB; ++c) {
    float v = acc[c];
    if (act) v = v > 0.0f ? v : kSlope * v;
    Y[(((int64_t)b * Co + co0 + c) * Ho + oy) * Ho + ox] = v;
  }
}

// Forward convolution on the matrix cores (FP32 MFMA 16x16x4), for c_out a
// multiple of 16 (at most 64): Y[co][p] = bias[co] + sum_j W[co][j] X[j][p]
// with X the im2col columns of the input (j = ci k^2 + tap).  A wave takes 16
// output pixels (A operand: 16 pixels x 4 columns j, gathered from the
// input) against every output channel (B operands: 4 columns x 16 channels
// of the BF16 weights, one per group of 16 channels); a block of four waves
// 64 consecutive pixels of one sample.  Lane layout as in the weight
// gradient: A row = lane & 15, k = lane >> 4; B k = lane >> 4, column = lane
// & 15; D row 4 (lane >> 4) + r, column lane & 15.
typedef float nnf4 __attribute__((ext_vector_type(4)));
template <int NG>
__global__ void __launch_bounds__(256)
k_conv_fwd_mfma(const float* __restrict__ A, int Ca, const float* __restrict__ B, int Cb, int H,
                const uint16_t* __restrict__ w, float* __restrict__ Y, int Ho, int k, int stride,
                int act, const int32_t* __restrict__ gate) {
  if (gate && !*gate) return;
  constexpr int Co = 16 * NG;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, b = blockIdx.y;
  const int i = l & 15, g = l >> 4;
  const int Ci = Ca + Cb, kk = k * k, J = Ci * kk, pad = k / 2;
  const int HH = Ho * Ho;
  const int p0 = blockIdx.x * 64 + wv * 16;
  const int pa = p0 + i;                       // this lane's A-operand pixel
  const bool pin = pa < HH;
  const int oy = pin ? pa / Ho : 0, ox = pin ? pa % Ho : 0;
  const int iy = oy * stride - pad, ix = ox * stride - pad;
  nnf4 acc[NG];
#pragma unroll
  for (int c = 0; c < NG; ++c) acc[c] = nnf4{0.0f, 0.0f, 0.0f, 0.0f};
  // column j = 4 s + g of this lane, walked as (ci, tap), tap = 3 dy + dx
  int ci = 0, tap = g;
  while (tap >= kk) { tap -= kk; ++ci; }
  for (int j = g; j - g < J; j += 4) {
    const bool jin = j < J;
    const int dy = k == 3 ? (tap >= 6 ? 2 : (tap >= 3 ? 1 : 0)) : 0, dx = tap - k * dy;
    const float x = (pin && jin) ? in_at(A, Ca, B, Cb, H, b, ci, iy + dy, ix + dx) : 0.0f;
#pragma unroll
    for (int c = 0; c < NG; ++c) {
      const float wt = jin ? bf2f(w[(int64_t)(16 * c + i) * J + j]) : 0.0f;
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wt, acc[c], 0, 0, 0);
    }
    tap += 4;
    while (tap >= kk) { tap -= kk; ++ci; }
  }
  const uint16_t* bias = w + (int64_t)Co * J;
#pragma unroll
  for (int c = 0; c < NG; ++c) {
    const int co = 16 * c + i;
    const float bv = bf2f(bias[co]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pr = p0 + 4 * g + r;
      if (pr >= HH) continue;
      float v = acc[c][r] + bv;
      if (act) v = v > 0.0f ? v : kSlope * v;
      Y[((int64_t)b * Co + co) * HH + pr] = v;
    }
  }
}

// G <- G * act'(y) in place (y the layer output; LeakyReLU is monotone, so
// the sign of y is the sign of the pre-activation).
__global__ void k_act_bwd(float* __restrict__ G, const float* __restrict__ Y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) G[i] = Y[i] > 0.0f ? G[i] : kSlope * G[i];
}

// Gradient w.r.t. the (concatenated) input: one thread per input pixel, CIB
// input channels per block.  dIn[ci][y][x] = sum_co sum_taps W[co][ci][tap]
// G[co][oy][ox] with oy*stride + dy - pad = y.  Channels < Ca go to dA
// (added when accA), the rest to dBf at full resolution (reduced later).
template <int CIB>
__global__ void __launch_bounds__(256)
k_conv_bwd_data(const float* __restrict__ G, int Co, int Ho, const uint16_t* __restrict__ w,
                int Ca, int Cb, int H, int k, int stride, float* __restrict__ dA, int accA,
                float* __restrict__ dBf) {
  extern __shared__ float wl[];
  const int Ci = Ca + Cb, kk = k * k, ci0 = blockIdx.y * CIB, b = blockIdx.z;
  for (int i = threadIdx.x; i < Co * CIB * kk; i += 256) {
    const int co = i / (CIB * kk), rem = i % (CIB * kk), c = rem / kk, t = rem % kk;
    wl[i] = bf2f(w[((int64_t)co * Ci + ci0 + c) * kk + t]);
  }
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= H * H) return;
  const int y = p / H, x = p % H, pad = k / 2;
  float acc[CIB];
#pragma unroll
  for (int c = 0; c < CIB; ++c) acc[c] = 0.0f;
  for (int dy = 0; dy < k; ++dy) {
    const int ty = y + pad - dy;
    if (ty < 0 || ty % stride) continue;
    const int oy = ty / stride;
    if (oy >= Ho) continue;
    for (int dx = 0; dx < k; ++dx) {
      const int tx = x + pad - dx;
      if (tx < 0 || tx % stride) continue;
      const int ox = tx / stride;
      if (ox >= Ho) continue;
      for (int co = 0; co < Co; ++co) {
        const float g = G[(((int64_t)b * Co + co) * Ho + oy) * Ho + ox];
        const float* wr = wl + (co * CIB) * kk + dy * k + dx;
#pragma unroll
        for (int c = 0; c < CIB; ++c) acc[c] = fmaf(wr[c * kk], g, acc[c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < CIB; ++c) {
    const int ci = ci0 + c;
    if (ci < Ca) {
      float* d = dA + (((int64_t)b * Ca + ci) * H + y) * H + x;
      *d = accA ? *d + acc[c] : acc[c];
    } else {
      dBf[(((int64_t)b * Cb + (ci - Ca)) * H + y) * H + x] = acc[c];
    }
  }
}

// dB[b][c][Y][X] = sum of the four fine children of dBf (nearest x2 upsampling).
__global__ void k_up_bwd(const float* __restrict__ dBf, float* __restrict__ dB, int C, int H, int batch) {
  const int Hh = H / 2;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)batch * C * Hh * Hh) return;
  const int X = i % Hh, Yy = (i / Hh) % Hh;
  const int64_t bc = i / ((int64_t)Hh * Hh);
  const float* s = dBf + bc * H * H;
  dB[i] = (s[(2 * Yy) * H + 2 * X] + s[(2 * Yy) * H + 2 * X + 1]) +
          (s[(2 * Yy + 1) * H + 2 * X] + s[(2 * Yy + 1) * H + 2 * X + 1]);
}

// Weight gradient: one block per (ci, co); each thread sums a strided set of
// output positions for the k*k taps (and the bias when ci == 0); fixed-order
// block reduction.
__global__ void __launch_bounds__(256)
k_conv_bwd_weight(const float* __restrict__ G, int Co, int Ho, const float* __restrict__ A, int Ca,
                  const float* __restrict__ B, int Cb, int H, int k, int stride, int batch,
                  float* __restrict__ gw) {
  __shared__ float red[10][8];
  const int ci = blockIdx.x, co = blockIdx.y, Ci = Ca + Cb, kk = k * k, pad = k / 2;
  float acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.0f;
  const int64_t tot = (int64_t)batch * Ho * Ho;
  for (int64_t q = threadIdx.x; q < tot; q += 256) {
    const int b = (int)(q / ((int64_t)Ho * Ho)), p = (int)(q % ((int64_t)Ho * Ho));
    const int oy = p / Ho, ox = p % Ho;
    const float g = G[(((int64_t)b * Co + co) * Ho + oy) * Ho + ox];
    for (int dy = 0; dy < k; ++dy)
      for (int dx = 0; dx < k; ++dx)
        acc[dy * k + dx] = fmaf(g, in_at(A, Ca, B, Cb, H, b, ci, oy * stride + dy - pad,
                                         ox * stride + dx - pad), acc[dy * k + dx]);
    acc[9] += g;
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    float v = acc[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (l == 0) red[t][w] = v;
  }
  __syncthreads();
  if (threadIdx.x < kk) {
    const int t = threadIdx.x;
    gw[((int64_t)co * Ci + ci) * kk + t] = (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  }
  if (ci == 0 && threadIdx.x == 0)
    gw[(int64_t)Co * Ci * kk + co] = (red[9][0] + red[9][1]) + (red[9][2] + red[9][3]);
}

// Weight gradient as a GEMM on the matrix cores (FP32 MFMA 16x16x4):
// dW[co][j] = sum over the output pixels q of G[co][q] X[j][q], with
// j = ci k^2 + tap and X the layer's input gathered at tap (the columns of
// an im2col matrix); column j = Ci k^2 (X = 1) gives the bias gradient.
// Block (c, jt): the pixels of chunk c, all output channels (16 NG), columns
// 64 jt..; each wave takes a quarter of the chunk's pixels and holds the
// whole 16 NG x 64 tile (NG x 4 products per step share the operands
// loaded for them); the four waves' sums are added in wave order in LDS and
// written to part[c][co][j], which k_wgrad_sum adds in chunk order (fixed
// order: reproducible bits).  Lane layout of the 16x16x4 product: A (16 x 4)
// row = lane & 15, k = lane >> 4; B (4 x 16) k = lane >> 4, column =
// lane & 15; D row 4 (lane >> 4) + r (r < 4), column lane & 15.
template <int NG>
__global__ void __launch_bounds__(256)
k_conv_bwd_weight_mfma(const float* __restrict__ G, int Co, int Ho, const float* __restrict__ A,
                       int Ca, const float* __restrict__ B, int Cb, int H, int k, int stride,
                       int64_t tot, int64_t chunk, float* __restrict__ part) {
  __shared__ float red[64 * NG * 16];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = l & 15, g = l >> 4;
  const int Ci = Ca + Cb, kk = k * k, J = Ci * kk, pad = k / 2;
  const int j0 = blockIdx.y * 64;
  // this lane's B columns j0 + 16 t + i: (input channel, tap), or the bias
  int cit[4], dyt[4], dxt[4];
  bool jw[4], jb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = j0 + 16 * t + i;
    jw[t] = j < J;
    jb[t] = j == J;
    const int tp = jw[t] ? j % kk : 0;
    cit[t] = jw[t] ? j / kk : 0;
    dyt[t] = tp / k;
    dxt[t] = tp % k;
  }
  // this wave's pixels: a quarter of the chunk (chunk is a multiple of 16)
  const int64_t sub = chunk / 4;
  const int64_t q0 = (int64_t)blockIdx.x * chunk + w * sub;
  const int64_t q1 = min(q0 + sub, tot);
  int64_t q = q0 + g;
  const int64_t HH = (int64_t)Ho * Ho;
  int b = (int)(q / HH);
  int rem = (int)(q % HH);
  int oy = rem / Ho, ox = rem % Ho;
  nnf4 acc[NG][4];
#pragma unroll
  for (int c = 0; c < NG; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[c][t] = nnf4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t p = q0; p < q1; p += 4) {
    const bool in = q < q1;
    float a[NG], x[4];
#pragma unroll
    for (int c = 0; c < NG; ++c) {
      const int co = 16 * c + i;
      a[c] = (in && co < Co) ? G[((int64_t)b * Co + co) * HH + (int64_t)oy * Ho + ox] : 0.0f;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x[t] = 0.0f;
      if (in) {
        if (jw[t])
          x[t] = in_at(A, Ca, B, Cb, H, b, cit[t], oy * stride + dyt[t] - pad,
                       ox * stride + dxt[t] - pad);
        else if (jb[t])
          x[t] = 1.0f;
      }
    }
#pragma unroll
    for (int c = 0; c < NG; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], x[t], acc[c][t], 0, 0, 0);
    q += 4;
    ox += 4;
    if (ox >= Ho) {   // Ho >= 4: at most one wrap per step
      ox -= Ho;
      if (++oy == Ho) { oy = 0; ++b; }
    }
  }
  // the four waves' sums, added in wave order
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww)
#pragma unroll
      for (int c = 0; c < NG; ++c)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float* d = &red[((c * 4 + t) * 4 + r) * 64 + l];
            *d = ww == 0 ? acc[c][t][r] : *d + acc[c][t][r];
          }
    __syncthreads();
  }
  if (w != 0) return;
  const int Jp = J + 1;
#pragma unroll
  for (int c = 0; c < NG; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = j0 + 16 * t + i;
      if (j >= Jp) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cr = 16 * c + 4 * g + r;
        if (cr < Co) part[((int64_t)blockIdx.x * Co + cr) * Jp + j] = red[((c * 4 + t) * 4 + r) * 64 + l];
      }
    }
}

// gw[co][j] = sum over the chunks in order of part[c][co][j] (j = J: the bias,
// stored after all weights).
__global__ void k_wgrad_sum(const float* __restrict__ part, int nch, int Co, int J,
                            float* __restrict__ gw) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int Jp = J + 1;
  if (idx >= (int64_t)Co * Jp) return;
  const int co = (int)(idx / Jp), j = (int)(idx % Jp);
  float s = 0.0f;
  for (int c = 0; c < nch; ++c) s += part[((int64_t)c * Co + co) * Jp + j];
  if (j < J) gw[(int64_t)co * J + j] = s;
  else gw[(int64_t)Co * J + co] = s;
}

__global__ void k_to_f32(const double* __restrict__ u, float* __restrict__ x, int64_t count,
                         const int32_t* __restrict__ gate) {
  if (gate && !*gate) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) x[i] = (float)u[i];
}
// out = clip(u + head, -OUT_BOUND, OUT_BOUND) (FP64).  The clip keeps the
// propagator bounded on states far from the training data (repeated
// application inside the coarse sweep); solutions of the equation stay well
// inside it.  Training uses the unclipped output.
constexpr double OUT_BOUND = 1.5;
__global__ void k_residual_out(const double* __restrict__ u, const float* __restrict__ h,
                               double* __restrict__ out, int64_t count,
                               const int32_t* __restrict__ gate) {
  if (gate && !*gate) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) out[i] = fmin(fmax(u[i] + (double)h[i], -OUT_BOUND), OUT_BOUND);
}
// MSE: dh = 2 (u + h - target)/count; per-block partial sums of squares
__global__ void k_mse(const double* __restrict__ u, const float* __restrict__ h,
                      const double* __restrict__ tgt, float* __restrict__ dh,
                      float* __restrict__ part, int64_t count) {
  __shared__ float red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float sq = 0.0f;
  if (i < count) {
    const float d = (float)(u[i] + (double)h[i] - tgt[i]);
    dh[i] = 2.0f * d / (float)count;
    sq = d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ void k_sum_parts(const float* __restrict__ part, int nparts, float scale,
                            float* __restrict__ out) {
  __shared__ float red[4];
  float s = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((red[0] + red[1]) + (red[2] + red[3])) * scale;
}

// Adam on the FP32 master weights, then the BF16 copy (round to nearest even).
__global__ void k_adam(float* __restrict__ wm, uint16_t* __restrict__ wb, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = wm[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  wm[i] = w;
  wb[i] = f2bf_rne(w);
}
__global__ void k_to_bf16(const float* __restrict__ wm, uint16_t* __restrict__ wb, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) wb[i] = f2bf_rne(wm[i]);
}

static inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// Parareal correction of one slice: U_{n+1} <- F_n + (g - G_old_n), G_old_n <- g,
// per-block partial sums of (U_{n+1}^{new} - U_{n+1}^{old})^2.  With
// predict != 0: U_{n+1} <- g, G_old_n <- g, no norm.
__global__ void k_pr_correct(double* __restrict__ Un1, const double* __restrict__ Fn,
                             double* __restrict__ Gn, const double* __restrict__ g, int64_t count,
                             double* __restrict__ part, int predict,
                             const int32_t* __restrict__ active) {
  __shared__ double red[4];
  if (active && !*active) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (i < count) {
    const double gv = g[i];
    if (predict) {
      Un1[i] = gv;
    } else {
      const double un = Fn[i] + (gv - Gn[i]);
      const double d = un - Un1[i];
      sq = d * d;
      Un1[i] = un;
    }
    Gn[i] = gv;
  }
  if (predict) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
// delta = sqrt(h^2 max_slices sum_blocks part) over the slices k..nslices-1
// (k = *kdev, 0 if kdev is null; part rows indexed by slice), fixed order; a
// NaN sets status bit 2.
__global__ void k_pr_delta(const double* __restrict__ part, int nb, int nslices, double h2,
                           double* __restrict__ delta, int32_t* __restrict__ status,
                           const int32_t* __restrict__ active, const int32_t* __restrict__ kdev) {
  if (threadIdx.x != 0) return;
  if (active && !*active) return;
  double mx = 0.0;
  bool bad = false;
  for (int sl = kdev ? *kdev : 0; sl < nslices; ++sl) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)sl * nb + b];
    if (!(s == s)) bad = true;
    mx = fmax(mx, s);
  }
  const double d = sqrt(h2 * mx);
  *delta = bad ? __builtin_nan("") : d;
  if (bad || d > 1e300) *status |= 2;
}

hipError_t pr_correct(double* Un1, const double* Fn, double* Gn, const double* g, int64_t count,
                      double* part, int predict, const int32_t* active, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_correct, dim3(blocks(count)), dim3(256), 0, s, Un1, Fn, Gn, g, count,
                     part, predict, active);
  return hipGetLastError();
}
hipError_t pr_delta(const double* part, int nb, int nslices, double h2, double* delta,
                    int32_t* status, const int32_t* active, hipStream_t s, const int32_t* kdev) {
  hipLaunchKernelGGL(k_pr_delta, dim3(1), dim3(64), 0, s, part, nb, nslices, h2, delta, status,
                     active, kdev);
  return hipGetLastError();
}
// The first corrected slice of iteration k = *kdev: U_{k+1} <- F_k (its
// G terms cancel: G(U_k) = G_old_k, slice k being final), with the per-block
// squares of the change in part row k.  Nothing when k >= nslices or the
// gate is off.
__global__ void k_pr_first(double* __restrict__ Ui, const double* __restrict__ Fi, int64_t P,
                           int nslices, double* __restrict__ part, int nb,
                           const int32_t* __restrict__ kdev, const int32_t* __restrict__ gate) {
  __shared__ double red[4];
  if (gate && !*gate) return;
  const int k = *kdev;
  if (k >= nslices) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sq = 0.0;
  if (i < P) {
    const double un = Fi[(int64_t)k * P + i];
    const double d = un - Ui[(int64_t)(k + 1) * P + i];
    sq = d * d;
    Ui[(int64_t)(k + 1) * P + i] = un;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)k * nb + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
hipError_t pr_first(double* Ui, const double* Fi, int64_t P, int nslices, double* part, int nb,
                    const int32_t* kdev, const int32_t* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_pr_first, dim3(blocks(P)), dim3(256), 0, s, Ui, Fi, P, nslices, part, nb,
                     kdev, gate);
  return hipGetLastError();
}
// gates[sl] = *live && sl > *kdev for the slices of one correction sweep
__global__ void k_slice_gates(const int32_t* __restrict__ live, const int32_t* __restrict__ kdev,
                              int nslices, int32_t* __restrict__ gates) {
  const int sl = blockIdx.x * 256 + threadIdx.x;
  if (sl < nslices) gates[sl] = (*live && sl > *kdev) ? 1 : 0;
}
hipError_t slice_gates(const int32_t* live, const int32_t* kdev, int nslices, int32_t* gates,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_slice_gates, dim3(blocks(nslices)), dim3(256), 0, s, live, kdev, nslices,
                     gates);
  return hipGetLastError();
}
// G_out <- g for masked slices (all when mask is null)
__global__ void k_masked_copy(double* __restrict__ dst, const double* __restrict__ src,
                              const uint8_t* __restrict__ mask, int64_t P, int nslices,
                              int64_t slice_base, const int32_t* __restrict__ gate) {
  if (gate && !*gate) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P * nslices) return;
  const int sl = (int)(i / P);
  if (mask && !mask[slice_base + sl]) return;
  dst[i] = src[i];
}
hipError_t masked_copy(double* dst, const double* src, const uint8_t* mask, int64_t P, int nslices,
                       int64_t slice_base, hipStream_t s, const int32_t* gate) {
  hipLaunchKernelGGL(k_masked_copy, dim3(blocks(P * nslices)), dim3(256), 0, s, dst, src, mask, P,
                     nslices, slice_base, gate);
  return hipGetLastError();
}

// ---------------------------------------------------------------- host launchers
hipError_t nn_forward(const uint16_t* w, const double* u, int batch, int n, float* ws,
                      const NNPlan& p, double* out, hipStream_t s, const int32_t* gate,
                      const double* base) {
  const int64_t cnt = (int64_t)batch * n * n;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_fwd<16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_to_f32, dim3(blocks(cnt)), dim3(256), 0, s, u, ws + p.x0, cnt, gate);
  for (int l = 0; l < NN_LAYERS; ++l) {
    const NNLayer& L = kNNLayers[l];
    const float* A;
    int Ca, Cb = 0;
    const float* B = nullptr;
    if (L.cat >= 0) {
      A = ws + p.act[L.cat];
      Ca = kNNLayers[L.cat].c_out;
      B = ws + p.act[l - 1];
      Cb = kNNLayers[l - 1].c_out;
    } else {
      A = l == 0 ? ws + p.x0 : ws + p.act[l - 1];
      Ca = L.c_in;
    }
    const int H = in_size(l, n), Ho = out_size(l, n);
    const uint16_t* wl = w + nn_param_offset(l);
    if (L.c_out % 16 == 0 && L.c_out <= 64) {
      const dim3 grid((unsigned)((int64_t)Ho * Ho + 63) / 64, batch);
      switch (L.c_out / 16) {
        case 1: hipLaunchKernelGGL(k_conv_fwd_mfma<1>, grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,
                                   ws + p.act[l], Ho, L.k, L.stride, L.act, gate); break;
        case 2: hipLaunchKernelGGL(k_conv_fwd_mfma<2>, grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,
                                   ws + p.act[l], Ho, L.k, L.stride, L.act, gate); break;
        case 3: hipLaunchKernelGGL(k_conv_fwd_mfma<3>, grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,
                                   ws + p.act[l], Ho, L.k, L.stride, L.act, gate); break;
        default: hipLaunchKernelGGL(k_conv_fwd_mfma<4>, grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,
                                    ws + p.act[l], Ho, L.k, L.stride, L.act, gate); break;
      }
    } else if (L.c_out >= 16) {
      const size_t lds = (size_t)16 * L.c_in * L.k * L.k * sizeof(float);
      hipLaunchKernelGGL(k_conv_fwd<16>, dim3(blocks((int64_t)Ho * Ho), L.c_out / 16, batch),
                         dim3(256), lds, s, A, Ca, B, Cb, H, wl, ws + p.act[l], L.c_out, Ho, L.k,
                         L.stride, L.act, gate);
    } else {
      const size_t lds = (size_t)L.c_in * L.k * L.k * sizeof(float);
      hipLaunchKernelGGL(k_conv_fwd<1>, dim3(blocks((int64_t)Ho * Ho), L.c_out, batch), dim3(256),
                         lds, s, A, Ca, B, Cb, H, wl, ws + p.act[l], L.c_out, Ho, L.k, L.stride,
                         L.act, gate);
    }
  }
  if (out)
    hipLaunchKernelGGL(k_residual_out, dim3(blocks(cnt)), dim3(256), 0, s, base ? base : u,
                       ws + p.act[NN_LAYERS - 1], out, cnt, gate);
  return hipGetLastError();
}

size_t nn_forward_floats(int batch, int n) {
  // the forward pass touches x0 and the activations, which come first in
  // the plan; the gradient buffers start right after them
  return nn_plan(batch, n).grad[0];
}

hipError_t nn_static_scratch(float** out) {
  static std::mutex mu;
  static float* ptr[64] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = (float*)p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

hipError_t nn_train_step(const uint16_t* w, const double* u, const double* tgt, int batch, int n,
                         float* ws, const NNPlan& p, float* grad, float* loss, hipStream_t s) {
  hipError_t e = nn_forward(w, u, batch, n, ws, p, nullptr, s);
  if (e != hipSuccess) return e;
  const int64_t cnt = (int64_t)batch * n * n;
  const int nb = (int)blocks(cnt);
  if (nb > 4096) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, u, ws + p.act[NN_LAYERS - 1], tgt,
                     ws + p.grad[NN_LAYERS - 1], ws + p.part, cnt);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, ws + p.part, nb, 1.0f / (float)cnt, loss);
  // gradient buffers of skip layers receive two contributions: the decoder
  // (written first, backward order) and the next encoder layer (added).
  bool written[NN_LAYERS] = {false};
  written[NN_LAYERS - 1] = true;
  for (int l = NN_LAYERS - 1; l >= 0; --l) {
    const NNLayer& L = kNNLayers[l];
    const int H = in_size(l, n), Ho = out_size(l, n);
    float* G = ws + p.grad[l];
    if (L.act) {
      const int64_t c = (int64_t)batch * L.c_out * Ho * Ho;
      hipLaunchKernelGGL(k_act_bwd, dim3(blocks(c)), dim3(256), 0, s, G, ws + p.act[l], c);
    }
    const float* A;
    const float* B = nullptr;
    int Ca, Cb = 0;
    float* dA = nullptr;
    int accA = 0;
    if (L.cat >= 0) {
      A = ws + p.act[L.cat];
      Ca = kNNLayers[L.cat].c_out;
      B = ws + p.act[l - 1];
      Cb = kNNLayers[l - 1].c_out;
      dA = ws + p.grad[L.cat];
      accA = written[L.cat] ? 1 : 0;
      written[L.cat] = true;
    } else {
      A = l == 0 ? ws + p.x0 : ws + p.act[l - 1];
      Ca = L.c_in;
      if (l > 0) {
        dA = ws + p.grad[l - 1];
        accA = written[l - 1] ? 1 : 0;
        written[l - 1] = true;
      }
    }
    const uint16_t* wl = w + nn_param_offset(l);
    float* gw = grad + nn_param_offset(l);
    {
      const int64_t tot = (int64_t)batch * Ho * Ho;
      const int nch = wgrad_chunks(tot), J = L.c_in * L.k * L.k;
      const dim3 grid(nch, (J + 1 + 63) / 64);
      const int64_t len = wgrad_chunk_len(tot);
      switch ((L.c_out + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_conv_bwd_weight_mfma<1>, grid, dim3(256), 0, s, G, L.c_out, Ho,
                                   A, Ca, B, Cb, H, L.k, L.stride, tot, len, ws + p.wpart); break;
        case 2: hipLaunchKernelGGL(k_conv_bwd_weight_mfma<2>, grid, dim3(256), 0, s, G, L.c_out, Ho,
                                   A, Ca, B, Cb, H, L.k, L.stride, tot, len, ws + p.wpart); break;
        case 3: hipLaunchKernelGGL(k_conv_bwd_weight_mfma<3>, grid, dim3(256), 0, s, G, L.c_out, Ho,
                                   A, Ca, B, Cb, H, L.k, L.stride, tot, len, ws + p.wpart); break;
        default: hipLaunchKernelGGL(k_conv_bwd_weight_mfma<4>, grid, dim3(256), 0, s, G, L.c_out,
                                    Ho, A, Ca, B, Cb, H, L.k, L.stride, tot, len, ws + p.wpart); break;
      }
      hipLaunchKernelGGL(k_wgrad_sum, dim3(blocks((int64_t)L.c_out * (J + 1))), dim3(256), 0, s,
                         ws + p.wpart, nch, L.c_out, J, gw);
    }
    if (l == 0) continue;
    const int CIB = (L.c_in % 16 == 0) ? 16 : 1;
    const size_t lds = (size_t)L.c_out * CIB * L.k * L.k * sizeof(float);
    if (CIB == 16)
      hipLaunchKernelGGL(k_conv_bwd_data<16>, dim3(blocks((int64_t)H * H), L.c_in / 16, batch),
                         dim3(256), lds, s, G, L.c_out, Ho, wl, Ca, Cb, H, L.k, L.stride, dA, accA,
                         ws + p.tmp);
    else
      hipLaunchKernelGGL(k_conv_bwd_data<1>, dim3(blocks((int64_t)H * H), L.c_in, batch), dim3(256),
                         lds, s, G, L.c_out, Ho, wl, Ca, Cb, H, L.k, L.stride, dA, accA, ws + p.tmp);
    if (L.cat >= 0) {
      // the upsampled part: gradient of layer l-1's output (first writer in
      // backward order for that buffer)
      const int64_t c = (int64_t)batch * Cb * (H / 2) * (H / 2);
      hipLaunchKernelGGL(k_up_bwd, dim3(blocks(c)), dim3(256), 0, s, ws + p.tmp, ws + p.grad[l - 1],
                         Cb, H, batch);
      written[l - 1] = true;
    }
  }
  return hipGetLastError();
}

hipError_t nn_adam(float* wm, uint16_t* wb, float* m, float* v, const float* g, int64_t count,
                   float lr, float b1, float b2, float eps, int t, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(blocks(count)), dim3(256), 0, s, wm, wb, m, v, g, count, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t nn_to_bf16(const float* wm, uint16_t* wb, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(count)), dim3(256), 0, s, wm, wb, count);
  return hipGetLastError();
}

}  // namespace chk
