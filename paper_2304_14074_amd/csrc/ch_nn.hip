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

// Tile count (16-pixel tiles times samples) from which the convolutions take
// two tiles a block.
constexpr int64_t kNNTwoTiles = 2048;
// Tile count below which the forward takes 16 waves a block (small grids at
// a small batch: the contraction split over more waves shortens each one's).
constexpr int64_t kNNWideTiles = 256;

// Chunks of the weight-gradient GEMM: a chunk is a band of R output rows of
// one sample, R >= 512 / Ho (at least 512 pixels where the map has them) and
// R >= batch Ho / 256 (at most about 256 chunks), fewer rows while the band's
// staged input would pass kWgradLds bytes; a single row may take up to
// kWgradLdsMax.  64 consecutive columns j = ci k^2 + tap span at
// most (62 + k^2) / k^2 + 1 channels: 8 for 3 x 3 layers, 64 for 1 x 1.
constexpr size_t kWgradLds = 96 * 1024, kWgradLdsMax = 150 * 1024;
static int wgrad_stage_channels(const NNLayer& L) {
  const int kk = L.k * L.k;
  return std::min(L.c_in, (62 + kk) / kk + 1);
}
static size_t wgrad_lds_bytes(const NNLayer& L, int Ho, int R) {
  const size_t rows = (size_t)(R - 1) * L.stride + L.k, cols = (size_t)(Ho - 1) * L.stride + L.k;
  return (size_t)wgrad_stage_channels(L) * rows * cols * sizeof(float);
}
static int wgrad_rows(const NNLayer& L, int batch, int Ho) {
  int R = std::max((512 + Ho - 1) / Ho, (int)(((int64_t)batch * Ho + 255) / 256));
  R = std::min(R, Ho);
  while (R > 1 && wgrad_lds_bytes(L, Ho, R) > kWgradLds) --R;
  return R;
}
static int64_t wgrad_chunks(const NNLayer& L, int batch, int Ho) {
  const int R = wgrad_rows(L, batch, Ho);
  return (int64_t)batch * ((Ho + R - 1) / R);
}

// Packed weights (FP32, from the BF16 parameters), one block per layer:
// forward layout  Wf[tap][ci][i][c] = W[16c + i][ci][tap]   (c < ceil(c_out/16))
// input-gradient  Wd[tap][co][i][c] = W[co][16c + i][tap]   (c < ceil(c_in/16))
// (zero where the channel is past c_out or c_in), so the 16 lanes of one
// MFMA operand row read one contiguous run.
static int64_t pack_layer_floats(int l, bool fwd) {
  const NNLayer& L = kNNLayers[l];
  const int kk = L.k * L.k;
  return fwd ? (int64_t)kk * L.c_in * 16 * ((L.c_out + 15) / 16)
             : (int64_t)kk * L.c_out * 16 * ((L.c_in + 15) / 16);
}
static int64_t pack_offset(int layer, bool fwd) {
  int64_t s = 0;
  for (int l = 0; l < layer; ++l) s += (pack_layer_floats(l, fwd) + 63) / 64 * 64;
  return s;
}
static int64_t pack_floats(bool fwd) { return pack_offset(NN_LAYERS, fwd); }

// Workspace layout (floats): x0 | for each layer: act | forward-packed weights | for each
// layer: grad | tmp | loss partials | weight-gradient partials | input-gradient-packed weights
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
  p.wpf = take((size_t)pack_floats(true));
  for (int l = 0; l < NN_LAYERS; ++l) {
    const int s = out_size(l, n);
    p.grad[l] = take((size_t)batch * kNNLayers[l].c_out * s * s);
  }
  p.tmp = take(maxin);
  p.part = take(4096);
  size_t wp = 0;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const NNLayer& L = kNNLayers[l];
    wp = std::max(wp, (size_t)wgrad_chunks(L, batch, out_size(l, n)) * L.c_out *
                          (L.c_in * L.k * L.k + 1));
  }
  p.wpart = take(wp);
  p.wpd = take((size_t)pack_floats(false));
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

// NG consecutive floats at p (p aligned to 4 NG bytes, as the packed rows are).
template <int NG>
__device__ __forceinline__ void ld_row(const float* __restrict__ p, float (&v)[NG]) {
  if constexpr (NG % 4 == 0) {
#pragma unroll
    for (int q = 0; q < NG / 4; ++q) {
      const float4 x = reinterpret_cast<const float4*>(p)[q];
      v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
  } else if constexpr (NG % 2 == 0) {
#pragma unroll
    for (int q = 0; q < NG / 2; ++q) {
      const float2 x = reinterpret_cast<const float2*>(p)[q];
      v[2 * q] = x.x; v[2 * q + 1] = x.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < NG; ++c) v[c] = p[c];
  }
}

// Every layer's weights into one packed layout (forward or input gradient),
// one thread per packed float (the padding of each layer's block included).
struct PackTab {
  int64_t woff[NN_LAYERS], poff[NN_LAYERS + 1];   // BF16 and packed offsets
  int co[NN_LAYERS], ci[NN_LAYERS], kk[NN_LAYERS];
};
__global__ void k_pack_weights(const uint16_t* __restrict__ w, float* __restrict__ out, PackTab t,
                               int fwd, const int32_t* __restrict__ gate) {
  if (gate && !*gate) return;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= t.poff[NN_LAYERS]) return;
  int l = 0;
  while (l + 1 < NN_LAYERS && d >= t.poff[l + 1]) ++l;
  const int64_t e = d - t.poff[l];
  const int Co = t.co[l], Ci = t.ci[l], kk = t.kk[l];
  const int NG = fwd ? (Co + 15) / 16 : (Ci + 15) / 16, M = fwd ? Ci : Co;
  const int c = (int)(e % NG), i = (int)((e / NG) % 16);
  const int64_t rest = e / (16 * NG);
  if (rest >= (int64_t)kk * M) {   // padding
    out[d] = 0.0f;
    return;
  }
  const int tap = (int)(rest / M), r = (int)(rest % M);
  const int co = fwd ? 16 * c + i : r, ci = fwd ? r : 16 * c + i;
  out[d] = (co < Co && ci < Ci) ? bf2f(w[t.woff[l] + ((int64_t)co * Ci + ci) * kk + tap]) : 0.0f;
}

// Convolutions on the matrix cores (FP32 MFMA 16x16x4, FP32 accumulation):
// implicit GEMMs whose contraction runs over pairs (tap, 16 channels).  A
// block takes T tiles of 16 pixels of one sample and every output column
// (16 NG); its four waves deal the pairs among themselves in turn, each
// keeps its own sums, and the waves' sums are added in wave order in LDS
// (fixed order: reproducible bits).  Per pair a lane issues its 4 T gathers
// and its 4 NG weight loads together, then the 4 T NG products (each weight
// serves the T tiles).  Lane layout of the 16x16x4 product: A (16 x 4) row
// = lane & 15, k = lane >> 4; B (4 x 16) k = lane >> 4, column = lane & 15;
// D row 4 (lane >> 4) + r (r < 4), column lane & 15.
typedef float nnf4 __attribute__((ext_vector_type(4)));

// The waves' sums of a block of W waves (M accumulators a lane): waves
// 1..W-1 park theirs in red, wave 0 adds them to its own in wave order.
// Returns false on waves 1..W-1.
template <int M, int W = 4>
__device__ __forceinline__ bool ks_reduce(nnf4 (&acc)[M], float* red, int wv, int l) {
  if (wv > 0)
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(((wv - 1) * M + m) * 4 + r) * 64 + l] = acc[m][r];
  __syncthreads();
  if (wv > 0) return false;
#pragma unroll 1
  for (int ww = 0; ww < W - 1; ++ww)
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][r] += red[((ww * M + m) * 4 + r) * 64 + l];
  return true;
}

// Forward: Y[co][p] = act(bias[co] + sum over (ci, tap) of W[co][ci][tap]
// X[ci][p + tap]), the input X either A alone or the concatenation [A (Ca
// channels), up2(B) (Cb channels)] with Ca a multiple of 16 when Cb > 0.
// A operand: 16 pixels x 4 channels gathered at the tap; B operands: 4
// channels x 16 output channels of the weights in the forward packed layout
// (wf, this layer's block; w for the BF16 biases); c_out <= 16 NG.  W waves
// a block (16 on small grids: more waves share the contraction).
template <int NG, int T, int W = 4>
__global__ void __launch_bounds__(64 * W)
k_conv_fwd_mfma(const float* __restrict__ A, int Ca, const float* __restrict__ B, int Cb, int H,
                const uint16_t* __restrict__ w, const float* __restrict__ wf,
                float* __restrict__ Y, int Co, int Ho, int k, int stride, int act,
                const int32_t* __restrict__ gate) {
  __shared__ float red[(W - 1) * T * NG * 4 * 64];
  if (gate && !*gate) return;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, b = blockIdx.y;
  const int i = l & 15, g = l >> 4;
  const int Ci = Ca + Cb, kk = k * k, pad = k / 2, nc = (Ci + 15) >> 4, items = kk * nc;
  const int HH = Ho * Ho, Hh = H >> 1;
  const int pbase = blockIdx.x * 16 * T;
  int oy[T], ox[T];
  bool pin[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {           // this lane's A-operand pixel of tile t
    const int pa = pbase + 16 * t + i;
    pin[t] = pa < HH;
    oy[t] = pin[t] ? pa / Ho : 0;
    ox[t] = pin[t] ? pa % Ho : 0;
  }
  nnf4 acc[T * NG];
#pragma unroll
  for (int m = 0; m < T * NG; ++m) acc[m] = nnf4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = wv; it < items; it += W) {
    const int tap = it / nc, c16 = it - tap * nc;
    const int dy = tap / k, dx = tap - dy * k;
    const int ci0 = 16 * c16 + g;
    const bool lowA = 16 * c16 < Ca;
    float x[T][4], wt[4][NG];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int yy = oy[t] * stride + dy - pad, xx = ox[t] * stride + dx - pad;
      const bool v = pin[t] && yy >= 0 && yy < H && xx >= 0 && xx < H;
      const float* src;
      int plane;
      if (lowA) {
        src = A + ((int64_t)b * Ca + ci0) * H * H + (v ? yy * H + xx : 0);
        plane = H * H;
      } else {
        src = B + ((int64_t)b * Cb + ci0 - Ca) * Hh * Hh + (v ? (yy >> 1) * Hh + (xx >> 1) : 0);
        plane = Hh * Hh;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) x[t][u] = (v && ci0 + 4 * u < Ci) ? src[4 * u * plane] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (ci0 + 4 * u < Ci) {
        ld_row<NG>(wf + ((int64_t)(tap * Ci + ci0 + 4 * u) * 16 + i) * NG, wt[u]);
      } else {
#pragma unroll
        for (int c = 0; c < NG; ++c) wt[u][c] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < NG; ++c)
          acc[t * NG + c] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(x[t][u], wt[u][c], acc[t * NG + c], 0, 0, 0);
  }
  if (!ks_reduce<T * NG, W>(acc, red, wv, l)) return;
  const uint16_t* bias = w + (int64_t)Co * Ci * kk;
#pragma unroll
  for (int c = 0; c < NG; ++c) {
    const int co = 16 * c + i;
    if (co >= Co) continue;
    const float bv = bf2f(bias[co]);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = pbase + 16 * t + 4 * g + r;
        if (pr >= HH) continue;
        float y = acc[t * NG + c][r] + bv;
        if (act) y = y > 0.0f ? y : kSlope * y;
        Y[((int64_t)b * Co + co) * HH + pr] = y;
      }
  }
}

// G <- G * act'(y) in place (y the layer output; LeakyReLU is monotone, so
// the sign of y is the sign of the pre-activation).
__global__ void k_act_bwd(float* __restrict__ G, const float* __restrict__ Y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) G[i] = Y[i] > 0.0f ? G[i] : kSlope * G[i];
}

// Gradient w.r.t. the (concatenated) input: dIn[ci][p] = sum over the pairs
// (co, tap) of W[co][ci][tap] G[co][q], q the output pixel that the tap joins
// to input pixel p (a zero where there is none: the border, or a tap that the
// stride skips; stride is 1 or 2).  A operand: 16 input pixels x 4 output
// channels gathered from G; B operands: 4 output channels x 16 input
// channels of the weights in the input-gradient packed layout (wd, this
// layer's block); c_in = Ca + Cb = 16 NG.  Channels < Ca go to
// dA (added when accA), the rest to dBf at full resolution (reduced later).
template <int NG, int T>
__global__ void __launch_bounds__(256)
k_conv_bwd_data_mfma(const float* __restrict__ G, int Co, int Ho, const float* __restrict__ wd,
                     int Ca, int Cb, int H, int k, int stride, float* __restrict__ dA, int accA,
                     float* __restrict__ dBf) {
  constexpr int Ci = 16 * NG;
  __shared__ float red[3 * T * NG * 4 * 64];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, b = blockIdx.y;
  const int i = l & 15, g = l >> 4;
  const int kk = k * k, pad = k / 2, sh = stride == 2 ? 1 : 0, nc = (Co + 15) >> 4;
  const int items = kk * nc, HH = H * H, HoHo = Ho * Ho;
  const int pbase = blockIdx.x * 16 * T;
  int y[T], x[T];
  bool pin[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {           // this lane's A-operand pixel of tile t
    const int pa = pbase + 16 * t + i;
    pin[t] = pa < HH;
    y[t] = pin[t] ? pa / H : 0;
    x[t] = pin[t] ? pa % H : 0;
  }
  nnf4 acc[T * NG];
#pragma unroll
  for (int m = 0; m < T * NG; ++m) acc[m] = nnf4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = wv; it < items; it += 4) {
    const int tap = it / nc, c16 = it - tap * nc;
    const int dy = tap / k, dx = tap - dy * k;
    const int co0 = 16 * c16 + g;
    float gv[T][4], wt[4][NG];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int ty = y[t] + pad - dy, tx = x[t] + pad - dx;
      const int oy = ty >> sh, ox = tx >> sh;
      const bool v = pin[t] && ty >= 0 && tx >= 0 && !(ty & sh) && !(tx & sh) && oy < Ho && ox < Ho;
      const float* src = G + ((int64_t)b * Co + co0) * HoHo + (v ? oy * Ho + ox : 0);
#pragma unroll
      for (int u = 0; u < 4; ++u) gv[t][u] = (v && co0 + 4 * u < Co) ? src[4 * u * HoHo] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (co0 + 4 * u < Co) {
        ld_row<NG>(wd + ((int64_t)(tap * Co + co0 + 4 * u) * 16 + i) * NG, wt[u]);
      } else {
#pragma unroll
        for (int c = 0; c < NG; ++c) wt[u][c] = 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int c = 0; c < NG; ++c)
          acc[t * NG + c] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(gv[t][u], wt[u][c], acc[t * NG + c], 0, 0, 0);
  }
  if (!ks_reduce<T * NG>(acc, red, wv, l)) return;
#pragma unroll
  for (int c = 0; c < NG; ++c) {
    const int ci = 16 * c + i;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = pbase + 16 * t + 4 * g + r;
        if (pr >= HH) continue;
        const float v = acc[t * NG + c][r];
        if (ci < Ca) {
          float* d = dA + ((int64_t)b * Ca + ci) * HH + pr;
          *d = accA ? *d + v : v;
        } else {
          dBf[((int64_t)b * Cb + (ci - Ca)) * HH + pr] = v;
        }
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

// Weight gradient as a GEMM on the matrix cores: dW[co][j] = sum over the
// output pixels q of G[co][q] X[j][q], with j = ci k^2 + tap and X the
// layer's input gathered at tap (the columns of an im2col matrix); column
// j = Ci k^2 (X = 1) gives the bias gradient.  A operand: 16 output channels
// x 4 pixels of G; B operand: 4 pixels x 16 columns.  Block (c, jt): chunk c
// (R output rows of one sample), every output channel (16 NG), columns
// 64 jt..  The block first stages the input that those columns read over the
// band (their channels, the band's input rows and every column, zero outside
// the map, the upsampled part of a concatenated input expanded) in LDS with
// coalesced loads; the im2col values then come from LDS.  Each wave takes a
// quarter of the band's pixels, 16 per pass, and holds the whole 16 NG x 64
// tile; the four waves' sums are added in wave order in LDS and written to
// part[c][co][j], which k_wgrad_sum adds in chunk order.
template <int NG>
__global__ void __launch_bounds__(256)
k_conv_bwd_weight_mfma(const float* __restrict__ G, int Co, int Ho, const float* __restrict__ A,
                       int Ca, const float* __restrict__ B, int Cb, int H, int k, int stride,
                       int R, int nband, float* __restrict__ part) {
  extern __shared__ float xs[];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = l & 15, g = l >> 4;
  const int Ci = Ca + Cb, kk = k * k, J = Ci * kk, pad = k / 2, Hh = H >> 1;
  const int b = blockIdx.x / nband, r0 = (blockIdx.x % nband) * R;
  const int nr = min(R, Ho - r0);                      // output rows of this band
  const int j0 = blockIdx.y * 64;
  const int ci_lo = j0 < J ? j0 / kk : 0;
  const int nch = j0 < J ? min(Ci - 1, (j0 + 63) / kk) - ci_lo + 1 : 0;
  const int rows = (nr - 1) * stride + k, cols = (Ho - 1) * stride + k;
  const int plane = rows * cols, ybase = r0 * stride - pad;
  // stage: xs[c][rr][cc] = input (ci_lo + c, ybase + rr, cc - pad)
  for (int idx = threadIdx.x; idx < nch * plane; idx += 256) {
    const int c = idx / plane, rem = idx - c * plane, rr = rem / cols, cc = rem - rr * cols;
    const int y = ybase + rr, x = cc - pad, ci = ci_lo + c;
    float v = 0.0f;
    if (y >= 0 && y < H && x >= 0 && x < H)
      v = ci < Ca ? A[(((int64_t)b * Ca + ci) * H + y) * H + x]
                  : B[(((int64_t)b * Cb + (ci - Ca)) * Hh + (y >> 1)) * Hh + (x >> 1)];
    xs[idx] = v;
  }
  // this lane's B columns j0 + 16 t + i: its offset in the staged input (the
  // channel's plane and the tap), or the bias
  int xo[4];
  bool jw[4], jb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = j0 + 16 * t + i;
    jw[t] = j < J;
    jb[t] = j == J;
    const int ci = jw[t] ? j / kk : ci_lo, tp = jw[t] ? j % kk : 0;
    xo[t] = (ci - ci_lo) * plane + (tp / k) * cols + tp % k;
  }
  __syncthreads();
  // this wave's pixels: a quarter of the band's, q = oy_rel Ho + ox
  const int P = nr * Ho, sub = (P + 63) / 64 * 16;
  const int q0 = w * sub, q1 = min(q0 + sub, P);
  int q = q0 + g, oy = q / Ho, ox = q % Ho;
  const float* Gb = G + ((int64_t)b * Co * Ho + r0) * Ho;   // (b, co = 0, row r0)
  const int64_t HH = (int64_t)Ho * Ho;
  nnf4 acc[NG][4];
#pragma unroll
  for (int c = 0; c < NG; ++c)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[c][t] = nnf4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int p = q0; p < q1; p += 16) {
    float a[4][NG], x[4][4];
    bool ain[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool in = q < q1;
      ain[s] = in;
      const int gq = in ? oy * Ho + ox : 0;
#pragma unroll
      for (int c = 0; c < NG; ++c) {
        const int co = 16 * c + i;
        a[s][c] = Gb[(int64_t)(co < Co ? co : 0) * HH + gq];
      }
      const int xq = in ? oy * stride * cols + ox * stride : 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) x[s][t] = xs[xo[t] + xq];
      q += 4;
      ox += 4;
      while (ox >= Ho) {
        ox -= Ho;
        ++oy;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < NG; ++c) {
        const float av = (ain[s] && 16 * c + i < Co) ? a[s][c] : 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float xb = jw[t] ? x[s][t] : (jb[t] ? 1.0f : 0.0f);
          acc[c][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, xb, acc[c][t], 0, 0, 0);
        }
      }
  }
  // the four waves' sums, added in wave order (the staged input is no longer
  // read: its LDS holds them)
  __syncthreads();
  float* red = xs;
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

// gw[co][j] = sum over the chunks of part[c][co][j] (j = J: the bias, stored
// after all weights).  A block takes 64 consecutive outputs; its four waves
// sum a quarter of the chunks each, in chunk order (eight loads issued
// together), and the quarters are added in order.
__global__ void __launch_bounds__(256)
k_wgrad_sum(const float* __restrict__ part, int nch, int Co, int J, float* __restrict__ gw) {
  __shared__ float qs[3][64];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + l;
  const int Jp = J + 1;
  const int64_t tot = (int64_t)Co * Jp;
  const int quarter = (nch + 3) / 4, c0 = w * quarter, c1 = min(nch, c0 + quarter);
  float s = 0.0f;
  if (idx < tot) {
    const float* src = part + idx;            // part[c][co][j] = part[c * Co * Jp + idx]
    int c = c0;
    for (; c + 8 <= c1; c += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(c + u) * tot];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < c1; ++c) s += src[(int64_t)c * tot];
  }
  if (w > 0) qs[w - 1][l] = s;
  __syncthreads();
  if (w > 0 || idx >= tot) return;
  s = ((s + qs[0][l]) + qs[1][l]) + qs[2][l];
  const int co = (int)(idx / Jp), j = (int)(idx % Jp);
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
static hipError_t pack_weights(const uint16_t* w, float* out, bool fwd, hipStream_t s,
                               const int32_t* gate) {
  PackTab t;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const NNLayer& L = kNNLayers[l];
    t.woff[l] = nn_param_offset(l);
    t.poff[l] = pack_offset(l, fwd);
    t.co[l] = L.c_out;
    t.ci[l] = L.c_in;
    t.kk[l] = L.k * L.k;
  }
  t.poff[NN_LAYERS] = pack_floats(fwd);
  hipLaunchKernelGGL(k_pack_weights, dim3(blocks(t.poff[NN_LAYERS])), dim3(256), 0, s, w, out, t,
                     fwd ? 1 : 0, gate);
  return hipGetLastError();
}

hipError_t nn_pack_forward(const uint16_t* w, float* ws, const NNPlan& p, hipStream_t s,
                           const int32_t* gate) {
  return pack_weights(w, ws + p.wpf, true, s, gate);
}

hipError_t nn_forward(const uint16_t* w, const double* u, int batch, int n, float* ws,
                      const NNPlan& p, double* out, hipStream_t s, const int32_t* gate,
                      const double* base, bool pack) {
  const int64_t cnt = (int64_t)batch * n * n;
  if (pack) {
    const hipError_t e = nn_pack_forward(w, ws, p, s, gate);
    if (e != hipSuccess) return e;
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
    const float* wf = ws + p.wpf + pack_offset(l, true);
    // the concatenated input's first part fills whole 16-channel pairs
    if ((Cb > 0 && Ca % 16) || L.c_out > 64) return hipErrorInvalidValue;
    // two 16-pixel tiles a block (each weight load serves both) once the
    // grid has work for every CU with them
    const int64_t tiles = ((int64_t)Ho * Ho + 15) / 16;
    const int T = tiles * batch >= kNNTwoTiles ? 2 : 1;
    // fewer tiles than kNNWideTiles: 16 waves a block share the contraction
    const bool wide = tiles * batch < kNNWideTiles;
    const dim3 grid((unsigned)((tiles + T - 1) / T), batch);
#define CH_FWD(NG)                                                                            \
  if (T == 2)                                                                                  \
    hipLaunchKernelGGL((k_conv_fwd_mfma<NG, 2>), grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,   \
                       wf, ws + p.act[l], L.c_out, Ho, L.k, L.stride, L.act, gate);            \
  else if (wide)                                                                               \
    hipLaunchKernelGGL((k_conv_fwd_mfma<NG, 1, 16>), grid, dim3(1024), 0, s, A, Ca, B, Cb, H,  \
                       wl, wf, ws + p.act[l], L.c_out, Ho, L.k, L.stride, L.act, gate);        \
  else                                                                                         \
    hipLaunchKernelGGL((k_conv_fwd_mfma<NG, 1>), grid, dim3(256), 0, s, A, Ca, B, Cb, H, wl,   \
                       wf, ws + p.act[l], L.c_out, Ho, L.k, L.stride, L.act, gate)
    switch ((L.c_out + 15) / 16) {
      case 1: CH_FWD(1); break;
      case 2: CH_FWD(2); break;
      case 3: CH_FWD(3); break;
      default: CH_FWD(4); break;
    }
#undef CH_FWD
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
  if (e == hipSuccess) e = pack_weights(w, ws + p.wpd, false, s, nullptr);
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
      const int J = L.c_in * L.k * L.k, R = wgrad_rows(L, batch, Ho);
      const int nband = (Ho + R - 1) / R;
      const int64_t nch = (int64_t)batch * nband;
      // the reduction reuses the staging LDS: at least 64 NG 16 floats
      const size_t lds = std::max(wgrad_lds_bytes(L, Ho, R),
                                  (size_t)64 * 16 * ((L.c_out + 15) / 16) * sizeof(float));
      if (lds > kWgradLdsMax || nch > 0x7fffffff) return hipErrorInvalidValue;
      const dim3 grid((unsigned)nch, (J + 1 + 63) / 64);
#define CH_WGRAD(NG)                                                                              \
  {                                                                                               \
    static bool attr = false;                                                                     \
    if (!attr) {                                                                                  \
      const hipError_t ea = hipFuncSetAttribute((const void*)k_conv_bwd_weight_mfma<NG>,           \
                                                hipFuncAttributeMaxDynamicSharedMemorySize,       \
                                                (int)kWgradLdsMax);                               \
      if (ea != hipSuccess) return ea;                                                            \
      attr = true;                                                                                \
    }                                                                                             \
    hipLaunchKernelGGL(k_conv_bwd_weight_mfma<NG>, grid, dim3(256), lds, s, G, L.c_out, Ho, A, Ca, \
                       B, Cb, H, L.k, L.stride, R, nband, ws + p.wpart);                          \
  }
      switch ((L.c_out + 15) / 16) {
        case 1: CH_WGRAD(1); break;
        case 2: CH_WGRAD(2); break;
        case 3: CH_WGRAD(3); break;
        default: CH_WGRAD(4); break;
      }
#undef CH_WGRAD
      hipLaunchKernelGGL(k_wgrad_sum, dim3((unsigned)(((int64_t)L.c_out * (J + 1) + 63) / 64)),
                         dim3(256), 0, s, ws + p.wpart, (int)nch, L.c_out, J, gw);
    }
    if (l == 0) continue;
    if (L.c_in % 16 || L.c_in > 128 || (L.stride != 1 && L.stride != 2))
      return hipErrorInvalidValue;
    const float* wd = ws + p.wpd + pack_offset(l, false);
    const int64_t dtiles = ((int64_t)H * H + 15) / 16;
    const int DT = dtiles * batch >= kNNTwoTiles ? 2 : 1;
    const dim3 dgrid((unsigned)((dtiles + DT - 1) / DT), batch);
#define CH_BWD_DATA(NG)                                                                         \
  if (DT == 2)                                                                                   \
    hipLaunchKernelGGL((k_conv_bwd_data_mfma<NG, 2>), dgrid, dim3(256), 0, s, G, L.c_out, Ho, wd, \
                       Ca, Cb, H, L.k, L.stride, dA, accA, ws + p.tmp);                          \
  else                                                                                           \
    hipLaunchKernelGGL((k_conv_bwd_data_mfma<NG, 1>), dgrid, dim3(256), 0, s, G, L.c_out, Ho, wd, \
                       Ca, Cb, H, L.k, L.stride, dA, accA, ws + p.tmp)
    switch (L.c_in / 16) {
      case 1: CH_BWD_DATA(1); break;
      case 2: CH_BWD_DATA(2); break;
      case 3: CH_BWD_DATA(3); break;
      case 4: CH_BWD_DATA(4); break;
      case 5: CH_BWD_DATA(5); break;
      case 6: CH_BWD_DATA(6); break;
      case 7: CH_BWD_DATA(7); break;
      default: CH_BWD_DATA(8); break;
    }
#undef CH_BWD_DATA
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
