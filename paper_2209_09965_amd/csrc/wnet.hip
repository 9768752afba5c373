// The paper's two-stage reconstruction network (the W-Net; paper Sec. 3.2.1-
// 3.2.3 and Sec. 3.5.1), inference in BF16:
//
//   D  a U-Net of 3x3 convs with the paper's depths, encoder 64/64/80/96 and
//      decoder 80/64/64 (two convs + ReLU per block, 2x2 average pooling,
//      bilinear x2 upsampling, [upsampled, skip] concatenation), whose last
//      decoder state gives the direct prediction O_d through a 1x1 conv.
//      Every conv runs on the library's MFMA conv kernel (BF16 operands,
//      FP32 accumulation), activations stored in BF16.
//   K  1x1 kernel predictors on D's hidden states H_0..H_3 (the decoder
//      states at full, 1/2 and 1/4 resolution and the bottleneck at 1/8):
//      encoder level l filters the image J_l with its predicted 5x5 kernel
//      (softmax of 25 logits, replicated border) and pools the result into
//      J_(l+1); decoder level l predicts 25 logits and a blend logit, blends
//      the encoder's filtered image with the upsampled coarser one by the
//      sigmoid of the blend logit and filters the blend.  K runs in FP32.
//
// The recurrent form (paper Sec. 3.2.4) keeps a state across frames: the
// previous frame's O_d, read by D's first conv as three more input channels,
// and each decoder block's previous output, read by the block's first conv
// as a third concatenated source after [upsampled, skip].  The decoder
// blocks write their outputs straight into the state (after the first conv
// has read the old one), so it costs no copies.
//
// Training (either form): the forward keeps K's per-level kernels, blend
// weights and blends; the backward runs K's adjoints in FP32 (finest
// decoder level to coarsest encoder level), adds K's gradients into D's
// states, then D's backward on the single-stage network's kernels (ReLU
// mask, MFMA weight gradient, input-gradient conv); Adam on the FP32 master.
// A recurrent form's state is a read-only input there (carried over one
// step, no gradient through it).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "net.h"
#include "net_kernels.h"

namespace fv {
namespace wnet {

using net::BF16;
using net::ConvArgs;

constexpr int kTaps = 25;
constexpr int kConv = 14;  // D's 3x3 convs; then the O_d head and K's seven 1x1 layers
constexpr int kLayersAll = kConv + 1 + 7;

struct Layer {
  int ci, co, k, level;
  int c0, c1, up0;  // conv inputs (3x3 layers): channels of source 0 / 1, upsampled source 0
  int c2;           // channels of the fed-back state (recurrent decoder blocks)
};

// Parameter order (each weight [Co][Ci][k][k], then the bias [Co]): D's convs
// e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b, the O_d head hd,
// then K: ke0 ke1 ke2 ke3 (encoder, 25 logits) and kd2 kd1 kd0 (decoder, 25
// logits and one blend logit).
const Layer kL[kLayersAll] = {
    {5, 64, 3, 0, 8, 0, 0},      {64, 64, 3, 0, 64, 0, 0},   {64, 64, 3, 1, 64, 0, 0},
    {64, 64, 3, 1, 64, 0, 0},    {64, 80, 3, 2, 64, 0, 0},   {80, 80, 3, 2, 80, 0, 0},
    {80, 96, 3, 3, 80, 0, 0},    {96, 96, 3, 3, 96, 0, 0},   {176, 80, 3, 2, 96, 80, 1},
    {80, 80, 3, 2, 80, 0, 0},    {144, 64, 3, 1, 80, 64, 1}, {64, 64, 3, 1, 64, 0, 0},
    {128, 64, 3, 0, 64, 64, 1},  {64, 64, 3, 0, 64, 0, 0},   {64, 3, 1, 0, 0, 0, 0},
    {64, kTaps, 1, 0, 0, 0, 0},  {64, kTaps, 1, 1, 0, 0, 0}, {80, kTaps, 1, 2, 0, 0, 0},
    {96, kTaps, 1, 3, 0, 0, 0},  {80, kTaps + 1, 1, 2, 0, 0, 0},
    {64, kTaps + 1, 1, 1, 0, 0, 0}, {64, kTaps + 1, 1, 0, 0, 0, 0},
};
// The recurrent form: e0a reads the 8 packed channels (the previous O_d
// last), each decoder block's first conv its own previous output last.
const Layer kLR[kLayersAll] = {
    {8, 64, 3, 0, 8, 0, 0},      {64, 64, 3, 0, 64, 0, 0},   {64, 64, 3, 1, 64, 0, 0},
    {64, 64, 3, 1, 64, 0, 0},    {64, 80, 3, 2, 64, 0, 0},   {80, 80, 3, 2, 80, 0, 0},
    {80, 96, 3, 3, 80, 0, 0},    {96, 96, 3, 3, 96, 0, 0},   {256, 80, 3, 2, 96, 80, 1, 80},
    {80, 80, 3, 2, 80, 0, 0},    {208, 64, 3, 1, 80, 64, 1, 64}, {64, 64, 3, 1, 64, 0, 0},
    {192, 64, 3, 0, 64, 64, 1, 64}, {64, 64, 3, 0, 64, 0, 0}, {64, 3, 1, 0, 0, 0, 0},
    {64, kTaps, 1, 0, 0, 0, 0},  {64, kTaps, 1, 1, 0, 0, 0}, {80, kTaps, 1, 2, 0, 0, 0},
    {96, kTaps, 1, 3, 0, 0, 0},  {80, kTaps + 1, 1, 2, 0, 0, 0},
    {64, kTaps + 1, 1, 1, 0, 0, 0}, {64, kTaps + 1, 1, 0, 0, 0, 0},
};
constexpr int kHead = 14, kKe0 = 15, kKd2 = 19;

// BF16 activation tensors of D
enum T {
  T_IN = 0, T_E0A, T_E0B, T_P0, T_E1A, T_E1B, T_P1, T_E2A, T_E2B, T_P2, T_E3A, T_E3B,
  T_D2A, T_D2B, T_D1A, T_D1B, T_D0A, T_D0B, kTensors
};
const int kTC[kTensors][2] = {  // channels, level
    {8, 0},  {64, 0}, {64, 0}, {64, 1}, {64, 1}, {64, 1}, {64, 2}, {80, 2}, {80, 2},
    {80, 3}, {96, 3}, {96, 3}, {80, 2}, {80, 2}, {64, 1}, {64, 1}, {64, 0}, {64, 0}};
// per conv: source 0, source 1 or -1, output, pooled output or -1
const int kIO[kConv][4] = {
    {T_IN, -1, T_E0A, -1},    {T_E0A, -1, T_E0B, T_P0}, {T_P0, -1, T_E1A, -1},
    {T_E1A, -1, T_E1B, T_P1}, {T_P1, -1, T_E2A, -1},    {T_E2A, -1, T_E2B, T_P2},
    {T_P2, -1, T_E3A, -1},    {T_E3A, -1, T_E3B, -1},   {T_E3B, T_E2B, T_D2A, -1},
    {T_D2A, -1, T_D2B, -1},   {T_D2B, T_E1B, T_D1A, -1}, {T_D1A, -1, T_D1B, -1},
    {T_D1B, T_E0B, T_D0A, -1}, {T_D0A, -1, T_D0B, -1}};
// K's hidden states H_0..H_3
const int kHidden[4] = {T_D0B, T_D1B, T_D2B, T_E3B};
// per conv: the fed-back tensor its first conv reads (recurrent form), or -1
const int kFeed[kConv] = {-1, -1, -1, -1, -1, -1, -1, -1, T_D2B, -1, T_D1B, -1, T_D0B, -1};

int64_t param_offset(const Layer* L, int layer) {
  int64_t off = 0;
  for (int l = 0; l < layer; ++l) off += (int64_t)L[l].co * L[l].ci * L[l].k * L[l].k + L[l].co;
  return off;
}
int64_t param_offset(int layer) { return param_offset(kL, layer); }

// The recurrent state, caller-owned device memory: O_d (FP32 [n h w 3]),
// then D's decoder outputs d2b, d1b, d0b (BF16 NHWC at 1/4, 1/2 and full
// resolution), each 256-byte aligned.
struct StatePlan {
  size_t od, t[kTensors];  // t[] set for T_D2B, T_D1B, T_D0B
  size_t bytes;
};

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

// Workspace: D's BF16 tensors, then FP32 images: O_d, the kernel weights and
// blend weights of the current K level (full-resolution sized), the pooled
// encoder inputs J_1..J_3, the encoder outputs Je_0..Je_3, the blend B and
// the decoder outputs J_2, J_1 (J_0 is the caller's output).
struct Plan {
  int n, h, w;
  size_t t[kTensors];
  size_t od, wk, av, jin[4], je[4], blend, jd[3];
  size_t bytes;
};

StatePlan make_state_plan(int n, int h, int w) {
  StatePlan p{};
  auto px = [&](int lv) { return (size_t)n * (h >> lv) * (w >> lv); };
  size_t off = 0;
  p.od = off;
  off += al(px(0) * 3 * 4);
  for (int t : {T_D2B, T_D1B, T_D0B}) {
    p.t[t] = off;
    off += al(px(kTC[t][1]) * kTC[t][0] * 2);
  }
  p.bytes = off;
  return p;
}

__global__ void __launch_bounds__(256) k_zero(uint4* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

Plan make_plan(int n, int h, int w) {
  Plan p;
  p.n = n;
  p.h = h;
  p.w = w;
  size_t off = 0;
  auto px = [&](int lv) { return (size_t)n * (h >> lv) * (w >> lv); };
  for (int t = 0; t < kTensors; ++t) {
    p.t[t] = off;
    off += al(px(kTC[t][1]) * kTC[t][0] * 2);
  }
  p.od = off;
  off += al(px(0) * 3 * 4);
  p.wk = off;
  off += al(px(0) * kTaps * 4);
  p.av = off;
  off += al(px(0) * 4);
  for (int l = 0; l < 4; ++l) {
    p.jin[l] = off;
    off += l ? al(px(l) * 3 * 4) : 0;
    p.je[l] = off;
    off += al(px(l) * 3 * 4);
  }
  p.blend = off;
  off += al(px(0) * 3 * 4);
  for (int l = 0; l < 3; ++l) {
    p.jd[l] = off;
    off += l ? al(px(l) * 3 * 4) : 0;
  }
  p.bytes = off;
  return p;
}

// 1x1 layer on a BF16 tensor of C channels (C a multiple of 8), T outputs.
// MODE 0: the T outputs as they are (O_d); 1: softmax over T = 25 (encoder
// kernels); 2: softmax over the first 25 and the sigmoid of the 26th (the
// decoder's kernels and blend weight).
template <int T, int MODE>
__global__ void __launch_bounds__(256) k_predict(const __bf16* __restrict__ h, int C,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ b, int64_t npx,
                                                 float* __restrict__ out,
                                                 float* __restrict__ aout) {
  extern __shared__ float sw[];  // w [T][C], then b [T]
  for (int i = threadIdx.x; i < T * C + T; i += 256) sw[i] = i < T * C ? w[i] : b[i - T * C];
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npx) return;
  float z[T];
  for (int t = 0; t < T; ++t) z[t] = sw[T * C + t];
  const uint4* src = (const uint4*)(h + p * C);
  for (int c8 = 0; c8 < C / 8; ++c8) {
    const uint4 u = src[c8];
    const uint32_t q[4] = {u.x, u.y, u.z, u.w};
    for (int j = 0; j < 8; ++j) {
      const float v = net::bf16_bits_to_f((q[j >> 1] >> (16 * (j & 1))) & 0xffffu);
      const int c = 8 * c8 + j;
      for (int t = 0; t < T; ++t) z[t] = fmaf(sw[t * C + c], v, z[t]);
    }
  }
  if constexpr (MODE == 0) {
    for (int t = 0; t < T; ++t) out[p * T + t] = z[t];
    return;
  }
  float m = z[0];
  for (int t = 1; t < kTaps; ++t) m = fmaxf(m, z[t]);
  float s = 0.f;
  for (int t = 0; t < kTaps; ++t) {
    z[t] = __expf(z[t] - m);
    s += z[t];
  }
  const float inv = 1.0f / s;
  for (int t = 0; t < kTaps; ++t) out[p * kTaps + t] = z[t] * inv;
  if constexpr (MODE == 2) {
    const float zb = z[kTaps];
    const float e = __expf(-fabsf(zb));
    aout[p] = zb >= 0.f ? 1.0f / (1.0f + e) : e / (1.0f + e);
  }
}

// out(p) = sum over the 5x5 taps k of wk[p][k] img(clamp(p + delta_k)), RGB,
// n images of h x w.
__global__ void __launch_bounds__(256) k_apply(const float* __restrict__ wk,
                                               const float* __restrict__ img, int n, int h,
                                               int w, float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t npx = (int64_t)n * h * w;
  if (p >= npx) return;
  const int x = (int)(p % w);
  const int64_t r = p / w;
  const int y = (int)(r % h);
  const int64_t base = (r / h) * h * w;
  float acc[3] = {0.f, 0.f, 0.f};
  for (int dy = -2; dy <= 2; ++dy) {
    const int yy = min(max(y + dy, 0), h - 1);
    for (int dx = -2; dx <= 2; ++dx) {
      const int xx = min(max(x + dx, 0), w - 1);
      const float k = wk[p * kTaps + 5 * (dy + 2) + (dx + 2)];
      const float* s = img + (base + (int64_t)yy * w + xx) * 3;
      for (int c = 0; c < 3; ++c) acc[c] = fmaf(k, s[c], acc[c]);
    }
  }
  for (int c = 0; c < 3; ++c) out[p * 3 + c] = acc[c];
}

// 2x2 average of an RGB image of h x w (h, w even) into (h/2) x (w/2).
__global__ void __launch_bounds__(256) k_pool3(const float* __restrict__ src, int n, int h,
                                               int w, float* __restrict__ dst) {
  const int ho = h / 2, wo = w / 2;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)n * ho * wo) return;
  const int x = (int)(p % wo);
  const int64_t r = p / wo;
  const int y = (int)(r % ho);
  const int64_t b = r / ho;
  for (int c = 0; c < 3; ++c) {
    float s = 0.f;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx)
        s += src[((b * h + 2 * y + dy) * w + 2 * x + dx) * 3 + c];
    dst[p * 3 + c] = 0.25f * s;
  }
}

// Source index and weight of bilinear x2 upsampling along one axis (half-pixel
// centres, edge clamp): output i samples the input at (i + 1/2) / 2 - 1/2.
__device__ __forceinline__ void up_axis(int i, int n, int* i0, int* i1, float* f) {
  float s = fminf(fmaxf((i + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(n - 1));
  const int a = (int)floorf(s);
  *i0 = a;
  *i1 = min(a + 1, n - 1);
  *f = s - (float)a;
}

// B = (1 - a) je + a up(jc): the decoder's blend of the encoder's filtered
// image je (h x w) with the upsampled coarser image jc ((h/2) x (w/2)).
__global__ void __launch_bounds__(256) k_blend(const float* __restrict__ je,
                                               const float* __restrict__ jc,
                                               const float* __restrict__ a, int n, int h, int w,
                                               float* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)n * h * w) return;
  const int x = (int)(p % w);
  const int64_t r = p / w;
  const int y = (int)(r % h);
  const int64_t b = r / h;
  const int hc = h / 2, wc = w / 2;
  int y0, y1, x0, x1;
  float fy, fx;
  up_axis(y, hc, &y0, &y1, &fy);
  up_axis(x, wc, &x0, &x1, &fx);
  const float* c00 = jc + ((b * hc + y0) * wc + x0) * 3;
  const float* c01 = jc + ((b * hc + y0) * wc + x1) * 3;
  const float* c10 = jc + ((b * hc + y1) * wc + x0) * 3;
  const float* c11 = jc + ((b * hc + y1) * wc + x1) * 3;
  const float av = a[p];
  for (int c = 0; c < 3; ++c) {
    const float top = c00[c] * (1.0f - fx) + c01[c] * fx;
    const float bot = c10[c] * (1.0f - fx) + c11[c] * fx;
    const float u = top * (1.0f - fy) + bot * fy;
    out[p * 3 + c] = (1.0f - av) * je[p * 3 + c] + av * u;
  }
}

static unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

// ------------------------------------------------------- K, backward pass

// Adjoint of out(p) = sum_k wk[p][k] img(clamp(p + d_k)) with respect to the
// kernel weights: dwk[p][k] = sum_c dout[p][c] img(clamp(p + d_k))[c].
__global__ void __launch_bounds__(256) k_apply_bwd_w(const float* __restrict__ dout,
                                                     const float* __restrict__ img, int n, int h,
                                                     int w, float* __restrict__ dwk) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)n * h * w) return;
  const int x = (int)(p % w);
  const int64_t r = p / w;
  const int y = (int)(r % h);
  const int64_t base = (r / h) * h * w;
  const float g0 = dout[p * 3], g1 = dout[p * 3 + 1], g2 = dout[p * 3 + 2];
  for (int dy = -2; dy <= 2; ++dy) {
    const int yy = min(max(y + dy, 0), h - 1);
    for (int dx = -2; dx <= 2; ++dx) {
      const int xx = min(max(x + dx, 0), w - 1);
      const float* q = img + (base + (int64_t)yy * w + xx) * 3;
      dwk[p * kTaps + 5 * (dy + 2) + (dx + 2)] = fmaf(g0, q[0], fmaf(g1, q[1], g2 * q[2]));
    }
  }
}

// Rows (columns) p of an axis of length n whose tap d, clamped, lands on q:
// q - d inside the image, widened to the image edge when q is an edge.
__device__ __forceinline__ void tap_range(int q, int d, int n, int* lo, int* hi) {
  *lo = max(q == 0 ? 0 : q - d, 0);
  *hi = min(q == n - 1 ? n - 1 : q - d, n - 1);
}

// Adjoint with respect to the image: dimg(q) = sum over (p, k) with
// clamp(p + d_k) = q of wk[p][k] dout[p], in a fixed order.
__global__ void __launch_bounds__(256) k_apply_bwd_img(const float* __restrict__ wk,
                                                       const float* __restrict__ dout, int n,
                                                       int h, int w, float* __restrict__ dimg) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (int64_t)n * h * w) return;
  const int qx = (int)(q % w);
  const int64_t r = q / w;
  const int qy = (int)(r % h);
  const int64_t base = (r / h) * h * w;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int dy = -2; dy <= 2; ++dy) {
    int ylo, yhi;
    tap_range(qy, dy, h, &ylo, &yhi);
    for (int dx = -2; dx <= 2; ++dx) {
      int xlo, xhi;
      tap_range(qx, dx, w, &xlo, &xhi);
      const int k = 5 * (dy + 2) + (dx + 2);
      for (int py = ylo; py <= yhi; ++py)
        for (int px = xlo; px <= xhi; ++px) {
          const int64_t pp = base + (int64_t)py * w + px;
          const float c = wk[pp * kTaps + k];
          a0 = fmaf(c, dout[pp * 3], a0);
          a1 = fmaf(c, dout[pp * 3 + 1], a1);
          a2 = fmaf(c, dout[pp * 3 + 2], a2);
        }
    }
  }
  dimg[q * 3] = a0;
  dimg[q * 3 + 1] = a1;
  dimg[q * 3 + 2] = a2;
}

// Softmax backward of the 25 kernel logits: dz[k] = wk[k] (dwk[k] - sum_j
// wk[j] dwk[j]); dz has `stride` values per pixel (25, or 26 with the blend).
__global__ void __launch_bounds__(256) k_softmax_bwd(const float* __restrict__ wk,
                                                     const float* __restrict__ dwk, int64_t npx,
                                                     int stride, float* __restrict__ dz) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npx) return;
  float dot = 0.f;
  for (int k = 0; k < kTaps; ++k) dot = fmaf(wk[p * kTaps + k], dwk[p * kTaps + k], dot);
  for (int k = 0; k < kTaps; ++k)
    dz[p * stride + k] = wk[p * kTaps + k] * (dwk[p * kTaps + k] - dot);
}

// Blend backward at a decoder level (h x w; jc the coarser image):
// B = (1 - a) je + a U with U = up(jc): dje = (1 - a) dB, dU = a dB and the
// blend logit's gradient sum_c (U - je) dB times a (1 - a) into dz[p][25].
__global__ void __launch_bounds__(256) k_blend_bwd(const float* __restrict__ je,
                                                   const float* __restrict__ jc,
                                                   const float* __restrict__ a,
                                                   const float* __restrict__ dB, int n, int h,
                                                   int w, float* __restrict__ dje,
                                                   float* __restrict__ dU,
                                                   float* __restrict__ dz) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)n * h * w) return;
  const int x = (int)(p % w);
  const int64_t r = p / w;
  const int y = (int)(r % h);
  const int64_t b = r / h;
  const int hc = h / 2, wc = w / 2;
  int y0, y1, x0, x1;
  float fy, fx;
  up_axis(y, hc, &y0, &y1, &fy);
  up_axis(x, wc, &x0, &x1, &fx);
  const float* c00 = jc + ((b * hc + y0) * wc + x0) * 3;
  const float* c01 = jc + ((b * hc + y0) * wc + x1) * 3;
  const float* c10 = jc + ((b * hc + y1) * wc + x0) * 3;
  const float* c11 = jc + ((b * hc + y1) * wc + x1) * 3;
  const float av = a[p];
  float da = 0.f;
  for (int c = 0; c < 3; ++c) {
    const float top = c00[c] * (1.0f - fx) + c01[c] * fx;
    const float bot = c10[c] * (1.0f - fx) + c11[c] * fx;
    const float u = top * (1.0f - fy) + bot * fy;
    const float g = dB[p * 3 + c];
    da = fmaf(u - je[p * 3 + c], g, da);
    dje[p * 3 + c] = (1.0f - av) * g;
    dU[p * 3 + c] = av * g;
  }
  dz[p * (kTaps + 1) + kTaps] = da * av * (1.0f - av);
}

// 1x1 layer backward, input side: dH[p][c] (+)= sum_t W[t][c] dz[p][t],
// summed over t in order.  A thread computes 4 consecutive channels of one
// pixel, so a wave loads and stores whole cache lines of dH; the dz rows of
// the block's pixels are staged in LDS with the weights.  C % 4 == 0.
__global__ void __launch_bounds__(256) k_predict_bwd_h(const float* __restrict__ dz, int T,
                                                       const float* __restrict__ W, int C,
                                                       int64_t npx, float* __restrict__ dh,
                                                       int acc) {
  extern __shared__ float sm[];  // W [T][C], then dz [pixels of the block][T]
  float* sw = sm;
  float* sd = sm + T * C;
  const int G = C >> 2;
  const int64_t e0 = (int64_t)blockIdx.x * 256, p0 = e0 / G;
  const int np = (int)(min((e0 + 255) / G, npx - 1) - p0 + 1);
  for (int i = threadIdx.x; i < T * C; i += 256) sw[i] = W[i];
  for (int i = threadIdx.x; i < np * T; i += 256) sd[i] = dz[p0 * T + i];
  __syncthreads();
  const int64_t e = e0 + threadIdx.x, p = e / G;
  if (p >= npx) return;
  const int c = (int)(e - p * G) * 4;
  const float* g = sd + (p - p0) * T;
  float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
  for (int t = 0; t < T; ++t) {
    const float gt = g[t];
    const float4 w = *(const float4*)(sw + t * C + c);
    v0 = fmaf(w.x, gt, v0);
    v1 = fmaf(w.y, gt, v1);
    v2 = fmaf(w.z, gt, v2);
    v3 = fmaf(w.w, gt, v3);
  }
  float4* o = (float4*)(dh + p * C + c);
  if (acc) {
    const float4 d = *o;
    v0 += d.x;
    v1 += d.y;
    v2 += d.z;
    v3 += d.w;
  }
  *o = make_float4(v0, v1, v2, v3);
}

// 1x1 layer backward, weight side: per pixel chunk, part[t][c] = sum_p
// dz[p][t] H[p][c] and part[t][C] = sum_p dz[p][t], each summed over the
// chunk's pixels in order.  64 pixels at a time in LDS (dz rows padded to an
// even Tp, H rows with the ones column and zeros to a multiple of 4); a
// thread owns tiles of 2 t x 4 outputs, one 8-byte and one 16-byte LDS read
// per pixel for 8 FMAs.  T <= 26, C % 8 == 0, C <= 96.
constexpr int kPwTp = 26, kPwKp = 100;
__global__ void __launch_bounds__(256) k_predict_wgrad(const float* __restrict__ dz, int T,
                                                       const __bf16* __restrict__ hb, int C,
                                                       int64_t npx, int chunks,
                                                       float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) float sd[64 * kPwTp];
  __shared__ __attribute__((aligned(16))) float sh[64 * kPwKp];
  const int chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t p0 = npx * chunk / chunks, p1 = npx * (chunk + 1) / chunks;
  const int Tp = (T + 1) & ~1, C1 = C + 1, Kp = (C1 + 3) & ~3, G8 = C >> 3, X = Kp - C;
  const int nkq = Kp >> 2, ntiles = (Tp >> 1) * nkq;
  const uint16_t* h16 = (const uint16_t*)hb;
  // this thread's fill items, the same in every batch: dz entries (pixel,
  // offset in the batch's rows or -1 for padding), H groups of 8 channels,
  // and one entry of the ones / zero columns
  constexpr int kD = (64 * kPwTp + 255) / 256, kH = (64 * 12 + 255) / 256;
  int dpp[kD], dsrc[kD];
#pragma unroll
  for (int u = 0; u < kD; ++u) {
    const int e = tid + 256 * u, pp = e / Tp, t = e - pp * Tp;
    dpp[u] = pp;
    dsrc[u] = e < 64 * Tp && t < T ? pp * T + t : -1;
  }
  const int xpp = tid / X, xk = C + tid - xpp * X;
  float acc[2][8];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[jj][i] = 0.f;
  for (int64_t base = p0; base < p1; base += 64) {
    const int cnt = (int)min((int64_t)64, p1 - base);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kD; ++u) {
      const int e = tid + 256 * u;
      if (e < 64 * Tp)
        sd[e] = dsrc[u] >= 0 && dpp[u] < cnt ? dz[base * T + dsrc[u]] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kH; ++u) {
      const int i = tid + 256 * u;
      if (i >= 64 * G8) break;
      const int pp = i / G8, g = i - pp * G8;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (pp < cnt) v = *(const uint4*)(h16 + (base + pp) * C + 8 * g);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      float f[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        f[2 * q] = net::bf16_bits_to_f(w[q] & 0xffffu);
        f[2 * q + 1] = net::bf16_bits_to_f(w[q] >> 16);
      }
      float4* d = (float4*)(sh + pp * Kp + 8 * g);
      d[0] = make_float4(f[0], f[1], f[2], f[3]);
      d[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
    if (tid < 64 * X) sh[xpp * Kp + xk] = xk == C && xpp < cnt ? 1.0f : 0.f;
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const int j = tid + 256 * jj;
      if (j >= ntiles) break;
      const int tp = j / nkq, kq = j - tp * nkq;
      float a[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = acc[jj][i];
      const float2* d2 = (const float2*)sd + tp;
      const float4* h4 = (const float4*)sh + kq;
#pragma unroll 4
      for (int pp = 0; pp < 64; ++pp) {
        const float2 d = d2[pp * (Tp >> 1)];
        const float4 h = h4[pp * nkq];
        a[0] = fmaf(d.x, h.x, a[0]);
        a[1] = fmaf(d.x, h.y, a[1]);
        a[2] = fmaf(d.x, h.z, a[2]);
        a[3] = fmaf(d.x, h.w, a[3]);
        a[4] = fmaf(d.y, h.x, a[4]);
        a[5] = fmaf(d.y, h.y, a[5]);
        a[6] = fmaf(d.y, h.z, a[6]);
        a[7] = fmaf(d.y, h.w, a[7]);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[jj][i] = a[i];
    }
  }
  const int nout = T * C1;
#pragma unroll
  for (int jj = 0; jj < 2; ++jj) {
    const int j = tid + 256 * jj;
    if (j >= ntiles) break;
    const int tp = j / nkq, kq = j - tp * nkq;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = 2 * tp + (i >> 2), k = 4 * kq + (i & 3);
      if (t < T && k < C1) part[(int64_t)chunk * nout + t * C1 + k] = acc[jj][i];
    }
  }
}

constexpr int kPredSlices = 32;  // first-stage slices of the chunk partials

// The chunk partials summed in a fixed order (deterministic): slice sl of
// the chunks first, then the slices in order (k_predict_reduce2).
__global__ void __launch_bounds__(256) k_predict_reduce(const float* __restrict__ part,
                                                        int chunks, int nout,
                                                        float* __restrict__ part2) {
  const int o = blockIdx.x * 256 + threadIdx.x, sl = blockIdx.y;
  if (o >= nout) return;
  const int c0 = chunks * sl / kPredSlices, c1 = chunks * (sl + 1) / kPredSlices;
  float s = 0.f;
  for (int c = c0; c < c1; ++c) s += part[(int64_t)c * nout + o];
  part2[sl * nout + o] = s;
}

// ... then the slices, stored in the parameter order (weights [t][c], then
// the T biases)
__global__ void __launch_bounds__(256) k_predict_reduce2(const float* __restrict__ part2, int T,
                                                         int C, float* __restrict__ grad) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  const int C1 = C + 1, nout = T * C1;
  if (o >= nout) return;
  float s = 0.f;
  for (int sl = 0; sl < kPredSlices; ++sl) s += part2[sl * nout + o];
  const int t = o / C1, k = o % C1;
  grad[k < C ? t * C + k : T * C + t] = s;
}

}  // namespace wnet
}  // namespace fv

struct fv_wnet {
  int device;
  int recurrent;                       // 1: the recurrent form (table kLR)
  const fv::wnet::Layer* L;            // its layer table
  float* master;                       // FP32 parameters, the order of the layer table
  void* w_bf16[fv::wnet::kConv];       // D's convs as swizzled BF16 MFMA fragments
  // training (plain form): gradient, Adam moments and step, the transposed
  // BF16 weights of D's input-gradient convolutions
  float* grad;
  float* adam_m;
  float* adam_v;
  int64_t step;
  void* w_bf16t[fv::wnet::kConv];
};

using namespace fv;
using namespace fv::wnet;

namespace {

// D's BF16 weight fragments from the FP32 master (and, for training, the
// transposed ones of the input-gradient convolutions).
fv_status refresh_bf16(fv_wnet* n, hipStream_t s) {
  fv_status st = FV_OK;
  for (int l = 0; st == FV_OK && l < kConv; ++l) {
    st = net::swizzle_bf16(n->master + param_offset(n->L, l), n->L[l].ci, n->L[l].co, 0,
                           n->w_bf16[l], s);
    if (st == FV_OK && n->w_bf16t[l])
      st = net::swizzle_bf16(n->master + param_offset(n->L, l), n->L[l].ci, n->L[l].co, 1,
                             n->w_bf16t[l], s, n->L[l].c0 + n->L[l].c1);
  }
  return st;
}

// What a training forward keeps of K for the backward pass: per level the
// encoder's kernel weights, and the decoder's kernel weights, blend weights
// and blends (inference reuses one buffer of each across levels).
struct KKeep {
  float* wke[4];
  float* wkd[3];
  float* av[3];
  float* bl[3];
};

fv_status reconstruct(const fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                      const float* frame_depth, void* state, size_t state_bytes, int reset,
                      int views, int width, int height, float* out_rgb, float* out_direct,
                      void* workspace, size_t ws_bytes, void* stream, const char* fn,
                      const KKeep* keep = nullptr) {
  if (!n || !frame_rgba || !mask || !out_rgb || !workspace)
    return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  const bool rec = state != nullptr;
  if (rec != (n->recurrent != 0))
    return fail(FV_ERR_INVALID_ARG,
                n->recurrent ? "%s: a recurrent network needs fv_wnet_reconstruct_recurrent"
                             : "%s: the plain network has no state (fv_wnet_reconstruct)",
                fn);
  fv_status st = net::check_frame(views, width, height, fn);
  if (st != FV_OK) return st;
  const Plan p = make_plan(views, height, width);
  if (ws_bytes < p.bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, p.bytes);
  if ((uintptr_t)workspace % 256)
    return fail(FV_ERR_INVALID_ARG, "%s: workspace not 256-byte aligned", fn);
  const StatePlan sp = make_state_plan(views, height, width);
  if (rec && state_bytes < sp.bytes)
    return fail(FV_ERR_CAPACITY, "%s: state %zu < %zu bytes", fn, state_bytes, sp.bytes);
  if (rec && (uintptr_t)state % 256)
    return fail(FV_ERR_INVALID_ARG, "%s: state not 256-byte aligned", fn);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  uint8_t* sb = (uint8_t*)state;
  const int64_t npx = (int64_t)views * height * width;
  // Inference writes the new state over the one it reads (decoder outputs
  // and O_d go straight into it); a training forward leaves it as its input
  // and keeps everything in the workspace
  const bool state_out = rec && !keep;
  auto tensor = [&](int t) -> uint8_t* {
    if (state_out && (t == T_D2B || t == T_D1B || t == T_D0B)) return sb + sp.t[t];
    return ws + p.t[t];
  };
  if (state_out && reset) {
    const int64_t n16 = (int64_t)(sp.bytes / 16);
    k_zero<<<blocks_of(n16), 256, 0, s>>>((uint4*)sb, n16);
    if ((st = launch_status("wnet: state reset")) != FV_OK) return st;
  }
  float* od_state = rec ? (float*)(sb + sp.od) : nullptr;
  // D: the packed input (with the previous O_d in the recurrent form), the
  // 14 convs (pooling fused into e0b, e1b, e2b), O_d
  st = net::pack_input_bf16(frame_rgba, mask, frame_depth, od_state, ws + p.t[T_IN], npx, s);
  if (st != FV_OK) return st;
  const Layer* LT = n->L;
  for (int l = 0; l < kConv; ++l) {
    const Layer& L = LT[l];
    ConvArgs a{};
    a.src0 = tensor(kIO[l][0]);
    a.src1 = kIO[l][1] >= 0 ? tensor(kIO[l][1]) : nullptr;
    a.src2 = rec && kFeed[l] >= 0 ? sb + sp.t[kFeed[l]] : nullptr;
    a.c0 = L.c0;
    a.c1 = L.c1;
    a.c2 = a.src2 ? L.c2 : 0;
    a.cip = net::cip_of(L.c0 + L.c1 + a.c2);
    a.up0 = L.up0;
    a.n = views;
    a.h = height >> L.level;
    a.w = width >> L.level;
    a.kc = net::kchunks_of(L.c0 + L.c1 + a.c2);
    a.wsw = (const uint8_t*)n->w_bf16[l];
    a.bias = n->master + param_offset(LT, l) + (int64_t)L.co * L.ci * 9;
    a.co = L.co;
    a.relu = 1;
    a.out = tensor(kIO[l][2]);
    a.out_ch = L.co;
    a.pool_out = kIO[l][3] >= 0 ? tensor(kIO[l][3]) : nullptr;
    st = net::launch_conv<BF16>(a, net::nblocks_of(L.co), s);
    if (st != FV_OK) return st;
  }
  float* od = state_out ? od_state : (out_direct && !keep) ? out_direct : (float*)(ws + p.od);
  {
    const Layer& L = LT[kHead];
    const float* w = n->master + param_offset(LT, kHead);
    k_predict<3, 0><<<blocks_of(npx), 256, (3 * L.ci + 3) * 4, s>>>(
        (const __bf16*)tensor(T_D0B), L.ci, w, w + 3 * L.ci, npx, od, nullptr);
    if ((st = launch_status("wnet: O_d")) != FV_OK) return st;
  }
  if (state_out && out_direct &&
      (st = hip_status(hipMemcpyAsync(out_direct, od, npx * 3 * sizeof(float),
                                      hipMemcpyDeviceToDevice, s), "wnet: O_d copy")) != FV_OK)
    return st;
  // K, encoder: J_0 = O_d; filter J_l with ke_l; pool into J_(l+1)
  float* wk = (float*)(ws + p.wk);
  float* av = (float*)(ws + p.av);
  const float* jin = od;
  for (int l = 0; l < 4; ++l) {
    const Layer& L = LT[kKe0 + l];
    const int h = height >> l, w = width >> l;
    const int64_t m = (int64_t)views * h * w;
    const float* wl = n->master + param_offset(LT, kKe0 + l);
    float* wkl = keep ? keep->wke[l] : wk;
    k_predict<kTaps, 1><<<blocks_of(m), 256, (kTaps * L.ci + kTaps) * 4, s>>>(
        (const __bf16*)tensor(kHidden[l]), L.ci, wl, wl + kTaps * L.ci, m, wkl, nullptr);
    float* je = (float*)(ws + p.je[l]);
    k_apply<<<blocks_of(m), 256, 0, s>>>(wkl, jin, views, h, w, je);
    if (l < 3) {
      float* nxt = (float*)(ws + p.jin[l + 1]);
      k_pool3<<<blocks_of(m / 4), 256, 0, s>>>(je, views, h, w, nxt);
      jin = nxt;
    }
    if ((st = launch_status("wnet: K encoder")) != FV_OK) return st;
  }
  // K, decoder: from J_3 = Je_3 up to J_0 = the output
  const float* jc = (const float*)(ws + p.je[3]);
  for (int l = 2; l >= 0; --l) {
    const int li = kKd2 + (2 - l);
    const Layer& L = LT[li];
    const int h = height >> l, w = width >> l;
    const int64_t m = (int64_t)views * h * w;
    const float* wl = n->master + param_offset(LT, li);
    float* wkl = keep ? keep->wkd[l] : wk;
    float* avl = keep ? keep->av[l] : av;
    float* bl = keep ? keep->bl[l] : (float*)(ws + p.blend);
    k_predict<kTaps + 1, 2><<<blocks_of(m), 256, ((kTaps + 1) * L.ci + kTaps + 1) * 4, s>>>(
        (const __bf16*)tensor(kHidden[l]), L.ci, wl, wl + (kTaps + 1) * L.ci, m, wkl, avl);
    k_blend<<<blocks_of(m), 256, 0, s>>>((const float*)(ws + p.je[l]), jc, avl, views, h, w, bl);
    float* dst = l ? (float*)(ws + p.jd[l]) : out_rgb;
    k_apply<<<blocks_of(m), 256, 0, s>>>(wkl, bl, views, h, w, dst);
    if ((st = launch_status("wnet: K decoder")) != FV_OK) return st;
    jc = dst;
  }
  return FV_OK;
}

// ---------------------------------------------------------------- training

// Workspace of a training step: the forward plan, what the forward keeps of
// K per level, FP32 gradients of D's tensors, the input-gradient conv output
// (tmp), the masked BF16 output gradient (dz), K's image gradients, the
// weight-gradient partial sums and the loss scratch.
struct TPlan {
  Plan f;
  size_t wke[4], wkd[3], av[3], bl[3];
  size_t g[kTensors];
  size_t tmp, dz, dz2, w0;
  size_t dja, djb, dje[3], db, du, dwk, dzk;
  size_t kpart, part, part2;
  size_t out, dout, tgt, ssim, red;
  size_t bytes;
  int chunks[kConv];
  int kchunks;
};

TPlan make_tplan(int n, int h, int w, const Layer* LT) {
  TPlan t;
  t.f = make_plan(n, h, w);
  size_t off = t.f.bytes;
  auto px = [&](int lv) { return (size_t)n * (h >> lv) * (w >> lv); };
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al(bytes);
    return o;
  };
  for (int l = 0; l < 4; ++l) t.wke[l] = take(px(l) * kTaps * 4);
  for (int l = 0; l < 3; ++l) {
    t.wkd[l] = take(px(l) * kTaps * 4);
    t.av[l] = take(px(l) * 4);
    t.bl[l] = take(px(l) * 3 * 4);
  }
  t.g[T_IN] = 0;
  for (int k = 1; k < kTensors; ++k) t.g[k] = take(px(kTC[k][1]) * kTC[k][0] * 4);
  size_t tmp = 0, dz = 0, part = 0, part2 = 0;
  for (int l = 0; l < kConv; ++l) {
    const Layer& L = LT[l];
    const int ci = L.c0 + L.c1 + L.c2;
    tmp = std::max(tmp, px(L.level) * (L.c0 + L.c1) * 4);
    dz = std::max(dz, px(L.level) * L.co * 2);
    t.chunks[l] = net::wgrad_chunks(n, h >> L.level, w >> L.level, ci, L.co);
    part = std::max(part, net::wgrad_part_bytes(t.chunks[l], ci, L.co));
    part2 = std::max(part2, net::wgrad_part2_bytes(ci, L.co));
  }
  t.tmp = take(tmp);
  t.dz = take(dz);
  t.dz2 = take(dz);
  t.w0 = take((size_t)(9 * kL[0].c0 * kL[0].co + kL[0].co) * 4);
  t.dja = take(px(0) * 3 * 4);
  t.djb = take(px(0) * 3 * 4);
  for (int l = 0; l < 3; ++l) t.dje[l] = take(px(l) * 3 * 4);
  t.db = take(px(0) * 3 * 4);
  t.du = take(px(0) * 3 * 4);
  t.dwk = take(px(0) * kTaps * 4);
  t.dzk = take(px(0) * (kTaps + 1) * 4);
  t.kchunks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (int64_t)px(0) / 256));
  t.kpart = take((size_t)t.kchunks * (kTaps + 1) * 97 * 4);
  t.part = take(part);
  // (also the 1x1 layers' first-stage sums: up to 26 x 97 outputs)
  part2 = std::max(part2, (size_t)kPredSlices * (kTaps + 1) * 97 * 4);
  t.part2 = take(part2);
  t.out = take(px(0) * 3 * 4);
  t.dout = take(px(0) * 3 * 4);
  t.tgt = take(px(0) * 3 * 4);
  t.ssim = take(net::loss_ssim_bytes(n, h, w));
  t.red = take(net::loss_red_bytes(n, h, w));
  t.bytes = off;
  return t;
}

fv_status train_check(const fv_wnet* n, int batch, int width, int height, const void* ws,
                      size_t ws_bytes, TPlan* tp, const char* fn, const void* state = nullptr,
                      size_t state_bytes = 0) {
  if (!n || !ws) return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  if ((state != nullptr) != (n->recurrent != 0))
    return fail(FV_ERR_INVALID_ARG,
                n->recurrent ? "%s: a recurrent network trains with a state (_recurrent call)"
                             : "%s: the plain network takes no state",
                fn);
  if (state) {
    const StatePlan sp = make_state_plan(batch, height, width);
    if (state_bytes < sp.bytes)
      return fail(FV_ERR_CAPACITY, "%s: state %zu < %zu bytes", fn, state_bytes, sp.bytes);
    if ((uintptr_t)state % 256) return fail(FV_ERR_INVALID_ARG, "%s: state not aligned", fn);
  }
  fv_status st = net::check_frame(batch, width, height, fn);
  if (st != FV_OK) return st;
  if (width < 16 || height < 16)
    return fail(FV_ERR_INVALID_ARG, "%s: training frames must be at least 16 x 16", fn);
  *tp = make_tplan(batch, height, width, n->L);
  if (ws_bytes < tp->bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, tp->bytes);
  if ((uintptr_t)ws % 256) return fail(FV_ERR_INVALID_ARG, "%s: workspace not aligned", fn);
  return FV_OK;
}

KKeep keep_of(const TPlan& t, uint8_t* ws) {
  KKeep k;
  for (int l = 0; l < 4; ++l) k.wke[l] = (float*)(ws + t.wke[l]);
  for (int l = 0; l < 3; ++l) {
    k.wkd[l] = (float*)(ws + t.wkd[l]);
    k.av[l] = (float*)(ws + t.av[l]);
    k.bl[l] = (float*)(ws + t.bl[l]);
  }
  return k;
}

// Gradient of a 1x1 layer applied to H (BF16, C channels) from dz (T per
// pixel): its weights and bias into grad, and dH (+)= W^T dz.
fv_status predict_backward(const fv_wnet* n, const TPlan& tp, uint8_t* ws, int layer,
                           const uint8_t* hten, float* gh, int acc, const float* dz, int T,
                           int64_t m, hipStream_t s) {
  const Layer& L = n->L[layer];
  const float* W = n->master + param_offset(n->L, layer);
  float* part = (float*)(ws + tp.kpart);
  const int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(tp.kchunks, m / 64));
  if (T > kPwTp || L.ci % 8 || L.ci + 1 > kPwKp)
    return fail(FV_ERR_UNSUPPORTED, "wnet: 1x1 layer %d -> %d", L.ci, T);
  const int groups = L.ci / 4;
  const size_t lds = ((size_t)T * L.ci + (size_t)(256 / groups + 2) * T) * 4;
  k_predict_bwd_h<<<blocks_of(m * groups), 256, lds, s>>>(dz, T, W, L.ci, m, gh, acc);
  k_predict_wgrad<<<chunks, 256, 0, s>>>(dz, T, (const __bf16*)hten, L.ci, m, chunks, part);
  const int nout = T * (L.ci + 1);
  float* part2 = (float*)(ws + tp.part2);
  k_predict_reduce<<<dim3(blocks_of(nout), kPredSlices), 256, 0, s>>>(part, chunks, nout, part2);
  k_predict_reduce2<<<blocks_of(nout), 256, 0, s>>>(part2, T, L.ci,
                                                    n->grad + param_offset(n->L, layer));
  return launch_status("wnet: 1x1 backward");
}

fv_status backward(fv_wnet* n, const float* dloss_dout, int views, int width, int height,
                   void* workspace, hipStream_t s, const uint8_t* state = nullptr) {
  const TPlan tp = make_tplan(views, height, width, n->L);
  const StatePlan sp = make_state_plan(views, height, width);
  const Plan& p = tp.f;
  uint8_t* ws = (uint8_t*)workspace;
  auto G = [&](int t) { return (float*)(ws + tp.g[t]); };
  auto px = [&](int lv) { return (int64_t)views * (height >> lv) * (width >> lv); };
  fv_status st = FV_OK;
  // ---- K decoder, finest level first: dJ is the gradient of J_l
  float* dj = (float*)(ws + tp.dja);
  float* djn = (float*)(ws + tp.djb);
  float* dB = (float*)(ws + tp.db);
  float* dU = (float*)(ws + tp.du);
  float* dwk = (float*)(ws + tp.dwk);
  float* dzk = (float*)(ws + tp.dzk);
  const float* djcur = dloss_dout;
  for (int l = 0; l < 3; ++l) {
    const int h = height >> l, w = width >> l;
    const int64_t m = px(l);
    const float* wk = (const float*)(ws + tp.wkd[l]);
    const float* B = (const float*)(ws + tp.bl[l]);
    const float* jc = l < 2 ? (const float*)(ws + p.jd[l + 1]) : (const float*)(ws + p.je[3]);
    k_apply_bwd_w<<<blocks_of(m), 256, 0, s>>>(djcur, B, views, h, w, dwk);
    k_apply_bwd_img<<<blocks_of(m), 256, 0, s>>>(wk, djcur, views, h, w, dB);
    k_softmax_bwd<<<blocks_of(m), 256, 0, s>>>(wk, dwk, m, kTaps + 1, dzk);
    k_blend_bwd<<<blocks_of(m), 256, 0, s>>>((const float*)(ws + p.je[l]), jc,
                                             (const float*)(ws + tp.av[l]), dB, views, h, w,
                                             (float*)(ws + tp.dje[l]), dU, dzk);
    if ((st = launch_status("wnet: K decoder backward")) != FV_OK) return st;
    // predictor kd_l reads H_l; the first contribution to its gradient
    st = predict_backward(n, tp, ws, kKd2 + (2 - l), ws + p.t[kHidden[l]], G(kHidden[l]), 0,
                          dzk, kTaps + 1, m, s);
    if (st != FV_OK) return st;
    // gradient of the coarser image J_(l+1) through the upsampling
    net::launch_upsample_bwd(dU, 3, 3, views, h / 2, w / 2, djn, 0, s);
    djcur = djn;
    std::swap(dj, djn);
  }
  // ---- K encoder, coarsest level first: d is the gradient of Je_l
  // (djcur holds that of J_3 = Je_3)
  float* d = (float*)djcur;
  for (int l = 3; l >= 0; --l) {
    const int h = height >> l, w = width >> l;
    const int64_t m = px(l);
    if (l < 3) {
      // Je_l feeds the decoder's blend (dje) and, pooled, the next level
      float* de = (float*)(ws + tp.dje[l]);
      net::launch_pool_bwd_add(d, views, h, w, 3, de, s);
      d = de;
    }
    const float* wk = (const float*)(ws + tp.wke[l]);
    const float* jin = l ? (const float*)(ws + p.jin[l]) : (const float*)(ws + p.od);
    float* dnext = (d == dj) ? djn : dj;
    k_apply_bwd_w<<<blocks_of(m), 256, 0, s>>>(d, jin, views, h, w, dwk);
    k_apply_bwd_img<<<blocks_of(m), 256, 0, s>>>(wk, d, views, h, w, dnext);
    k_softmax_bwd<<<blocks_of(m), 256, 0, s>>>(wk, dwk, m, kTaps, dzk);
    if ((st = launch_status("wnet: K encoder backward")) != FV_OK) return st;
    // H_3 has no decoder predictor: ke3 is its first contribution
    st = predict_backward(n, tp, ws, kKe0 + l, ws + p.t[kHidden[l]], G(kHidden[l]), l < 3, dzk,
                          kTaps, m, s);
    if (st != FV_OK) return st;
    d = dnext;
  }
  // d is the gradient of O_d: the head hd (64 -> 3) on d0b
  st = predict_backward(n, tp, ws, kHead, ws + p.t[T_D0B], G(T_D0B), 1, d, 3, px(0), s);
  if (st != FV_OK) return st;
  // ---- D, last conv first
  float* tmp = (float*)(ws + tp.tmp);
  uint8_t* dz = ws + tp.dz;       // masked output gradient of conv l
  uint8_t* dz_next = ws + tp.dz2;  // of conv l - 1, when the dgrad stores it
  bool dz_ready = false;
  float* part = (float*)(ws + tp.part);
  float* part2 = (float*)(ws + tp.part2);
  for (int l = kConv - 1; l >= 0; --l) {
    const Layer& L = n->L[l];
    const int hh = height >> L.level, ww = width >> L.level;
    const int64_t m = px(L.level);
    const bool feed = state && kFeed[l] >= 0;  // reads a fed-back state
    const int ci = L.c0 + L.c1;                 // the channels whose gradient flows on
    if (!dz_ready) net::launch_relu_mask(G(kIO[l][2]), ws + p.t[kIO[l][2]], dz, m * L.co / 8, s);
    dz_ready = false;
    ConvArgs in{};
    in.src0 = ws + p.t[kIO[l][0]];
    in.src1 = kIO[l][1] >= 0 ? ws + p.t[kIO[l][1]] : nullptr;
    in.c0 = L.c0;
    in.c1 = L.c1;
    in.src2 = feed ? state + sp.t[kFeed[l]] : nullptr;
    in.c2 = feed ? L.c2 : 0;
    in.up0 = L.up0;
    in.n = views;
    in.h = hh;
    in.w = ww;
    const int ci_w = ci + in.c2;  // the weight gradient's input channels
    if (l == 0 && L.ci == ci) {
      // the recurrent form's first conv reads all 8 packed channels
      return net::conv_wgrad(in, dz, ci, L.co, tp.chunks[l], part, part2,
                             n->grad + param_offset(n->L, 0), s);
    }
    if (l == 0) {
      // the packed input has 8 channels; the layer's parameters cover 5
      float* g0 = (float*)(ws + tp.w0);
      if ((st = net::conv_wgrad(in, dz, ci, L.co, tp.chunks[l], part, part2, g0, s)) != FV_OK)
        return st;
      float* gdst = n->grad + param_offset(n->L, 0);
      st = hip_status(hipMemcpy2DAsync(gdst, L.ci * 9 * sizeof(float), g0, ci * 9 * sizeof(float),
                                       L.ci * 9 * sizeof(float), L.co, hipMemcpyDeviceToDevice,
                                       s), "wnet: e0a gradient");
      if (st == FV_OK)
        st = hip_status(hipMemcpyAsync(gdst + (int64_t)L.co * L.ci * 9,
                                       g0 + (int64_t)L.co * ci * 9, L.co * sizeof(float),
                                       hipMemcpyDeviceToDevice, s), "wnet: e0a bias gradient");
      return st;
    }
    st = net::conv_wgrad(in, dz, ci_w, L.co, tp.chunks[l], part, part2,
                         n->grad + param_offset(n->L, l), s);
    if (st != FV_OK) return st;
    // input gradient: conv with the transposed weights, FP32 output
    ConvArgs a{};
    a.src0 = dz;
    a.c0 = L.co;
    a.cip = net::cip_of(L.co);
    a.n = views;
    a.h = hh;
    a.w = ww;
    a.wsw = (const uint8_t*)n->w_bf16t[l];
    a.kc = net::kchunks_of(L.co);
    a.co = ci;
    a.out_fp32 = 1;
    a.out_ch = ci;
    const bool concat = kIO[l][1] >= 0;
    // The input is conv l - 1's output with no other consumer (not one of
    // K's inputs): the conv stores that conv's masked BF16 gradient directly,
    // the same bits as the FP32 gradient through the ReLU mask.
    const bool gated = !concat && kIO[l][0] == kIO[l - 1][2];
    uint8_t* obase = gated ? dz_next : (uint8_t*)(concat ? tmp : G(kIO[l][0]));
    const uint8_t* gbase = ws + p.t[kIO[l][0]];
    if (gated) a.out_fp32 = 0;
    // in groups of images whose output stays below the conv's 2 GiB buffer
    // range (the conv works image by image)
    const int64_t img_out = (int64_t)hh * ww * ci * (gated ? 2 : 4);
    const int64_t img_in = (int64_t)hh * ww * L.co * 2;
    const int grp = (int)std::max<int64_t>(
        1, std::min<int64_t>(views, ((((int64_t)1) << 31) - 64 - 1) / img_out));
    for (int b0 = 0; b0 < views; b0 += grp) {
      a.n = std::min(grp, views - b0);
      a.src0 = dz + b0 * img_in;
      a.out = obase + b0 * img_out;
      a.gate = gated ? gbase + b0 * img_out : nullptr;
      if ((st = net::launch_conv<BF16>(a, net::nblocks_of(ci), s)) != FV_OK) return st;
    }
    if (gated) {
      std::swap(dz, dz_next);
      dz_ready = true;
    }
    // The last contribution to conv l - 1's output gradient (the upsample
    // backward for e3b, d2b, d1b after K's; the pool backward for e0b, e1b,
    // e2b after the skip's) stores that conv's masked BF16 gradient instead.
    bool next_ready = false;
    if (concat) {
      // the upsampled source (e3b, d2b, d1b) is also one of K's inputs,
      // whose gradient K has already written: add to it
      next_ready = kIO[l][0] == kIO[l - 1][2];
      net::launch_upsample_bwd(tmp, ci, L.c0, views, hh / 2, ww / 2, G(kIO[l][0]), 1, s,
                               next_ready ? ws + p.t[kIO[l][0]] : nullptr,
                               next_ready ? dz_next : nullptr);
      net::launch_split_skip(tmp, ci, L.c0, L.c1, m, G(kIO[l][1]), s);
    }
    // a pooled input's gradient flows back to the pooled tensor's source
    int src = -1;
    if (kIO[l][0] == T_P0) src = T_E0B;
    if (kIO[l][0] == T_P1) src = T_E1B;
    if (kIO[l][0] == T_P2) src = T_E2B;
    if (src >= 0) {
      next_ready = src == kIO[l - 1][2];
      net::launch_pool_bwd_add(G(kIO[l][0]), views, hh * 2, ww * 2, L.c0, G(src), s,
                               next_ready ? ws + p.t[src] : nullptr,
                               next_ready ? dz_next : nullptr);
    }
    if (next_ready) {
      std::swap(dz, dz_next);
      dz_ready = true;
    }
    if ((st = launch_status("wnet: D backward")) != FV_OK) return st;
  }
  return st;
}

}  // namespace

extern "C" {

size_t fv_wnet_param_count(void) { return (size_t)param_offset(kL, kLayersAll); }
size_t fv_wnet_param_count_recurrent(void) { return (size_t)param_offset(kLR, kLayersAll); }

fv_status fv_wnet_create(const float* host_params, size_t n_params, fv_wnet** out) {
  clear_error();
  if (!host_params || !out) return fail(FV_ERR_INVALID_ARG, "fv_wnet_create: null pointer");
  const int64_t P0 = param_offset(kL, kLayersAll), P1 = param_offset(kLR, kLayersAll);
  if ((int64_t)n_params != P0 && (int64_t)n_params != P1)
    return fail(FV_ERR_INVALID_ARG,
                "fv_wnet_create: %zu parameters, expected %lld (plain) or %lld (recurrent)",
                n_params, (long long)P0, (long long)P1);
  fv_wnet* n = new fv_wnet();
  std::memset(n->w_bf16, 0, sizeof n->w_bf16);
  std::memset(n->w_bf16t, 0, sizeof n->w_bf16t);
  n->grad = n->adam_m = n->adam_v = nullptr;
  n->step = 0;
  n->recurrent = (int64_t)n_params == P1;
  n->L = n->recurrent ? kLR : kL;
  n->master = nullptr;
  const int64_t P = (int64_t)n_params;
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return fail(FV_ERR_DEVICE, "fv_wnet_create: hipGetDevice");
  }
  bool ok = hipMalloc(&n->master, P * sizeof(float)) == hipSuccess;
  for (int l = 0; ok && l < kConv; ++l)
    ok = hipMalloc(&n->w_bf16[l], net::swizzled_elems(n->L[l].ci, n->L[l].co) * 2) ==
         hipSuccess;
  {
    ok = ok && hipMalloc(&n->grad, P * sizeof(float)) == hipSuccess &&
         hipMalloc(&n->adam_m, P * sizeof(float)) == hipSuccess &&
         hipMalloc(&n->adam_v, P * sizeof(float)) == hipSuccess;
    // transposed weights of the input-gradient convs: only the gradients of
    // [upsampled, skip] are used (a fed-back state is an input)
    for (int l = 1; ok && l < kConv; ++l)
      ok = hipMalloc(&n->w_bf16t[l],
                     net::swizzled_elems(n->L[l].co, n->L[l].c0 + n->L[l].c1) * 2) ==
           hipSuccess;
    if (ok)
      ok = hipMemset(n->adam_m, 0, P * sizeof(float)) == hipSuccess &&
           hipMemset(n->adam_v, 0, P * sizeof(float)) == hipSuccess &&
           hipMemset(n->grad, 0, P * sizeof(float)) == hipSuccess;
  }
  if (!ok) {
    fv_wnet_destroy(n);
    return fail(FV_ERR_NOMEM, "fv_wnet_create: allocation");
  }
  fv_status st = hip_status(hipMemcpy(n->master, host_params, P * sizeof(float),
                                      hipMemcpyHostToDevice), "fv_wnet_create: upload");
  if (st == FV_OK) st = refresh_bf16(n, nullptr);
  if (st == FV_OK) st = hip_status(hipDeviceSynchronize(), "fv_wnet_create: sync");
  if (st != FV_OK) {
    fv_wnet_destroy(n);
    return st;
  }
  *out = n;
  return FV_OK;
}

fv_status fv_wnet_destroy(fv_wnet* n) {
  clear_error();
  if (!n) return FV_OK;
  (void)hipFree(n->master);
  (void)hipFree(n->grad);
  (void)hipFree(n->adam_m);
  (void)hipFree(n->adam_v);
  for (int l = 0; l < kConv; ++l) {
    (void)hipFree(n->w_bf16[l]);
    (void)hipFree(n->w_bf16t[l]);
  }
  delete n;
  return FV_OK;
}

int fv_wnet_is_recurrent(const fv_wnet* n) { return n && n->recurrent ? 1 : 0; }

fv_status fv_wnet_workspace(int views, int width, int height, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(FV_ERR_INVALID_ARG, "fv_wnet_workspace: null bytes");
  fv_status st = net::check_frame(views, width, height, "fv_wnet_workspace");
  if (st != FV_OK) return st;
  *bytes = make_plan(views, height, width).bytes;
  return FV_OK;
}

fv_status fv_wnet_state_bytes(int views, int width, int height, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(FV_ERR_INVALID_ARG, "fv_wnet_state_bytes: null bytes");
  fv_status st = net::check_frame(views, width, height, "fv_wnet_state_bytes");
  if (st != FV_OK) return st;
  *bytes = make_state_plan(views, height, width).bytes;
  return FV_OK;
}

fv_status fv_wnet_state_layout(int views, int width, int height, size_t* od_offset,
                               size_t* d2_offset, size_t* d1_offset, size_t* d0_offset) {
  clear_error();
  if (!od_offset || !d2_offset || !d1_offset || !d0_offset)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_state_layout: null pointer");
  fv_status st = net::check_frame(views, width, height, "fv_wnet_state_layout");
  if (st != FV_OK) return st;
  const StatePlan sp = make_state_plan(views, height, width);
  *od_offset = sp.od;
  *d2_offset = sp.t[T_D2B];
  *d1_offset = sp.t[T_D1B];
  *d0_offset = sp.t[T_D0B];
  return FV_OK;
}

fv_status fv_wnet_reconstruct(const fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                              const float* frame_depth, int views, int width, int height,
                              float* out_rgb, float* out_direct, void* workspace,
                              size_t ws_bytes, void* stream) {
  clear_error();
  return reconstruct(n, frame_rgba, mask, frame_depth, nullptr, 0, 0, views, width, height,
                     out_rgb, out_direct, workspace, ws_bytes, stream, "fv_wnet_reconstruct");
}

fv_status fv_wnet_reconstruct_recurrent(const fv_wnet* n, const float* frame_rgba,
                                        const uint8_t* mask, const float* frame_depth,
                                        void* state, size_t state_bytes, int reset, int views,
                                        int width, int height, float* out_rgb,
                                        float* out_direct, void* workspace, size_t ws_bytes,
                                        void* stream) {
  clear_error();
  if (!state) return fail(FV_ERR_INVALID_ARG, "fv_wnet_reconstruct_recurrent: null state");
  return reconstruct(n, frame_rgba, mask, frame_depth, state, state_bytes, reset, views, width,
                     height, out_rgb, out_direct, workspace, ws_bytes, stream,
                     "fv_wnet_reconstruct_recurrent");
}

}  // extern "C"

extern "C" {

fv_status fv_wnet_train_workspace(const fv_wnet* n, int batch, int width, int height,
                                  size_t* bytes) {
  clear_error();
  if (!n || !bytes) return fail(FV_ERR_INVALID_ARG, "fv_wnet_train_workspace: null pointer");
  fv_status st = net::check_frame(batch, width, height, "fv_wnet_train_workspace");
  if (st != FV_OK) return st;
  *bytes = make_tplan(batch, height, width, n->L).bytes;
  return FV_OK;
}

fv_status fv_wnet_forward_train(fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                                const float* frame_depth, int batch, int width, int height,
                                float* out_rgb, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  TPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_wnet_forward_train");
  if (st != FV_OK) return st;
  const KKeep k = keep_of(tp, (uint8_t*)workspace);
  return reconstruct(n, frame_rgba, mask, frame_depth, nullptr, 0, 0, batch, width, height,
                     out_rgb, nullptr, workspace, ws_bytes, stream, "fv_wnet_forward_train", &k);
}

fv_status fv_wnet_backward(fv_wnet* n, const float* dloss_dout, int batch, int width,
                           int height, float* grad_out, void* workspace, size_t ws_bytes,
                           void* stream) {
  clear_error();
  TPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_wnet_backward");
  if (st != FV_OK) return st;
  if (!dloss_dout) return fail(FV_ERR_INVALID_ARG, "fv_wnet_backward: null dloss_dout");
  hipStream_t s = (hipStream_t)stream;
  if ((st = backward(n, dloss_dout, batch, width, height, workspace, s)) != FV_OK) return st;
  if (grad_out)
    st = hip_status(hipMemcpyAsync(grad_out, n->grad, param_offset(n->L, kLayersAll) * 4,
                                   hipMemcpyDeviceToDevice, s), "fv_wnet_backward: copy");
  return st;
}

fv_status fv_wnet_forward_train_recurrent(fv_wnet* n, const float* frame_rgba,
                                          const uint8_t* mask, const float* frame_depth,
                                          const void* state, size_t state_bytes, int batch,
                                          int width, int height, float* out_rgb,
                                          void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  TPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_wnet_forward_train_recurrent", state, state_bytes);
  if (st != FV_OK) return st;
  const KKeep k = keep_of(tp, (uint8_t*)workspace);
  return reconstruct(n, frame_rgba, mask, frame_depth, const_cast<void*>(state), state_bytes, 0,
                     batch, width, height, out_rgb, nullptr, workspace, ws_bytes, stream,
                     "fv_wnet_forward_train_recurrent", &k);
}

fv_status fv_wnet_backward_recurrent(fv_wnet* n, const float* dloss_dout, const void* state,
                                     size_t state_bytes, int batch, int width, int height,
                                     float* grad_out, void* workspace, size_t ws_bytes,
                                     void* stream) {
  clear_error();
  TPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_wnet_backward_recurrent", state, state_bytes);
  if (st != FV_OK) return st;
  if (!dloss_dout) return fail(FV_ERR_INVALID_ARG, "fv_wnet_backward_recurrent: null dloss");
  hipStream_t s = (hipStream_t)stream;
  if ((st = backward(n, dloss_dout, batch, width, height, workspace, s,
                     (const uint8_t*)state)) != FV_OK)
    return st;
  if (grad_out)
    st = hip_status(hipMemcpyAsync(grad_out, n->grad, param_offset(n->L, kLayersAll) * 4,
                                   hipMemcpyDeviceToDevice, s), "fv_wnet_backward: copy");
  return st;
}

fv_status fv_wnet_loss_temporal(const fv_wnet* n, const float* out_rgb,
                                const float* target_rgba, int batch, int width, int height,
                                float weight, float* loss, float* dloss_dout, void* workspace,
                                size_t ws_bytes, void* stream) {
  clear_error();
  if (!n || !workspace || !out_rgb || !target_rgba || !loss || !dloss_dout)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_loss_temporal: null pointer");
  fv_status st = net::check_frame(batch, width, height, "fv_wnet_loss_temporal");
  if (st != FV_OK) return st;
  if (batch % 2)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_loss_temporal: batch %d is not a set of pairs",
                batch);
  if (!(weight >= 0.0f && std::isfinite(weight)))
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_loss_temporal: weight must be finite and >= 0");
  const TPlan tp = make_tplan(batch, height, width, n->L);
  if (ws_bytes < tp.bytes)
    return fail(FV_ERR_CAPACITY, "fv_wnet_loss_temporal: workspace %zu < %zu bytes", ws_bytes,
                tp.bytes);
  return net::tloss_run(out_rgb, target_rgba, batch / 2, height, width, weight, loss,
                        dloss_dout, (double*)((uint8_t*)workspace + tp.red),
                        (hipStream_t)stream);
}

fv_status fv_wnet_loss(const fv_wnet* n, const float* out_rgb, const float* target_rgba,
                       int batch, int width, int height, float* loss3, float* dloss_dout,
                       void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (!n || !workspace || !out_rgb || !target_rgba || !loss3 || !dloss_dout)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_loss: null pointer");
  fv_status st = net::check_frame(batch, width, height, "fv_wnet_loss");
  if (st != FV_OK) return st;
  const TPlan tp = make_tplan(batch, height, width, n->L);
  if (ws_bytes < tp.bytes)
    return fail(FV_ERR_CAPACITY, "fv_wnet_loss: workspace %zu < %zu bytes", ws_bytes, tp.bytes);
  uint8_t* ws = (uint8_t*)workspace;
  return net::loss_run(out_rgb, target_rgba, batch, height, width, loss3, dloss_dout,
                       (float*)(ws + tp.tgt), ws + tp.ssim, (double*)(ws + tp.red),
                       (hipStream_t)stream);
}

fv_status fv_wnet_adam(fv_wnet* n, float lr, float beta1, float beta2, float eps, void* stream) {
  clear_error();
  if (!n) return fail(FV_ERR_INVALID_ARG, "fv_wnet_adam: null net");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_adam: bad hyper-parameters");
  hipStream_t s = (hipStream_t)stream;
  n->step += 1;
  fv_status st = net::adam_run(n->master, n->adam_m, n->adam_v, n->grad,
                               param_offset(kL, kLayersAll), lr, beta1, beta2, eps, n->step, s);
  if (st == FV_OK) st = refresh_bf16(n, s);
  return st;
}

fv_status fv_wnet_train_step(fv_wnet* n, const float* frame_rgba, const uint8_t* mask,
                             const float* frame_depth, const float* target_rgba, int batch,
                             int width, int height, float lr, float* loss3, void* workspace,
                             size_t ws_bytes, void* stream) {
  clear_error();
  TPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_wnet_train_step");
  if (st != FV_OK) return st;
  if (!target_rgba || !loss3) return fail(FV_ERR_INVALID_ARG, "fv_wnet_train_step: null pointer");
  uint8_t* ws = (uint8_t*)workspace;
  hipStream_t s = (hipStream_t)stream;
  float* out = (float*)(ws + tp.out);
  float* dout = (float*)(ws + tp.dout);
  if ((st = fv_wnet_forward_train(n, frame_rgba, mask, frame_depth, batch, width, height, out,
                                  workspace, ws_bytes, stream)) != FV_OK)
    return st;
  if ((st = net::loss_run(out, target_rgba, batch, height, width, loss3, dout,
                          (float*)(ws + tp.tgt), ws + tp.ssim, (double*)(ws + tp.red), s)) !=
      FV_OK)
    return st;
  if ((st = backward(n, dout, batch, width, height, workspace, s)) != FV_OK) return st;
  return fv_wnet_adam(n, lr, 0.9f, 0.999f, 1e-8f, stream);
}

fv_status fv_wnet_get_params(const fv_wnet* n, float* host_out, size_t n_params) {
  clear_error();
  if (!n || !host_out) return fail(FV_ERR_INVALID_ARG, "fv_wnet_get_params: null pointer");
  const int64_t P = param_offset(n->L, kLayersAll);
  if ((int64_t)n_params != P)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_get_params: %zu parameters, the network has %lld",
                n_params, (long long)P);
  return hip_status(hipMemcpy(host_out, n->master, P * sizeof(float), hipMemcpyDeviceToHost),
                    "fv_wnet_get_params");
}

fv_status fv_wnet_set_params(fv_wnet* n, const float* host_params, size_t n_params) {
  clear_error();
  if (!n || !host_params) return fail(FV_ERR_INVALID_ARG, "fv_wnet_set_params: null pointer");
  const int64_t P = param_offset(n->L, kLayersAll);
  if ((int64_t)n_params != P)
    return fail(FV_ERR_INVALID_ARG, "fv_wnet_set_params: %zu parameters, the network has %lld",
                n_params, (long long)P);
  fv_status st = hip_status(hipMemcpy(n->master, host_params, P * sizeof(float),
                                      hipMemcpyHostToDevice), "fv_wnet_set_params");
  if (st == FV_OK) st = refresh_bf16(n, nullptr);
  if (st == FV_OK) st = hip_status(hipDeviceSynchronize(), "fv_wnet_set_params: sync");
  return st;
}

}  // extern "C"
