// Reconstruction network: forward kernels, the handle, FP8 calibration and
// fv_reconstruct (paper: "Reconstruction Network", "Model Precision &
// Optimization").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "net.h"
#include "net_kernels.h"

namespace fv {
namespace net {

const LayerDesc kLayers[kNumLayers] = {
    // name   ci  co  k lvl  c0  c1 up0
    {"e0a", 8, 32, 3, 0, 8, 0, 0},     {"e0b", 32, 32, 3, 0, 32, 0, 0},
    {"e1a", 32, 48, 3, 1, 32, 0, 0},   {"e1b", 48, 48, 3, 1, 48, 0, 0},
    {"e2a", 48, 64, 3, 2, 48, 0, 0},   {"e2b", 64, 64, 3, 2, 64, 0, 0},
    {"e3a", 64, 96, 3, 3, 64, 0, 0},   {"e3b", 96, 96, 3, 3, 96, 0, 0},
    {"d2a", 160, 64, 3, 2, 96, 64, 1}, {"d2b", 64, 64, 3, 2, 64, 0, 0},
    {"d1a", 112, 48, 3, 1, 64, 48, 1}, {"d1b", 48, 48, 3, 1, 48, 0, 0},
    {"d0a", 80, 32, 3, 0, 48, 32, 1},  {"d0b", 32, 32, 3, 0, 32, 0, 0},
    {"hd", 32, 3, 1, 0, 32, 0, 0},     {"hk", 32, 25, 1, 0, 32, 0, 0},
};

const TensorDesc kTensors[kNumTensors] = {
    {8, 0},  {32, 0}, {32, 0}, {32, 1}, {48, 1}, {48, 1}, {48, 2}, {64, 2}, {64, 2},
    {64, 3}, {96, 3}, {96, 3}, {64, 2}, {64, 2}, {48, 1}, {48, 1}, {32, 0}, {32, 0},
};

// Per conv layer: (src0, src1 or -1, output) tensors.
const int kLayerIO[kNumConv][3] = {
    {T_IN, -1, T_E0A},    {T_E0A, -1, T_E0B}, {T_P0, -1, T_E1A},   {T_E1A, -1, T_E1B},
    {T_P1, -1, T_E2A},    {T_E2A, -1, T_E2B}, {T_P2, -1, T_E3A},   {T_E3A, -1, T_E3B},
    {T_E3B, T_E2B, T_D2A}, {T_D2A, -1, T_D2B}, {T_D2B, T_E1B, T_D1A}, {T_D1A, -1, T_D1B},
    {T_D1B, T_E0B, T_D0A}, {T_D0A, -1, T_D0B},
};

int64_t param_offset(int layer) {
  int64_t off = 0;
  for (int i = 0; i < layer; ++i) {
    const LayerDesc& L = kLayers[i];
    off += (int64_t)L.co * L.ci * L.k * L.k + L.co;
  }
  return off;
}

int64_t param_count() { return param_offset(kNumLayers); }

int64_t external_param_count(int recurrent) {
  return param_count() - (recurrent ? 0 : (int64_t)kLayers[0].co * kFedBack * 9);
}

// The first conv's weights are [32][8][3][3] inside and [32][5][3][3] in the
// plain form's external vector; everything after them is shifted alike.
void params_to_internal(const float* ext, int recurrent, float* in) {
  const int64_t n = param_count();
  if (recurrent) {
    std::memcpy(in, ext, n * sizeof(float));
    return;
  }
  const int co = kLayers[0].co, ci = kLayers[0].ci, ce = ci - kFedBack;
  for (int o = 0; o < co; ++o)
    for (int c = 0; c < ci; ++c)
      for (int t = 0; t < 9; ++t)
        in[((int64_t)o * ci + c) * 9 + t] = c < ce ? ext[((int64_t)o * ce + c) * 9 + t] : 0.0f;
  const int64_t wi = (int64_t)co * ci * 9, we = (int64_t)co * ce * 9;
  std::memcpy(in + wi, ext + we, (n - wi) * sizeof(float));
}

void params_to_external(const float* in, int recurrent, float* ext) {
  const int64_t n = param_count();
  if (recurrent) {
    std::memcpy(ext, in, n * sizeof(float));
    return;
  }
  const int co = kLayers[0].co, ci = kLayers[0].ci, ce = ci - kFedBack;
  for (int o = 0; o < co; ++o)
    std::memcpy(ext + (int64_t)o * ce * 9, in + (int64_t)o * ci * 9, ce * 9 * sizeof(float));
  const int64_t wi = (int64_t)co * ci * 9, we = (int64_t)co * ce * 9;
  std::memcpy(ext + we, in + wi, (n - wi) * sizeof(float));
}

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

Plan make_plan(int n, int h, int w, size_t elem) {
  Plan p;
  p.n = n;
  p.h = h;
  p.w = w;
  p.elem = elem;
  size_t off = 0;
  for (int t = 0; t < kNumTensors; ++t) {
    const int lv = kTensors[t].level;
    p.t[t] = off;
    off += align256((size_t)n * (h >> lv) * (w >> lv) * kTensors[t].channels * elem);
  }
  p.od = off;
  off += align256((size_t)n * h * w * 3 * sizeof(float));
  p.wk = off;
  off += align256((size_t)n * h * w * 25 * sizeof(float));
  p.absmax = off;
  off += align256(64 * sizeof(float));
  p.bytes = off;
  return p;
}

// ------------------------------------------------------------------ kernels

// Sparse frame -> 8-channel network input
// [M r, M g, M b, M, M depth/2, O_d,prev r, g, b] (the back-projected sparse
// image with its mask and depth; paper: the network reconstructs from the
// sparse RGB input; the last three are the previous frame's direct
// prediction in the recurrent form, Sec. 3.2.4, else 0).  The frame is not
// read where M = 0; the previous O_d is read everywhere.
template <class E>
__global__ void __launch_bounds__(256) k_pack(const float4* __restrict__ rgba,
                                              const uint8_t* __restrict__ mask,
                                              const float* __restrict__ depth,
                                              const float* __restrict__ prev, uint8_t* out,
                                              int64_t npx, float inv_scale,
                                              float* __restrict__ absmax) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (p < npx && mask[p]) {
    const float4 c = rgba[p];
    v[0] = c.x;
    v[1] = c.y;
    v[2] = c.z;
    v[3] = 1.0f;
    v[4] = depth ? 0.5f * depth[p] : 0.0f;
  }
  if (p < npx && prev) {
    v[5] = prev[p * 3 + 0];
    v[6] = prev[p * 3 + 1];
    v[7] = prev[p * 3 + 2];
  }
  if (absmax) {
    float m = 0.f;
    for (int i = 0; i < 8; ++i) m = fmaxf(m, fabsf(v[i]));
    wave_absmax(absmax, m);
  }
  if (p >= npx) return;
  for (int i = 0; i < 8; ++i) v[i] *= inv_scale;
  E::store8(out + p * 8 * E::kBytes, v);
}

template <class E>
__global__ void __launch_bounds__(256) k_avgpool2(const uint8_t* __restrict__ src,
                                                  uint8_t* __restrict__ dst, int n, int h, int w,
                                                  int c) {
  // one thread = one output pixel x 8 channels
  const int groups = c / 8;
  const int64_t total = (int64_t)n * (h / 2) * (w / 2) * groups;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int g = (int)(e % groups);
  const int64_t pix = e / groups;
  const int ox = (int)(pix % (w / 2));
  const int64_t r = pix / (w / 2);
  const int oy = (int)(r % (h / 2));
  const int b = (int)(r / (h / 2));
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      float v[8];
      const int64_t sp = ((int64_t)b * h + 2 * oy + dy) * w + 2 * ox + dx;
      E::load8(src + (sp * c + g * 8) * E::kBytes, v);
      for (int i = 0; i < 8; ++i) acc[i] += v[i];
    }
  for (int i = 0; i < 8; ++i) acc[i] *= 0.25f;
  E::store8(dst + (pix * c + g * 8) * E::kBytes, acc);
}

// Heads: O_d = 1x1 conv (32 -> 3), logits = 1x1 conv (32 -> 25), w = softmax,
// out(p) = sum_k w_k(p) O_d(clamp(p + delta_k)) over the 5x5 taps.
// One 16x16 output tile per block.  The two 1x1 convs are one MFMA GEMM
// [400 halo pixels x 32] x [32 x 32] (BF16 operands, FP32 accumulation; FP8
// activations are widened in registers) whose 28 used columns land in LDS;
// softmax and the kernel application run in FP32.
// 8 stored channels of one pixel as BF16 (exact for E4M3 codes; the FP8
// tensor scale is folded into the FP8-mode head weights).
template <class E>
__device__ __forceinline__ bf16x8_t heads_frag(const typename Chunk8<E>::T& raw);

template <>
__device__ __forceinline__ bf16x8_t heads_frag<FP8>(const uint2& raw) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)raw.x, 1.0f, false);
  const bf16x2_t p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)raw.x, 1.0f, true);
  const bf16x2_t p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)raw.y, 1.0f, false);
  const bf16x2_t p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)raw.y, 1.0f, true);
  return bf16x8_t{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}

template <>
__device__ __forceinline__ bf16x8_t heads_frag<BF16>(const uint4& raw) {
  return __builtin_bit_cast(bf16x8_t, raw);
}

// The two 1x1 heads and the kernel-prediction output (Sec. 3.2, "Direct
// Prediction" and "Kernel Prediction"): per pixel O_d = hd . h + b_d and
// logits = hk . h + b_k (h = the 32 decoder channels), w = softmax(logits)
// over the 25 taps, O = sum_q w_q O_d(pixel + offset_q) with edge-replicated
// O_d.  Block = 16 x 16 output pixels.  Both heads run on MFMA with the head
// weights as the A operand, so a lane holds 4 output channels of one pixel:
// O_d of the 20 x 20 halo goes to LDS, while the logits of a tile pixel stay
// in the registers of the 4 lanes that own it and the softmax and the 5 x 5
// sum reduce across those lanes.  All global loads of a wave are issued
// before the first MFMA.
template <class E>
__global__ void __launch_bounds__(256) k_heads(const uint8_t* __restrict__ hdec, int n, int h,
                                               int w, const float* __restrict__ params,
                                               const __bf16* __restrict__ whs,
                                               int64_t off_hd, int64_t off_hk,
                                               float* __restrict__ out_rgb,
                                               float* __restrict__ out_od,
                                               float* __restrict__ out_wk) {
  constexpr int HW = 20, HB = HW * HW / 16;  // halo width, halo blocks of 16 pixels
  constexpr int KH = (HB + 3) / 4;           // halo blocks per wave (at most)
  using Raw = typename Chunk8<E>::T;
  __shared__ float4 s_od[HW * HW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 16, b = blockIdx.z;
  const uint8_t* img = hdec + (int64_t)b * h * w * 32 * E::kBytes + 8 * grp * E::kBytes;
  Raw rh[KH], rc[4];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hb = min(wave + 4 * k, HB - 1);  // (a repeated block is not stored)
    const int hp = hb * 16 + col, r = hp / HW, c = hp - r * HW;
    const int y = min(max(y0 - 2 + r, 0), h - 1), x = min(max(x0 - 2 + c, 0), w - 1);
    rh[k] = *(const Raw*)(img + ((int64_t)y * w + x) * 32 * E::kBytes);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int y = min(y0 + wave * 4 + m, h - 1), x = min(x0 + col, w - 1);
    rc[m] = *(const Raw*)(img + ((int64_t)y * w + x) * 32 * E::kBytes);
  }
  // A operands: rows 0-15 = [hd 0-2, hk 0-12], rows 16-31 = [hk 13-24, 4 zero]
  const bf16x8_t w0 = *(const bf16x8_t*)(whs + (size_t)lane * 8);
  const bf16x8_t w1 = *(const bf16x8_t*)(whs + (size_t)(64 + lane) * 8);
  // this lane's 8 output channels: 4 grp + i (block 0) and 16 + 4 grp + i
  // (block 1); channel c < 3 is O_d, 3 <= c < 28 the logit of tap c - 3.
  // Slots that are not taps get a -inf logit bias: their softmax weight is 0.
  float bias[8];
  int tap_off[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int c = (j < 4 ? 0 : 16) + 4 * grp + (j & 3);
    const bool tap = c >= 3 && c < 28;
    bias[j] = tap ? params[off_hk + 800 + c - 3] : -INFINITY;
    const int q = tap ? c - 3 : 0;
    tap_off[j] = (q / 5) * HW + q % 5;
  }
  float bd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) bd[i] = params[off_hd + 96 + i];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int hb = wave + 4 * k;
    const f32x4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
        w0, heads_frag<E>(rh[k]), f32x4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    if (hb < HB && grp == 0)
      s_od[hb * 16 + col] = make_float4(d[0] + bd[0], d[1] + bd[1], d[2] + bd[2], 0.f);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int ty = wave * 4 + m, y = y0 + ty, x = x0 + col;
    const bf16x8_t f = heads_frag<E>(rc[m]);
    const f32x4_t d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, f, f32x4_t{0.f, 0.f, 0.f, 0.f},
                                                               0, 0, 0);
    const f32x4_t d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, f, f32x4_t{0.f, 0.f, 0.f, 0.f},
                                                               0, 0, 0);
    float lg[8];
    float mx = -INFINITY;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      lg[j] = (j < 4 ? d0[j] : d1[j - 4]) + bias[j];
      mx = fmaxf(mx, lg[j]);
    }
    mx = pair_max32(pair_max16(mx));
    float den = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      lg[j] = __expf(lg[j] - mx);
      den += lg[j];
    }
    den = pair_sum32(pair_sum16(den));
    const float inv = __builtin_amdgcn_rcpf(den);  // hardware reciprocal (1 ulp)
    const float4* win = s_od + ty * HW + col;  // top-left of this pixel's 5 x 5 window
    float o0 = 0.f, o1 = 0.f, o2 = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      lg[j] *= inv;
      const float4 od = win[tap_off[j]];
      o0 = fmaf(lg[j], od.x, o0);
      o1 = fmaf(lg[j], od.y, o1);
      o2 = fmaf(lg[j], od.z, o2);
    }
    o0 = pair_sum32(pair_sum16(o0));
    o1 = pair_sum32(pair_sum16(o1));
    o2 = pair_sum32(pair_sum16(o2));
    if (y >= h || x >= w) continue;
    const int64_t p = ((int64_t)b * h + y) * w + x;
    if (grp == 0) {
      out_rgb[p * 3 + 0] = o0;
      out_rgb[p * 3 + 1] = o1;
      out_rgb[p * 3 + 2] = o2;
      if (out_od) {
        out_od[p * 3 + 0] = d0[0] + bd[0];
        out_od[p * 3 + 1] = d0[1] + bd[1];
        out_od[p * 3 + 2] = d0[2] + bd[2];
      }
    }
    if (out_wk) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = (j < 4 ? 0 : 16) + 4 * grp + (j & 3);
        if (c >= 3 && c < 28) out_wk[p * 25 + c - 3] = lg[j];
      }
    }
  }
}

// Head weights [hd (3 rows); hk (25 rows); 4 zero rows] x 32 inputs as the
// two BF16 MFMA B fragments (n block 0: rows 0-15, n block 1: rows 16-31).
__global__ void k_swizzle_heads(const float* __restrict__ hd, const float* __restrict__ hk,
                                __bf16* __restrict__ out, float scale) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= 2 * 512) return;
  const int j = e & 7, l = (e >> 3) & 63, nb = e >> 9;
  const int nrow = nb * 16 + (l & 15), k = 8 * (l >> 4) + j;
  float v = 0.f;
  if (nrow < 3)
    v = hd[nrow * 32 + k];
  else if (nrow < 28)
    v = hk[(nrow - 3) * 32 + k];
  out[e] = (__bf16)(v * scale);
}

// Master FP32 weights of a 3x3 layer -> swizzled BF16 MFMA B fragments.
// transposed = 1 builds the weights of the input-gradient convolution
// (in/out channels swapped, taps mirrored).
__global__ void __launch_bounds__(256) k_swizzle_bf16(const float* __restrict__ w, int ci, int co,
                                                      int transposed, int kc, int nb,
                                                      int out_limit, __bf16* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)kc * nb * 512;
  if (e >= total) return;
  const int j = (int)(e & 7), l = (int)((e >> 3) & 63);
  const int nbi = (int)((e >> 9) % nb);
  const int c = (int)(e / (512 * (int64_t)nb));
  // GEMM view: input channels (K side) and output channels (N side)
  const int in_ch = transposed ? co : ci, out_ch = min(transposed ? ci : co, out_limit);
  const int cip = cip_of(in_ch);
  const int kk = c * 32 + 8 * (l >> 4) + j;
  const int tap = kk / cip, kin = kk - tap * cip;
  const int nout = nbi * 16 + (l & 15);
  float v = 0.f;
  if (tap < 9 && kin < in_ch && nout < out_ch) {
    if (!transposed)
      v = w[((int64_t)nout * ci + kin) * 9 + tap];
    else
      v = w[((int64_t)kin * ci + nout) * 9 + (8 - tap)];
  }
  out[e] = (__bf16)v;
}

__global__ void __launch_bounds__(256) k_f32_to_fp8(const float* __restrict__ src,
                                                    uint8_t* __restrict__ dst, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  dst[e] = FP8::enc(src[e]);
}

__global__ void k_zero_f32(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------- launchers

template <class E, int NB, int R>
void conv_launch(const ConvArgs& a, hipStream_t s) {
  static bool attr_set = false;
  const size_t lds = conv_lds_bytes<E, R>(a.cip, a.c0, a.up0, a.kc, NB, a.co, a.b_lds) +
                     (!a.fuse0 ? 0
                      : a.f_mixed ? fuse0_lds_bytes<BF16, R>(a.f_kc)
                                  : fuse0_lds_bytes<E, R>(a.f_kc));
  if (!attr_set) {
    hipFuncSetAttribute((const void*)k_conv3x3<E, NB, R>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  // one block per tile, tiles in (image, row, column) order
  const dim3 grid((a.w + 15) / 16, (a.h + 4 * R - 1) / (4 * R), a.n);
  k_conv3x3<E, NB, R><<<grid, 256, lds, s>>>(a);
}

template <class E, int NB>
void conv_nb(const ConvArgs& a, int R, hipStream_t s) {
  if (R == 4)
    conv_launch<E, NB, 4>(a, s);
  else if (R == 2)
    conv_launch<E, NB, 2>(a, s);
  else
    conv_launch<E, NB, 1>(a, s);
}

template <class E>
fv_status launch_conv(const ConvArgs& args, int nb, hipStream_t s) {
  ConvArgs a = args;
  // source sizes for the kernel's buffer-load range checks (loads outside the
  // image use an offset of 2 GiB, so every source must stay below that)
  const int64_t px = (int64_t)a.n * a.h * a.w;
  const int64_t b0 = (a.up0 ? (int64_t)a.n * (a.h >> 1) * (a.w >> 1) : px) * a.c0 * E::kBytes;
  const int64_t b1 = a.src1 ? px * a.c1 * E::kBytes : 0;
  const int64_t b2 = a.src2 ? px * a.c2 * E::kBytes : 0;
  const int64_t bmax = std::max(b0, std::max(b1, b2));
  if (bmax >= ((int64_t)1 << 31) - 64)
    return fail(FV_ERR_UNSUPPORTED, "conv: an input tensor of %lld bytes (limit 2 GiB)",
                (long long)bmax);
  if (a.src2 && (!a.src1 || (a.c0 + a.c1) % 8 || a.c2 <= 0))
    return fail(FV_ERR_UNSUPPORTED, "conv: a third source needs the second and 8-aligned groups");
  if (!a.src2) a.c2 = 0;
  a.src0_bytes = (uint32_t)b0;
  a.src1_bytes = (uint32_t)b1;
  a.src2_bytes = (uint32_t)b2;
  const int64_t bo = px * a.out_ch * (a.out_fp32 ? 4 : E::kBytes);
  const int64_t bp = a.pool_out ? (int64_t)a.n * (a.h >> 1) * (a.w >> 1) * a.out_ch * E::kBytes : 0;
  if (bo >= ((int64_t)1 << 31) - 64)
    return fail(FV_ERR_UNSUPPORTED, "conv: an output tensor of %lld bytes (limit 2 GiB)",
                (long long)bo);
  a.out_bytes = (uint32_t)bo;
  a.pool_bytes = (uint32_t)bp;
  if (a.gate && (E::kBytes != 2 || a.out_fp32 || a.pool_out || a.relu || a.absmax))
    return fail(FV_ERR_UNSUPPORTED, "conv: a gated output is a plain BF16 store");
  auto magic = [](uint32_t d) { return d > 1 ? (uint32_t)(((uint64_t)1 << 32) / d + 1) : 0u; };
  if (a.up0 && (a.c0 % 8 || a.c0 < 16 || (a.h | a.w) & 1))
    return fail(FV_ERR_UNSUPPORTED, "conv: upsampled source with %d channels at %d x %d", a.c0,
                a.w, a.h);
  // FP8 fill items of 16 channels when no item straddles a source boundary
  a.wide = E::kBytes == 1 && a.cip % 16 == 0 && a.c0 % 16 == 0 && a.c1 % 16 == 0 &&
           a.c2 % 16 == 0;
  const uint32_t iw = a.wide ? 16u : 8u;
  const uint32_t g0 = a.up0 ? (uint32_t)a.c0 / iw : 0u;
  a.gmagic = magic((uint32_t)a.cip / iw - g0);
  a.umagic = magic(g0);
  a.umagic8 = magic((uint32_t)a.c0 >> 3);  // (exact for the 2 x 2 block items too)
  // rows per wave: the largest R that still gives at least two blocks per CU
  // (256 CUs) and whose patch fits in 48 KB of LDS (64 KB for BF16, whose
  // wide concatenating layers would otherwise drop to one row per wave); the
  // weights are staged in LDS only while the block's LDS stays within 40 KB
  // (four blocks per CU)
  auto lds_of = [&](int r, int bl) {
    return r == 4 ? conv_lds_bytes<E, 4>(a.cip, a.c0, a.up0, a.kc, nb, a.co, bl)
                  : r == 2 ? conv_lds_bytes<E, 2>(a.cip, a.c0, a.up0, a.kc, nb, a.co, bl)
                           : conv_lds_bytes<E, 1>(a.cip, a.c0, a.up0, a.kc, nb, a.co, bl);
  };
  const size_t patch_max = (E::kBytes == 2 ? 64 : 48) * 1024;
  int R = 4;
  while (R > 1) {
    const int64_t blocks = (int64_t)((a.w + 15) / 16) * ((a.h + 4 * R - 1) / (4 * R)) * a.n;
    if (lds_of(R, 0) <= patch_max && blocks >= 512) break;
    R >>= 1;
  }
  if (nb >= 7 && R == 4) R = 2;  // 112+ accumulators per lane would spill
  a.b_lds = (size_t)a.kc * nb * 64 * E::kFragBytes <= kMaxLdsWeights && lds_of(R, 1) <= 40 * 1024;
  if (a.fuse0) {
    // the fused first layer keeps both layers' weights in LDS
    if (nb != 2 || a.up0 || a.co != 32 || a.cip != 32)
      return fail(FV_ERR_UNSUPPORTED, "conv: fused first layer needs a 32 -> 32 conv");
    a.b_lds = 1;
  }
  if (a.co % 8 || a.co > 256) return fail(FV_ERR_UNSUPPORTED, "conv: %d output channels", a.co);
  // the fused 2x2 pooling needs both rows of a pair in one wave
  uint8_t* pool_out = a.pool_out;
  if (pool_out && (R == 1 || a.out_fp32 || a.out_ch != a.co || (a.h | a.w) & 1)) a.pool_out = nullptr;
  switch (nb) {
    case 1: conv_nb<E, 1>(a, R, s); break;
    case 2: conv_nb<E, 2>(a, R, s); break;
    case 3: conv_nb<E, 3>(a, R, s); break;
    case 4: conv_nb<E, 4>(a, R, s); break;
    case 5: conv_nb<E, 5>(a, R, s); break;
    case 6: conv_nb<E, 6>(a, R, s); break;
    case 7: conv_nb<E, 7>(a, R, s); break;
    case 10: conv_nb<E, 10>(a, R, s); break;
    default:
      // 8, 9 and 11 blocks (128, 144, 176 channels): the W-Net's input-
      // gradient convolutions, BF16 only
      if constexpr (E::kBytes == 2) {
        if (nb == 8) {
          conv_nb<E, 8>(a, R, s);
          break;
        }
        if (nb == 9) {
          conv_nb<E, 9>(a, R, s);
          break;
        }
        if (nb == 11) {
          conv_nb<E, 11>(a, R, s);
          break;
        }
      }
      return fail(FV_ERR_UNSUPPORTED, "conv: %d output blocks", nb);
  }
  if (pool_out && !a.pool_out) {
    const int64_t total = (int64_t)a.n * (a.h / 2) * (a.w / 2) * (a.co / 8);
    k_avgpool2<E><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(a.out, pool_out, a.n, a.h,
                                                                  a.w, a.co);
  }
  return launch_status("conv3x3");
}

template fv_status launch_conv<BF16>(const ConvArgs&, int, hipStream_t);
template fv_status launch_conv<FP8>(const ConvArgs&, int, hipStream_t);

fv_status swizzle_bf16(const float* w, int ci, int co, int transposed, void* out, hipStream_t s,
                       int out_limit) {
  const int in_ch = transposed ? co : ci;
  const int out_ch = std::min(transposed ? ci : co, out_limit);
  const int kc = kchunks_of(in_ch), nb = nblocks_of(out_ch);
  const int64_t total = (int64_t)kc * nb * 512;
  k_swizzle_bf16<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(w, ci, co, transposed, kc, nb,
                                                                 out_ch, (__bf16*)out);
  return launch_status("swizzle");
}

size_t swizzled_elems(int in_ch, int out_ch) {
  return (size_t)kchunks_of(in_ch) * nblocks_of(out_ch) * 512;
}

fv_status refresh_bf16(fv_net* n, hipStream_t s) {
  k_swizzle_heads<<<4, 256, 0, s>>>(n->master + param_offset(14), n->master + param_offset(15),
                                    (__bf16*)n->w_heads, 1.0f);
  for (int l = 0; l < kNumConv; ++l) {
    fv_status st = swizzle_bf16(n->master + param_offset(l), kLayers[l].ci, kLayers[l].co, 0,
                                n->w_bf16[l], s);
    if (st == FV_OK && l > 0)
      st = swizzle_bf16(n->master + param_offset(l), kLayers[l].ci, kLayers[l].co, 1,
                        n->w_bf16t[l], s);
    if (st != FV_OK) return st;
  }
  return FV_OK;
}

// Runs the forward pass; prec 1 = BF16, 2 = FP8.  With absmax != nullptr the
// BF16 pass records per-tensor maxima (calibration).  Steps first .. last
// only (0 .. 13 the 3x3 convs, 14 the heads; the packed input is part of
// step 0): a later step reads the tensors an earlier one left in ws.
template <class E>
fv_status forward_impl(const fv_net* net, const Plan& p, uint8_t* ws, const float* frame,
                       const uint8_t* mask, const float* depth, const float* prev,
                       float* out_rgb, float* out_od, float* out_wk, float* absmax,
                       hipStream_t s, bool fuse_first, int first, int last) {
  const bool fp8 = E::kBytes == 1;
  const int64_t npx = (int64_t)p.n * p.h * p.w;
  const float in_inv = fp8 ? 1.0f / net->act_scale[T_IN] : 1.0f;
  fv_status st = FV_OK;
  if (!fuse_first && first == 0) {
    k_pack<E><<<(unsigned)((npx + 255) / 256), 256, 0, s>>>(
        (const float4*)frame, mask, depth, prev, ws + p.t[T_IN], npx, in_inv,
        absmax ? absmax + T_IN : nullptr);
    st = launch_status("pack");
    if (st != FV_OK) return st;
  }
  for (int l = first; l < kNumConv && l <= last; ++l) {
    // the packed input and the first conv are computed inside the second
    // conv's blocks (their tensors are not written)
    if (fuse_first && l == 0) continue;
    const LayerDesc& L = kLayers[l];
    const int* io = kLayerIO[l];
    ConvArgs a{};
    a.src0 = ws + p.t[io[0]];
    a.src1 = io[1] >= 0 ? ws + p.t[io[1]] : nullptr;
    a.c0 = L.c0;
    a.c1 = L.c1;
    a.cip = cip_of(L.c0 + L.c1);
    a.up0 = L.up0;
    a.n = p.n;
    a.h = p.h >> L.level;
    a.w = p.w >> L.level;
    a.kc = fp8 ? kchunks128_of(L.c0 + L.c1) : kchunks_of(L.c0 + L.c1);
    a.co = L.co;
    a.relu = 1;
    a.out = ws + p.t[io[2]];
    a.out_ch = L.co;
    a.out_fp32 = 0;
    a.absmax = absmax ? absmax + io[2] : nullptr;
    if (fp8) {
      a.wsw = (const uint8_t*)net->w_fp8[l];
      a.alpha = net->alpha_fp8[l];
      a.bias = net->bias_fp8[l];
    } else {
      a.wsw = (const uint8_t*)net->w_bf16[l];
      a.alpha = nullptr;
      a.bias = net->master + param_offset(l) + (int64_t)L.co * L.ci * 9;
    }
    if (fuse_first && l == 1) {
      const LayerDesc& L0 = kLayers[0];
      a.fuse0 = 1;
      a.f_rgba = (const float4*)frame;
      a.f_mask = mask;
      a.f_depth = depth;
      a.f_prev = prev;
      // under FP8 the first layer runs in BF16: its input is the sampled
      // colours (and, recurrent, the fed-back O_d), which the output has to
      // carry to well below E4M3's 6 % steps
      const bool mixed = fp8;
      const bool f8 = fp8 && !mixed;
      a.f_mixed = mixed;
      a.f_inv = f8 ? in_inv : 1.0f;
      a.f_wsw = (const uint8_t*)(f8 ? net->w_fp8[0] : net->w_bf16[0]);
      a.f_kc = f8 ? kchunks128_of(L0.ci) : kchunks_of(L0.ci);
      a.f_alpha = f8 ? net->alpha_fp8[0] : mixed ? net->mix0_ab : nullptr;
      a.f_bias = f8 ? net->bias_fp8[0]
                 : mixed ? net->mix0_ab + L0.co
                         : net->master + param_offset(0) + (int64_t)L0.co * L0.ci * 9;
    }
    // the encoder's second conv of levels 0-2 also writes the pooled input
    // of the next level
    a.pool_out = l == 1 ? ws + p.t[T_P0] : l == 3 ? ws + p.t[T_P1] : l == 5 ? ws + p.t[T_P2] : nullptr;
    st = launch_conv<E>(a, nblocks_of(L.co), s);
    if (st != FV_OK) return st;
  }
  if (last < kNumConv) return FV_OK;
  dim3 grid((p.w + 15) / 16, (p.h + 15) / 16, p.n);
  k_heads<E><<<grid, 256, 0, s>>>(ws + p.t[T_D0B], p.n, p.h, p.w, net->master,
                                  (const __bf16*)(fp8 ? net->w_heads_fp8 : net->w_heads),
                                  param_offset(14), param_offset(15), out_rgb, out_od, out_wk);
  return launch_status("heads");
}

template fv_status forward_impl<BF16>(const fv_net*, const Plan&, uint8_t*, const float*,
                                      const uint8_t*, const float*, const float*, float*, float*,
                                      float*, float*, hipStream_t, bool, int, int);
template fv_status forward_impl<FP8>(const fv_net*, const Plan&, uint8_t*, const float*,
                                     const uint8_t*, const float*, const float*, float*, float*,
                                     float*, float*, hipStream_t, bool, int, int);

// Nearest E4M3 value of v (ties to even, saturated at +-448), in double:
// 3 mantissa bits, so the spacing in [2^(e-1), 2^e) is 2^(e-4), and 2^-9
// below 2^-6 (subnormals).
static double e4m3_nearest(double v) {
  const double a = std::fabs(v);
  if (a >= 448.0) return std::copysign(448.0, v);
  int e = 0;
  (void)std::frexp(a, &e);
  const int se = std::max(e - 4, -9);
  const double q = std::ldexp(std::nearbyint(std::ldexp(a, -se)), se);
  return std::copysign(std::min(q, 448.0), v);
}

// FP8 weights: fold the per-input-channel activation scales into the
// weights, quantise per output channel (E4M3, |q| <= 448), and fold the
// output scale into alpha and bias.  The quantisation runs in double on the
// host (W s_in is exact there, one rounding for the division), so every
// code is the nearest E4M3 value of W' / omega; the device conversion of
// these exact values is exact.
fv_status build_fp8(fv_net* n, hipStream_t s) {
  const int64_t P = param_count();
  std::vector<float> host((size_t)P);
  fv_status st = hip_status(hipMemcpy(host.data(), n->master, P * sizeof(float),
                                      hipMemcpyDeviceToHost), "fp8: read weights");
  if (st != FV_OK) return st;
  for (int l = 0; l < kNumConv; ++l) {
    const LayerDesc& L = kLayers[l];
    const int* io = kLayerIO[l];
    const int cin = L.c0 + L.c1, cip = cip_of(cin);
    const float s_out = n->act_scale[io[2]];
    const float* W = host.data() + param_offset(l);
    const float* B = W + (int64_t)L.co * L.ci * 9;
    auto in_scale = [&](int ci) {
      return n->act_scale[ci < L.c0 ? io[0] : io[1]];
    };
    std::vector<double> wscale(L.co);
    std::vector<float> alpha(L.co), bias(L.co);
    for (int co = 0; co < L.co; ++co) {
      double m = 0.0;
      for (int ci = 0; ci < L.ci; ++ci)
        for (int t = 0; t < 9; ++t)
          m = std::max(m, std::fabs((double)W[((int64_t)co * L.ci + ci) * 9 + t] *
                                    (double)in_scale(ci)));
      wscale[co] = m > 0.0 ? m / 448.0 : 1.0;
      alpha[co] = (float)(wscale[co] / (double)s_out);
      bias[co] = (float)((double)B[co] / (double)s_out);
    }
    // fragments [chunk][n block][64 lanes][32 bytes]: lane ln holds output
    // channel 16 nb + ln % 16 at K positions 128 c + 32 (ln / 16) + j
    const int kc = kchunks128_of(cin), nb = nblocks_of(L.co);
    std::vector<float> sw((size_t)kc * nb * 2048, 0.f);
    for (size_t e = 0; e < sw.size(); ++e) {
      const int j = (int)(e & 31), ln = (int)((e >> 5) & 63);
      const int nbi = (int)((e >> 11) % nb);
      const int c = (int)(e / (2048 * (size_t)nb));
      const int kk = c * 128 + 32 * (ln >> 4) + j;
      const int tap = kk / cip, ci = kk - tap * cip;
      const int co = nbi * 16 + (ln & 15);
      if (tap < 9 && ci < L.ci && co < L.co)
        sw[e] = (float)e4m3_nearest((double)W[((int64_t)co * L.ci + ci) * 9 + tap] *
                                    (double)in_scale(ci) / wscale[co]);
    }
    float* tmp = nullptr;
    if (hipMalloc(&tmp, sw.size() * sizeof(float)) != hipSuccess)
      return fail(FV_ERR_NOMEM, "fp8: staging");
    st = hip_status(hipMemcpy(tmp, sw.data(), sw.size() * sizeof(float), hipMemcpyHostToDevice),
                    "fp8: upload");
    if (st == FV_OK) {
      k_f32_to_fp8<<<(unsigned)((sw.size() + 255) / 256), 256, 0, s>>>(
          tmp, (uint8_t*)n->w_fp8[l], (int64_t)sw.size());
      st = launch_status("fp8: quantise");
    }
    if (st == FV_OK) st = hip_status(hipStreamSynchronize(s), "fp8: sync");
    (void)hipFree(tmp);
    if (st != FV_OK) return st;
    st = hip_status(hipMemcpy(n->alpha_fp8[l], alpha.data(), L.co * sizeof(float),
                              hipMemcpyHostToDevice), "fp8: alpha");
    if (st == FV_OK)
      st = hip_status(hipMemcpy(n->bias_fp8[l], bias.data(), L.co * sizeof(float),
                                hipMemcpyHostToDevice), "fp8: bias");
    if (st != FV_OK) return st;
  }
  {
    // BF16 first layer under FP8: FP32 accumulators
    // times 1 / (output scale), bias / (output scale)
    const LayerDesc& L0 = kLayers[0];
    const float s_out = n->act_scale[T_E0A];
    std::vector<float> ab(2 * L0.co);
    for (int co = 0; co < L0.co; ++co) {
      ab[co] = 1.0f / s_out;
      ab[L0.co + co] = host[param_offset(0) + (int64_t)L0.co * L0.ci * 9 + co] / s_out;
    }
    st = hip_status(hipMemcpy(n->mix0_ab, ab.data(), ab.size() * sizeof(float),
                              hipMemcpyHostToDevice), "fp8: first-layer scales");
    if (st != FV_OK) return st;
  }
  // heads on FP8 decoder outputs: the tensor scale folded into the weights
  k_swizzle_heads<<<4, 256, 0, s>>>(n->master + param_offset(14), n->master + param_offset(15),
                                    (__bf16*)n->w_heads_fp8, n->act_scale[T_D0B]);
  st = launch_status("fp8: heads");
  if (st == FV_OK) st = hip_status(hipStreamSynchronize(s), "fp8: sync");
  if (st != FV_OK) return st;
  n->fp8_ready = 1;
  return FV_OK;
}

fv_status pack_input_bf16(const float* frame, const uint8_t* mask, const float* depth,
                          const float* prev, uint8_t* out, int64_t npx, hipStream_t s) {
  k_pack<BF16><<<(unsigned)((npx + 255) / 256), 256, 0, s>>>((const float4*)frame, mask, depth,
                                                           prev, out, npx, 1.0f, nullptr);
  return launch_status("pack");
}

fv_status check_frame(int views, int W, int H, const char* fn) {
  if (views <= 0 || W < 8 || H < 8 || W % 8 || H % 8 || W > 16384 || H > 16384)
    return fail(FV_ERR_INVALID_ARG,
                "%s: frame %d x %d x %d: width and height must be multiples of 8 in [8, 16384]",
                fn, views, W, H);
  return FV_OK;
}

}  // namespace net
}  // namespace fv

using namespace fv;
using namespace fv::net;

extern "C" {

size_t fv_net_param_count(void) { return (size_t)external_param_count(0); }

int fv_net_input_channels(const fv_net* n) {
  if (!n) return -1;
  return n->recurrent ? kLayers[0].ci : kLayers[0].ci - kFedBack;
}

fv_status fv_net_create(const float* host_params, size_t n_params, fv_net** out) {
  clear_error();
  if (!host_params || !out) return fail(FV_ERR_INVALID_ARG, "fv_net_create: null pointer");
  *out = nullptr;
  if (n_params != (size_t)external_param_count(0) && n_params != (size_t)external_param_count(1))
    return fail(FV_ERR_INVALID_ARG,
                "fv_net_create: %zu parameters, expected %lld (plain) or %lld (recurrent)",
                n_params, (long long)external_param_count(0), (long long)external_param_count(1));
  fv_net* n = new fv_net();
  memset(n, 0, sizeof(*n));
  n->recurrent = n_params == (size_t)external_param_count(1);
  std::vector<float> internal((size_t)param_count());
  params_to_internal(host_params, n->recurrent, internal.data());
  n_params = internal.size();
  if (hipGetDevice(&n->device) != hipSuccess) {
    delete n;
    return fail(FV_ERR_DEVICE, "fv_net_create: hipGetDevice");
  }
  const size_t pb = n_params * sizeof(float);
  bool ok = hipMalloc(&n->master, pb) == hipSuccess && hipMalloc(&n->adam_m, pb) == hipSuccess &&
            hipMalloc(&n->w_heads, 2 * 512 * 2) == hipSuccess &&
            hipMalloc(&n->w_heads_fp8, 2 * 512 * 2) == hipSuccess &&
            hipMalloc(&n->adam_v, pb) == hipSuccess && hipMalloc(&n->grad, pb) == hipSuccess &&
            hipMalloc(&n->mix0_ab, 2 * kLayers[0].co * sizeof(float)) == hipSuccess;
  for (int l = 0; ok && l < kNumConv; ++l) {
    const size_t e = swizzled_elems(kLayers[l].c0 + kLayers[l].c1, kLayers[l].co);
    const size_t et = swizzled_elems(kLayers[l].co, kLayers[l].c0 + kLayers[l].c1);
    const size_t e8 = (size_t)kchunks128_of(kLayers[l].c0 + kLayers[l].c1) *
                      nblocks_of(kLayers[l].co) * 2048;
    ok = hipMalloc(&n->w_bf16[l], e * 2) == hipSuccess && hipMalloc(&n->w_fp8[l], e8) == hipSuccess &&
         hipMalloc(&n->w_bf16t[l], et * 2) == hipSuccess &&
         hipMalloc(&n->alpha_fp8[l], kLayers[l].co * sizeof(float)) == hipSuccess &&
         hipMalloc(&n->bias_fp8[l], kLayers[l].co * sizeof(float)) == hipSuccess;
  }
  if (!ok) {
    fv_net_destroy(n);
    return fail(FV_ERR_NOMEM, "fv_net_create: allocation failed");
  }
  fv_status st = hip_status(hipMemcpy(n->master, internal.data(), pb, hipMemcpyHostToDevice),
                            "fv_net_create: upload");
  if (st == FV_OK) st = hip_status(hipMemset(n->adam_m, 0, pb), "fv_net_create: adam");
  if (st == FV_OK) st = hip_status(hipMemset(n->adam_v, 0, pb), "fv_net_create: adam");
  if (st == FV_OK) st = hip_status(hipMemset(n->grad, 0, pb), "fv_net_create: grad");
  if (st == FV_OK) st = refresh_bf16(n, nullptr);
  if (st == FV_OK) st = hip_status(hipDeviceSynchronize(), "fv_net_create: sync");
  if (st != FV_OK) {
    fv_net_destroy(n);
    return st;
  }
  *out = n;
  return FV_OK;
}

fv_status fv_net_destroy(fv_net* n) {
  if (!n) return FV_OK;
  (void)hipFree(n->master);
  (void)hipFree(n->adam_m);
  (void)hipFree(n->adam_v);
  (void)hipFree(n->grad);
  (void)hipFree(n->w_heads);
  (void)hipFree(n->w_heads_fp8);
  (void)hipFree(n->mix0_ab);
  for (int l = 0; l < kNumConv; ++l) {
    (void)hipFree(n->w_bf16[l]);
    (void)hipFree(n->w_bf16t[l]);
    (void)hipFree(n->w_fp8[l]);
    (void)hipFree(n->alpha_fp8[l]);
    (void)hipFree(n->bias_fp8[l]);
  }
  delete n;
  return FV_OK;
}

fv_status fv_net_get_params(const fv_net* n, float* host_params, size_t n_params) {
  clear_error();
  if (!n || !host_params) return fail(FV_ERR_INVALID_ARG, "fv_net_get_params: null pointer");
  if (n_params != (size_t)external_param_count(n->recurrent))
    return fail(FV_ERR_INVALID_ARG, "fv_net_get_params: size %zu, the network has %lld",
                n_params, (long long)external_param_count(n->recurrent));
  std::vector<float> internal((size_t)param_count());
  fv_status st = hip_status(hipMemcpy(internal.data(), n->master, internal.size() * sizeof(float),
                                      hipMemcpyDeviceToHost), "fv_net_get_params");
  if (st == FV_OK) params_to_external(internal.data(), n->recurrent, host_params);
  return st;
}

fv_status fv_net_set_params(fv_net* n, const float* host_params, size_t n_params) {
  clear_error();
  if (!n || !host_params) return fail(FV_ERR_INVALID_ARG, "fv_net_set_params: null pointer");
  if (n_params != (size_t)external_param_count(n->recurrent))
    return fail(FV_ERR_INVALID_ARG, "fv_net_set_params: size %zu, the network has %lld",
                n_params, (long long)external_param_count(n->recurrent));
  std::vector<float> internal((size_t)param_count());
  params_to_internal(host_params, n->recurrent, internal.data());
  fv_status st = hip_status(hipMemcpy(n->master, internal.data(),
                                      internal.size() * sizeof(float), hipMemcpyHostToDevice),
                            "fv_net_set_params");
  if (st == FV_OK) st = refresh_bf16(n, nullptr);
  if (st == FV_OK) st = hip_status(hipDeviceSynchronize(), "fv_net_set_params: sync");
  n->fp8_ready = 0;
  return st;
}

fv_status fv_reconstruct_workspace(const fv_net* n, int precision, int views, int width,
                                   int height, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(FV_ERR_INVALID_ARG, "fv_reconstruct_workspace: null pointer");
  if (precision == FV_RECON_PULLPUSH)
    return fv_pullpush_workspace(views, width, height, bytes);
  if (!n) return fail(FV_ERR_INVALID_ARG, "fv_reconstruct_workspace: null network");
  if (precision != FV_PREC_BF16 && precision != FV_PREC_FP8)
    return fail(FV_ERR_UNSUPPORTED, "fv_reconstruct_workspace: precision %d", precision);
  fv_status st = check_frame(views, width, height, "fv_reconstruct_workspace");
  if (st != FV_OK) return st;
  *bytes = make_plan(views, height, width, precision == FV_PREC_FP8 ? 1 : 2).bytes;
  return FV_OK;
}

static fv_status reconstruct(const fv_net* n, int precision, const float* frame_rgba,
                             const uint8_t* mask, const float* frame_depth, const float* prev,
                             int views, int width, int height, float* out_rgb,
                             float* out_direct, void* workspace, size_t ws_bytes, void* stream,
                             const char* fn, int first = 0, int last = kNumConv) {
  clear_error();
  if (precision == FV_RECON_PULLPUSH) {
    if (prev || out_direct)
      return fail(FV_ERR_INVALID_ARG, "%s: pull-push has no direct prediction or feedback", fn);
    return pullpush_run(frame_rgba, mask, views, width, height, out_rgb, workspace, ws_bytes,
                        (hipStream_t)stream, fn);
  }
  if (first < 0 || last > kNumConv || first > last)
    return fail(FV_ERR_INVALID_ARG, "%s: steps %d .. %d (0 .. %d)", fn, first, last, kNumConv);
  // the frame is read by the first two steps (the fused first layer), the
  // output is written by the last one (the heads)
  const bool need_frame = first <= 1, need_out = last == kNumConv;
  if (!n || !workspace || (need_frame && (!frame_rgba || !mask)) || (need_out && !out_rgb))
    return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  if (prev && !n->recurrent)
    return fail(FV_ERR_INVALID_ARG, "%s: the network has no recurrent input", fn);
  if (precision != FV_PREC_BF16 && precision != FV_PREC_FP8)
    return fail(FV_ERR_UNSUPPORTED, "%s: precision %d", fn, precision);
  fv_status st = check_frame(views, width, height, fn);
  if (st != FV_OK) return st;
  if (precision == FV_PREC_FP8 && !n->fp8_ready)
    return fail(FV_ERR_INVALID_ARG, "%s: FP8 requested before fv_net_calibrate", fn);
  const Plan p = make_plan(views, height, width, precision == FV_PREC_FP8 ? 1 : 2);
  if (ws_bytes < p.bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, p.bytes);
  if ((uintptr_t)workspace % 256)
    return fail(FV_ERR_INVALID_ARG, "%s: workspace not 256-byte aligned", fn);
  hipStream_t s = (hipStream_t)stream;
  if (precision == FV_PREC_FP8)
    return forward_impl<FP8>(n, p, (uint8_t*)workspace, frame_rgba, mask, frame_depth, prev,
                             out_rgb, out_direct, nullptr, nullptr, s, true, first, last);
  return forward_impl<BF16>(n, p, (uint8_t*)workspace, frame_rgba, mask, frame_depth, prev,
                            out_rgb, out_direct, nullptr, nullptr, s, true, first, last);
}

fv_status fv_reconstruct(const fv_net* n, int precision, const float* frame_rgba,
                         const uint8_t* mask, const float* frame_depth, int views, int width,
                         int height, float* out_rgb, float* out_direct, void* workspace,
                         size_t ws_bytes, void* stream) {
  return reconstruct(n, precision, frame_rgba, mask, frame_depth, nullptr, views, width, height,
                     out_rgb, out_direct, workspace, ws_bytes, stream, "fv_reconstruct");
}

fv_status fv_reconstruct_steps(const fv_net* n, int precision, int first, int last,
                               const float* frame_rgba, const uint8_t* mask,
                               const float* frame_depth, const float* prev_direct, int views,
                               int width, int height, float* out_rgb, float* out_direct,
                               void* workspace, size_t ws_bytes, void* stream) {
  return reconstruct(n, precision, frame_rgba, mask, frame_depth, prev_direct, views, width,
                     height, out_rgb, out_direct, workspace, ws_bytes, stream,
                     "fv_reconstruct_steps", first, last);
}

fv_status fv_reconstruct_tensor(int precision, int views, int width, int height, int tensor,
                                size_t* offset, int* channels, int* level) {
  clear_error();
  if (!offset || !channels || !level)
    return fail(FV_ERR_INVALID_ARG, "fv_reconstruct_tensor: null pointer");
  if (precision != FV_PREC_BF16 && precision != FV_PREC_FP8)
    return fail(FV_ERR_UNSUPPORTED, "fv_reconstruct_tensor: precision %d", precision);
  if (tensor < 0 || tensor >= kNumTensors)
    return fail(FV_ERR_INVALID_ARG, "fv_reconstruct_tensor: tensor %d (0 .. %d)", tensor,
                kNumTensors - 1);
  fv_status st = check_frame(views, width, height, "fv_reconstruct_tensor");
  if (st != FV_OK) return st;
  const Plan p = make_plan(views, height, width, precision == FV_PREC_FP8 ? 1 : 2);
  *offset = p.t[tensor];
  *channels = kTensors[tensor].channels;
  *level = kTensors[tensor].level;
  return FV_OK;
}

fv_status fv_reconstruct_recurrent(const fv_net* n, int precision, const float* frame_rgba,
                                   const uint8_t* mask, const float* frame_depth,
                                   const float* prev_direct, int views, int width, int height,
                                   float* out_rgb, float* out_direct, void* workspace,
                                   size_t ws_bytes, void* stream) {
  return reconstruct(n, precision, frame_rgba, mask, frame_depth, prev_direct, views, width,
                     height, out_rgb, out_direct, workspace, ws_bytes, stream,
                     "fv_reconstruct_recurrent");
}

static fv_status calibrate(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                           const float* frame_depth, const float* prev, int views, int width,
                           int height, void* workspace, size_t ws_bytes, void* stream,
                           const char* fn) {
  clear_error();
  if (!n || !frame_rgba || !mask || !workspace)
    return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  if (prev && !n->recurrent)
    return fail(FV_ERR_INVALID_ARG, "%s: the network has no recurrent input", fn);
  fv_status st = check_frame(views, width, height, fn);
  if (st != FV_OK) return st;
  const Plan p = make_plan(views, height, width, 2);
  if (ws_bytes < p.bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes (BF16 plan)", fn, ws_bytes,
                p.bytes);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  float* amax = (float*)(ws + p.absmax);
  k_zero_f32<<<1, 64, 0, s>>>(amax, 64);
  if ((st = launch_status("calibrate: clear")) != FV_OK) return st;
  float* tmp_rgb = (float*)(ws + p.od);  // the O_d slot is free in this pass
  st = forward_impl<BF16>(n, p, ws, frame_rgba, mask, frame_depth, prev, tmp_rgb, nullptr,
                          nullptr, amax, s, false, 0, kNumConv);
  if (st != FV_OK) return st;
  float host[64];
  st = hip_status(hipMemcpyAsync(host, amax, sizeof host, hipMemcpyDeviceToHost, s),
                  "calibrate: read");
  if (st == FV_OK) st = hip_status(hipStreamSynchronize(s), "calibrate: sync");
  if (st != FV_OK) return st;
  for (int t = 0; t < kNumTensors; ++t)
    n->act_scale[t] = FV_FP8_HEADROOM * std::max(host[t], 1e-6f) / 448.0f;
  n->act_scale[T_P0] = n->act_scale[T_E0B];
  n->act_scale[T_P1] = n->act_scale[T_E1B];
  n->act_scale[T_P2] = n->act_scale[T_E2B];
  return build_fp8(n, s);
}

fv_status fv_net_set_fp8_scales(fv_net* n, const float* host_scales, int count,
                                void* stream) {
  clear_error();
  if (!n || !host_scales) return fail(FV_ERR_INVALID_ARG, "fv_net_set_fp8_scales: null pointer");
  if (count != FV_NET_FP8_TENSORS)
    return fail(FV_ERR_INVALID_ARG, "fv_net_set_fp8_scales: count %d, expected %d", count,
                FV_NET_FP8_TENSORS);
  for (int i = 0; i < count; ++i)
    if (!(host_scales[i] > 0.f) || !std::isfinite(host_scales[i]))
      return fail(FV_ERR_INVALID_ARG, "fv_net_set_fp8_scales: scale %d is %g", i,
                  (double)host_scales[i]);
  n->act_scale[T_IN] = host_scales[0];
  for (int l = 0; l < kNumConv; ++l) n->act_scale[kLayerIO[l][2]] = host_scales[1 + l];
  n->act_scale[T_P0] = n->act_scale[T_E0B];
  n->act_scale[T_P1] = n->act_scale[T_E1B];
  n->act_scale[T_P2] = n->act_scale[T_E2B];
  return build_fp8(n, (hipStream_t)stream);
}

fv_status fv_net_calibrate(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                           const float* frame_depth, int views, int width, int height,
                           void* workspace, size_t ws_bytes, void* stream) {
  return calibrate(n, frame_rgba, mask, frame_depth, nullptr, views, width, height, workspace,
                   ws_bytes, stream, "fv_net_calibrate");
}

fv_status fv_net_calibrate_recurrent(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                                     const float* frame_depth, const float* prev_direct,
                                     int views, int width, int height, void* workspace,
                                     size_t ws_bytes, void* stream) {
  return calibrate(n, frame_rgba, mask, frame_depth, prev_direct, views, width, height,
                   workspace, ws_bytes, stream, "fv_net_calibrate_recurrent");
}

}  // extern "C"
