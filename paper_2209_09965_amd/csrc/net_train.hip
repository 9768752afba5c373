// Reconstruction network: training (paper: "Loss", "Training").
//
// Forward in BF16 with every activation kept, loss 0.9 (1 - SSIM) + 0.1 L1
// (SSIM in place of the unavailable VGG19-LPIPS term), backward through the
// kernel-prediction and direct heads, every conv (input gradient = the MFMA
// conv kernel with transposed weights, weight gradient = FP32 partial sums per
// pixel chunk reduced in a fixed order, so a step is deterministic), the
// bilinear upsampling and the average pooling; Adam on FP32 master weights.
#include <algorithm>
#include <utility>
#include <vector>

#include "net.h"
#include "net_kernels.h"

namespace fv {
namespace net {

template <class E>
fv_status forward_impl(const fv_net* net, const Plan& p, uint8_t* ws, const float* frame,
                       const uint8_t* mask, const float* depth, const float* prev,
                       float* out_rgb, float* out_od, float* out_wk, float* absmax,
                       hipStream_t s, bool fuse_first, int first, int last);
fv_status refresh_bf16(fv_net* n, hipStream_t s);
fv_status check_frame(int views, int W, int H, const char* fn);

static size_t al(size_t v) { return (v + 255) / 256 * 256; }

constexpr int kWgRows = 16;        // tile rows of the weight-gradient kernel (x 16 columns)
constexpr int kHeadChunks = 1024;  // pixel chunks of the heads' weight gradient
constexpr int kReduceSlices = 32;  // first-stage slices of the weight-gradient reduction

static int64_t px_at(const Plan& p, int level) {
  return (int64_t)p.n * (p.h >> level) * (p.w >> level);
}

TrainPlan make_train_plan(int n, int h, int w) {
  TrainPlan t;
  t.f = make_plan(n, h, w, 2);
  size_t off = t.f.bytes;
  t.g[T_IN] = 0;
  for (int k = 1; k < kNumTensors; ++k) {
    t.g[k] = off;
    off += al((size_t)px_at(t.f, kTensors[k].level) * kTensors[k].channels * 4);
  }
  size_t tmp = (size_t)px_at(t.f, 0) * 28 * 4, dz = 0, part = 0;
  for (int l = 0; l < kNumConv; ++l) {
    const LayerDesc& L = kLayers[l];
    const int64_t px = px_at(t.f, L.level);
    tmp = std::max(tmp, (size_t)px * L.ci * 4);
    dz = std::max(dz, (size_t)px * L.co * 2);
    const int64_t tiles =
        (int64_t)n * (((h >> L.level) + kWgRows - 1) / kWgRows) * (((w >> L.level) + 15) / 16);
    // about 2048 blocks per weight-gradient launch (channel groups x chunks)
    const int64_t groups = (int64_t)((L.ci + 31) / 32) * ((L.co + 31) / 32);
    t.chunks[l] = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 2048 / groups));
    part = std::max(part, (size_t)t.chunks[l] * (9 * (size_t)L.ci * L.co + L.co) * 4);
  }
  part = std::max(part, (size_t)kHeadChunks * 28 * 33 * 4);
  size_t part2 = 0;
  for (int l = 0; l < kNumConv; ++l)
    part2 = std::max(part2, (size_t)kReduceSlices * (9 * (size_t)kLayers[l].ci * kLayers[l].co +
                                                     kLayers[l].co) * 4);
  t.tmp = off;
  off += al(tmp);
  t.dz = off;
  off += al(dz);
  t.dz2 = off;
  off += al(dz);
  t.target = off;
  off += al((size_t)n * h * w * 3 * 4);
  t.dout = off;
  off += al((size_t)n * h * w * 3 * 4);
  const size_t q = (size_t)n * 3;
  t.ssim = off;
  off += al(q * h * (w - 10) * 4 * 5) + al(q * (h - 10) * (w - 10) * 4 * 3) +
         al(q * h * (w - 10) * 4 * 3);
  t.part = off;
  off += al(part);
  t.part2 = off;
  off += al(part2);
  t.red = off;
  const int64_t vblocks = ((int64_t)q * (h - 10) * (w - 10) + 255) / 256;
  const int64_t lblocks = ((int64_t)q * h * w + 255) / 256;
  off += al((size_t)(vblocks + lblocks) * 8);
  t.bytes = off;
  return t;
}

// ------------------------------------------------------------------ loss

__constant__ float c_gauss[11];

// horizontal 11-tap filter of x, t, x^2, t^2, x t (valid columns)
// One thread per output pixel and all 3 colour planes (12 contiguous bytes
// of each image per tap, lanes adjacent in x); every output sums its 11 taps
// in tap order.
__global__ void __launch_bounds__(256) k_ssim_h(const float* __restrict__ out,
                                                const float* __restrict__ tgt, int n, int h, int w,
                                                float* __restrict__ hq) {
  const int wv = w - 10;
  const int64_t q = (int64_t)n * 3;
  const int64_t total = q * h * wv;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (image, row, column)
  if (e >= (int64_t)n * h * wv) return;
  const int x = (int)(e % wv);
  const int64_t r = e / wv;
  const int y = (int)(r % h), b = (int)(r / h);
  float s[3][5];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int j = 0; j < 5; ++j) s[c][j] = 0.f;
  for (int k = 0; k < 11; ++k) {
    const int64_t p = ((int64_t)b * h + y) * w + x + k;
    const float g = c_gauss[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float a = out[p * 3 + c], t = tgt[p * 3 + c];
      s[c][0] = fmaf(g, a, s[c][0]);
      s[c][1] = fmaf(g, t, s[c][1]);
      s[c][2] = fmaf(g, a * a, s[c][2]);
      s[c][3] = fmaf(g, t * t, s[c][3]);
      s[c][4] = fmaf(g, a * t, s[c][4]);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t eo = (((int64_t)b * 3 + c) * h + y) * wv + x;  // plane b*3+c
#pragma unroll
    for (int k = 0; k < 5; ++k) hq[k * total + eo] = s[c][k];
  }
}

// vertical filter -> SSIM map and its partial derivatives w.r.t. mu_x,
// E[x^2] and E[x t]; block sums of the map (double) for the loss value
// A thread of the vertical passes computes kSsimRows consecutive output rows
// of one column, sliding over the input rows it shares between them; every
// output sums its 11 taps in tap order.
constexpr int kSsimRows = 8;

__global__ void __launch_bounds__(256) k_ssim_v(const float* __restrict__ hq, int n, int h, int w,
                                                float* __restrict__ dmap,
                                                double* __restrict__ red) {
  __shared__ double sh[256];
  const int wv = w - 10, hv = h - 10, nyb = (hv + kSsimRows - 1) / kSsimRows;
  const int64_t q = (int64_t)n * 3;
  const int64_t htot = q * h * wv, vtot = q * hv * wv;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sval = 0.0;
  if (e < q * nyb * wv) {
    const int x = (int)(e % wv);
    const int64_t r = e / wv;
    const int y0 = (int)(r % nyb) * kSsimRows;
    const int64_t pl = r / nyb;
    float m[kSsimRows][5];
#pragma unroll
    for (int o = 0; o < kSsimRows; ++o)
#pragma unroll
      for (int j = 0; j < 5; ++j) m[o][j] = 0.f;
    // input row y0 + t feeds output y0 + o with tap k = t - o
#pragma unroll
    for (int t = 0; t < kSsimRows + 10; ++t) {
      if (y0 + t >= h) break;
      const int64_t hi = (pl * h + y0 + t) * wv + x;
      float v[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) v[j] = hq[j * htot + hi];
#pragma unroll
      for (int o = 0; o < kSsimRows; ++o) {
        const int k = t - o;
        if (k >= 0 && k < 11)
#pragma unroll
          for (int j = 0; j < 5; ++j) m[o][j] = fmaf(c_gauss[k], v[j], m[o][j]);
      }
    }
    const float C1 = 1e-4f, C2 = 9e-4f;
#pragma unroll
    for (int o = 0; o < kSsimRows; ++o) {
      if (y0 + o >= hv) break;
      const float mx = m[o][0], my = m[o][1];
      const float vx = m[o][2] - mx * mx, vy = m[o][3] - my * my, cxy = m[o][4] - mx * my;
      const float A1 = 2 * mx * my + C1, A2 = 2 * cxy + C2;
      const float B1 = mx * mx + my * my + C1, B2 = vx + vy + C2;
      const float S = A1 * A2 / (B1 * B2);
      sval += S;
      const int64_t ev = (pl * hv + y0 + o) * wv + x;
      dmap[ev] = (2 * my * A2 - 2 * my * A1) / (B1 * B2) - S * (2 * mx / B1 - 2 * mx / B2);
      dmap[vtot + ev] = -S / B2;
      dmap[2 * vtot + ev] = 2 * A1 / (B1 * B2);
    }
  }
  sh[threadIdx.x] = sval;
  __syncthreads();
  for (int st = 128; st; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}

// adjoint of the vertical filter for the three partial maps
__global__ void __launch_bounds__(256) k_ssim_vt(const float* __restrict__ dmap, int n, int h,
                                                 int w, float* __restrict__ va) {
  const int wv = w - 10, hv = h - 10, nyb = (h + kSsimRows - 1) / kSsimRows;
  const int64_t q = (int64_t)n * 3;
  const int64_t htot = q * h * wv, vtot = q * hv * wv;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= q * nyb * wv) return;
  const int x = (int)(e % wv);
  const int64_t r = e / wv;
  const int y0 = (int)(r % nyb) * kSsimRows;
  const int64_t pl = r / nyb;
  float s[kSsimRows][3];
#pragma unroll
  for (int o = 0; o < kSsimRows; ++o)
#pragma unroll
    for (int j = 0; j < 3; ++j) s[o][j] = 0.f;
  // map row yy = y0 + kSsimRows - 1 - t feeds output y0 + o with tap
  // k = y0 + o - yy, increasing with t as each output's sum requires
#pragma unroll
  for (int t = 0; t < kSsimRows + 10; ++t) {
    const int yy = y0 + kSsimRows - 1 - t;
    if (yy < 0 || yy >= hv) continue;
    const int64_t vi = (pl * hv + yy) * wv + x;
    float v[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) v[j] = dmap[j * vtot + vi];
#pragma unroll
    for (int o = 0; o < kSsimRows; ++o) {
      const int k = o - (kSsimRows - 1) + t;
      if (k >= 0 && k < 11)
#pragma unroll
        for (int j = 0; j < 3; ++j) s[o][j] = fmaf(c_gauss[k], v[j], s[o][j]);
    }
  }
#pragma unroll
  for (int o = 0; o < kSsimRows; ++o) {
    if (y0 + o >= h) break;
    const int64_t ev = (pl * h + y0 + o) * wv + x;
#pragma unroll
    for (int j = 0; j < 3; ++j) va[j * htot + ev] = s[o][j];
  }
}

// adjoint of the horizontal filter, combined into d loss / d out, plus the
// L1 term and its block sums
// one thread per pixel and all 3 colour planes, like k_ssim_h
__global__ void __launch_bounds__(256) k_ssim_ht(const float* __restrict__ va,
                                                 const float* __restrict__ out,
                                                 const float* __restrict__ tgt, int n, int h,
                                                 int w, float ssim_scale, float l1_scale,
                                                 float* __restrict__ dout,
                                                 double* __restrict__ red) {
  __shared__ double sh[256];
  const int wv = w - 10;
  const int64_t q = (int64_t)n * 3;
  const int64_t htot = q * h * wv;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (image, row, column)
  double l1 = 0.0;
  if (e < (int64_t)n * h * w) {
    const int x = (int)(e % w);
    const int64_t r = e / w;
    const int y = (int)(r % h), b = (int)(r / h);
    float s[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 3; ++j) s[c][j] = 0.f;
    for (int k = 0; k < 11; ++k) {
      const int xx = x - k;
      if (xx < 0 || xx >= wv) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t hi = (((int64_t)b * 3 + c) * h + y) * wv + xx;  // plane b*3+c
#pragma unroll
        for (int j = 0; j < 3; ++j) s[c][j] = fmaf(c_gauss[k], va[j * htot + hi], s[c][j]);
      }
    }
    const int64_t p = ((int64_t)b * h + y) * w + x;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float a = out[p * 3 + c], t = tgt[p * 3 + c];
      const float dssim = s[c][0] + 2.0f * a * s[c][1] + t * s[c][2];
      const float sg = (a > t) ? 1.0f : (a < t ? -1.0f : 0.0f);
      dout[p * 3 + c] = -0.9f * ssim_scale * dssim + 0.1f * l1_scale * sg;
      l1 += fabs((double)a - (double)t);
    }
  }
  sh[threadIdx.x] = l1;
  __syncthreads();
  for (int st = 128; st; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}

// fixed-order sums of the block partials -> [loss, ssim, l1]
__global__ void __launch_bounds__(1024) k_loss_final(const double* __restrict__ rs, int ns,
                                                     const double* __restrict__ rl, int nl,
                                                     double ssim_scale, double l1_scale,
                                                     float* __restrict__ out) {
  __shared__ double a[1024], c[1024];
  double sa = 0.0, sc = 0.0;
  for (int i = threadIdx.x; i < ns; i += 1024) sa += rs[i];
  for (int i = threadIdx.x; i < nl; i += 1024) sc += rl[i];
  a[threadIdx.x] = sa;
  c[threadIdx.x] = sc;
  __syncthreads();
  for (int st = 512; st; st >>= 1) {
    if (threadIdx.x < st) {
      a[threadIdx.x] += a[threadIdx.x + st];
      c[threadIdx.x] += c[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ssim = a[0] * ssim_scale, l1 = c[0] * l1_scale;
    out[0] = (float)(0.9 * (1.0 - ssim) + 0.1 * l1);
    out[1] = (float)ssim;
    out[2] = (float)l1;
  }
}

// Temporal loss, finite-difference term, over batch pairs (2i, 2i + 1):
// d = (out_2i+1 - out_2i) - (target_2i+1 - target_2i) per channel; |d| is
// summed per block in FP64 and d L / d out (+-gscale by the sign of d) is
// added to dloss.
__global__ void __launch_bounds__(256) k_tloss(const float* __restrict__ out,
                                               const float4* __restrict__ tgt, int64_t pairs,
                                               int64_t hw, float gscale,
                                               float* __restrict__ dloss,
                                               double* __restrict__ red) {
  __shared__ double sh[256];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double ad = 0.0;
  if (e < pairs * hw * 3) {
    const int64_t pr = e / (hw * 3), rem = e - pr * hw * 3;
    const int64_t px = rem / 3;
    const int c = (int)(rem - px * 3);
    const int64_t i0 = 2 * pr * hw * 3 + rem, i1 = i0 + hw * 3;
    const float4 a = tgt[2 * pr * hw + px], b = tgt[(2 * pr + 1) * hw + px];
    const float t0 = c == 0 ? a.x : c == 1 ? a.y : a.z;
    const float t1 = c == 0 ? b.x : c == 1 ? b.y : b.z;
    const float d = (out[i1] - out[i0]) - (t1 - t0);
    ad = fabs((double)d);
    const float g = d > 0.0f ? gscale : (d < 0.0f ? -gscale : 0.0f);
    dloss[i1] += g;
    dloss[i0] -= g;
  }
  sh[threadIdx.x] = ad;
  __syncthreads();
  for (int st = 128; st; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}

// fixed-order sum of the block partials -> L_t
__global__ void k_tloss_final(const double* __restrict__ red, int nb, double scale,
                              float* __restrict__ out) {
  __shared__ double a[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += red[i];
  a[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st; st >>= 1) {
    if (threadIdx.x < st) a[threadIdx.x] += a[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(a[0] * scale);
}

__global__ void __launch_bounds__(256) k_rgb_of_rgba(const float4* __restrict__ src,
                                                     float* __restrict__ dst, int64_t npx) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npx) return;
  const float4 v = src[p];
  dst[p * 3 + 0] = v.x;
  dst[p * 3 + 1] = v.y;
  dst[p * 3 + 2] = v.z;
}

// A finished output gradient stored as the next layer back needs it: dz =
// BF16(v x [gate > 0]), the ReLU derivative of the forward activation gate
// (BF16), exactly as the ReLU mask pass would store it.
__device__ __forceinline__ float relu_gate(const uint8_t* gate, int64_t i, float v) {
  return bf16_bits_to_f(((const uint16_t*)gate)[i]) > 0.f ? v : 0.f;
}
// the same for V consecutive channels from element i (V = 4: 8-byte accesses)
template <int V>
__device__ __forceinline__ void store_gated(uint8_t* dz, const uint8_t* gate, int64_t i,
                                            const float* v) {
  if constexpr (V == 4) {
    const uint2 gb = *(const uint2*)(gate + i * 2);
    const float r[4] = {bf16_bits_to_f(gb.x & 0xffffu) > 0.f ? v[0] : 0.f,
                        bf16_bits_to_f(gb.x >> 16) > 0.f ? v[1] : 0.f,
                        bf16_bits_to_f(gb.y & 0xffffu) > 0.f ? v[2] : 0.f,
                        bf16_bits_to_f(gb.y >> 16) > 0.f ? v[3] : 0.f};
    BF16::store4(dz + i * 2, r);
  } else {
    BF16::store1(dz + i * 2, relu_gate(gate, i, v[0]));
  }
}

// ----------------------------------------------------------- heads backward

// Per pixel: d w_k = sum_c dout_c(p) O_d,c(clamp(p + delta_k)); d logits by
// the softmax Jacobian; d O_d(p) gathered from every pixel whose clamped tap
// lands on p; d H_d = W_heads^T [d O_d; d logits].  Writes d28 = [d O_d,
// d logits] (for the heads' weight gradient) and, as H_d has no other
// consumer, the last conv's masked output gradient: dz = BF16(d H_d x
// [H_d > 0]) (H_d: the stored BF16 activation).
// Block = one 16 x 16 tile of one image.  The kernel weights, O_d and dout
// of the tile and its 2-pixel border are staged in LDS, rows and columns
// clamped to the image (what the clamped taps read; every pixel a gather
// visits lies inside the image and within 2 pixels of the tile).  The
// outputs then leave through the same LDS in whole 16-byte units.
constexpr int kHT = 16, kHH = kHT + 4;  // tile side, tile + border
__global__ void __launch_bounds__(256) k_heads_bwd(const float* __restrict__ dout,
                                                   const float* __restrict__ od,
                                                   const float* __restrict__ wk, int h, int w,
                                                   const float* __restrict__ params,
                                                   int64_t off_hd, int64_t off_hk,
                                                   float* __restrict__ d28,
                                                   const uint8_t* __restrict__ hd_act,
                                                   uint8_t* __restrict__ dz) {
  // the BF16-rounded head weights (the forward's), [28 outputs][32 inputs]
  __shared__ float sw[28 * 32];
  // kernel weights of the bordered tile [20 x 20 pixels][25]; afterwards the
  // outputs: d28 (28 floats a pixel), then gh (rows padded to 36 floats)
  __shared__ __attribute__((aligned(16))) float swk[kHH * kHH * 25];
  __shared__ float sod[kHH * kHH * 3], sdo[kHH * kHH * 3];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kHT, y0 = blockIdx.y * kHT, b = blockIdx.z;
  for (int i = tid; i < 28 * 32; i += 256)
    sw[i] = (float)(__bf16)(i < 3 * 32 ? params[off_hd + i] : params[off_hk + i - 3 * 32]);
  // every staging load is issued before the first LDS store (one memory
  // round trip per block): 40 kernel-weight values and 10 of O_d / dout per
  // thread
  constexpr int kNW = kHH * kHH * 25, kNO = kHH * kHH * 3;
  constexpr int kUW = (kNW + 255) / 256, kUO = (kNO + 255) / 256;
  float vw[kUW], vo[kUO], vd[kUO];
#pragma unroll
  for (int u = 0; u < kUW; ++u) {
    const int e = tid + 256 * u;
    if (e < kNW) {
      const int pix = e / 25, k = e - 25 * pix, r = pix / kHH, c = pix - r * kHH;
      const int yy = min(max(y0 - 2 + r, 0), h - 1), xx = min(max(x0 - 2 + c, 0), w - 1);
      vw[u] = wk[(((int64_t)b * h + yy) * w + xx) * 25 + k];
    }
  }
#pragma unroll
  for (int u = 0; u < kUO; ++u) {
    const int e = tid + 256 * u;
    if (e < kNO) {
      const int pix = e / 3, j = e - 3 * pix, r = pix / kHH, c = pix - r * kHH;
      const int yy = min(max(y0 - 2 + r, 0), h - 1), xx = min(max(x0 - 2 + c, 0), w - 1);
      const int64_t q = ((int64_t)b * h + yy) * w + xx;
      vo[u] = od[q * 3 + j];
      vd[u] = dout[q * 3 + j];
    }
  }
#pragma unroll
  for (int u = 0; u < kUW; ++u)
    if (tid + 256 * u < kNW) swk[tid + 256 * u] = vw[u];
#pragma unroll
  for (int u = 0; u < kUO; ++u)
    if (tid + 256 * u < kNO) {
      sod[tid + 256 * u] = vo[u];
      sdo[tid + 256 * u] = vd[u];
    }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4, x = x0 + tx, y = y0 + ty;
  float d[28];
  if (x < w && y < h) {
    const int c0 = (ty + 2) * kHH + tx + 2;  // this pixel in the bordered tile
    const float g0 = sdo[c0 * 3], g1 = sdo[c0 * 3 + 1], g2 = sdo[c0 * 3 + 2];
    float dw[25], wl[25];
    float dot = 0.f;
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        const int k = 5 * (dy + 2) + (dx + 2);
        const int qn = c0 + dy * kHH + dx;  // clamp(p + delta_k), as staged
        dw[k] = g0 * sod[qn * 3] + g1 * sod[qn * 3 + 1] + g2 * sod[qn * 3 + 2];
        wl[k] = swk[c0 * 25 + k];
        dot = fmaf(wl[k], dw[k], dot);
      }
    for (int k = 0; k < 25; ++k) d[3 + k] = wl[k] * (dw[k] - dot);
    // d O_d(p): every pixel q whose clamped tap k lands on p, in the order
    // (dy, dx, qy, qx); per axis the q are p - d inside the image, widened to
    // the edge when p is an edge pixel
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int dy = -2; dy <= 2; ++dy) {
      const int ylo = max(y == 0 ? 0 : y - dy, 0), yhi = min(y == h - 1 ? h - 1 : y - dy, h - 1);
      for (int dx = -2; dx <= 2; ++dx) {
        const int xlo = max(x == 0 ? 0 : x - dx, 0), xhi = min(x == w - 1 ? w - 1 : x - dx, w - 1);
        const int k = 5 * (dy + 2) + (dx + 2);
        for (int py = ylo; py <= yhi; ++py)
          for (int px = xlo; px <= xhi; ++px) {
            const int qn = (py - y0 + 2) * kHH + (px - x0 + 2);
            const float wq = swk[qn * 25 + k];
            a0 = fmaf(wq, sdo[qn * 3], a0);
            a1 = fmaf(wq, sdo[qn * 3 + 1], a1);
            a2 = fmaf(wq, sdo[qn * 3 + 2], a2);
          }
      }
    }
    d[0] = a0;
    d[1] = a1;
    d[2] = a2;
  } else {
    for (int j = 0; j < 28; ++j) d[j] = 0.f;
  }
  __syncthreads();  // the kernel weights are no longer needed: stage outputs
  const int nx = min(kHT, w - x0), ny = min(kHT, h - y0);
  float4* so4 = (float4*)swk;
  for (int q = 0; q < 7; ++q)
    so4[tid * 7 + q] = make_float4(d[4 * q], d[4 * q + 1], d[4 * q + 2], d[4 * q + 3]);
  __syncthreads();
  // d28: per tile row 7 nx units of 16 bytes, contiguous in memory
  for (int e = tid; e < ny * 7 * kHT; e += 256) {
    const int r = e / (7 * kHT), u = e - r * 7 * kHT;
    if (u < 7 * nx)
      ((float4*)(d28 + (((int64_t)b * h + y0 + r) * w + x0) * 28))[u] = so4[r * 7 * kHT + u];
  }
  __syncthreads();
  for (int k4 = 0; k4 < 8; ++k4) {
    float v[4];
    for (int i = 0; i < 4; ++i) {
      float sacc = 0.f;
      for (int c = 0; c < 28; ++c) sacc = fmaf(sw[c * 32 + 4 * k4 + i], d[c], sacc);
      v[i] = sacc;
    }
    so4[tid * 9 + k4] = make_float4(v[0], v[1], v[2], v[3]);
  }
  __syncthreads();
  for (int e = tid; e < ny * 8 * kHT; e += 256) {
    const int r = e / (8 * kHT), u = e - r * 8 * kHT;
    if (u < 8 * nx) {
      const float4 g4 = so4[(r * kHT + (u >> 3)) * 9 + (u & 7)];
      const float g[4] = {g4.x, g4.y, g4.z, g4.w};
      store_gated<4>(dz, hd_act, (((int64_t)b * h + y0 + r) * w + x0) * 32 + 4 * u, g);
    }
  }
}

// Heads weight gradient partials: per chunk of pixels, d W[q][k] = sum d28[q] h[k]
// and d b[q] = sum d28[q] (28 x 33 outputs), each summed over the chunk's
// pixels in order.  Pixels are staged 64 at a time in LDS (h rows with the
// ones column, padded with zeros to 36); a thread owns 4 consecutive
// outputs of one q: one 4-byte and one 16-byte LDS read per pixel for 4
// FMAs (28 x 9 = 252 tiles).
__global__ void __launch_bounds__(256) k_heads_wgrad(const float* __restrict__ d28,
                                                     const uint8_t* __restrict__ hdec,
                                                     int64_t npx, int chunks,
                                                     float* __restrict__ part) {
  constexpr int Kp = 36, NKQ = Kp / 4;
  __shared__ __attribute__((aligned(16))) float sd[64 * 28];
  __shared__ __attribute__((aligned(16))) float shv[64 * Kp];
  const int chunk = blockIdx.x, tid = threadIdx.x;
  const int64_t p0 = npx * chunk / chunks, p1 = npx * (chunk + 1) / chunks;
  const int qq = tid / NKQ, kq = tid - qq * NKQ;  // this thread's tile (tid < 252)
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const uint16_t* h16 = (const uint16_t*)hdec;
  // fill items: pixel tid / 4's channel group tid % 4 (8 channels), and one
  // entry of columns 32..35 (ones for the bias, then zeros)
  const int hpp = tid >> 2, hg = tid & 3;
  const int xpp = tid >> 2, xk = 32 + (tid & 3);
  for (int64_t base = p0; base < p1; base += 64) {
    const int cnt = (int)min((int64_t)64, p1 - base);
    __syncthreads();
    for (int e = tid; e < 64 * 28; e += 256) sd[e] = e < cnt * 28 ? d28[base * 28 + e] : 0.f;
    {
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (hpp < cnt) v = *(const uint4*)(h16 + (base + hpp) * 32 + 8 * hg);
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
      float f[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        f[2 * i] = bf16_bits_to_f(wv[i] & 0xffffu);
        f[2 * i + 1] = bf16_bits_to_f(wv[i] >> 16);
      }
      float4* dst = (float4*)(shv + hpp * Kp + 8 * hg);
      dst[0] = make_float4(f[0], f[1], f[2], f[3]);
      dst[1] = make_float4(f[4], f[5], f[6], f[7]);
      shv[xpp * Kp + xk] = xk == 32 && xpp < cnt ? 1.0f : 0.f;
    }
    __syncthreads();
    if (tid < 28 * NKQ) {
      float a0 = acc[0], a1 = acc[1], a2 = acc[2], a3 = acc[3];
      const float4* h4 = (const float4*)shv + kq;
#pragma unroll 8
      for (int pp = 0; pp < 64; ++pp) {
        const float d = sd[pp * 28 + qq];
        const float4 hv = h4[pp * NKQ];
        a0 = fmaf(d, hv.x, a0);
        a1 = fmaf(d, hv.y, a1);
        a2 = fmaf(d, hv.z, a2);
        a3 = fmaf(d, hv.w, a3);
      }
      acc[0] = a0;
      acc[1] = a1;
      acc[2] = a2;
      acc[3] = a3;
    }
  }
  if (tid < 28 * NKQ) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * kq + i;
      if (k < 33) part[(int64_t)chunk * 28 * 33 + qq * 33 + k] = acc[i];
    }
  }
}

// The heads' gradient: the first-stage sums of the chunk partials (slices
// of chunks, by k_wgrad_reduce) summed in slice order, into the parameters.
__global__ void k_heads_reduce(const float* __restrict__ part2, int64_t off_hd, int64_t off_hk,
                               float* __restrict__ grad) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= 28 * 33) return;
  float s = 0.f;
  for (int sl = 0; sl < kReduceSlices; ++sl) s += part2[sl * 28 * 33 + o];
  const int qq = o / 33, k = o % 33;
  if (qq < 3)
    grad[k < 32 ? off_hd + qq * 32 + k : off_hd + 96 + qq] = s;
  else
    grad[k < 32 ? off_hk + (qq - 3) * 32 + k : off_hk + 800 + (qq - 3)] = s;
}

// -------------------------------------------------------- conv backward

// dz = g * [y > 0] (ReLU derivative) stored as BF16 for the MFMA dgrad
__global__ void __launch_bounds__(256) k_relu_mask(const float* __restrict__ g,
                                                   const uint8_t* __restrict__ y,
                                                   uint8_t* __restrict__ dz, int64_t n8) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n8) return;
  float yv[8], v[8];
  BF16::load8(y + e * 16, yv);
  for (int i = 0; i < 8; ++i) v[i] = yv[i] > 0.f ? g[e * 8 + i] : 0.f;
  BF16::store8(dz + e * 16, v);
}

// Input channels ch..ch+7 of a conv layer at pixel (y, x) of image b, as the
// forward kernel's patch fill defines them (concat of the bilinearly
// upsampled source 0, rounded to BF16 as the forward pass stores it, source
// 1 and source 2; zero outside the image), as BF16 bits.  ch is a multiple
// of 8 and so are c0 and c0 + c1, so a group never straddles two sources.
__device__ __forceinline__ uint4 conv_input8(const ConvArgs& a, int b, int y, int x, int ch) {
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  const int c01 = a.c0 + a.c1;
  if (y < 0 || y >= a.h || x < 0 || x >= a.w || ch >= c01 + (a.src2 ? a.c2 : 0)) return zero;
  if (ch >= c01)  // the third source (a fed-back state), c2 channels
    return *(const uint4*)((const uint16_t*)a.src2 +
                           (((int64_t)b * a.h + y) * a.w + x) * a.c2 + (ch - c01));
  if (ch >= a.c0)
    return *(const uint4*)((const uint16_t*)a.src1 +
                           (((int64_t)b * a.h + y) * a.w + x) * a.c1 + (ch - a.c0));
  const uint16_t* s0 = (const uint16_t*)a.src0;
  if (!a.up0) return *(const uint4*)(s0 + (((int64_t)b * a.h + y) * a.w + x) * a.c0 + ch);
  const int hh = a.h >> 1, ww = a.w >> 1;
  const float sy = fminf(fmaxf((y + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(hh - 1));
  const float sx = fminf(fmaxf((x + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(ww - 1));
  const int ly0 = (int)sy, lx0 = (int)sx;
  const int ly1 = min(ly0 + 1, hh - 1), lx1 = min(lx0 + 1, ww - 1);
  const float fy = sy - (float)ly0, fx = sx - (float)lx0;
  const int64_t base = (int64_t)b * hh * ww;
  const uint4 q00 = *(const uint4*)(s0 + (base + (int64_t)ly0 * ww + lx0) * a.c0 + ch);
  const uint4 q01 = *(const uint4*)(s0 + (base + (int64_t)ly0 * ww + lx1) * a.c0 + ch);
  const uint4 q10 = *(const uint4*)(s0 + (base + (int64_t)ly1 * ww + lx0) * a.c0 + ch);
  const uint4 q11 = *(const uint4*)(s0 + (base + (int64_t)ly1 * ww + lx1) * a.c0 + ch);
  const uint32_t w00[4] = {q00.x, q00.y, q00.z, q00.w}, w01[4] = {q01.x, q01.y, q01.z, q01.w};
  const uint32_t w10[4] = {q10.x, q10.y, q10.z, q10.w}, w11[4] = {q11.x, q11.y, q11.z, q11.w};
  uint32_t o[4];
  for (int i = 0; i < 4; ++i) {
    uint32_t packed = 0;
    for (int hi = 0; hi < 2; ++hi) {
      const int sh = 16 * hi;
      const float v00 = bf16_bits_to_f((w00[i] >> sh) & 0xffffu);
      const float v01 = bf16_bits_to_f((w01[i] >> sh) & 0xffffu);
      const float v10 = bf16_bits_to_f((w10[i] >> sh) & 0xffffu);
      const float v11 = bf16_bits_to_f((w11[i] >> sh) & 0xffffu);
      const float top = fmaf(fx, v01 - v00, v00), bot = fmaf(fx, v11 - v10, v10);
      // the forward pass stores the blended value in BF16
      const __bf16 v = (__bf16)fmaf(fy, bot - top, top);
      packed |= (uint32_t)__builtin_bit_cast(uint16_t, v) << sh;
    }
    o[i] = packed;
  }
  return make_uint4(o[0], o[1], o[2], o[3]);
}

// Weight gradient of a 3x3 layer on MFMA: per tap, dW[co][ci] = sum over
// pixels p of dz[p][co] x[p + tap][ci], a GEMM whose K dimension is the
// pixels (BF16 operands as stored by the forward pass and the ReLU mask,
// FP32 accumulation).  Block = 32 output x 32 input channels for all 9 taps
// and one chunk of 16 x 16-pixel tiles; wave w owns the 16 x 16 channel pair
// (w / 2, w % 2) and keeps its 9 tap accumulators (plus the bias, sum of dz,
// as an MFMA against ones) in registers.  Each tile's dz and input patch
// (18 x 18 pixels) are staged in LDS transposed, channel-major, so a lane's
// MFMA operand (8 consecutive pixels of one channel) is one 16-byte read;
// the three horizontal taps of one row share a 10-pixel window (a 16- and a
// 4-byte read, shifted by one and two pixels in registers).  K step s of a
// tile is rows 2s, 2s+1: lane group g takes row 2s + g/2, columns 8 (g%2)
// .. +7, the same pixels in both operands.  Partial sums go to part[chunk]
// and are summed in chunk order by k_wgrad_reduce, so the result is
// deterministic.
constexpr int kWgXRow = 24;                             // patch row in LDS (18 used)
constexpr int kWgXStride = (kWgRows + 2) * kWgXRow * 2 + 16;  // bytes per input channel
constexpr int kWgDStride = kWgRows * 16 * 2 + 16;              // bytes per output channel

__global__ void __launch_bounds__(256) k_wgrad(ConvArgs a, const uint8_t* __restrict__ dz,
                                               int ci_total, int co_total, int cig_n,
                                               int chunks, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint8_t sx[32 * kWgXStride];
  __shared__ __attribute__((aligned(16))) uint8_t sd[32 * kWgDStride];
  const int cig = blockIdx.x % cig_n, cog = blockIdx.x / cig_n;
  const int chunk = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int mt = wave >> 1, ns = wave & 1;
  const int g = lane >> 4, li = lane & 15, c8 = 8 * (g & 1);
  const int ci0 = cig * 32, co0 = cog * 32;
  const int tiles_x = (a.w + 15) / 16, tiles_y = (a.h + kWgRows - 1) / kWgRows;
  const int64_t tiles = (int64_t)a.n * tiles_x * tiles_y;
  const int64_t t0 = tiles * chunk / chunks, t1 = tiles * (chunk + 1) / chunks;
  const bool bias = cig == 0 && ns == 0;
  f32x4_t acc[9], accb = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const bf16x8_t ones = __builtin_bit_cast(bf16x8_t, make_uint4(0x3f803f80u, 0x3f803f80u,
                                                               0x3f803f80u, 0x3f803f80u));
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t t = t0; t < t1; ++t) {
    const int tx = (int)(t % tiles_x);
    const int64_t rr = t / tiles_x;
    const int ty = (int)(rr % tiles_y), b = (int)(rr / tiles_y);
    const int x0 = tx * 16, y0 = ty * kWgRows;
    __syncthreads();
    for (int e = tid; e < (kWgRows + 2) * 18 * 4; e += 256) {
      const int grp = e & 3, pix = e >> 2;
      const int r = pix / 18, c = pix - r * 18;
      const int ch = ci0 + 8 * grp;
      const uint4 v = ch < ci_total ? conv_input8(a, b, y0 - 1 + r, x0 - 1 + c, ch) : zero;
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      uint8_t* dst = sx + (8 * grp) * kWgXStride + (r * kWgXRow + c) * 2;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        *(uint16_t*)(dst + j * kWgXStride) = (uint16_t)(w[j >> 1] >> (16 * (j & 1)));
    }
    for (int e = tid; e < kWgRows * 16 * 4; e += 256) {
      const int grp = e & 3, pix = e >> 2;
      const int r = pix >> 4, c = pix & 15;
      const int y = y0 + r, x = x0 + c, co = co0 + 8 * grp;
      uint4 v = zero;
      if (y < a.h && x < a.w && co < co_total)
        v = *(const uint4*)(dz + ((((int64_t)b * a.h + y) * a.w + x) * co_total + co) * 2);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      uint8_t* dst = sd + (8 * grp) * kWgDStride + (r * 16 + c) * 2;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        *(uint16_t*)(dst + j * kWgDStride) = (uint16_t)(w[j >> 1] >> (16 * (j & 1)));
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kWgRows / 2; ++ks) {
      const int row = 2 * ks + (g >> 1);
      const bf16x8_t af =
          *(const bf16x8_t*)(sd + (mt * 16 + li) * kWgDStride + (row * 16 + c8) * 2);
      if (bias) accb = BF16::mma(af, ones, accb);
      const uint8_t* xb = sx + (ns * 16 + li) * kWgXStride + c8 * 2;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const uint8_t* p = xb + (row + dy) * kWgXRow * 2;
        const uint4 v = *(const uint4*)p;
        const uint32_t e4 = *(const uint32_t*)(p + 16);
        const uint4 v1 = make_uint4(__builtin_amdgcn_alignbit(v.y, v.x, 16),
                                    __builtin_amdgcn_alignbit(v.z, v.y, 16),
                                    __builtin_amdgcn_alignbit(v.w, v.z, 16),
                                    __builtin_amdgcn_alignbit(e4, v.w, 16));
        const uint4 v2 = make_uint4(v.y, v.z, v.w, e4);
        acc[3 * dy] = BF16::mma(af, __builtin_bit_cast(bf16x8_t, v), acc[3 * dy]);
        acc[3 * dy + 1] = BF16::mma(af, __builtin_bit_cast(bf16x8_t, v1), acc[3 * dy + 1]);
        acc[3 * dy + 2] = BF16::mma(af, __builtin_bit_cast(bf16x8_t, v2), acc[3 * dy + 2]);
      }
    }
  }
  // lane (g, li) holds D[4 g + r][li] of its pair: output channel
  // co0 + 16 mt + 4 g + r, input channel ci0 + 16 ns + li
  float* pp = part + (int64_t)chunk * (9 * (int64_t)ci_total * co_total + co_total);
  const int ci = ci0 + ns * 16 + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int co = co0 + mt * 16 + 4 * g + r;
    if (co < co_total && ci < ci_total)
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) pp[((int64_t)co * ci_total + ci) * 9 + tp] = acc[tp][r];
    if (bias && li == 0 && co < co_total) pp[9 * (int64_t)ci_total * co_total + co] = accb[r];
  }
}

// Sum of the chunk partials in two fixed-order stages: slice s of
// kReduceSlices sums chunks [s chunks / S, (s + 1) chunks / S) in order,
// then the slices are summed in order (deterministic for any hardware).
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* __restrict__ part, int chunks,
                                                      int64_t count, float* __restrict__ part2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int sl = blockIdx.y;
  if (e >= count) return;
  const int c0 = (int)((int64_t)chunks * sl / kReduceSlices);
  const int c1 = (int)((int64_t)chunks * (sl + 1) / kReduceSlices);
  float s = 0.f;
  for (int c = c0; c < c1; ++c) s += part[(int64_t)c * count + e];
  part2[(int64_t)sl * count + e] = s;
}

__global__ void __launch_bounds__(256) k_wgrad_reduce2(const float* __restrict__ part2,
                                                       int64_t count, float* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  float s = 0.f;
  for (int sl = 0; sl < kReduceSlices; ++sl) s += part2[(int64_t)sl * count + e];
  grad[e] = s;
}

// Gradient of a bilinear x2 upsampling (half-pixel centres, edge clamp):
// low-resolution pixel q gathers output rows (columns) 2q - 1 .. 2q + 2 with
// the weights the forward blend gave it, 1/4, 3/4, 3/4, 1/4, where the edge
// clamp turns the 3/4 of the first (last) sample into 1 and drops the tap
// outside the image.  These are exactly the values of the clamped formula.
__device__ __forceinline__ float up_tap(int j, int q, int nlow) {
  if (j == 0) return q > 0 ? 0.25f : 0.0f;
  if (j == 1) return q == 0 ? 1.0f : 0.75f;
  if (j == 2) return q == nlow - 1 ? 1.0f : 0.75f;
  return q < nlow - 1 ? 0.25f : 0.0f;
}

// V consecutive channels per thread (V = 4 when the channel counts allow
// 16-byte accesses); taps in row, then column order
// (with dz set: the masked BF16 gradient instead of glow, see store_gated)
template <int V>
__global__ void __launch_bounds__(256) k_upsample_bwd(const float* __restrict__ gup, int ch_stride,
                                                      int c0, int n, int hl, int wl,
                                                      float* __restrict__ glow, int acc,
                                                      const uint8_t* __restrict__ gate,
                                                      uint8_t* __restrict__ dz) {
  const int cg = c0 / V;
  const int64_t total = (int64_t)n * hl * wl * cg;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int c = (int)(e % cg) * V;
  const int64_t pix = e / cg;
  const int qx = (int)(pix % wl);
  const int64_t r = pix / wl;
  const int qy = (int)(r % hl), b = (int)(r / hl);
  const int h = 2 * hl, w = 2 * wl;
  float s[V];
#pragma unroll
  for (int v = 0; v < V; ++v) s[v] = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float wy = up_tap(j, qy, hl);
    if (wy == 0.f) continue;
    const int y = 2 * qy - 1 + j;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float wx = up_tap(i, qx, wl);
      if (wx == 0.f) continue;
      const int x = 2 * qx - 1 + i;
      const float* g = gup + (((int64_t)b * h + y) * w + x) * ch_stride + c;
      float gv[V];
      if constexpr (V == 4) {
        const float4 t = *(const float4*)g;
        gv[0] = t.x;
        gv[1] = t.y;
        gv[2] = t.z;
        gv[3] = t.w;
      } else {
        gv[0] = g[0];
      }
#pragma unroll
      for (int v = 0; v < V; ++v) s[v] = fmaf(wy * wx, gv[v], s[v]);
    }
  }
  float* o = glow + pix * c0 + c;
#pragma unroll
  for (int v = 0; v < V; ++v) s[v] = acc ? o[v] + s[v] : s[v];
  if (dz) {
    store_gated<V>(dz, gate, pix * c0 + c, s);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = s[v];
  }
}

// copy channels [c0, c0 + c1) of the transposed-conv output into the skip
// tensor's gradient (first contribution), V channels per thread
template <int V>
__global__ void __launch_bounds__(256) k_split_skip(const float* __restrict__ tmp, int ch_stride,
                                                    int c0, int c1, int64_t npx,
                                                    float* __restrict__ gskip) {
  const int cg = c1 / V;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= npx * cg) return;
  const int c = (int)(e % cg) * V;
  const int64_t p = e / cg;
  const float* src = tmp + p * ch_stride + c0 + c;
  float* dst = gskip + p * c1 + c;
  if constexpr (V == 4)
    *(float4*)dst = *(const float4*)src;
  else
    *dst = *src;
}

// gradient of 2x2 average pooling, added to the pooled tensor's source, V
// channels per thread
template <int V>
__global__ void __launch_bounds__(256) k_pool_bwd_add(const float* __restrict__ gp, int n, int h,
                                                      int w, int c, float* __restrict__ g,
                                                      const uint8_t* __restrict__ gate,
                                                      uint8_t* __restrict__ dz) {
  const int cg = c / V;
  const int64_t total = (int64_t)n * h * w * cg;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int ch = (int)(e % cg) * V;
  const int64_t pix = e / cg;
  const int x = (int)(pix % w);
  const int64_t r = pix / w;
  const int y = (int)(r % h), b = (int)(r / h);
  const float* src = gp + (((int64_t)b * (h / 2) + y / 2) * (w / 2) + x / 2) * c + ch;
  float* dst = g + pix * c + ch;
  float res[V];
  if constexpr (V == 4) {
    const float4 t = *(const float4*)src;
    float4 d = *(float4*)dst;
    d.x += 0.25f * t.x;
    d.y += 0.25f * t.y;
    d.z += 0.25f * t.z;
    d.w += 0.25f * t.w;
    res[0] = d.x;
    res[1] = d.y;
    res[2] = d.z;
    res[3] = d.w;
  } else {
    res[0] = *dst + 0.25f * *src;
  }
  if (dz) {
    store_gated<V>(dz, gate, pix * c + ch, res);
  } else if constexpr (V == 4) {
    *(float4*)dst = make_float4(res[0], res[1], res[2], res[3]);
  } else {
    *dst = res[0];
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ th, float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }


}  // namespace net
}  // namespace fv

using namespace fv;
using namespace fv::net;

static fv_status upload_gauss() {
  static bool done = false;
  if (done) return FV_OK;
  float g[11], sum = 0.f;
  double gd[11], sd = 0.0;
  for (int i = 0; i < 11; ++i) {
    const double x = i - 5.0;
    gd[i] = std::exp(-x * x / (2.0 * 1.5 * 1.5));
    sd += gd[i];
  }
  for (int i = 0; i < 11; ++i) {
    g[i] = (float)(gd[i] / sd);
    sum += g[i];
  }
  (void)sum;
  fv_status st = hip_status(hipMemcpyToSymbol(HIP_SYMBOL(c_gauss), g, sizeof g), "gauss upload");
  if (st == FV_OK) done = true;
  return st;
}

// ---------------------------------------------------- shared with the W-Net

namespace fv {
namespace net {

size_t loss_ssim_bytes(int n, int h, int w) {
  const size_t q = (size_t)n * 3;
  return al(q * h * (w - 10) * 4 * 5) + al(q * (h - 10) * (w - 10) * 4 * 3) +
         al(q * h * (w - 10) * 4 * 3);
}

size_t loss_red_bytes(int n, int h, int w) {
  const int64_t q = (int64_t)n * 3;
  const int64_t vblocks = (q * (h - 10) * (w - 10) + 255) / 256;
  const int64_t lblocks = (q * h * w + 255) / 256;
  return al((size_t)(vblocks + lblocks) * 8);
}

fv_status loss_run(const float* out_rgb, const float* target_rgba, int n, int h, int w,
                   float* loss3, float* dloss_dout, float* tgt, uint8_t* ssim, double* red,
                   hipStream_t s) {
  fv_status st = upload_gauss();
  if (st != FV_OK) return st;
  const int64_t npx = (int64_t)n * h * w;
  k_rgb_of_rgba<<<nblk(npx), 256, 0, s>>>((const float4*)target_rgba, tgt, npx);
  const int64_t q = (int64_t)n * 3;
  const int64_t htot = q * h * (w - 10), vtot = q * (h - 10) * (w - 10);
  float* hq = (float*)ssim;
  float* dmap = (float*)(ssim + al(htot * 4 * 5));
  float* va = (float*)(ssim + al(htot * 4 * 5) + al(vtot * 4 * 3));
  const int64_t nyv = (h - 10 + kSsimRows - 1) / kSsimRows, nyt = (h + kSsimRows - 1) / kSsimRows;
  const unsigned nbv = nblk(q * nyv * (w - 10)), nbl = nblk((int64_t)n * h * w);
  k_ssim_h<<<nblk((int64_t)n * h * (w - 10)), 256, 0, s>>>(out_rgb, tgt, n, h, w, hq);
  k_ssim_v<<<nbv, 256, 0, s>>>(hq, n, h, w, dmap, red);
  k_ssim_vt<<<nblk(q * nyt * (w - 10)), 256, 0, s>>>(dmap, n, h, w, va);
  const double ssim_scale = 1.0 / (double)vtot, l1_scale = 1.0 / (double)(q * h * w);
  k_ssim_ht<<<nbl, 256, 0, s>>>(va, out_rgb, tgt, n, h, w, (float)ssim_scale, (float)l1_scale,
                                dloss_dout, red + nbv);
  k_loss_final<<<1, 1024, 0, s>>>(red, (int)nbv, red + nbv, (int)nbl, ssim_scale, l1_scale,
                                   loss3);
  return launch_status("loss");
}

fv_status tloss_run(const float* out_rgb, const float* target_rgba, int pairs, int h, int w,
                    float weight, float* loss, float* dloss_dout, double* red, hipStream_t s) {
  const int64_t hw = (int64_t)h * w, cnt = (int64_t)pairs * hw * 3;
  const unsigned nb = nblk(cnt);
  k_tloss<<<nb, 256, 0, s>>>(out_rgb, (const float4*)target_rgba, pairs, hw,
                             (float)((double)weight / (double)cnt), dloss_dout, red);
  k_tloss_final<<<1, 256, 0, s>>>(red, (int)nb, 1.0 / (double)cnt, loss);
  return launch_status("temporal loss");
}

void launch_relu_mask(const float* g, const uint8_t* y, uint8_t* dz, int64_t n8, hipStream_t s) {
  k_relu_mask<<<nblk(n8), 256, 0, s>>>(g, y, dz, n8);
}

// (the 4-channel forms need 16-byte aligned tensors, which workspace
// offsets are, and channel counts that are multiples of 4)
void launch_upsample_bwd(const float* gup, int ch_stride, int c0, int n, int hl, int wl,
                         float* glow, int acc, hipStream_t s, const uint8_t* gate, uint8_t* dz) {
  if (c0 % 4 == 0 && ch_stride % 4 == 0)
    k_upsample_bwd<4><<<nblk((int64_t)n * hl * wl * c0 / 4), 256, 0, s>>>(
        gup, ch_stride, c0, n, hl, wl, glow, acc, gate, dz);
  else
    k_upsample_bwd<1><<<nblk((int64_t)n * hl * wl * c0), 256, 0, s>>>(
        gup, ch_stride, c0, n, hl, wl, glow, acc, gate, dz);
}

void launch_split_skip(const float* tmp, int ch_stride, int c0, int c1, int64_t npx,
                       float* gskip, hipStream_t s) {
  if (c0 % 4 == 0 && c1 % 4 == 0 && ch_stride % 4 == 0)
    k_split_skip<4><<<nblk(npx * c1 / 4), 256, 0, s>>>(tmp, ch_stride, c0, c1, npx, gskip);
  else
    k_split_skip<1><<<nblk(npx * c1), 256, 0, s>>>(tmp, ch_stride, c0, c1, npx, gskip);
}

void launch_pool_bwd_add(const float* gp, int n, int h, int w, int c, float* g, hipStream_t s,
                         const uint8_t* gate, uint8_t* dz) {
  if (c % 4 == 0)
    k_pool_bwd_add<4><<<nblk((int64_t)n * h * w * c / 4), 256, 0, s>>>(gp, n, h, w, c, g, gate,
                                                                       dz);
  else
    k_pool_bwd_add<1><<<nblk((int64_t)n * h * w * c), 256, 0, s>>>(gp, n, h, w, c, g, gate, dz);
}

int wgrad_chunks(int n, int h, int w, int ci, int co) {
  const int64_t tiles = (int64_t)n * ((h + kWgRows - 1) / kWgRows) * ((w + 15) / 16);
  const int64_t groups = (int64_t)((ci + 31) / 32) * ((co + 31) / 32);
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 2048 / groups));
}

size_t wgrad_part_bytes(int chunks, int ci, int co) {
  return (size_t)chunks * (9 * (size_t)ci * co + co) * 4;
}

size_t wgrad_part2_bytes(int ci, int co) {
  return (size_t)kReduceSlices * (9 * (size_t)ci * co + co) * 4;
}

fv_status conv_wgrad(const ConvArgs& in, const uint8_t* dz, int ci, int co, int chunks,
                     float* part, float* part2, float* grad, hipStream_t s) {
  const int cig_n = (ci + 31) / 32;
  dim3 gw((unsigned)(cig_n * ((co + 31) / 32)), (unsigned)chunks);
  k_wgrad<<<gw, 256, 0, s>>>(in, dz, ci, co, cig_n, chunks, part);
  const int64_t cnt = 9 * (int64_t)ci * co + co;
  k_wgrad_reduce<<<dim3(nblk(cnt), kReduceSlices), 256, 0, s>>>(part, chunks, cnt, part2);
  k_wgrad_reduce2<<<nblk(cnt), 256, 0, s>>>(part2, cnt, grad);
  return launch_status("wgrad");
}

fv_status adam_run(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                   float b2, float eps, int64_t step, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
  k_adam<<<nblk(n), 256, 0, s>>>(th, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return launch_status("adam");
}

}  // namespace net
}  // namespace fv

extern "C" {

fv_status fv_train_workspace(const fv_net* n, int batch, int width, int height, size_t* bytes) {
  clear_error();
  if (!n || !bytes) return fail(FV_ERR_INVALID_ARG, "fv_train_workspace: null pointer");
  fv_status st = check_frame(batch, width, height, "fv_train_workspace");
  if (st != FV_OK) return st;
  if (width < 16 || height < 16)
    return fail(FV_ERR_INVALID_ARG, "fv_train_workspace: training tiles must be >= 16 x 16");
  *bytes = make_train_plan(batch, height, width).bytes;
  return FV_OK;
}

static fv_status train_check(const fv_net* n, int batch, int width, int height, void* ws,
                             size_t ws_bytes, TrainPlan* tp, const char* fn) {
  if (!n || !ws) return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  fv_status st = check_frame(batch, width, height, fn);
  if (st != FV_OK) return st;
  if (width < 16 || height < 16)
    return fail(FV_ERR_INVALID_ARG, "%s: training tiles must be >= 16 x 16", fn);
  *tp = make_train_plan(batch, height, width);
  if (ws_bytes < tp->bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, tp->bytes);
  if ((uintptr_t)ws % 256) return fail(FV_ERR_INVALID_ARG, "%s: workspace not aligned", fn);
  return FV_OK;
}

static fv_status forward_train(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                               const float* frame_depth, const float* prev, int batch,
                               int width, int height, float* out_rgb, void* workspace,
                               size_t ws_bytes, void* stream, const char* fn) {
  clear_error();
  TrainPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp, fn);
  if (st != FV_OK) return st;
  if (!frame_rgba || !mask || !out_rgb) return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  if (prev && !n->recurrent)
    return fail(FV_ERR_INVALID_ARG, "%s: the network has no recurrent input", fn);
  uint8_t* ws = (uint8_t*)workspace;
  return forward_impl<BF16>(n, tp.f, ws, frame_rgba, mask, frame_depth, prev, out_rgb,
                            (float*)(ws + tp.f.od), (float*)(ws + tp.f.wk), nullptr,
                            (hipStream_t)stream, false, 0, kNumConv);
}

fv_status fv_net_forward_train(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                               const float* frame_depth, int batch, int width, int height,
                               float* out_rgb, void* workspace, size_t ws_bytes, void* stream) {
  return forward_train(n, frame_rgba, mask, frame_depth, nullptr, batch, width, height, out_rgb,
                       workspace, ws_bytes, stream, "fv_net_forward_train");
}

fv_status fv_net_forward_train_recurrent(fv_net* n, const float* frame_rgba,
                                         const uint8_t* mask, const float* frame_depth,
                                         const float* prev_direct, int batch, int width,
                                         int height, float* out_rgb, void* workspace,
                                         size_t ws_bytes, void* stream) {
  return forward_train(n, frame_rgba, mask, frame_depth, prev_direct, batch, width, height,
                       out_rgb, workspace, ws_bytes, stream, "fv_net_forward_train_recurrent");
}

fv_status fv_net_loss(const fv_net* n, const float* out_rgb, const float* target_rgba, int batch,
                      int width, int height, float* loss3, float* dloss_dout, void* workspace,
                      size_t ws_bytes, void* stream) {
  clear_error();
  TrainPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp, "fv_net_loss");
  if (st != FV_OK) return st;
  if (!out_rgb || !target_rgba || !loss3 || !dloss_dout)
    return fail(FV_ERR_INVALID_ARG, "fv_net_loss: null pointer");
  uint8_t* ws = (uint8_t*)workspace;
  return loss_run(out_rgb, target_rgba, batch, height, width, loss3, dloss_dout,
                  (float*)(ws + tp.target), ws + tp.ssim, (double*)(ws + tp.red),
                  (hipStream_t)stream);
}

fv_status fv_net_loss_temporal(const fv_net* n, const float* out_rgb, const float* target_rgba,
                               int batch, int width, int height, float weight, float* loss,
                               float* dloss_dout, void* workspace, size_t ws_bytes,
                               void* stream) {
  clear_error();
  TrainPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_net_loss_temporal");
  if (st != FV_OK) return st;
  if (!out_rgb || !target_rgba || !loss || !dloss_dout)
    return fail(FV_ERR_INVALID_ARG, "fv_net_loss_temporal: null pointer");
  if (batch % 2)
    return fail(FV_ERR_INVALID_ARG, "fv_net_loss_temporal: batch %d is not a set of pairs",
                batch);
  if (!(weight >= 0.0f && std::isfinite(weight)))
    return fail(FV_ERR_INVALID_ARG, "fv_net_loss_temporal: weight must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  const int64_t hw = (int64_t)height * width, pairs = batch / 2;
  const int64_t cnt = pairs * hw * 3;
  // the block partials fit in the loss partial-sum region (half the L1 blocks)
  double* red = (double*)(ws + tp.red);
  const unsigned nb = nblk(cnt);
  k_tloss<<<nb, 256, 0, s>>>(out_rgb, (const float4*)target_rgba, pairs, hw,
                             (float)((double)weight / (double)cnt), dloss_dout, red);
  k_tloss_final<<<1, 256, 0, s>>>(red, (int)nb, 1.0 / (double)cnt, loss);
  return launch_status("fv_net_loss_temporal");
}

fv_status fv_net_backward(fv_net* n, const float* dloss_dout, int batch, int width, int height,
                          float* grad_out, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  TrainPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp,
                             "fv_net_backward");
  if (st != FV_OK) return st;
  if (!dloss_dout) return fail(FV_ERR_INVALID_ARG, "fv_net_backward: null dloss_dout");
  hipStream_t s = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)workspace;
  const Plan& p = tp.f;
  const int64_t npx = (int64_t)p.n * p.h * p.w;
  float* grad = n->grad;
  float* tmp = (float*)(ws + tp.tmp);
  uint8_t* dz = ws + tp.dz;       // masked output gradient of layer l
  uint8_t* dz_next = ws + tp.dz2;  // of layer l - 1, when layer l's kernels store it
  bool dz_ready = true;            // dz already holds layer l's masked gradient
  float* part = (float*)(ws + tp.part);
  auto G = [&](int t) { return (float*)(ws + tp.g[t]); };
  // heads (they also store the last conv's masked output gradient in dz)
  k_heads_bwd<<<dim3((p.w + kHT - 1) / kHT, (p.h + kHT - 1) / kHT, p.n), 256, 0, s>>>(
      dloss_dout, (const float*)(ws + p.od), (const float*)(ws + p.wk), p.h, p.w, n->master,
      param_offset(14), param_offset(15), tmp, ws + p.t[T_D0B], dz);
  const int hchunks = kHeadChunks;
  k_heads_wgrad<<<hchunks, 256, 0, s>>>(tmp, ws + p.t[T_D0B], npx, hchunks, part);
  float* part2 = (float*)(ws + tp.part2);
  k_wgrad_reduce<<<dim3(nblk(28 * 33), kReduceSlices), 256, 0, s>>>(part, hchunks, 28 * 33,
                                                                    part2);
  k_heads_reduce<<<4, 256, 0, s>>>(part2, param_offset(14), param_offset(15), grad);
  if ((st = launch_status("heads backward")) != FV_OK) return st;
  for (int l = kNumConv - 1; l >= 0; --l) {
    const LayerDesc& L = kLayers[l];
    const int* io = kLayerIO[l];
    const int hh = p.h >> L.level, ww = p.w >> L.level;
    const int64_t px = (int64_t)p.n * hh * ww;
    // ReLU derivative, BF16 copy of the output gradient (unless a kernel of
    // layer l + 1 or the heads stored it)
    if (!dz_ready)
      k_relu_mask<<<nblk(px * L.co / 8), 256, 0, s>>>(G(io[2]), ws + p.t[io[2]], dz,
                                                      px * L.co / 8);
    dz_ready = false;
    // weight + bias gradient
    ConvArgs in{};
    in.src0 = ws + p.t[io[0]];
    in.src1 = io[1] >= 0 ? ws + p.t[io[1]] : nullptr;
    in.c0 = L.c0;
    in.c1 = L.c1;
    in.up0 = L.up0;
    in.n = p.n;
    in.h = hh;
    in.w = ww;
    const int ci_tot = l == 0 ? L.ci : L.c0 + L.c1;
    const int cig_n = (ci_tot + 31) / 32;
    dim3 gw((unsigned)(cig_n * ((L.co + 31) / 32)), (unsigned)tp.chunks[l]);
    k_wgrad<<<gw, 256, 0, s>>>(in, dz, ci_tot, L.co, cig_n, tp.chunks[l], part);
    const int64_t cnt = 9 * (int64_t)ci_tot * L.co + L.co;
    k_wgrad_reduce<<<dim3(nblk(cnt), kReduceSlices), 256, 0, s>>>(part, tp.chunks[l], cnt, part2);
    k_wgrad_reduce2<<<nblk(cnt), 256, 0, s>>>(part2, cnt, grad + param_offset(l));
    if ((st = launch_status("wgrad")) != FV_OK) return st;
    if (l == 0) break;  // no gradient w.r.t. the network input
    // input gradient: conv with transposed weights, FP32 output
    ConvArgs a{};
    a.src0 = dz;
    a.src1 = nullptr;
    a.c0 = L.co;
    a.c1 = 0;
    a.cip = cip_of(L.co);
    a.up0 = 0;
    a.n = p.n;
    a.h = hh;
    a.w = ww;
    a.wsw = (const uint8_t*)n->w_bf16t[l];
    a.kc = kchunks_of(L.co);
    a.alpha = nullptr;
    a.bias = nullptr;
    a.co = L.c0 + L.c1;
    a.relu = 0;
    a.out_fp32 = 1;
    a.out_ch = L.c0 + L.c1;
    a.absmax = nullptr;
    const bool concat = io[1] >= 0;
    a.out = (uint8_t*)(concat ? tmp : G(io[0]));
    // The input is layer l - 1's output with no other consumer: the conv
    // stores that layer's masked BF16 gradient directly (the same bits as
    // the FP32 gradient through k_relu_mask).
    const bool gated = !concat && io[0] == kLayerIO[l - 1][2];
    if (gated) {
      a.out_fp32 = 0;
      a.out = dz_next;
      a.gate = ws + p.t[io[0]];
    }
    if ((st = launch_conv<BF16>(a, nblocks_of(L.c0 + L.c1), s)) != FV_OK) return st;
    if (gated) {
      std::swap(dz, dz_next);
      dz_ready = true;
    }
    // The upsampled source (e3b, d2b, d1b) is layer l - 1's output with no
    // other consumer, and the pooled source (e0b, e1b, e2b) gets its last
    // contribution (its skip gradient came earlier): either kernel stores
    // layer l - 1's masked BF16 gradient instead of the FP32 one.
    bool next_ready = false;
    if (concat) {
      const int hl = hh / 2, wl = ww / 2;
      next_ready = io[0] == kLayerIO[l - 1][2];
      launch_upsample_bwd(tmp, L.c0 + L.c1, L.c0, p.n, hl, wl, G(io[0]), 0, s,
                          next_ready ? ws + p.t[io[0]] : nullptr, next_ready ? dz_next : nullptr);
      launch_split_skip(tmp, L.c0 + L.c1, L.c0, L.c1, px, G(io[1]), s);
    }
    // the pooled input's gradient flows back to the pooled tensor's source
    int src = -1;
    if (io[0] == T_P0) src = T_E0B;
    if (io[0] == T_P1) src = T_E1B;
    if (io[0] == T_P2) src = T_E2B;
    if (src >= 0) {
      next_ready = src == kLayerIO[l - 1][2];
      launch_pool_bwd_add(G(io[0]), p.n, hh * 2, ww * 2, L.c0, G(src), s,
                          next_ready ? ws + p.t[src] : nullptr, next_ready ? dz_next : nullptr);
    }
    if (next_ready) {
      std::swap(dz, dz_next);
      dz_ready = true;
    }
    if ((st = launch_status("dgrad")) != FV_OK) return st;
  }
  if (grad_out) {
    // in the external layout of the network's form
    const int64_t P = param_count();
    if (n->recurrent) {
      st = hip_status(hipMemcpyAsync(grad_out, grad, P * sizeof(float), hipMemcpyDeviceToDevice,
                                     s), "fv_net_backward: copy grads");
    } else {
      const LayerDesc& L0 = kLayers[0];
      const int ce = L0.ci - kFedBack;
      const int64_t wi = (int64_t)L0.co * L0.ci * 9, we = (int64_t)L0.co * ce * 9;
      st = hip_status(hipMemcpy2DAsync(grad_out, ce * 9 * sizeof(float), grad,
                                       L0.ci * 9 * sizeof(float), ce * 9 * sizeof(float), L0.co,
                                       hipMemcpyDeviceToDevice, s),
                      "fv_net_backward: copy grads");
      if (st == FV_OK)
        st = hip_status(hipMemcpyAsync(grad_out + we, grad + wi, (P - wi) * sizeof(float),
                                       hipMemcpyDeviceToDevice, s),
                        "fv_net_backward: copy grads");
    }
  }
  return st;
}

fv_status fv_net_adam(fv_net* n, float lr, float beta1, float beta2, float eps, void* stream) {
  clear_error();
  if (!n) return fail(FV_ERR_INVALID_ARG, "fv_net_adam: null net");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(FV_ERR_INVALID_ARG, "fv_net_adam: bad hyper-parameters");
  hipStream_t s = (hipStream_t)stream;
  n->step += 1;
  // bias corrections 1 - beta^t, formed in double: in FP32 the subtraction
  // of a rounded beta^t close to 1 would lose most of the difference's bits
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)n->step));
  const int64_t P = param_count();
  k_adam<<<nblk(P), 256, 0, s>>>(n->master, n->adam_m, n->adam_v, n->grad, P, lr, beta1, beta2,
                                 eps, c1, c2);
  fv_status st = launch_status("fv_net_adam");
  if (st == FV_OK) st = refresh_bf16(n, s);
  n->fp8_ready = 0;
  return st;
}

fv_status fv_train_step(fv_net* n, const float* frame_rgba, const uint8_t* mask,
                        const float* frame_depth, const float* target_rgba, int batch,
                        int width, int height, float lr, float* loss3, void* workspace,
                        size_t ws_bytes, void* stream) {
  clear_error();
  TrainPlan tp;
  fv_status st = train_check(n, batch, width, height, workspace, ws_bytes, &tp, "fv_train_step");
  if (st != FV_OK) return st;
  uint8_t* ws = (uint8_t*)workspace;
  // network output in the (not yet used) transposed-conv buffer, loss
  // gradient in its own slot
  float* yout = (float*)(ws + tp.tmp);
  float* out = (float*)(ws + tp.dout);
  if ((st = fv_net_forward_train(n, frame_rgba, mask, frame_depth, batch, width, height, yout,
                                 workspace, ws_bytes, stream)) != FV_OK)
    return st;
  if ((st = fv_net_loss(n, yout, target_rgba, batch, width, height, loss3, out, workspace,
                        ws_bytes, stream)) != FV_OK)
    return st;
  if ((st = fv_net_backward(n, out, batch, width, height, nullptr, workspace, ws_bytes,
                            stream)) != FV_OK)
    return st;
  return fv_net_adam(n, lr, 0.9f, 0.999f, 1e-8f, stream);
}

}  // extern "C"
