// Internal declarations of the reconstruction network (not part of the ABI).
//
// Network (paper: "Reconstruction Network"): a 4-level U-Net (32/48/64/96
// channels, two 3x3 conv + ReLU per block, 2x2 average pooling, bilinear x2
// upsampling, concatenated skips) whose last decoder state feeds a direct
// RGB head (O_d, 1x1 conv) and a kernel-prediction head (1x1 conv -> 25
// logits -> softmax -> 5x5 kernel applied to O_d).
//
// Activations are NHWC.  Convolutions are implicit GEMMs on MFMA: the GEMM
// K index is tap-major, k = tap * CiP + ci with CiP = Ci rounded up to 8, and
// is cut into 32-wide chunks; weights are pre-arranged ("swizzled") so each
// lane loads its MFMA B fragment with one 16-byte (bf16) / 8-byte (fp8) load.
#pragma once

#include "common.h"

namespace fv {
namespace net {

constexpr int kNumLayers = 16;
constexpr int kNumConv = 14;  // 3x3 layers; 14 and 15 are the 1x1 heads

struct LayerDesc {
  const char* name;
  int ci, co, k;
  int level;      // resolution level of the output (0 = full)
  int c0, c1;     // input channels from source 0 / source 1 (concat skip)
  int up0;        // source 0 is bilinearly upsampled x2 on load
};

// Canonical layer order (also the order of the flat parameter vector:
// each layer's weight [Co][Ci][k][k] then its bias [Co]).  Inside the
// library the first conv always reads 8 input channels: the 5 of the sparse
// frame and 3 for the previous frame's direct prediction O_d (the recurrent
// form, paper Sec. 3.2.4).  The plain network keeps zero weights on those
// channels and its parameter vector leaves them out (external layout).
extern const LayerDesc kLayers[kNumLayers];
constexpr int kFedBack = 3;  // fed-back channels of the recurrent form

__host__ __device__ inline int cip_of(int ci) { return (ci + 7) / 8 * 8; }
// K chunks of a 3x3 conv over ci input channels: 32 wide (BF16 MFMA) or
// 128 wide (FP8 MFMA); K = 9 taps x cip, zero-padded to whole chunks.
__host__ __device__ inline int kchunks_of(int ci) { return (9 * cip_of(ci) + 31) / 32; }
__host__ __device__ inline int kchunks128_of(int ci) { return (9 * cip_of(ci) + 127) / 128; }
__host__ __device__ inline int nblocks_of(int co) { return (co + 15) / 16; }

// Offsets of each layer's weight / bias in the internal parameter vector.
int64_t param_offset(int layer);
int64_t param_count();
// Length of the external parameter vector of either form.
int64_t external_param_count(int recurrent);
// External <-> internal layout (they differ in the first conv's weights of
// the plain form only).
void params_to_internal(const float* ext, int recurrent, float* internal);
void params_to_external(const float* internal, int recurrent, float* ext);

// Activation tensors of one forward pass (indices into Plan::t).
enum Tensor {
  T_IN = 0, T_E0A, T_E0B, T_P0, T_E1A, T_E1B, T_P1, T_E2A, T_E2B, T_P2, T_E3A, T_E3B,
  T_D2A, T_D2B, T_D1A, T_D1B, T_D0A, T_D0B, kNumTensors
};

struct TensorDesc {
  int channels, level;
};
extern const TensorDesc kTensors[kNumTensors];

// Per conv layer: (source 0, source 1 or -1, output) tensor indices.
extern const int kLayerIO[kNumConv][3];

// Byte layout of a forward-pass workspace for batch n at H x W.
struct Plan {
  int n, h, w;
  size_t elem;                 // bytes per activation element (2 bf16, 1 fp8)
  size_t t[kNumTensors];       // byte offsets of the activation tensors
  size_t od, wk, absmax;       // O_d (f32 x3), softmax weights (f32 x25), calibration maxima
  size_t bytes;                // total
};
Plan make_plan(int n, int h, int w, size_t elem);

// Training workspace: the BF16 forward plan followed by FP32 gradients of
// every activation tensor, a transposed-conv output buffer, the masked BF16
// output gradient of the current layer, weight-gradient partial sums and
// loss scratch.
struct TrainPlan {
  Plan f;
  size_t g[kNumTensors];  // FP32 gradient of each activation tensor (not T_IN)
  size_t tmp;             // FP32 [px at level][Ci] of the current layer
  size_t dz, dz2;         // BF16 masked gradient of the current layer output
                          // (two buffers: an input-gradient conv reads one
                          // and stores the next layer's into the other)
  size_t target;          // FP32 copy of the target RGB (loss)
  size_t dout;            // FP32 d loss / d out [n h w 3]
  size_t ssim;            // SSIM maps: 5 filtered row maps + 3 partial maps
  size_t part;            // weight-gradient partial sums (per pixel chunk)
  size_t part2;           // their first-stage sums (per slice of chunks)
  size_t red;             // loss partial sums
  size_t bytes;
  int chunks[kNumConv];   // pixel chunks of each layer's weight gradient
};
TrainPlan make_train_plan(int n, int h, int w);

// Shared with the W-Net (wnet.hip): BF16 weight fragments of a 3x3 layer,
// their element count, the 8-channel BF16 input packing (the last three the
// previous O_d, [n h w 3] FP32, or zero when prev is null) and the frame
// checks of the reconstruction entry points.
// (out_limit: build only the first out_limit output channels of the GEMM,
// the input channels of a transposed conv whose other gradients are unused)
fv_status swizzle_bf16(const float* w, int ci, int co, int transposed, void* out, hipStream_t s,
                       int out_limit = 1 << 30);
size_t swizzled_elems(int in_ch, int out_ch);
fv_status pack_input_bf16(const float* frame, const uint8_t* mask, const float* depth,
                          const float* prev, uint8_t* out, int64_t npx, hipStream_t s);
fv_status check_frame(int views, int W, int H, const char* fn);

// Training pieces shared with the W-Net (net_train.hip): the loss (SSIM +
// L1, its scratch: target RGB, SSIM maps, partial sums), the backward
// elementwise kernels, the MFMA weight gradient of a 3x3 conv (with its
// chunk count and partial-sum sizes) and Adam.
size_t loss_ssim_bytes(int n, int h, int w);
size_t loss_red_bytes(int n, int h, int w);
fv_status loss_run(const float* out_rgb, const float* target_rgba, int n, int h, int w,
                   float* loss3, float* dloss_dout, float* tgt, uint8_t* ssim, double* red,
                   hipStream_t s);
// the temporal finite-difference loss over batch pairs (2i, 2i + 1); its
// block partial sums fit in loss_red_bytes' region
fv_status tloss_run(const float* out_rgb, const float* target_rgba, int pairs, int h, int w,
                    float weight, float* loss, float* dloss_dout, double* red, hipStream_t s);
void launch_relu_mask(const float* g, const uint8_t* y, uint8_t* dz, int64_t n8, hipStream_t s);
// With dz set, the upsample and pool backward do not store the finished
// FP32 gradient but dz = BF16(gradient x [gate > 0]), the masked output
// gradient the ReLU mask pass would make from it (gate: the forward
// activation, BF16, same layout).
void launch_upsample_bwd(const float* gup, int ch_stride, int c0, int n, int hl, int wl,
                         float* glow, int acc, hipStream_t s, const uint8_t* gate = nullptr,
                         uint8_t* dz = nullptr);
void launch_split_skip(const float* tmp, int ch_stride, int c0, int c1, int64_t npx,
                       float* gskip, hipStream_t s);
void launch_pool_bwd_add(const float* gp, int n, int h, int w, int c, float* g, hipStream_t s,
                         const uint8_t* gate = nullptr, uint8_t* dz = nullptr);
int wgrad_chunks(int n, int h, int w, int ci, int co);
size_t wgrad_part_bytes(int chunks, int ci, int co);
size_t wgrad_part2_bytes(int ci, int co);
struct ConvArgs;
fv_status conv_wgrad(const ConvArgs& in, const uint8_t* dz, int ci, int co, int chunks,
                     float* part, float* part2, float* grad, hipStream_t s);
fv_status adam_run(float* th, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                   float b2, float eps, int64_t step, hipStream_t s);

}  // namespace net
}  // namespace fv

// The network handle: FP32 master parameters + Adam state, the swizzled
// BF16 copy used by training and BF16 inference, and the FP8 copy with its
// scales (valid after fv_net_calibrate).
struct fv_net {
  int device;
  float* master;          // [P] canonical order
  float* adam_m;          // [P]
  float* adam_v;          // [P]
  float* grad;            // [P]
  int64_t step;           // Adam steps taken
  void* w_bf16[fv::net::kNumConv];
  void* w_bf16t[fv::net::kNumConv];     // transposed (input-gradient) weights
  void* w_heads;                        // the two 1x1 heads as BF16 MFMA fragments
  void* w_heads_fp8;                    // the same times the FP8 decoder-output scale
  void* w_fp8[fv::net::kNumConv];
  float* alpha_fp8[fv::net::kNumConv];  // per-output-channel dequant x requant factor
  float* bias_fp8[fv::net::kNumConv];   // bias / output scale
  float act_scale[fv::net::kNumTensors];  // FP8 per-tensor activation scales
  int fp8_ready;
  int recurrent;  // 1: the first conv reads the previous frame's O_d
  float* mix0_ab;  // [2 x 32] scale / bias of the BF16 first layer under FP8
};
