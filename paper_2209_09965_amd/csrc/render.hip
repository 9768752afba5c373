// The foveated frame as one call, with the dense march kept as the quality
// reference and the fallback of the reconstruction (paper Sec. 3, the pipeline of
// Fig. 2: sample map -> compaction -> sparse march -> back-projection ->
// reconstruction; the conventional renderer it replaces is the dense march).
//
// A renderer owns every intermediate buffer of the frame.  Every
// check_every-th frame it also marches the dense frame and scores the
// reconstruction against it (PSNR over clamped RGB, reduced on the device in
// a fixed order, read back with one synchronisation).  Below min_psnr_db the
// frame is replaced by the dense frame and the renderer stays in fallback,
// marching dense frames, until a later check frame scores at or above the
// threshold again.
#include <cstring>

#include "common.h"

struct fv_renderer {
  int device, views, W, H;
  fv_render_policy pol;
  uint64_t frame;     // frames rendered so far
  int fallback;       // 1: frames are dense until the next passing check
  uint32_t* ray_idx;  // [views W H]
  uint32_t* count;    // [1]
  uint8_t* mask;      // [views W H]
  float* sparse;      // [views W H 4] back-projected sparse frame
  float* depth;       // [views W H]
  float* dense;       // [views W H 4] dense frame (checks and fallback)
  double* partial;    // MSE partial sums [kMseBlocks + 1]
  void* ws_mask;
  void* ws_march;
  void* ws_recon;
  size_t n_mask, n_march, n_recon;
};

namespace fv {
namespace {

constexpr int kMseBlocks = 1024;

// Squared clamped differences of RGB (3 per pixel) against RGBA (4 per
// pixel): one FP64 partial per block, each block summing a fixed strided set.
__global__ void __launch_bounds__(256) k_mse_partial(const float* __restrict__ rgb,
                                                     const float4* __restrict__ ref, size_t npx,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < npx; p += (size_t)gridDim.x * 256) {
    const float4 r = ref[p];
    const float rr[3] = {r.x, r.y, r.z};
    for (int c = 0; c < 3; ++c) {
      const float a = fminf(fmaxf(rgb[p * 3 + c], 0.0f), 1.0f);
      const float b = fminf(fmaxf(rr[c], 0.0f), 1.0f);
      const double d = (double)a - (double)b;
      acc += d * d;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mse_final(double* part, int n, double inv_count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  part[n] = s * inv_count;
}

// RGB of an RGBA frame.
__global__ void __launch_bounds__(256) k_rgba_to_rgb(const float4* __restrict__ src,
                                                     float* __restrict__ dst, size_t npx) {
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npx) return;
  const float4 v = src[p];
  dst[p * 3 + 0] = v.x;
  dst[p * 3 + 1] = v.y;
  dst[p * 3 + 2] = v.z;
}

void release(fv_renderer* r) {
  if (!r) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(r->device);
  (void)hipDeviceSynchronize();  // frames in flight may still use the buffers
  void* ptrs[] = {r->ray_idx, r->count,   r->mask,    r->sparse,   r->depth,
                  r->dense,   r->partial, r->ws_mask, r->ws_march, r->ws_recon};
  for (void* p : ptrs) (void)hipFree(p);
  (void)hipSetDevice(cur);
  delete r;
}

fv_status mse_of(const float* rgb, const float* rgba, size_t npx, double* part, double* out,
                 hipStream_t s) {
  k_mse_partial<<<kMseBlocks, 256, 0, s>>>(rgb, (const float4*)rgba, npx, part);
  fv_status st = launch_status("fv_render_frame: mse");
  if (st != FV_OK) return st;
  k_mse_final<<<1, 64, 0, s>>>(part, kMseBlocks, 1.0 / (3.0 * (double)npx));
  if ((st = launch_status("fv_render_frame: mse")) != FV_OK) return st;
  st = hip_status(hipMemcpyAsync(out, part + kMseBlocks, sizeof(double), hipMemcpyDeviceToHost, s),
                  "fv_render_frame: read mse");
  if (st == FV_OK) st = hip_status(hipStreamSynchronize(s), "fv_render_frame: sync");
  return st;
}

}  // namespace
}  // namespace fv

extern "C" {

fv_status fv_renderer_create(int views, int width, int height, const fv_render_policy* policy,
                             fv_renderer** out) {
  fv::clear_error();
  if (!policy || !out) return fv::fail(FV_ERR_INVALID_ARG, "fv_renderer_create: null pointer");
  *out = nullptr;
  if (views <= 0 || views > 8 || width < 8 || height < 8 || width % 8 || height % 8 ||
      width > 16384 || height > 16384 || (uint64_t)views * width * height >= (1ull << 32))
    return fv::fail(FV_ERR_INVALID_ARG,
                    "fv_renderer_create: frame %d x %d x %d (1..8 views, W and H multiples of 8 "
                    "in [8, 16384])", views, width, height);
  if (policy->precision != FV_PREC_BF16 && policy->precision != FV_PREC_FP8 &&
      policy->precision != FV_RECON_PULLPUSH)
    return fv::fail(FV_ERR_UNSUPPORTED, "fv_renderer_create: precision %d", policy->precision);
  if (policy->check_every < 0 || !std::isfinite(policy->min_psnr_db))
    return fv::fail(FV_ERR_INVALID_ARG, "fv_renderer_create: check_every < 0 or bad threshold");
  fv_renderer* r = new fv_renderer();
  memset(r, 0, sizeof(*r));
  r->views = views;
  r->W = width;
  r->H = height;
  r->pol = *policy;
  if (hipGetDevice(&r->device) != hipSuccess) {
    delete r;
    return fv::fail(FV_ERR_DEVICE, "fv_renderer_create: hipGetDevice");
  }
  const size_t npx = (size_t)views * width * height;
  fv_status st = fv_fovea_mask_workspace(width, height, views, &r->n_mask);
  if (st == FV_OK) st = fv_raymarch_sparse_workspace((uint32_t)npx, &r->n_march);
  if (st == FV_OK) {
    // a network's workspace is allocated by the first frame (its size
    // depends on the handle)
    r->n_recon = policy->precision == FV_RECON_PULLPUSH
                     ? fv::pullpush_workspace_bytes(views, width, height)
                     : 0;
  }
  if (st != FV_OK) {
    delete r;
    return st;
  }
  bool ok = hipMalloc(&r->ray_idx, npx * 4) == hipSuccess &&
            hipMalloc(&r->count, 256) == hipSuccess && hipMalloc(&r->mask, npx) == hipSuccess &&
            hipMalloc(&r->sparse, npx * 16) == hipSuccess &&
            hipMalloc(&r->depth, npx * 4) == hipSuccess &&
            hipMalloc(&r->dense, npx * 16) == hipSuccess &&
            hipMalloc(&r->partial, (fv::kMseBlocks + 1) * sizeof(double)) == hipSuccess &&
            hipMalloc(&r->ws_mask, r->n_mask) == hipSuccess &&
            hipMalloc(&r->ws_march, r->n_march) == hipSuccess;
  if (!ok) {
    fv::release(r);
    return fv::fail(FV_ERR_NOMEM, "fv_renderer_create: allocation failed");
  }
  *out = r;
  return FV_OK;
}

fv_status fv_renderer_destroy(fv_renderer* r) {
  fv::release(r);
  return FV_OK;
}

fv_status fv_render_frame(fv_renderer* r, const fv_volume* vol, const float* tf_rgba, int tf_n,
                          const fv_camera* cams, const fv_march_params* mp,
                          const fv_fovea_params* fp, const fv_net* net, float* out_rgb,
                          fv_frame_info* info, void* stream) {
  fv::clear_error();
  if (!r || !vol || !tf_rgba || !cams || !mp || !fp || !out_rgb || !info)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_render_frame: null pointer");
  if (r->pol.precision != FV_RECON_PULLPUSH && !net)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_render_frame: the policy's precision needs a network");
  hipStream_t s = (hipStream_t)stream;
  const int V = r->views, W = r->W, H = r->H;
  const size_t npx = (size_t)V * W * H;
  const bool check = r->pol.check_every > 0 && r->frame % (uint64_t)r->pol.check_every == 0;
  info->dense = 0;
  info->checked = check ? 1 : 0;
  info->psnr_db = NAN;
  info->frame = r->frame;
  fv_status st = FV_OK;
  // the network workspace is sized on first use (it depends on the handle)
  if (r->pol.precision != FV_RECON_PULLPUSH) {
    size_t need = 0;
    st = fv_reconstruct_workspace(net, r->pol.precision, V, W, H, &need);
    if (st != FV_OK) return st;
    if (need > r->n_recon) {
      if (r->ws_recon) {
        (void)hipDeviceSynchronize();  // earlier frames may still read it
        (void)hipFree(r->ws_recon);
        r->ws_recon = nullptr;
      }
      if (hipMalloc(&r->ws_recon, need) != hipSuccess)
        return fv::fail(FV_ERR_NOMEM, "fv_render_frame: workspace allocation failed");
      r->n_recon = need;
    }
  } else if (!r->ws_recon) {
    if (hipMalloc(&r->ws_recon, r->n_recon) != hipSuccess)
      return fv::fail(FV_ERR_NOMEM, "fv_render_frame: workspace allocation failed");
  }
  const bool foveated = check || !r->fallback;
  if (foveated) {
    st = fv_fovea_mask(fp, W, H, V, r->mask, r->ray_idx, (uint32_t)npx, r->count, r->ws_mask,
                       r->n_mask, stream);
    if (st == FV_OK)
      st = fv_raymarch_sparse(vol, tf_rgba, tf_n, cams, V, W, H, mp, r->ray_idx, r->count,
                              (uint32_t)npx, nullptr, nullptr, r->sparse, r->depth, nullptr,
                              r->ws_march, r->n_march, stream);
    if (st == FV_OK)
      st = fv_reconstruct(net, r->pol.precision, r->sparse, r->mask,
                          r->pol.precision == FV_RECON_PULLPUSH ? nullptr : r->depth, V, W, H,
                          out_rgb, nullptr, r->ws_recon, r->n_recon, stream);
    if (st != FV_OK) return st;
  }
  if (check || r->fallback) {
    st = fv_raymarch_dense(vol, tf_rgba, tf_n, cams, V, W, H, mp, r->dense, nullptr, nullptr,
                           stream);
    if (st != FV_OK) return st;
  }
  if (check) {
    double mse = 0.0;
    st = fv::mse_of(out_rgb, r->dense, npx, r->partial, &mse, s);
    if (st != FV_OK) return st;
    const double psnr = mse > 0.0 ? 10.0 * std::log10(1.0 / mse) : INFINITY;
    info->psnr_db = (float)psnr;
    r->fallback = !(psnr >= (double)r->pol.min_psnr_db);
  }
  if (r->fallback) {
    fv::k_rgba_to_rgb<<<(unsigned)((npx + 255) / 256), 256, 0, s>>>((const float4*)r->dense,
                                                                    out_rgb, npx);
    if ((st = fv::launch_status("fv_render_frame: dense output")) != FV_OK) return st;
    info->dense = 1;
  }
  info->fallback = r->fallback;
  ++r->frame;
  return FV_OK;
}

}  // extern "C"
