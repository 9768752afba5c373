// Reconstruction without a network: pull-push hole filling on an image
// pyramid (Gortler et al., "The Lumigraph", SIGGRAPH 1996, Sec. 3.3), the
// baseline that shows what the paper's learned reconstruction (Sec. 3.2)
// gains, and the cheap full-frame fill of a sparse frame.
//
// Level l+1 has ceil(H_l/2) x ceil(W_l/2) pixels, down to 1 x 1.  Pull:
// t = min(w, 1) per child, w' = sum t, c' = sum t c / w'.  Push: f_l =
// t c_l + (1 - t) bilinear(f_{l+1}) at the half-pixel centre, clamped.
// Level 0 is read from the back-projected frame and the sample map.
//
// Launches (all on the caller's stream, no host synchronisation):
//   k_pull   one thread per coarse pixel, levels 0 -> 1 -> ... -> lt
//   k_tail   one workgroup per view: the pyramid from level lt (at most
//            kTailPx pixels from there to the top) pulled and pushed in LDS
//   k_push   one thread per fine pixel, levels lt -> ... -> 1 -> 0; level 0
//            writes the RGB output
// Each pulled level is a float4 (c.rgb, w) per pixel in the workspace; the
// push overwrites c.rgb with the finished f (each thread its own pixel).
#include <vector>

#include "common.h"

namespace fv {
namespace {

constexpr int kMaxLevels = 40;
constexpr int kTailPx = 2048;  // pixels of the LDS tail (32 KiB of float4)

struct Level {
  int h, w;
  size_t off;  // float4 offset of this level in the workspace (level >= 1)
};

struct Pyramid {
  int n = 0;       // levels, level 0 = the frame
  int lt = 0;      // first level handled by the LDS tail
  Level lv[kMaxLevels];
  size_t bytes = 0;  // workspace bytes
};

Pyramid make_pyramid(int views, int H, int W) {
  Pyramid p;
  int h = H, w = W;
  size_t off = 0;
  while (true) {
    Level& L = p.lv[p.n++];
    L.h = h;
    L.w = w;
    L.off = off;
    if (p.n > 1) off += ((size_t)views * h * w + 15) / 16 * 16;
    if (h == 1 && w == 1) break;
    h = (h + 1) / 2;
    w = (w + 1) / 2;
  }
  // tail: the first level from which the rest of the pyramid fits in LDS
  size_t rest = 0;
  p.lt = p.n;
  for (int l = p.n - 1; l >= 0; --l) {
    rest += (size_t)p.lv[l].h * p.lv[l].w;
    if (rest > (size_t)kTailPx) break;
    p.lt = l;
  }
  p.bytes = (off * 16 + 255) / 256 * 256;
  if (p.bytes == 0) p.bytes = 256;
  return p;
}

struct PPArgs {
  const float4* frame;
  const uint8_t* mask;
  float4* ws;
  float* out;
  int views;
};

// Pulled value of child (y, x) of level l (level 0 straight from the frame).
__device__ __forceinline__ float4 child(const PPArgs& a, const Level& L, int l, int view, int y,
                                        int x) {
  const size_t i = ((size_t)view * L.h + y) * L.w + x;
  if (l == 0) {
    // an unsampled pixel's frame entry is never read (it may hold anything)
    if (!a.mask[i]) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const float4 c = a.frame[i];
    return make_float4(c.x, c.y, c.z, 1.0f);
  }
  return a.ws[L.off + i];
}

// Sum of the clamped children of coarse pixel (y, x); returns (c, w').
__device__ __forceinline__ float4 pull_sum(float4 q[4], int nq) {
  float sw = 0.0f, sr = 0.0f, sg = 0.0f, sb = 0.0f;
  for (int k = 0; k < nq; ++k) {
    const float t = fminf(q[k].w, 1.0f);
    sw += t;
    sr = fmaf(t, q[k].x, sr);
    sg = fmaf(t, q[k].y, sg);
    sb = fmaf(t, q[k].z, sb);
  }
  if (sw > 0.0f) return make_float4(sr / sw, sg / sw, sb / sw, sw);
  return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

__global__ void __launch_bounds__(256) k_pull(PPArgs a, Level F, Level C, int lf) {
  const size_t n = (size_t)a.views * C.h * C.w;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % C.w);
  const size_t r = i / C.w;
  const int y = (int)(r % C.h), view = (int)(r / C.h);
  float4 q[4];
  int nq = 0;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int fy = 2 * y + dy, fx = 2 * x + dx;
      if (fy < F.h && fx < F.w) q[nq++] = child(a, F, lf, view, fy, fx);
    }
  a.ws[C.off + i] = pull_sum(q, nq);
}

// Bilinear source along one axis: fine index i of a level of n_f pixels
// samples the coarser level (n_c pixels) at (i + 1/2)/2 - 1/2, clamped.
__device__ __forceinline__ void axis_src(int i, int n_c, int& i0, int& i1, float& f) {
  float s = ((float)i + 0.5f) * 0.5f - 0.5f;
  s = fminf(fmaxf(s, 0.0f), (float)(n_c - 1));
  i0 = (int)s;
  i1 = min(i0 + 1, n_c - 1);
  f = s - (float)i0;
}

__device__ __forceinline__ float3 blend_push(float4 own, float3 u) {
  const float t = fminf(own.w, 1.0f), o = 1.0f - t;
  return make_float3(fmaf(t, own.x, o * u.x), fmaf(t, own.y, o * u.y), fmaf(t, own.z, o * u.z));
}

__device__ __forceinline__ float3 lerp3(float3 a, float3 b, float f) {
  return make_float3(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y), fmaf(f, b.z - a.z, a.z));
}

// Push from level lf+1 (C, finished) into level lf (F): level 0 writes out.
__global__ void __launch_bounds__(256) k_push(PPArgs a, Level F, Level C, int lf) {
  const size_t n = (size_t)a.views * F.h * F.w;
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % F.w);
  const size_t r = i / F.w;
  const int y = (int)(r % F.h), view = (int)(r / F.h);
  int y0, y1, x0, x1;
  float fy, fx;
  axis_src(y, C.h, y0, y1, fy);
  axis_src(x, C.w, x0, x1, fx);
  const float4* cl = a.ws + C.off + (size_t)view * C.h * C.w;
  auto at = [&](int yy, int xx) {
    const float4 v = cl[(size_t)yy * C.w + xx];
    return make_float3(v.x, v.y, v.z);
  };
  const float3 u = lerp3(lerp3(at(y0, x0), at(y0, x1), fx), lerp3(at(y1, x0), at(y1, x1), fx), fy);
  const float4 own = child(a, F, lf, view, y, x);
  const float3 f = blend_push(own, u);
  if (lf == 0) {
    a.out[i * 3 + 0] = f.x;
    a.out[i * 3 + 1] = f.y;
    a.out[i * 3 + 2] = f.z;
  } else {
    a.ws[F.off + i] = make_float4(f.x, f.y, f.z, own.w);
  }
}

struct TailArgs {
  int lt, n;          // first tail level, number of levels
  Level lv[kMaxLevels];
  int loff[kMaxLevels];  // float4 offset of each tail level in LDS
};

// One workgroup per view: level lt (pulled already, or the frame when lt is
// 0) up to the top and back, in LDS.
__global__ void __launch_bounds__(256) k_tail(PPArgs a, TailArgs t) {
  __shared__ float4 s[kTailPx];
  const int view = blockIdx.x;
  {
    const Level& L = t.lv[t.lt];
    for (int i = threadIdx.x; i < L.h * L.w; i += 256)
      s[t.loff[t.lt] + i] = child(a, L, t.lt, view, i / L.w, i % L.w);
  }
  __syncthreads();
  for (int l = t.lt; l + 1 < t.n; ++l) {
    const Level &F = t.lv[l], &C = t.lv[l + 1];
    for (int i = threadIdx.x; i < C.h * C.w; i += 256) {
      const int y = i / C.w, x = i % C.w;
      float4 q[4];
      int nq = 0;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int fy = 2 * y + dy, fx = 2 * x + dx;
          if (fy < F.h && fx < F.w) q[nq++] = s[t.loff[l] + fy * F.w + fx];
        }
      s[t.loff[l + 1] + i] = pull_sum(q, nq);
    }
    __syncthreads();
  }
  for (int l = t.n - 2; l >= t.lt; --l) {
    const Level &F = t.lv[l], &C = t.lv[l + 1];
    for (int i = threadIdx.x; i < F.h * F.w; i += 256) {
      const int y = i / F.w, x = i % F.w;
      int y0, y1, x0, x1;
      float fy, fx;
      axis_src(y, C.h, y0, y1, fy);
      axis_src(x, C.w, x0, x1, fx);
      auto at = [&](int yy, int xx) {
        const float4 v = s[t.loff[l + 1] + yy * C.w + xx];
        return make_float3(v.x, v.y, v.z);
      };
      const float3 u =
          lerp3(lerp3(at(y0, x0), at(y0, x1), fx), lerp3(at(y1, x0), at(y1, x1), fx), fy);
      const float4 own = s[t.loff[l] + i];
      const float3 f = blend_push(own, u);
      s[t.loff[l] + i] = make_float4(f.x, f.y, f.z, own.w);
    }
    __syncthreads();
  }
  // the top level alone (a 1 x 1 frame) is its own result: f = c
  const Level& L = t.lv[t.lt];
  for (int i = threadIdx.x; i < L.h * L.w; i += 256) {
    const float4 v = s[t.loff[t.lt] + i];
    const size_t g = (size_t)view * L.h * L.w + i;
    if (t.lt == 0) {
      a.out[g * 3 + 0] = v.x;
      a.out[g * 3 + 1] = v.y;
      a.out[g * 3 + 2] = v.z;
    } else {
      a.ws[L.off + g] = v;
    }
  }
}

fv_status check(int views, int W, int H, const char* fn) {
  if (views <= 0 || W <= 0 || H <= 0 || W > 65535 || H > 65535)
    return fail(FV_ERR_INVALID_ARG, "%s: bad frame %d x %d x %d", fn, views, W, H);
  if ((uint64_t)views * W * H >= (1ull << 32))
    return fail(FV_ERR_INVALID_ARG, "%s: views*W*H must be < 2^32", fn);
  return FV_OK;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Shared with fv_reconstruct's FV_RECON_PULLPUSH mode.
size_t pullpush_workspace_bytes(int views, int W, int H) {
  return make_pyramid(views, H, W).bytes;
}

fv_status pullpush_run(const float* frame_rgba, const uint8_t* mask, int views, int W, int H,
                       float* out_rgb, void* workspace, size_t ws_bytes, hipStream_t s,
                       const char* fn) {
  fv_status st = check(views, W, H, fn);
  if (st != FV_OK) return st;
  if (!frame_rgba || !mask || !out_rgb || !workspace)
    return fail(FV_ERR_INVALID_ARG, "%s: null pointer", fn);
  const Pyramid p = make_pyramid(views, H, W);
  if (ws_bytes < p.bytes)
    return fail(FV_ERR_CAPACITY, "%s: workspace %zu < %zu bytes", fn, ws_bytes, p.bytes);
  if ((uintptr_t)workspace % 256)
    return fail(FV_ERR_INVALID_ARG, "%s: workspace not 256-byte aligned", fn);
  PPArgs a{(const float4*)frame_rgba, mask, (float4*)workspace, out_rgb, views};
  for (int l = 0; l < p.lt; ++l) {
    k_pull<<<blocks_for((size_t)views * p.lv[l + 1].h * p.lv[l + 1].w), 256, 0, s>>>(
        a, p.lv[l], p.lv[l + 1], l);
    if ((st = launch_status(fn)) != FV_OK) return st;
  }
  TailArgs t;
  t.lt = p.lt;
  t.n = p.n;
  int off = 0;
  for (int l = 0; l < p.n; ++l) {
    t.lv[l] = p.lv[l];
    t.loff[l] = l >= p.lt ? off : 0;
    if (l >= p.lt) off += p.lv[l].h * p.lv[l].w;
  }
  k_tail<<<views, 256, 0, s>>>(a, t);
  if ((st = launch_status(fn)) != FV_OK) return st;
  for (int l = p.lt - 1; l >= 0; --l) {
    k_push<<<blocks_for((size_t)views * p.lv[l].h * p.lv[l].w), 256, 0, s>>>(a, p.lv[l],
                                                                           p.lv[l + 1], l);
    if ((st = launch_status(fn)) != FV_OK) return st;
  }
  return FV_OK;
}

}  // namespace fv

extern "C" {

fv_status fv_pullpush_workspace(int views, int width, int height, size_t* bytes) {
  fv::clear_error();
  if (!bytes) return fv::fail(FV_ERR_INVALID_ARG, "fv_pullpush_workspace: null bytes");
  fv_status st = fv::check(views, width, height, "fv_pullpush_workspace");
  if (st != FV_OK) return st;
  *bytes = fv::pullpush_workspace_bytes(views, width, height);
  return FV_OK;
}

fv_status fv_reconstruct_pullpush(const float* frame_rgba, const uint8_t* mask, int views,
                                  int width, int height, float* out_rgb, void* workspace,
                                  size_t ws_bytes, void* stream) {
  fv::clear_error();
  return fv::pullpush_run(frame_rgba, mask, views, width, height, out_rgb, workspace, ws_bytes,
                          (hipStream_t)stream, "fv_reconstruct_pullpush");
}

}  // extern "C"
