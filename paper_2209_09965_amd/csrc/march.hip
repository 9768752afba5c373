// Direct volume ray marching, dense (every pixel) and sparse (the compacted
// pixel list of the sample map, with back-projection to the full frame).
// Paper: "Foveated Rendering" (the ray-marching renderer), "Rendering",
// "Stream Compaction" (render the packed list, project results back).
//
// One ray per lane, FP32 compositing.  Ray set-up and the per-sample voxel
// position are computed in FP64 and split into an integer voxel index and an
// FP32 fraction, so the sample position carries no FP32 drift along long
// rays; everything after the split (32 voxel fetches for a shaded sample,
// trilinear blends, TF lookup from LDS, Blinn-Phong, compositing) is FP32.
// The dense and the sparse kernel call the same march_ray(), so the two give
// bit-identical pixels.
#include "common.h"

namespace fv {
namespace {

constexpr int kMaxViews = 8;

struct CamD {
  double o[3], f[3], r[3], u[3];
  double sx, sy;  // tan(fovy/2) * W/H, tan(fovy/2)
};

struct MarchArgs {
  const void* vol;
  int64_t px, py;  // padded row / slice pitch in elements
  int n[3];
  double h;        // voxel edge in world units
  double half[3];  // box half extents
  const float4* tf;
  int W, H, views;
  uint32_t total;  // views * W * H
  double step;
  float alpha_stop;
  float light[3];  // normalised, towards the light
  float ka, kd, ks, shininess;
  int ipow;        // shininess as a small integer, or -1
  float bg[3];
  CamD cam[kMaxViews];
};

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ float tri(float v000, float v100, float v010, float v110, float v001,
                                     float v101, float v011, float v111, float wx, float wy,
                                     float wz) {
  const float c00 = lerpf(v000, v100, wx), c10 = lerpf(v010, v110, wx);
  const float c01 = lerpf(v001, v101, wx), c11 = lerpf(v011, v111, wx);
  return lerpf(lerpf(c00, c10, wy), lerpf(c01, c11, wy), wz);
}

__device__ __forceinline__ float pow_small(float x, int n, float p) {
  if (n < 0) return powf(x, p);
  float r = 1.0f;
  while (n) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

struct RayOut {
  float4 rgba;
  float depth;
  uint32_t samples;
};

template <int DT, bool SHADE>
__device__ __forceinline__ RayOut march_ray(const MarchArgs& a, const float4* __restrict__ tfs,
                                            int view, int x, int y) {
  using VT = typename Voxel<DT>::T;
  RayOut out;
  out.depth = 0.0f;
  out.samples = 0;
  const CamD& c = a.cam[view];
  const double pxn = (2.0 * ((double)x + 0.5) / a.W - 1.0) * c.sx;
  const double pyn = (1.0 - 2.0 * ((double)y + 0.5) / a.H) * c.sy;
  double d[3];
  for (int i = 0; i < 3; ++i) d[i] = c.f[i] + pxn * c.r[i] + pyn * c.u[i];
  const double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) d[i] /= dl;
  // slab test
  double tn = -INFINITY, tf = INFINITY;
  bool miss = false;
  for (int i = 0; i < 3; ++i) {
    if (d[i] == 0.0) {
      if (c.o[i] < -a.half[i] || c.o[i] > a.half[i]) miss = true;
      continue;
    }
    const double ta = (-a.half[i] - c.o[i]) / d[i], tb = (a.half[i] - c.o[i]) / d[i];
    tn = fmax(tn, fmin(ta, tb));
    tf = fmin(tf, fmax(ta, tb));
  }
  tn = fmax(tn, 0.0);
  if (miss || !(tf > tn)) {
    out.rgba = make_float4(a.bg[0], a.bg[1], a.bg[2], 0.0f);
    return out;
  }
  const double L = (tf - tn) / a.h;
  const int64_t N = (int64_t)ceil(L / a.step);
  double qe[3];
  for (int i = 0; i < 3; ++i) qe[i] = (c.o[i] + d[i] * tn + a.half[i]) / a.h - 0.5;
  float hv[3] = {0.f, 0.f, 0.f};
  if (SHADE) {
    double hd[3];
    for (int i = 0; i < 3; ++i) hd[i] = (double)a.light[i] - d[i];
    double hl = sqrt(hd[0] * hd[0] + hd[1] * hd[1] + hd[2] * hd[2]);
    hl = fmax(hl, 1e-30);
    for (int i = 0; i < 3; ++i) hv[i] = (float)(hd[i] / hl);
  }
  const VT* __restrict__ vol = (const VT*)a.vol;
  const int64_t sy = a.px, sz = a.px * a.py;
  float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.0f, D = 0.0f;
  uint32_t ns = 0;
  for (int64_t k = 0; k < N; ++k) {
    const double a0 = (double)k * a.step;
    const double b0 = fmin((double)(k + 1) * a.step, L);
    const double m = 0.5 * (a0 + b0);
    const float len = (float)(b0 - a0);
    const float t = (float)(tn + a.h * m);
    int ii[3];
    float w[3];
    for (int i = 0; i < 3; ++i) {
      const double q = qe[i] + d[i] * m;
      const double fq = floor(q);
      int iq = (int)fq;
      w[i] = (float)(q - fq);
      iq = min(max(iq, -1), a.n[i] - 1);
      ii[i] = iq;
    }
    const VT* b = vol + ((int64_t)(ii[2] + 2) * sz + (int64_t)(ii[1] + 2) * sy + (ii[0] + 2));
    const float v000 = Voxel<DT>::f(b[0]), v100 = Voxel<DT>::f(b[1]);
    const float v010 = Voxel<DT>::f(b[sy]), v110 = Voxel<DT>::f(b[sy + 1]);
    const float v001 = Voxel<DT>::f(b[sz]), v101 = Voxel<DT>::f(b[sz + 1]);
    const float v011 = Voxel<DT>::f(b[sz + sy]), v111 = Voxel<DT>::f(b[sz + sy + 1]);
    const float v = tri(v000, v100, v010, v110, v001, v101, v011, v111, w[0], w[1], w[2]);
    // transfer function: linear interpolation between the 256 entries
    const float xv = fminf(fmaxf(v, 0.0f), 1.0f) * 255.0f;
    const int j = min((int)xv, 254);
    const float fr = xv - (float)j;
    const float4 e0 = tfs[j], e1 = tfs[j + 1];
    float r = lerpf(e0.x, e1.x, fr), g = lerpf(e0.y, e1.y, fr), bl = lerpf(e0.z, e1.z, fr);
    const float sig = lerpf(e0.w, e1.w, fr);
    const float alpha = -expm1f(-sig * len);
    if (SHADE) {
      // one-voxel central differences of the interpolated field
      const float xm00 = Voxel<DT>::f(b[-1]), xm10 = Voxel<DT>::f(b[sy - 1]);
      const float xm01 = Voxel<DT>::f(b[sz - 1]), xm11 = Voxel<DT>::f(b[sz + sy - 1]);
      const float xp00 = Voxel<DT>::f(b[2]), xp10 = Voxel<DT>::f(b[sy + 2]);
      const float xp01 = Voxel<DT>::f(b[sz + 2]), xp11 = Voxel<DT>::f(b[sz + sy + 2]);
      const float ym00 = Voxel<DT>::f(b[-sy]), ym10 = Voxel<DT>::f(b[-sy + 1]);
      const float ym01 = Voxel<DT>::f(b[sz - sy]), ym11 = Voxel<DT>::f(b[sz - sy + 1]);
      const float yp00 = Voxel<DT>::f(b[2 * sy]), yp10 = Voxel<DT>::f(b[2 * sy + 1]);
      const float yp01 = Voxel<DT>::f(b[sz + 2 * sy]), yp11 = Voxel<DT>::f(b[sz + 2 * sy + 1]);
      const float zm00 = Voxel<DT>::f(b[-sz]), zm10 = Voxel<DT>::f(b[-sz + 1]);
      const float zm01 = Voxel<DT>::f(b[-sz + sy]), zm11 = Voxel<DT>::f(b[-sz + sy + 1]);
      const float zp00 = Voxel<DT>::f(b[2 * sz]), zp10 = Voxel<DT>::f(b[2 * sz + 1]);
      const float zp01 = Voxel<DT>::f(b[2 * sz + sy]), zp11 = Voxel<DT>::f(b[2 * sz + sy + 1]);
      const float gx = 0.5f * tri(v100 - xm00, xp00 - v000, v110 - xm10, xp10 - v010,
                                  v101 - xm01, xp01 - v001, v111 - xm11, xp11 - v011, w[0], w[1],
                                  w[2]);
      const float gy = 0.5f * tri(v010 - ym00, v110 - ym10, yp00 - v000, yp10 - v100,
                                  v011 - ym01, v111 - ym11, yp01 - v001, yp11 - v101, w[0], w[1],
                                  w[2]);
      const float gz = 0.5f * tri(v001 - zm00, v101 - zm10, v011 - zm01, v111 - zm11,
                                  zp00 - v000, zp10 - v100, zp01 - v010, zp11 - v110, w[0], w[1],
                                  w[2]);
      const float inv = rsqrtf(fmaxf(gx * gx + gy * gy + gz * gz, 1e-8f));
      const float nx = -gx * inv, ny = -gy * inv, nz = -gz * inv;
      const float ndl = fabsf(nx * a.light[0] + ny * a.light[1] + nz * a.light[2]);
      const float ndh = fabsf(nx * hv[0] + ny * hv[1] + nz * hv[2]);
      const float spec = a.ks * pow_small(ndh, a.ipow, a.shininess);
      const float diff = a.ka + a.kd * ndl;
      r = r * diff + spec;
      g = g * diff + spec;
      bl = bl * diff + spec;
    }
    const float wgt = T * alpha;
    C0 = fmaf(wgt, r, C0);
    C1 = fmaf(wgt, g, C1);
    C2 = fmaf(wgt, bl, C2);
    D = fmaf(wgt, t, D);
    T *= (1.0f - alpha);
    ++ns;
    if (1.0f - T >= a.alpha_stop) break;
  }
  out.rgba = make_float4(fmaf(T, a.bg[0], C0), fmaf(T, a.bg[1], C1), fmaf(T, a.bg[2], C2),
                         1.0f - T);
  out.depth = D;
  out.samples = ns;
  return out;
}

__device__ __forceinline__ void add_samples(unsigned long long* nsamp, uint32_t ns) {
  unsigned long long s = ns;
  for (int off = 32; off; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(nsamp, s);
}

// Dense: a 256-thread block covers a 16x16 pixel block as four 8x8 wave tiles.
template <int DT, bool SHADE>
__global__ void __launch_bounds__(256) k_march_dense(MarchArgs a, float4* __restrict__ rgba,
                                                     float* __restrict__ depth,
                                                     unsigned long long* __restrict__ nsamp) {
  __shared__ float4 tfs[FV_TF_ENTRIES];
  tfs[threadIdx.x] = a.tf[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
  const int view = blockIdx.z;
  uint32_t ns = 0;
  if (x < a.W && y < a.H) {
    const RayOut r = march_ray<DT, SHADE>(a, tfs, view, x, y);
    const uint32_t lin = (uint32_t)view * (uint32_t)a.W * (uint32_t)a.H + (uint32_t)y * a.W + x;
    rgba[lin] = r.rgba;
    if (depth) depth[lin] = r.depth;
    ns = r.samples;
  }
  if (nsamp) add_samples(nsamp, ns);
}

// Sparse: grid-stride over the compacted list; results go to the compact
// buffers and/or back to their pixels in the full frame.
template <int DT, bool SHADE>
__global__ void __launch_bounds__(256) k_march_sparse(
    MarchArgs a, const uint32_t* __restrict__ ray_idx, const uint32_t* __restrict__ count,
    uint32_t capacity, float4* __restrict__ rgba_c, float* __restrict__ depth_c,
    float4* __restrict__ rgba_f, float* __restrict__ depth_f,
    unsigned long long* __restrict__ nsamp) {
  __shared__ float4 tfs[FV_TF_ENTRIES];
  tfs[threadIdx.x] = a.tf[threadIdx.x];
  __syncthreads();
  const uint32_t n = min(*count, capacity);
  const uint32_t wh = (uint32_t)a.W * (uint32_t)a.H;
  uint32_t ns = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t lin = ray_idx[i];
    if (lin >= a.total) continue;
    const int view = (int)(lin / wh);
    const uint32_t rem = lin - (uint32_t)view * wh;
    const int y = (int)(rem / (uint32_t)a.W), x = (int)(rem - (uint32_t)y * a.W);
    const RayOut r = march_ray<DT, SHADE>(a, tfs, view, x, y);
    if (rgba_c) rgba_c[i] = r.rgba;
    if (depth_c) depth_c[i] = r.depth;
    if (rgba_f) rgba_f[lin] = r.rgba;
    if (depth_f) depth_f[lin] = r.depth;
    ns += r.samples;
  }
  if (nsamp) add_samples(nsamp, ns);
}

// ---------------------------------------------------------------- host side

fv_status fill_args(const fv_volume* v, const float* tf, int tf_n, const fv_camera* cams,
                    int views, int W, int H, const fv_march_params* mp, MarchArgs* a,
                    const char* fn) {
  if (!v || !tf || !cams || !mp) return fail(FV_ERR_INVALID_ARG, "%s: null argument", fn);
  if (W <= 0 || H <= 0 || views <= 0 || W > 65535 || H > 65535)
    return fail(FV_ERR_INVALID_ARG, "%s: bad frame %d x %d x %d", fn, views, W, H);
  if (views > kMaxViews)
    return fail(FV_ERR_INVALID_ARG, "%s: at most %d views per launch", fn, kMaxViews);
  if ((uint64_t)views * W * H >= (1ull << 32))
    return fail(FV_ERR_INVALID_ARG, "%s: views*W*H must be < 2^32", fn);
  if (tf_n != FV_TF_ENTRIES)
    return fail(FV_ERR_INVALID_ARG, "%s: tf_n must be %d", fn, FV_TF_ENTRIES);
  if (!(mp->step_vox >= 1.0f / 64.0f && mp->step_vox <= 64.0f))
    return fail(FV_ERR_INVALID_ARG, "%s: step_vox must be in [1/64, 64]", fn);
  if (!(mp->alpha_stop > 0.0f && mp->alpha_stop <= 1.0f))
    return fail(FV_ERR_INVALID_ARG, "%s: alpha_stop must be in (0, 1]", fn);
  if (mp->shading != 0 && mp->shading != 1)
    return fail(FV_ERR_UNSUPPORTED, "%s: shading must be 0 or 1", fn);
  a->vol = v->data;
  a->px = v->px;
  a->py = v->py;
  int nmax = 0;
  for (int i = 0; i < 3; ++i) {
    a->n[i] = v->n[i];
    nmax = v->n[i] > nmax ? v->n[i] : nmax;
  }
  a->h = 1.0 / nmax;
  for (int i = 0; i < 3; ++i) a->half[i] = v->n[i] * a->h / 2.0;
  a->tf = (const float4*)tf;
  a->W = W;
  a->H = H;
  a->views = views;
  a->total = (uint32_t)((uint64_t)views * W * H);
  a->step = mp->step_vox;
  a->alpha_stop = mp->alpha_stop;
  double L[3] = {mp->light_dir[0], mp->light_dir[1], mp->light_dir[2]};
  const double ll = std::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
  if (mp->shading && !(ll > 0.0 && std::isfinite(ll)))
    return fail(FV_ERR_INVALID_ARG, "%s: light_dir must be non-zero", fn);
  for (int i = 0; i < 3; ++i) a->light[i] = ll > 0.0 ? (float)(L[i] / ll) : 0.0f;
  a->ka = mp->ka;
  a->kd = mp->kd;
  a->ks = mp->ks;
  a->shininess = mp->shininess;
  const float sh = mp->shininess;
  a->ipow = (sh >= 0.0f && sh <= 256.0f && sh == std::floor(sh)) ? (int)sh : -1;
  for (int i = 0; i < 3; ++i) a->bg[i] = mp->bg[i];
  for (int k = 0; k < views; ++k) {
    const fv_camera& cm = cams[k];
    double e[3], t[3], up[3];
    for (int i = 0; i < 3; ++i) {
      e[i] = cm.eye[i];
      t[i] = cm.target[i];
      up[i] = cm.up[i];
      if (!std::isfinite(e[i]) || !std::isfinite(t[i]) || !std::isfinite(up[i]))
        return fail(FV_ERR_INVALID_ARG, "%s: camera %d not finite", fn, k);
    }
    if (!(cm.fovy_deg > 0.0f && cm.fovy_deg < 180.0f) || !std::isfinite(cm.eye_offset))
      return fail(FV_ERR_INVALID_ARG, "%s: camera %d fovy/eye_offset out of range", fn, k);
    CamD& c = a->cam[k];
    double fl = 0.0;
    for (int i = 0; i < 3; ++i) {
      c.f[i] = t[i] - e[i];
      fl += c.f[i] * c.f[i];
    }
    fl = std::sqrt(fl);
    if (!(fl > 0.0)) return fail(FV_ERR_INVALID_ARG, "%s: camera %d eye == target", fn, k);
    for (int i = 0; i < 3; ++i) c.f[i] /= fl;
    c.r[0] = c.f[1] * up[2] - c.f[2] * up[1];
    c.r[1] = c.f[2] * up[0] - c.f[0] * up[2];
    c.r[2] = c.f[0] * up[1] - c.f[1] * up[0];
    const double rl = std::sqrt(c.r[0] * c.r[0] + c.r[1] * c.r[1] + c.r[2] * c.r[2]);
    if (!(rl > 0.0)) return fail(FV_ERR_INVALID_ARG, "%s: camera %d up parallel to view", fn, k);
    for (int i = 0; i < 3; ++i) c.r[i] /= rl;
    c.u[0] = c.r[1] * c.f[2] - c.r[2] * c.f[1];
    c.u[1] = c.r[2] * c.f[0] - c.r[0] * c.f[2];
    c.u[2] = c.r[0] * c.f[1] - c.r[1] * c.f[0];
    const double th = std::tan((double)cm.fovy_deg * M_PI / 360.0);
    c.sx = th * ((double)W / H);
    c.sy = th;
    for (int i = 0; i < 3; ++i) c.o[i] = e[i] + (double)cm.eye_offset * c.r[i];
  }
  return FV_OK;
}

template <int DT, bool SHADE>
void launch_dense(const MarchArgs& a, float* rgba, float* depth, uint64_t* ns, hipStream_t s) {
  dim3 grid((a.W + 15) / 16, (a.H + 15) / 16, a.views);
  k_march_dense<DT, SHADE><<<grid, 256, 0, s>>>(a, (float4*)rgba, depth,
                                                (unsigned long long*)ns);
}

template <int DT, bool SHADE>
void launch_sparse(const MarchArgs& a, const uint32_t* idx, const uint32_t* count,
                   uint32_t capacity, float* rc, float* dc, float* rf, float* df, uint64_t* ns,
                   hipStream_t s) {
  const uint64_t blocks = ((uint64_t)capacity + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
  k_march_sparse<DT, SHADE><<<grid, 256, 0, s>>>(a, idx, count, capacity, (float4*)rc, dc,
                                                 (float4*)rf, df, (unsigned long long*)ns);
}

}  // namespace
}  // namespace fv

extern "C" {

fv_status fv_raymarch_dense(const fv_volume* v, const float* tf_rgba, int tf_n,
                            const fv_camera* cams, int views, int width, int height,
                            const fv_march_params* mp, float* frame_rgba, float* frame_depth,
                            uint64_t* sample_count, void* stream) {
  fv::clear_error();
  fv::MarchArgs a;
  fv_status st =
      fv::fill_args(v, tf_rgba, tf_n, cams, views, width, height, mp, &a, "fv_raymarch_dense");
  if (st != FV_OK) return st;
  if (!frame_rgba) return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_dense: null frame_rgba");
  hipStream_t s = (hipStream_t)stream;
  const bool sh = mp->shading != 0;
  switch (v->dt) {
    case FV_U8:
      sh ? fv::launch_dense<FV_U8, true>(a, frame_rgba, frame_depth, sample_count, s)
         : fv::launch_dense<FV_U8, false>(a, frame_rgba, frame_depth, sample_count, s);
      break;
    case FV_F16:
      sh ? fv::launch_dense<FV_F16, true>(a, frame_rgba, frame_depth, sample_count, s)
         : fv::launch_dense<FV_F16, false>(a, frame_rgba, frame_depth, sample_count, s);
      break;
    default:
      sh ? fv::launch_dense<FV_F32, true>(a, frame_rgba, frame_depth, sample_count, s)
         : fv::launch_dense<FV_F32, false>(a, frame_rgba, frame_depth, sample_count, s);
  }
  return fv::launch_status("fv_raymarch_dense");
}

fv_status fv_raymarch_sparse_workspace(size_t* bytes) {
  fv::clear_error();
  if (!bytes) return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse_workspace: null bytes");
  *bytes = 256;
  return FV_OK;
}

fv_status fv_raymarch_sparse(const fv_volume* v, const float* tf_rgba, int tf_n,
                             const fv_camera* cams, int views, int width, int height,
                             const fv_march_params* mp, const uint32_t* ray_idx,
                             const uint32_t* count, uint32_t capacity, float* rgba_compact,
                             float* depth_compact, float* frame_rgba, float* frame_depth,
                             uint64_t* sample_count, void* workspace, size_t ws_bytes,
                             void* stream) {
  fv::clear_error();
  fv::MarchArgs a;
  fv_status st =
      fv::fill_args(v, tf_rgba, tf_n, cams, views, width, height, mp, &a, "fv_raymarch_sparse");
  if (st != FV_OK) return st;
  if (!ray_idx || !count || !workspace)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: null ray_idx, count or workspace");
  if (ws_bytes < 256)
    return fv::fail(FV_ERR_CAPACITY, "fv_raymarch_sparse: workspace %zu < 256 bytes", ws_bytes);
  if (capacity == 0 || capacity > a.total)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: capacity %u not in [1, %u]", capacity,
                    a.total);
  if (!rgba_compact && !depth_compact && !frame_rgba && !frame_depth)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: no output given");
  hipStream_t s = (hipStream_t)stream;
  const bool sh = mp->shading != 0;
#define FV_SPARSE(DT)                                                                          \
  (sh ? fv::launch_sparse<DT, true>(a, ray_idx, count, capacity, rgba_compact, depth_compact, \
                                    frame_rgba, frame_depth, sample_count, s)                 \
      : fv::launch_sparse<DT, false>(a, ray_idx, count, capacity, rgba_compact,               \
                                     depth_compact, frame_rgba, frame_depth, sample_count, s))
  switch (v->dt) {
    case FV_U8:
      FV_SPARSE(FV_U8);
      break;
    case FV_F16:
      FV_SPARSE(FV_F16);
      break;
    default:
      FV_SPARSE(FV_F32);
  }
#undef FV_SPARSE
  return fv::launch_status("fv_raymarch_sparse");
}

}  // extern "C"
