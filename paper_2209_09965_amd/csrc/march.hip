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

// The kernels' DT template argument: the voxel dtype (fv_dtype), plus
// kBricked for a volume in the bricked layout.
constexpr int kBricked = 4;
template <int DT>
using Vx = Voxel<DT & 3>;

struct CamD {
  double o[3], f[3], r[3], u[3];
  double sx, sy;  // tan(fovy/2) * W/H, tan(fovy/2)
};

struct MarchArgs {
  const void* vol;
  uint32_t vol_bytes;  // size of the padded copy (< 2^32)
  int64_t px, py;  // row / slice pitch in elements (of the bricks when brick)
  int nb[2];        // bricks along x and y (bricked layout)
  int n[3];
  double h;        // voxel edge in world units
  double half[3];  // box half extents
  const float4* tf;
  int W, H, views;
  uint32_t total;  // views * W * H
  double step;
  float alpha_stop;
  float light[3];  // normalised, towards the light
  double lightd[3];  // the same in FP64 (shadow-ray positions)
  double shadow_step;  // shadow-ray segment length in voxels (0: no shadows)
  int lanes;           // lanes per ray of the sparse march (0: chosen per launch)
  float ka, kd, ks, shininess;
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

// x^p for x in [0, 1], p >= 0: exp2(p log2 x) with the hardware log/exp
// (relative error a few 1e-6 at p = 32); x = 0 gives 0 (p > 0) and p = 0
// gives 1.
__device__ __forceinline__ float pow01(float x, float p) {
  return p > 0.0f ? __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x)) : 1.0f;
}

template <typename VT>
__device__ __forceinline__ VT buffer_voxel(__amdgpu_buffer_rsrc_t rs, int voff, int soff);
template <>
__device__ __forceinline__ float buffer_voxel<float>(__amdgpu_buffer_rsrc_t rs, int voff,
                                                     int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
template <>
__device__ __forceinline__ _Float16 buffer_voxel<_Float16>(__amdgpu_buffer_rsrc_t rs, int voff,
                                                           int soff) {
  return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0));
}
template <>
__device__ __forceinline__ uint8_t buffer_voxel<uint8_t>(__amdgpu_buffer_rsrc_t rs, int voff,
                                                         int soff) {
  return __builtin_amdgcn_raw_buffer_load_b8(rs, voff, soff, 0);
}

struct RayOut {
  float4 rgba;
  float depth;
  uint32_t samples;
};

// Per-ray marching state.  Full segments k sample at m_k = (k + 1/2) step
// voxel lengths from the entry, so the sample position in voxel index space
// is q_k = q0 + k qs with q0 = qe + d step/2 and qs = d step (FP64); only the
// last segment may be shorter (length last_len): its midpoint is
// q0 + klast qs with klast = N - 3/2 + last_len / (2 step).
struct RayState {
  double q0[3], qs[3];
  double klast;
  float t0, tstep, tlast;  // world-space distance of full / last samples
  float last_len;
  float hv[3];
  int N, k;
  float C0, C1, C2, T, D;
};

// Ray set-up: camera ray through the pixel centre, slab test, segment count.
// Returns false on a miss.
template <bool SHADE>
__device__ __forceinline__ bool ray_setup(const MarchArgs& a, int view, int x, int y,
                                          RayState& s) {
  const CamD& c = a.cam[view];
  const double pxn = (2.0 * ((double)x + 0.5) / a.W - 1.0) * c.sx;
  const double pyn = (1.0 - 2.0 * ((double)y + 0.5) / a.H) * c.sy;
  double d[3];
  for (int i = 0; i < 3; ++i) d[i] = c.f[i] + pxn * c.r[i] + pyn * c.u[i];
  const double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) d[i] /= dl;
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
  if (miss || !(tf > tn)) return false;
  const double L = (tf - tn) / a.h;
  s.N = (int)ceil(L / a.step);
  const double mh = 0.5 * a.step;
  const double la = (double)(s.N - 1) * a.step;  // start of the last segment
  const double lm = 0.5 * (la + L);                // its midpoint
  for (int i = 0; i < 3; ++i) {
    const double qe = (c.o[i] + d[i] * tn + a.half[i]) / a.h - 0.5;
    s.q0[i] = qe + d[i] * mh;
    s.qs[i] = d[i] * a.step;
  }
  s.klast = (double)s.N - 1.5 + (L - la) / (2.0 * a.step);
  s.t0 = (float)(tn + a.h * mh);
  s.tstep = (float)(a.h * a.step);
  s.tlast = (float)(tn + a.h * lm);
  s.last_len = (float)(L - la);
  if (SHADE) {
    double hd[3];
    for (int i = 0; i < 3; ++i) hd[i] = (double)a.light[i] - d[i];
    double hl = sqrt(hd[0] * hd[0] + hd[1] * hd[1] + hd[2] * hd[2]);
    hl = fmax(hl, 1e-30);
    for (int i = 0; i < 3; ++i) s.hv[i] = (float)(hd[i] / hl);
  }
  s.k = 0;
  s.C0 = s.C1 = s.C2 = 0.f;
  s.T = 1.0f;
  s.D = 0.0f;
  return true;
}

// Element offset of the stencil's first voxel, (i - 1, j - 1, k - 1) for the
// cell (i, j, k) with each index in [-1, n - 1]; the other stencil voxels
// follow at the uniform row / slice pitches a.px, a.px a.py.  Bricked
// layout: cell index c = i + 1 lies in brick c / 16, whose stored voxel
// (c mod 16) along that axis is voxel i - 1.
template <int DT>
__device__ __forceinline__ uint32_t stencil_base(const MarchArgs& a, const int ii[3]) {
  const uint32_t c0 = (uint32_t)(ii[0] + 1), c1 = (uint32_t)(ii[1] + 1),
                 c2 = (uint32_t)(ii[2] + 1);
  if constexpr ((DT & kBricked) != 0) {
    const uint32_t b = ((c2 / kBrick) * (uint32_t)a.nb[1] + c1 / kBrick) * (uint32_t)a.nb[0] +
                       c0 / kBrick;
    return b * (uint32_t)kBrickVox +
           ((c2 % kBrick) * kBrickRow + c1 % kBrick) * kBrickRow + c0 % kBrick;
  }
  return c2 * (uint32_t)(a.px * a.py) + c1 * (uint32_t)a.px + c0;
}

// The voxels one sample reads, as stored (converted to float when used):
// the 8 corners of its cell and, when shading, the 24 more voxels of the
// one-voxel central differences (the 4 x 2 x 2, 2 x 4 x 2 and 2 x 2 x 4 arms).
// Stencil voxel (x, y, z) is at offset (x - 1, y - 1, z - 1) from the cell's
// minimum corner.
template <int DT, bool SHADE>
struct Stencil {
  typename Vx<DT>::T c[8];            // centre cell, index x + 2 y + 4 z
  typename Vx<DT>::T g[SHADE ? 24 : 1];  // arms: x-, x+, y-, y+, z-, z+ (4 each)
  float w[3];                            // trilinear weights
};

// Issues the voxel loads of sample k of the ray (k = N - 1 is the last,
// possibly shorter, segment).  Nothing here waits for the loads, so the
// caller can composite the previous sample while they are in flight.  A lane
// with live == false issues its loads at an offset past the end of the
// buffer: the hardware range check returns zeros without touching memory,
// which lets a wave run the pipelined loop without branching around idle
// lanes.
template <int DT, bool SHADE>
__device__ __forceinline__ void gather(const MarchArgs& a, const RayState& s, int k,
                                       Stencil<DT, SHADE>& st, bool live = true) {
  using VT = typename Vx<DT>::T;
  const double kk = k == s.N - 1 ? s.klast : (double)k;
  int ii[3];
  for (int i = 0; i < 3; ++i) {
    const double q = fma(kk, s.qs[i], s.q0[i]);
    const double fq = floor(q);
    st.w[i] = (float)(q - fq);
    ii[i] = min(max((int)fq, -1), a.n[i] - 1);
  }
  // Voxel gathers as buffer loads: the VGPR offset addresses the stencil's
  // minimum corner (i0-1, j0-1, k0-1); the (y, z) row offsets are uniform
  // (SGPR) and x is the immediate, so a gather costs no vector ALU work.
  // Reads outside the buffer return 0 (hardware range check).
  constexpr int EB = (int)sizeof(VT);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.vol, (short)0, (int)a.vol_bytes, 0x00020000);
  const int sy = (int)a.px * EB, sz = (int)(a.px * a.py) * EB;
  const uint32_t oi = stencil_base<DT>(a, ii) * EB;
  const int o = (int)(live ? oi : a.vol_bytes);
#define FV_V(x, y, z) buffer_voxel<VT>(rs, o + (x) * EB, (y) * sy + (z) * sz)
  for (int z = 0; z < 2; ++z)
    for (int y = 0; y < 2; ++y)
      for (int x = 0; x < 2; ++x) st.c[x + 2 * y + 4 * z] = FV_V(1 + x, 1 + y, 1 + z);
  if (SHADE) {
    for (int j = 0; j < 4; ++j) {
      const int u = 1 + (j & 1), v = 1 + (j >> 1);
      st.g[0 + j] = FV_V(0, u, v);    // x - 1
      st.g[4 + j] = FV_V(3, u, v);    // x + 2
      st.g[8 + j] = FV_V(u, 0, v);    // y - 1
      st.g[12 + j] = FV_V(u, 3, v);   // y + 2
      st.g[16 + j] = FV_V(u, v, 0);   // z - 1
      st.g[20 + j] = FV_V(u, v, 3);   // z + 2
    }
  }
#undef FV_V
}

// dst = c ? src : dst, element by element.
template <int DT, bool SHADE>
__device__ __forceinline__ void select_stencil(bool c, const Stencil<DT, SHADE>& src,
                                               Stencil<DT, SHADE>& dst) {
  for (int i = 0; i < 8; ++i) dst.c[i] = c ? src.c[i] : dst.c[i];
  if (SHADE)
    for (int i = 0; i < 24; ++i) dst.g[i] = c ? src.g[i] : dst.g[i];
  for (int i = 0; i < 3; ++i) dst.w[i] = c ? src.w[i] : dst.w[i];
}

// Voxel index space position of segment k (the last one may be shorter).
__device__ __forceinline__ double seg_pos(const RayState& s, int k, int i) {
  const double kk = k == s.N - 1 ? s.klast : (double)k;
  return fma(kk, s.qs[i], s.q0[i]);
}

constexpr int kMaxShadowSegs = 1 << 20;  // a bound on every shadow loop
constexpr int kShadowBufs = 2;           // shadow segments in flight per lane

// Global ray-marched shadow: transmittance from the sample at voxel-index
// position q towards the (directional) light.  The shadow ray runs to where
// it leaves the box [-1/2, n - 1/2]^3, in segments of shadow_step voxel
// lengths sampled at their midpoints (the last one shorter), and the light is
// attenuated by exp(-sum sigma_j len_j).  Positions are FP64 and split into a
// cell and FP32 weights like the primary samples; the two-buffer loop issues
// the loads of segment j + 1 before segment j is blended.
template <int DT>
__device__ __forceinline__ float shadow_transmittance(const MarchArgs& a,
                                                      const float4* __restrict__ tfs,
                                                      const double q[3]) {
  using VT = typename Vx<DT>::T;
  double L = INFINITY;
  for (int i = 0; i < 3; ++i) {
    const double l = a.lightd[i];
    if (l == 0.0) continue;
    const double face = l > 0.0 ? (double)a.n[i] - 0.5 : -0.5;
    L = fmin(L, (face - q[i]) / l);
  }
  if (!(L > 0.0)) return 1.0f;
  const double ds = a.shadow_step;
  const int ns = (int)fmin(ceil(L / ds), (double)kMaxShadowSegs);
  constexpr int EB = (int)sizeof(VT);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.vol, (short)0, (int)a.vol_bytes, 0x00020000);
  const int sy = (int)a.px * EB, sz = (int)(a.px * a.py) * EB;
  struct Cell {
    VT c[8];
    float w[3];
    float len;
  };
  auto load = [&](int j, Cell& cl) {
    const double a0 = (double)j * ds, b0 = fmin((double)(j + 1) * ds, L);
    const double m = 0.5 * (a0 + b0);
    cl.len = (float)(b0 - a0);
    int ii[3];
    for (int i = 0; i < 3; ++i) {
      const double p = fma(m, a.lightd[i], q[i]);
      const double fp = floor(p);
      cl.w[i] = (float)(p - fp);
      ii[i] = min(max((int)fp, -1), a.n[i] - 1);
    }
    const int o = (int)(stencil_base<DT>(a, ii) * EB);
    for (int z = 0; z < 2; ++z)
      for (int y = 0; y < 2; ++y)
        for (int x = 0; x < 2; ++x)
          cl.c[x + 2 * y + 4 * z] =
              buffer_voxel<VT>(rs, o + (1 + x) * EB, (1 + y) * sy + (1 + z) * sz);
  };
  auto sigma = [&](const Cell& cl) {
#define FV_C(x, y, z) Vx<DT>::f(cl.c[(x) + 2 * (y) + 4 * (z)])
    const float v = tri(FV_C(0, 0, 0), FV_C(1, 0, 0), FV_C(0, 1, 0), FV_C(1, 1, 0),
                        FV_C(0, 0, 1), FV_C(1, 0, 1), FV_C(0, 1, 1), FV_C(1, 1, 1), cl.w[0],
                        cl.w[1], cl.w[2]);
#undef FV_C
    const float xv = fminf(fmaxf(v, 0.0f), 1.0f) * 255.0f;
    const int j = min((int)xv, 254);
    return lerpf(tfs[j].w, tfs[j + 1].w, xv - (float)j);
  };
  // kShadowBufs cells in flight: at the top of each pass C[u] holds segment
  // j + u (indices past the last segment are clamped to it, loaded and never
  // blended)
  constexpr int NS = kShadowBufs;
  float tau = 0.0f;
  Cell C[NS];
#pragma unroll
  for (int u = 0; u < NS - 1; ++u) load(min(u, ns - 1), C[u]);
  int j = 0;
  bool more = true;
  while (more) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      if (!more) break;
      load(min(j + NS - 1, ns - 1), C[(u + NS - 1) % NS]);
      tau = fmaf(sigma(C[u]), C[u].len, tau);
      more = ++j < ns;
    }
  }
  return __expf(-tau);
}

// The shaded result of one segment: colour, transmittance exp(-sigma l) and
// the world-space distance of its sample point.
struct Segment {
  float r, g, b, tr, t;
};

// One segment k from its gathered voxels: trilinear sample (plus the
// central-difference gradient and Blinn-Phong when shading, with the light
// attenuated by the shadow ray's transmittance when SHADOW) and TF lookup.
template <int DT, bool SHADE, bool SHADOW = false>
__device__ __forceinline__ Segment shade(const MarchArgs& a, const float4* __restrict__ tfs,
                                         const RayState& s, int k,
                                         const Stencil<DT, SHADE>& st) {
  const bool last = k == s.N - 1;
  float len, t;
  if (last) {
    len = s.last_len;
    t = s.tlast;
  } else {
    len = (float)a.step;
    t = fmaf((float)k, s.tstep, s.t0);
  }
  const float wx = st.w[0], wy = st.w[1], wz = st.w[2];
#define FV_C(x, y, z) Vx<DT>::f(st.c[(x) + 2 * (y) + 4 * (z)])
  const float v000 = FV_C(0, 0, 0), v100 = FV_C(1, 0, 0);
  const float v010 = FV_C(0, 1, 0), v110 = FV_C(1, 1, 0);
  const float v001 = FV_C(0, 0, 1), v101 = FV_C(1, 0, 1);
  const float v011 = FV_C(0, 1, 1), v111 = FV_C(1, 1, 1);
#undef FV_C
  const float v = tri(v000, v100, v010, v110, v001, v101, v011, v111, wx, wy, wz);
  // transfer function: linear interpolation between the 256 entries
  const float xv = fminf(fmaxf(v, 0.0f), 1.0f) * 255.0f;
  const int j = min((int)xv, 254);
  const float fr = xv - (float)j;
  const float4 e0 = tfs[j], e1 = tfs[j + 1];
  float r = lerpf(e0.x, e1.x, fr), g = lerpf(e0.y, e1.y, fr), bl = lerpf(e0.z, e1.z, fr);
  const float sig = lerpf(e0.w, e1.w, fr);
  // segment transmittance exp(-sigma l) (hardware exp)
  const float tr = __expf(-sig * len);
  if (SHADE) {
    // one-voxel central differences of the interpolated field; arm entry j
    // holds the voxel at (u, v) = (j & 1, j >> 1) across the arm's axis
#define FV_G(i) Vx<DT>::f(st.g[i])
    const float xm00 = FV_G(0), xm10 = FV_G(1), xm01 = FV_G(2), xm11 = FV_G(3);
    const float xp00 = FV_G(4), xp10 = FV_G(5), xp01 = FV_G(6), xp11 = FV_G(7);
    const float ym00 = FV_G(8), ym10 = FV_G(9), ym01 = FV_G(10), ym11 = FV_G(11);
    const float yp00 = FV_G(12), yp10 = FV_G(13), yp01 = FV_G(14), yp11 = FV_G(15);
    const float zm00 = FV_G(16), zm10 = FV_G(17), zm01 = FV_G(18), zm11 = FV_G(19);
    const float zp00 = FV_G(20), zp10 = FV_G(21), zp01 = FV_G(22), zp11 = FV_G(23);
#undef FV_G
    // x arms: (u, v) = (y, z); y arms: (x, z); z arms: (x, y)
    const float gx = 0.5f * tri(v100 - xm00, xp00 - v000, v110 - xm10, xp10 - v010, v101 - xm01,
                                xp01 - v001, v111 - xm11, xp11 - v011, wx, wy, wz);
    const float gy = 0.5f * tri(v010 - ym00, v110 - ym10, yp00 - v000, yp10 - v100, v011 - ym01,
                                v111 - ym11, yp01 - v001, yp11 - v101, wx, wy, wz);
    const float gz = 0.5f * tri(v001 - zm00, v101 - zm10, v011 - zm01, v111 - zm11, zp00 - v000,
                                zp10 - v100, zp01 - v010, zp11 - v110, wx, wy, wz);
    const float inv = rsqrtf(fmaxf(gx * gx + gy * gy + gz * gz, 1e-8f));
    const float nx = -gx * inv, ny = -gy * inv, nz = -gz * inv;
    const float ndl = fabsf(nx * a.light[0] + ny * a.light[1] + nz * a.light[2]);
    const float ndh = fabsf(nx * s.hv[0] + ny * s.hv[1] + nz * s.hv[2]);
    float spec = a.ks * pow01(ndh, a.shininess);
    float diff;
    if constexpr (SHADOW) {
      // the light reaching the sample (diffuse and specular) is attenuated
      const double q[3] = {seg_pos(s, k, 0), seg_pos(s, k, 1), seg_pos(s, k, 2)};
      const float ts = shadow_transmittance<DT>(a, tfs, q);
      diff = a.ka + ts * (a.kd * ndl);
      spec = ts * spec;
    } else {
      diff = a.ka + a.kd * ndl;
    }
    r = r * diff + spec;
    g = g * diff + spec;
    bl = bl * diff + spec;
  }
  return Segment{r, g, bl, tr, t};
}

// Front-to-back compositing of the ray's next segment (opacity 1 - tr).
// Advances k; returns true when the ray is finished (last segment or early
// termination).
__device__ __forceinline__ bool accumulate(const MarchArgs& a, RayState& s, const Segment& o) {
  const bool last = s.k == s.N - 1;
  const float alpha = 1.0f - o.tr;
  const float wgt = s.T * alpha;
  s.C0 = fmaf(wgt, o.r, s.C0);
  s.C1 = fmaf(wgt, o.g, s.C1);
  s.C2 = fmaf(wgt, o.b, s.C2);
  s.D = fmaf(wgt, o.t, s.D);
  s.T *= o.tr;
  ++s.k;
  return last || 1.0f - s.T >= a.alpha_stop;
}

template <int DT, bool SHADE, bool SHADOW>
__device__ __forceinline__ bool composite(const MarchArgs& a, const float4* __restrict__ tfs,
                                          RayState& s, const Stencil<DT, SHADE>& st) {
  return accumulate(a, s, shade<DT, SHADE, SHADOW>(a, tfs, s, s.k, st));
}

__device__ __forceinline__ RayOut ray_finish(const MarchArgs& a, const RayState& s) {
  RayOut o;
  o.rgba = make_float4(fmaf(s.T, a.bg[0], s.C0), fmaf(s.T, a.bg[1], s.C1),
                       fmaf(s.T, a.bg[2], s.C2), 1.0f - s.T);
  o.depth = s.D;
  o.samples = (uint32_t)s.k;
  return o;
}

__device__ __forceinline__ RayOut ray_miss(const MarchArgs& a) {
  RayOut o;
  o.rgba = make_float4(a.bg[0], a.bg[1], a.bg[2], 0.0f);
  o.depth = 0.0f;
  o.samples = 0;
  return o;
}

// The march loop is software-pipelined: the gathers of sample k + 1 are
// issued before sample k is composited (two stencil buffers, A and B), so the
// memory latency of one sample overlaps the arithmetic of the previous one.
// The sample after the last is never read: its index is clamped to N - 1.
template <int DT, bool SHADE, bool SHADOW>
__device__ __forceinline__ RayOut march_ray(const MarchArgs& a, const float4* __restrict__ tfs,
                                            int view, int x, int y) {
  RayState s;
  if (!ray_setup<SHADE>(a, view, x, y, s)) return ray_miss(a);
  if (s.N > 0) {
    Stencil<DT, SHADE> A, B;
    gather(a, s, 0, A);
    while (true) {
      gather(a, s, min(s.k + 1, s.N - 1), B);
      if (composite<DT, SHADE, SHADOW>(a, tfs, s, A)) break;
      gather(a, s, min(s.k + 1, s.N - 1), A);
      if (composite<DT, SHADE, SHADOW>(a, tfs, s, B)) break;
    }
  }
  return ray_finish(a, s);
}

__device__ __forceinline__ void add_samples(unsigned long long* nsamp, uint32_t ns) {
  unsigned long long s = ns;
  for (int off = 32; off; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(nsamp, s);
}

// Dense: a 256-thread block covers a 16x16 pixel block as four 8x8 wave tiles.
// With a sample map (naive rejection), a thread whose pixel is not sampled
// returns at once; the others march as in the dense frame.
template <int DT, bool SHADE, bool SHADOW>
__global__ void __launch_bounds__(256) k_march_dense(MarchArgs a, const uint8_t* __restrict__ mask,
                                                     float4* __restrict__ rgba,
                                                     float* __restrict__ depth,
                                                     unsigned long long* __restrict__ nsamp) {
  __shared__ float4 tfs[FV_TF_ENTRIES];
  tfs[threadIdx.x] = a.tf[threadIdx.x];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  const int y = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
  const int view = blockIdx.z;
  const uint32_t lin = (uint32_t)view * (uint32_t)a.W * (uint32_t)a.H + (uint32_t)y * a.W + x;
  uint32_t ns = 0;
  if (x < a.W && y < a.H && (!mask || mask[lin])) {
    const RayOut r = march_ray<DT, SHADE, SHADOW>(a, tfs, view, x, y);
    rgba[lin] = r.rgba;
    if (depth) depth[lin] = r.depth;
    ns = r.samples;
  }
  if (nsamp) add_samples(nsamp, ns);
}

// Ray set-up of the compacted list, done once per listed ray by a kernel of
// its own, so the march kernel's claim step only loads the state (the FP64
// set-up and its temporaries stay out of the march loop's registers).  One
// record per list slot, structure of arrays in the sparse workspace.
struct SetupList {
  double* q[7];  // q0 x y z, qs x y z, klast
  float* f[7];   // t0, tstep, tlast, last_len, half vector x y z
  int* n;        // segments N >= 1, 0 for a miss, -1 for an invalid list entry
};

constexpr int kSetupDoubles = 7, kSetupFloats = 7;

__host__ __device__ inline size_t setup_stride(uint32_t capacity, size_t elem) {
  return ((size_t)capacity * elem + 255) & ~(size_t)255;
}

// Workspace header: the claim counter (word 0) and kHitCounters counters of
// the rays that reach the volume, one per 128-byte line (word 32 j), so the
// set-up pass's atomics spread over many lines.
constexpr int kHitCounters = 31;
constexpr size_t kWsHeader = 4096;

inline size_t sparse_workspace_bytes(uint32_t capacity) {
  return kWsHeader + kSetupDoubles * setup_stride(capacity, 8) +
         (kSetupFloats + 1) * setup_stride(capacity, 4);
}

inline SetupList setup_list(void* ws, uint32_t capacity) {
  SetupList l;
  char* p = (char*)ws + kWsHeader;
  for (int i = 0; i < kSetupDoubles; ++i, p += setup_stride(capacity, 8)) l.q[i] = (double*)p;
  for (int i = 0; i < kSetupFloats; ++i, p += setup_stride(capacity, 4)) l.f[i] = (float*)p;
  l.n = (int*)p;
  return l;
}

template <bool SHADE>
__global__ void __launch_bounds__(256) k_setup_list(MarchArgs a,
                                                    const uint32_t* __restrict__ ray_idx,
                                                    const uint32_t* __restrict__ count,
                                                    uint32_t capacity, SetupList l,
                                                    uint32_t* __restrict__ queue) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const bool listed = i < min(*count, capacity);
  const uint32_t lin = listed ? ray_idx[i] : 0u;
  bool hit = false;
  RayState s;
  if (listed && lin < a.total) {
    const uint32_t wh = (uint32_t)a.W * (uint32_t)a.H;
    const int view = (int)(lin / wh);
    const uint32_t rem = lin - (uint32_t)view * wh;
    const int y = (int)(rem / (uint32_t)a.W), x = (int)(rem - (uint32_t)y * a.W);
    // a zero-length ray inside the box finishes with the same output as a miss
    hit = ray_setup<SHADE>(a, view, x, y, s) && s.N > 0;
  }
  // rays that reach the volume: one atomic per wave, on one of the header's
  // counters (cleared before this kernel)
  const uint64_t hm = __ballot(hit);
  if (hm && (threadIdx.x & 63) == __ffsll((long long)hm) - 1) {
    const uint32_t wv = (blockIdx.x * 256u + threadIdx.x) >> 6;
    atomicAdd(queue + 32 * (1 + wv % kHitCounters), (uint32_t)__popcll(hm));
  }
  if (!listed) return;
  if (!hit) {
    l.n[i] = lin < a.total ? 0 : -1;
    return;
  }
  for (int j = 0; j < 3; ++j) {
    l.q[j][i] = s.q0[j];
    l.q[3 + j][i] = s.qs[j];
  }
  l.q[6][i] = s.klast;
  l.f[0][i] = s.t0;
  l.f[1][i] = s.tstep;
  l.f[2][i] = s.tlast;
  l.f[3][i] = s.last_len;
  for (int j = 0; j < 3; ++j) l.f[4 + j][i] = SHADE ? s.hv[j] : 0.0f;
  l.n[i] = s.N;
}

// Sparse, persistent: every wave claims rays from a global queue (one atomic
// per claim) in list order.  A wave claims once all its lanes are idle
// (their rays finished or missed the box), checked every kStepsPerRefill
// segments: one claim takes consecutive list entries, so a wave's lanes step
// through neighbouring pixels in lock step and fetch neighbouring voxels.
// (Refilling lanes as soon as half a wave was idle, or one by one, was
// slower: lanes at different depths share no cache lines.)  Results go to
// the compact buffers and/or back to their pixels (back-projection).
// The loop is software-pipelined kSparseAhead steps ahead: each lane keeps
// the voxels of its next kSparseAhead samples in flight.
//
// When the list holds few rays for the lanes resident on the device, one ray
// would otherwise take one lane for its whole length, and the frame would
// last as long as its longest ray.  Then G = 2, 4 or 8 consecutive lanes
// march one ray together: lane r of the group shades segments k + r, and
// every lane of the group composites the group's G segments in ray order,
// with the same operations as the single-lane march, so the pixel is the
// same bit for bit and the group's lanes keep identical ray state.
constexpr int kStepsPerRefill = 9;
constexpr int kSparseAhead = 2;
// With shadows each segment runs its own shadow loop, whose length depends
// on where the sample is: one primary sample ahead and a register budget for
// two waves per SIMD (the shadowed full list took 30.7 ms with one wave and
// two samples ahead, 21.5 ms with this), and the idle check every 4
// segments (with whole-wave claims the lanes' shadow loops stay about
// equally long: 21.5 -> 10.5 ms, the dense march's time for the same rays).
constexpr int kSparseAheadShadow = 1;
constexpr int kStepsPerRefillShadow = 4;
// G is the largest of 1, 2, 4, 8 with h G^2 <= kGroupRule, h = (rays that
// reach the volume) / (resident lanes).  Measured on the 1080p noise volume:
// the best G was 1 at h = 11 (2 within 3 %), 2 at h = 2.2 to 2.5, 4 at
// h = 0.55 and 8 at h = 0.11 (a larger G shortens each ray's critical path
// and costs the exchange and the repeated compositing).
constexpr int kGroupRule = 16;
// With shadows the lanes of a group also march neighbouring shadow rays (one
// per segment of the same primary ray), which share cache lines: grouping pays
// at higher densities.  Forced-G probe with shadows (fovea map / full list /
// p = 0.05, ms): G = 1: 16.1 / 10.4 / 15.6; G = 4: 3.46 / 9.38 / 2.35; this
// rule (G = 4 / 2 / 8): 3.45 / 8.68 / 1.21.
constexpr int kGroupRuleShadow = 64;

// Value of v held by lane Q of this lane's group of G (G a power of two).
template <int G, int Q>
__device__ __forceinline__ float group_get(float v) {
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 2 || G == 4) {
    // quad permutation: lane i of each quad reads lane p_i of the quad
    constexpr int p0 = G == 2 ? Q : Q, p2 = G == 2 ? 2 + Q : Q;
    constexpr int ctrl = p0 | (p0 << 2) | (p2 << 4) | (p2 << 6);
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), ctrl, 0xF, 0xF, true));
  } else {
    const int lane = threadIdx.x & 63;
    return __shfl(v, (lane & ~(G - 1)) | Q, 64);
  }
}

template <int G, int Q = 0>
__device__ __forceinline__ bool group_accumulate(const MarchArgs& a, RayState& s,
                                                 const Segment& o, bool fin) {
  if constexpr (Q == G) {
    return fin;
  } else {
    const Segment q{group_get<G, Q>(o.r), group_get<G, Q>(o.g), group_get<G, Q>(o.b),
                    group_get<G, Q>(o.tr), group_get<G, Q>(o.t)};
    if (!fin) fin = accumulate(a, s, q);
    return group_accumulate<G, Q + 1>(a, s, o, fin);
  }
}

template <int DT, bool SHADE, bool SHADOW, int G>
__device__ __forceinline__ void march_list(const MarchArgs& a, const float4* __restrict__ tfs,
                                           const uint32_t* __restrict__ ray_idx, uint32_t n,
                                           const SetupList& l, float4* __restrict__ rgba_c,
                                           float* __restrict__ depth_c,
                                           float4* __restrict__ rgba_f,
                                           float* __restrict__ depth_f, uint32_t& ns,
                                           uint32_t* __restrict__ queue) {
  constexpr int NB = (SHADOW ? kSparseAheadShadow : kSparseAhead) + 1;
  constexpr int kSteps = SHADOW ? kStepsPerRefillShadow : kStepsPerRefill;
  static_assert(kSteps % NB == 0, "steps per refill round: a multiple of the buffers");
  const int lane = threadIdx.x & 63, r = lane & (G - 1);
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  // Idle lanes run the loop body too, so their state and buffers start
  // defined (zero) rather than uninitialised.  Every lane of a group holds
  // the same ray state.
  RayState s{};
  s.N = 1;
  Stencil<DT, SHADE> S[NB]{};
  bool active = false, exhausted = false, done = false;
  uint32_t slot = 0, lin = 0;
  RayOut fin{};  // a ray finished in this round, stored at the round's end
  auto store = [&](const RayOut& o) {
    if (rgba_c) rgba_c[slot] = o.rgba;
    if (depth_c) depth_c[slot] = o.depth;
    if (rgba_f) rgba_f[lin] = o.rgba;
    if (depth_f) depth_f[lin] = o.depth;
  };
  while (true) {
    const bool want = !active && !exhausted;
    const uint64_t m = __ballot(want);  // G bits per idle group
    bool fresh = false;  // claimed a ray this round that needs marching
    if (m && !__ballot(active)) {
      const int leader = __ffsll((long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(queue, (uint32_t)__popcll(m) / G);
      base = __shfl(base, leader, 64);
      if (want) {
        slot = base + (uint32_t)__popcll(m & lt) / G;
        if (slot >= n) {
          exhausted = true;
        } else {
          const int N = l.n[slot];
          if (N >= 0) lin = ray_idx[slot];
          if (N > 0) {
            for (int j = 0; j < 3; ++j) {
              s.q0[j] = l.q[j][slot];
              s.qs[j] = l.q[3 + j][slot];
            }
            s.klast = l.q[6][slot];
            s.t0 = l.f[0][slot];
            s.tstep = l.f[1][slot];
            s.tlast = l.f[2][slot];
            s.last_len = l.f[3][slot];
            for (int j = 0; j < 3; ++j) s.hv[j] = l.f[4 + j][slot];
            s.N = N;
            s.k = 0;
            s.C0 = s.C1 = s.C2 = 0.f;
            s.T = 1.0f;
            s.D = 0.0f;
            active = fresh = true;
          } else if (N == 0 && r == 0) {
            store(ray_miss(a));
          }
        }
      }
    }
    // first gathers of the new rays, outside the divergent claim code (so the
    // stencil registers are not copied around it)
    if (__ballot(fresh)) {
      Stencil<DT, SHADE> F[NB - 1];
#pragma unroll
      for (int j = 0; j < NB - 1; ++j) gather(a, s, min(r + G * j, s.N - 1), F[j], fresh);
#pragma unroll
      for (int j = 0; j < NB - 1; ++j) select_stencil(fresh, F[j], S[j]);
    }
    if (!__ballot(active)) {
      if (!__ballot(!exhausted)) break;
      continue;
    }
    // Every lane runs the loop body (idle lanes gather nothing and their
    // state is discarded); only active lanes take a finished ray's result,
    // which is written once the round is over (stores inside the loop would
    // hold their addresses in registers across it).  At the top of each
    // group of NB steps, S[j] holds the voxels of segment k + r + G j.
    // Segments past the last one are clamped to it: they are shaded but
    // never composited.
#pragma unroll 1
    for (int it = 0; it < kSteps; it += NB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        gather(a, s, min(s.k + r + G * (NB - 1), s.N - 1), S[(j + NB - 1) % NB], active);
        const Segment o =
            shade<DT, SHADE, SHADOW>(a, tfs, s, G == 1 ? s.k : min(s.k + r, s.N - 1), S[j]);
        if (group_accumulate<G>(a, s, o, false) && active) {
          fin = ray_finish(a, s);
          done = true;
          active = false;
        }
      }
    }
    if (done) {
      if (r == 0) {
        store(fin);
        ns += fin.samples;
      }
      done = false;
    }
  }
}

template <int DT, bool SHADE, bool SHADOW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SHADOW ? 2 : 1)))
k_march_sparse(
    MarchArgs a, const uint32_t* __restrict__ ray_idx, const uint32_t* __restrict__ count,
    uint32_t capacity, SetupList l, float4* __restrict__ rgba_c, float* __restrict__ depth_c,
    float4* __restrict__ rgba_f, float* __restrict__ depth_f,
    unsigned long long* __restrict__ nsamp, uint32_t* __restrict__ queue) {
  __shared__ float4 tfs[FV_TF_ENTRIES];
  tfs[threadIdx.x] = a.tf[threadIdx.x];
  __syncthreads();
  const uint32_t n = min(*count, capacity);
  // lanes per ray, from the rays that reach the volume (counted by the set-up
  // pass) and the lanes of the persistent grid (the same for every wave)
  const int lane = threadIdx.x & 63;
  uint32_t hc = lane < kHitCounters ? queue[32 * (1 + lane)] : 0u;
  for (int off = 32; off; off >>= 1) hc += __shfl_xor(hc, off, 64);
  const uint64_t hits = hc, lanes = (uint64_t)gridDim.x * 256u;
  int g = a.lanes;
  if (g == 0) {
    g = 1;
    while (g < 8 &&
           hits * (uint64_t)(4 * g * g) <= lanes * (SHADOW ? kGroupRuleShadow : kGroupRule))
      g *= 2;
  }
  uint32_t ns = 0;
  switch (g) {
    case 8:
      march_list<DT, SHADE, SHADOW, 8>(a, tfs, ray_idx, n, l, rgba_c, depth_c, rgba_f, depth_f, ns, queue);
      break;
    case 4:
      march_list<DT, SHADE, SHADOW, 4>(a, tfs, ray_idx, n, l, rgba_c, depth_c, rgba_f, depth_f, ns, queue);
      break;
    case 2:
      march_list<DT, SHADE, SHADOW, 2>(a, tfs, ray_idx, n, l, rgba_c, depth_c, rgba_f, depth_f, ns, queue);
      break;
    default:
      march_list<DT, SHADE, SHADOW, 1>(a, tfs, ray_idx, n, l, rgba_c, depth_c, rgba_f, depth_f, ns, queue);
  }
  if (nsamp) add_samples(nsamp, ns);
}

// Clears the workspace header's counters.
__global__ void k_clear_queue(uint32_t* q) {
  if (threadIdx.x <= kHitCounters) q[32 * threadIdx.x] = 0u;
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
  a->vol_bytes = (uint32_t)v->bytes;
  a->nb[0] = v->nb[0];
  a->nb[1] = v->nb[1];
  a->px = v->brick ? kBrickRow : v->px;
  a->py = v->brick ? kBrickRow : v->py;
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
  for (int i = 0; i < 3; ++i) a->lightd[i] = ll > 0.0 ? L[i] / ll : 0.0;
  if (!(mp->shadow_step == 0.0f || (mp->shadow_step >= 1.0f / 64.0f && mp->shadow_step <= 64.0f)))
    return fail(FV_ERR_INVALID_ARG, "%s: shadow_step must be 0 or in [1/64, 64]", fn);
  a->shadow_step = mp->shading ? (double)mp->shadow_step : 0.0;
  if (!(mp->lanes_per_ray == 0 || mp->lanes_per_ray == 1 || mp->lanes_per_ray == 2 ||
        mp->lanes_per_ray == 4 || mp->lanes_per_ray == 8))
    return fail(FV_ERR_INVALID_ARG, "%s: lanes_per_ray must be 0, 1, 2, 4 or 8", fn);
  a->lanes = mp->lanes_per_ray;
  a->ka = mp->ka;
  a->kd = mp->kd;
  a->ks = mp->ks;
  a->shininess = mp->shininess;
  if (mp->shading && !(mp->shininess >= 0.0f && mp->shininess <= 1024.0f))
    return fail(FV_ERR_INVALID_ARG, "%s: shininess must be in [0, 1024]", fn);
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

template <int DT, bool SHADE, bool SHADOW>
void launch_dense(const MarchArgs& a, const uint8_t* mask, float* rgba, float* depth,
                  uint64_t* ns, hipStream_t s) {
  dim3 grid((a.W + 15) / 16, (a.H + 15) / 16, a.views);
  k_march_dense<DT, SHADE, SHADOW><<<grid, 256, 0, s>>>(a, mask, (float4*)rgba, depth,
                                                (unsigned long long*)ns);
}

fv_status dense_entry(const char* who, const fv_volume* v, const float* tf_rgba, int tf_n,
                      const fv_camera* cams, int views, int width, int height,
                      const fv_march_params* mp, const uint8_t* mask, bool need_mask,
                      float* frame_rgba, float* frame_depth, uint64_t* sample_count,
                      void* stream) {
  clear_error();
  MarchArgs a;
  fv_status st = fill_args(v, tf_rgba, tf_n, cams, views, width, height, mp, &a, who);
  if (st != FV_OK) return st;
  if (!frame_rgba) return fail(FV_ERR_INVALID_ARG, "%s: null frame_rgba", who);
  if (need_mask && !mask) return fail(FV_ERR_INVALID_ARG, "%s: null mask", who);
  hipStream_t s = (hipStream_t)stream;
  // 0: emission-absorption, 1: Blinn-Phong, 2: Blinn-Phong with shadows
  const int mode = mp->shading == 0 ? 0 : (a.shadow_step > 0.0 ? 2 : 1);
#define FV_DENSE(DT)                                                                         \
  (mode == 0   ? launch_dense<DT, false, false>(a, mask, frame_rgba, frame_depth, sample_count, s) \
   : mode == 1 ? launch_dense<DT, true, false>(a, mask, frame_rgba, frame_depth, sample_count, s)  \
               : launch_dense<DT, true, true>(a, mask, frame_rgba, frame_depth, sample_count, s))
  switch (v->dt + (v->brick ? kBricked : 0)) {
    case FV_U8:
      FV_DENSE(FV_U8);
      break;
    case FV_F16:
      FV_DENSE(FV_F16);
      break;
    case FV_F32:
      FV_DENSE(FV_F32);
      break;
    case FV_U8 + kBricked:
      FV_DENSE(FV_U8 + kBricked);
      break;
    case FV_F16 + kBricked:
      FV_DENSE(FV_F16 + kBricked);
      break;
    default:
      FV_DENSE(FV_F32 + kBricked);
  }
#undef FV_DENSE
  return launch_status(who);
}

template <int DT, bool SHADE, bool SHADOW>
void launch_sparse(const MarchArgs& a, const uint32_t* idx, const uint32_t* count,
                   uint32_t capacity, float* rc, float* dc, float* rf, float* df, uint64_t* ns,
                   void* ws, hipStream_t s) {
  uint32_t* queue = (uint32_t*)ws;
  const SetupList l = setup_list(ws, capacity);
  // persistent grid: as many blocks as can be resident at once
  static int per_cu = 0, cus = 0;
  if (!per_cu) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_march_sparse<DT, SHADE, SHADOW>, 256,
                                                     0) != hipSuccess || per_cu < 1)
      per_cu = 4;
    if (cus < 1) cus = 256;
  }
  const uint64_t need = ((uint64_t)capacity + 255) / 256;
  uint64_t grid = (uint64_t)per_cu * cus;
  if (grid > need) grid = need;
  k_clear_queue<<<1, 64, 0, s>>>(queue);
  k_setup_list<SHADE><<<(unsigned)need, 256, 0, s>>>(a, idx, count, capacity, l, queue);
  k_march_sparse<DT, SHADE, SHADOW><<<(unsigned)grid, 256, 0, s>>>(a, idx, count, capacity, l,
                                                           (float4*)rc, dc, (float4*)rf, df,
                                                           (unsigned long long*)ns, queue);
}

}  // namespace
}  // namespace fv

extern "C" {

fv_status fv_raymarch_dense(const fv_volume* v, const float* tf_rgba, int tf_n,
                            const fv_camera* cams, int views, int width, int height,
                            const fv_march_params* mp, float* frame_rgba, float* frame_depth,
                            uint64_t* sample_count, void* stream) {
  return fv::dense_entry("fv_raymarch_dense", v, tf_rgba, tf_n, cams, views, width, height, mp,
                         nullptr, false, frame_rgba, frame_depth, sample_count, stream);
}

fv_status fv_raymarch_masked(const fv_volume* v, const float* tf_rgba, int tf_n,
                             const fv_camera* cams, int views, int width, int height,
                             const fv_march_params* mp, const uint8_t* mask, float* frame_rgba,
                             float* frame_depth, uint64_t* sample_count, void* stream) {
  return fv::dense_entry("fv_raymarch_masked", v, tf_rgba, tf_n, cams, views, width, height, mp,
                         mask, true, frame_rgba, frame_depth, sample_count, stream);
}

fv_status fv_raymarch_sparse_workspace(uint32_t capacity, size_t* bytes) {
  fv::clear_error();
  if (!bytes) return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse_workspace: null bytes");
  if (capacity == 0)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse_workspace: capacity 0");
  *bytes = fv::sparse_workspace_bytes(capacity);
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
  if (capacity == 0 || capacity > a.total)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: capacity %u not in [1, %u]", capacity,
                    a.total);
  if (ws_bytes < fv::sparse_workspace_bytes(capacity))
    return fv::fail(FV_ERR_CAPACITY, "fv_raymarch_sparse: workspace %zu < %zu bytes", ws_bytes,
                    fv::sparse_workspace_bytes(capacity));
  if (((uintptr_t)workspace & 255) != 0)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: workspace not 256-byte aligned");
  if (!rgba_compact && !depth_compact && !frame_rgba && !frame_depth)
    return fv::fail(FV_ERR_INVALID_ARG, "fv_raymarch_sparse: no output given");
  hipStream_t s = (hipStream_t)stream;
  // 0: emission-absorption, 1: Blinn-Phong, 2: Blinn-Phong with shadows
  const int mode = mp->shading == 0 ? 0 : (a.shadow_step > 0.0 ? 2 : 1);
#define FV_SPARSE_M(DT, SH, SW)                                                         \
  fv::launch_sparse<DT, SH, SW>(a, ray_idx, count, capacity, rgba_compact, depth_compact, \
                                frame_rgba, frame_depth, sample_count, workspace, s)
#define FV_SPARSE(DT)                                                                     \
  (mode == 0 ? FV_SPARSE_M(DT, false, false)                                            \
             : mode == 1 ? FV_SPARSE_M(DT, true, false) : FV_SPARSE_M(DT, true, true))
  switch (v->dt + (v->brick ? fv::kBricked : 0)) {
    case FV_U8:
      FV_SPARSE(FV_U8);
      break;
    case FV_F16:
      FV_SPARSE(FV_F16);
      break;
    case FV_F32:
      FV_SPARSE(FV_F32);
      break;
    case FV_U8 + fv::kBricked:
      FV_SPARSE(FV_U8 + fv::kBricked);
      break;
    case FV_F16 + fv::kBricked:
      FV_SPARSE(FV_F16 + fv::kBricked);
      break;
    default:
      FV_SPARSE(FV_F32 + fv::kBricked);
  }
#undef FV_SPARSE
#undef FV_SPARSE_M
  return fv::launch_status("fv_raymarch_sparse");
}

}  // extern "C"
