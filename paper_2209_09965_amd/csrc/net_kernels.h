// Device-side building blocks of the reconstruction network: element traits
// for BF16 and FP8 (OCP E4M3) activations/weights and the implicit-GEMM 3x3
// convolution on MFMA.
#pragma once

#include <type_traits>

#include "net.h"

namespace fv {
namespace net {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

__device__ __forceinline__ float bf16_bits_to_f(uint32_t b16) { return __uint_as_float(b16 << 16); }

struct BF16 {
  static constexpr int kBytes = 2;
  static constexpr int kPad = 8;  // LDS pixel padding (elements): 16-byte skew
  typedef bf16x8_t Frag;
  static __device__ __forceinline__ Frag frag(const uint8_t* p) { return *(const Frag*)p; }
  static __device__ __forceinline__ Frag zero() {
    const uint4 z = make_uint4(0, 0, 0, 0);
    return __builtin_bit_cast(Frag, z);
  }
  static __device__ __forceinline__ f32x4_t mma(Frag a, Frag b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void copy8(uint8_t* dst, const uint8_t* src) {
    *(uint4*)dst = *(const uint4*)src;
  }
  static __device__ __forceinline__ void zero8(uint8_t* dst) { *(uint4*)dst = make_uint4(0, 0, 0, 0); }
  static __device__ __forceinline__ void load8(const uint8_t* p, float v[8]) {
    const uint4 u = *(const uint4*)p;
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = bf16_bits_to_f(w[i] & 0xffffu);
      v[2 * i + 1] = bf16_bits_to_f(w[i] >> 16);
    }
  }
  static __device__ __forceinline__ uint32_t enc_bits(float v) {
    const __bf16 h = (__bf16)v;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
  }
  static __device__ __forceinline__ void store8(uint8_t* p, const float v[8]) {
    uint4 u;
    u.x = enc_bits(v[0]) | (enc_bits(v[1]) << 16);
    u.y = enc_bits(v[2]) | (enc_bits(v[3]) << 16);
    u.z = enc_bits(v[4]) | (enc_bits(v[5]) << 16);
    u.w = enc_bits(v[6]) | (enc_bits(v[7]) << 16);
    *(uint4*)p = u;
  }
  static __device__ __forceinline__ void load32(const uint8_t* p, float v[32]) {
    for (int g = 0; g < 4; ++g) load8(p + g * 16, v + 8 * g);
  }
  static __device__ __forceinline__ void store1(uint8_t* p, float v) {
    *(uint16_t*)p = (uint16_t)enc_bits(v);
  }
};

struct FP8 {
  static constexpr int kBytes = 1;
  static constexpr int kPad = 16;  // 16-byte skew
  typedef long Frag;
  static __device__ __forceinline__ Frag frag(const uint8_t* p) { return *(const long*)p; }
  static __device__ __forceinline__ Frag zero() { return 0; }
  static __device__ __forceinline__ f32x4_t mma(Frag a, Frag b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void copy8(uint8_t* dst, const uint8_t* src) {
    *(uint2*)dst = *(const uint2*)src;
  }
  static __device__ __forceinline__ void zero8(uint8_t* dst) { *(uint2*)dst = make_uint2(0, 0); }
  static __device__ __forceinline__ float sat(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }
  static __device__ __forceinline__ uint8_t enc(float v) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(sat(v), 0.0f, 0, false) & 0xff);
  }
  static __device__ __forceinline__ void load8(const uint8_t* p, float v[8]) {
    const uint2 u = *(const uint2*)p;
    v[0] = __builtin_amdgcn_cvt_f32_fp8((int)u.x, 0);
    v[1] = __builtin_amdgcn_cvt_f32_fp8((int)u.x, 1);
    v[2] = __builtin_amdgcn_cvt_f32_fp8((int)u.x, 2);
    v[3] = __builtin_amdgcn_cvt_f32_fp8((int)u.x, 3);
    v[4] = __builtin_amdgcn_cvt_f32_fp8((int)u.y, 0);
    v[5] = __builtin_amdgcn_cvt_f32_fp8((int)u.y, 1);
    v[6] = __builtin_amdgcn_cvt_f32_fp8((int)u.y, 2);
    v[7] = __builtin_amdgcn_cvt_f32_fp8((int)u.y, 3);
  }
  static __device__ __forceinline__ void store8(uint8_t* p, const float v[8]) {
    int lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[0]), sat(v[1]), lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[2]), sat(v[3]), lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[4]), sat(v[5]), hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[6]), sat(v[7]), hi, true);
    *(uint2*)p = make_uint2((uint32_t)lo, (uint32_t)hi);
  }
  static __device__ __forceinline__ void load32(const uint8_t* p, float v[32]) {
    for (int g = 0; g < 4; ++g) load8(p + g * 8, v + 8 * g);
  }
  static __device__ __forceinline__ void store1(uint8_t* p, float v) { *p = enc(v); }
};

__device__ __forceinline__ void wave_absmax(float* dst, float m) {
  for (int off = 32; off; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax((unsigned int*)dst, __float_as_uint(m));
}

// One 3x3 convolution as an implicit GEMM: M = output pixels, N = output
// channels, K = 9 taps x input channels.
struct ConvArgs {
  const uint8_t* src0;  // NHWC, c0 channels; half resolution if up0
  const uint8_t* src1;  // NHWC, c1 channels (concatenated after src0), or null
  int c0, c1, cip;      // cip = c0 + c1 rounded up to 8
  int up0;
  int n, h, w;          // output size
  const uint8_t* wsw;   // swizzled B fragments [kc][nb][64 lanes][8]
  int kc;
  const float* alpha;   // per-output-channel multiplier, or null (= 1)
  const float* bias;    // per-output-channel bias, or null
  int co, relu;
  uint8_t* out;         // NHWC, out_ch channel stride
  int out_ch, out_fp32;
  float* absmax;        // per-tensor running maximum (calibration), or null
};

// Low-resolution staging for an upsampled source 0: the tile's output rows
// [y0-1, y0+4R] and columns [x0-1, x0+16] read low-resolution rows
// [y0/2-1, y0/2+2R] and columns [x0/2-1, x0/2+8] (half-pixel centres), so a
// (2R+2) x 10 patch of source-0 pixels (clamped to the image) is loaded once.
template <int R>
struct LowPatch {
  static constexpr int kRows = 2 * R + 2, kCols = 10;
};

// 8 channels [ch, ch+8) of one patch pixel (output coordinates y, x):
// zero outside the image; else source 0 (bilinear x2 from the staged
// low-resolution patch when up0), then source 1, then zero up to cip.
template <class E, int R>
__device__ __forceinline__ void fill_group(const ConvArgs& a, const uint8_t* low, int b, int y0,
                                           int x0, int y, int x, int ch, uint8_t* dst) {
  if (y < 0 || y >= a.h || x < 0 || x >= a.w) {
    E::zero8(dst);
    return;
  }
  if (ch < a.c0) {
    if (!a.up0) {
      E::copy8(dst, a.src0 + ((((int64_t)b * a.h + y) * a.w + x) * a.c0 + ch) * E::kBytes);
      return;
    }
    const int hh = a.h >> 1, ww = a.w >> 1;
    const float sy = fminf(fmaxf((y + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(hh - 1));
    const float sx = fminf(fmaxf((x + 0.5f) * 0.5f - 0.5f, 0.0f), (float)(ww - 1));
    const int ly0 = (int)sy, lx0 = (int)sx;
    const int ly1 = min(ly0 + 1, hh - 1), lx1 = min(lx0 + 1, ww - 1);
    const float fy = sy - (float)ly0, fx = sx - (float)lx0;
    const int oy = (y0 >> 1) - 1, ox = (x0 >> 1) - 1;
    const int rs = LowPatch<R>::kCols * a.c0;
    const uint8_t* p = low + ch * E::kBytes;
    float v00[8], v01[8], v10[8], v11[8], r[8];
    E::load8(p + ((ly0 - oy) * rs + (lx0 - ox) * a.c0) * E::kBytes, v00);
    E::load8(p + ((ly0 - oy) * rs + (lx1 - ox) * a.c0) * E::kBytes, v01);
    E::load8(p + ((ly1 - oy) * rs + (lx0 - ox) * a.c0) * E::kBytes, v10);
    E::load8(p + ((ly1 - oy) * rs + (lx1 - ox) * a.c0) * E::kBytes, v11);
    for (int i = 0; i < 8; ++i) {
      const float top = fmaf(fx, v01[i] - v00[i], v00[i]);
      const float bot = fmaf(fx, v11[i] - v10[i], v10[i]);
      r[i] = fmaf(fy, bot - top, top);
    }
    E::store8(dst, r);
    return;
  }
  if (ch < a.c0 + a.c1) {
    E::copy8(dst, a.src1 + ((((int64_t)b * a.h + y) * a.w + x) * a.c1 + (ch - a.c0)) * E::kBytes);
    return;
  }
  E::zero8(dst);
}

// Bytes of dynamic LDS k_conv3x3<E, NB, R> needs.
template <class E, int R>
__host__ __device__ inline size_t conv_lds_bytes(int cip, int c0, int up0, int co) {
  size_t patch = (size_t)(4 * R + 2) * 18 * (cip + E::kPad) * E::kBytes;
  size_t low = up0 ? (size_t)LowPatch<R>::kRows * LowPatch<R>::kCols * c0 * E::kBytes : 0;
  size_t outt = (size_t)4 * R * 16 * (co + E::kPad) * E::kBytes;
  size_t a = patch + low;
  return a > outt ? a : outt;
}

// Block = 4 waves; output tile = (4 R) rows x 16 columns of one image; wave w
// owns rows [w R, w R + R), each row one 16-pixel M block.  The input patch
// (tile + 1-pixel halo, all cip channels) is staged in LDS once; per 32-wide
// K chunk each lane reads its A fragment (8 channels of one pixel at one tap)
// from LDS; B fragments (pre-swizzled weights) come from global memory one
// chunk ahead of their use.  The epilogue transposes the tile through LDS
// and writes whole 16-byte channel groups.
template <class E, int NB, int R>
__global__ void __launch_bounds__(256) k_conv3x3(ConvArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  constexpr int PR = 4 * R + 2, PC = 18;
  const int S = a.cip + E::kPad;  // patch pixel stride in elements
  const int x0 = blockIdx.x * 16, y0 = blockIdx.y * (4 * R), b = blockIdx.z;
  const int tid = threadIdx.x;
  uint8_t* low = smem + (size_t)PR * PC * S * E::kBytes;
  if (a.up0) {
    const int hh = a.h >> 1, ww = a.w >> 1, g0 = a.c0 >> 3;
    const int tot = LowPatch<R>::kRows * LowPatch<R>::kCols * g0;
    constexpr int kB = 4;
    using V = typename std::conditional<E::kBytes == 2, uint4, uint2>::type;
    for (int base = tid; base < tot; base += 256 * kB) {
      V v[kB];
      for (int u = 0; u < kB; ++u) {
        const int e = base + u * 256;
        if (e >= tot) continue;
        const int g = e % g0, pix = e / g0;
        const int r = pix / LowPatch<R>::kCols, c = pix - r * LowPatch<R>::kCols;
        const int ly = min(max((y0 >> 1) - 1 + r, 0), hh - 1);
        const int lx = min(max((x0 >> 1) - 1 + c, 0), ww - 1);
        v[u] = *(const V*)(a.src0 + ((((int64_t)b * hh + ly) * ww + lx) * a.c0 + g * 8) * E::kBytes);
      }
      for (int u = 0; u < kB; ++u) {
        const int e = base + u * 256;
        if (e < tot) *(V*)(low + (size_t)e * 8 * E::kBytes) = v[u];
      }
    }
    __syncthreads();
  }
  const int groups = a.cip >> 3;
  const int total = PR * PC * groups;
  if (!a.up0) {
    // plain copy: issue a batch of global loads before the LDS stores so
    // several loads per thread are in flight
    constexpr int kB = 6;
    using V = typename std::conditional<E::kBytes == 2, uint4, uint2>::type;
    for (int base = tid; base < total; base += 256 * kB) {
      V v[kB];
      int dst[kB];
      for (int u = 0; u < kB; ++u) {
        const int e = base + u * 256;
        dst[u] = -1;
        V z;
        memset(&z, 0, sizeof z);
        v[u] = z;
        if (e >= total) continue;
        const int g = e % groups, pix = e / groups;
        const int r = pix / PC, c = pix - r * PC;
        const int y = y0 - 1 + r, x = x0 - 1 + c, ch = g * 8;
        dst[u] = pix * S + ch;
        if (y < 0 || y >= a.h || x < 0 || x >= a.w) continue;
        const uint8_t* src = ch < a.c0
            ? a.src0 + ((((int64_t)b * a.h + y) * a.w + x) * a.c0 + ch) * E::kBytes
            : (ch < a.c0 + a.c1
                   ? a.src1 + ((((int64_t)b * a.h + y) * a.w + x) * a.c1 + (ch - a.c0)) * E::kBytes
                   : nullptr);
        if (src) v[u] = *(const V*)src;
      }
      for (int u = 0; u < kB; ++u)
        if (dst[u] >= 0) *(V*)(smem + (size_t)dst[u] * E::kBytes) = v[u];
    }
  } else {
    for (int e = tid; e < total; e += 256) {
      const int g = e % groups, pix = e / groups;
      const int r = pix / PC, c = pix - r * PC;
      fill_group<E, R>(a, low, b, y0, x0, y0 - 1 + r, x0 - 1 + c, g * 8,
                       smem + ((size_t)pix * S + g * 8) * E::kBytes);
    }
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  f32x4_t acc[R][NB];
  for (int rr = 0; rr < R; ++rr)
    for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int col = lane & 15;
  const uint8_t* wl = a.wsw + (size_t)lane * 8 * E::kBytes;
  // this lane's K position (c * 32 + 8 * (lane / 16)) as (tap, channel),
  // advanced incrementally (no division in the loop)
  int ci = 8 * (lane >> 4), tap = 0;
  while (ci >= a.cip) {
    ci -= a.cip;
    ++tap;
  }
  auto load_a = [&](int tp, int cc, typename E::Frag* af) {
    if (tp < 9) {
      const int ky = tp / 3, kx = tp - ky * 3;
      for (int rr = 0; rr < R; ++rr) {
        const int pix = (wave * R + rr + ky) * PC + col + kx;
        af[rr] = E::frag(smem + ((size_t)pix * S + cc) * E::kBytes);
      }
    } else {
      for (int rr = 0; rr < R; ++rr) af[rr] = E::zero();
    }
  };
  typename E::Frag acur[R], anext[R], bcur[NB], bnext[NB];
  load_a(tap, ci, acur);
  for (int nb = 0; nb < NB; ++nb) bcur[nb] = E::frag(wl + (size_t)nb * 512 * E::kBytes);
  for (int c = 0; c < a.kc; ++c) {
    const bool more = c + 1 < a.kc;
    if (more) {
      ci += 32;
      while (ci >= a.cip) {
        ci -= a.cip;
        ++tap;
      }
      for (int nb = 0; nb < NB; ++nb)
        bnext[nb] = E::frag(wl + ((size_t)(c + 1) * NB + nb) * 512 * E::kBytes);
      load_a(tap, ci, anext);
    }
    for (int nb = 0; nb < NB; ++nb)
      for (int rr = 0; rr < R; ++rr) acc[rr][nb] = E::mma(acur[rr], bcur[nb], acc[rr][nb]);
    if (more) {
      for (int nb = 0; nb < NB; ++nb) bcur[nb] = bnext[nb];
      for (int rr = 0; rr < R; ++rr) acur[rr] = anext[rr];
    }
  }
  // epilogue: bias, ReLU, (calibration max), then store
  float mx = 0.f;
  const int OS = a.co + E::kPad;  // LDS output pixel stride (elements)
  if (!a.out_fp32) __syncthreads();  // the patch is dead; reuse LDS for the output tile
  for (int rr = 0; rr < R; ++rr) {
    const int ty = wave * R + rr;
    const int y = y0 + ty;
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 16 + col;
      if (n >= a.co) continue;
      const float al = a.alpha ? a.alpha[n] : 1.0f;
      const float bi = a.bias ? a.bias[n] : 0.0f;
      for (int i = 0; i < 4; ++i) {
        const int tx = 4 * (lane >> 4) + i;
        float v = fmaf(acc[rr][nb][i], al, bi);
        if (a.relu) v = fmaxf(v, 0.0f);
        if (y < a.h && x0 + tx < a.w) mx = fmaxf(mx, fabsf(v));
        if (a.out_fp32) {
          if (y < a.h && x0 + tx < a.w)
            ((float*)a.out)[(((int64_t)b * a.h + y) * a.w + x0 + tx) * a.out_ch + n] = v;
        } else {
          E::store1(smem + ((size_t)(ty * 16 + tx) * OS + n) * E::kBytes, v);
        }
      }
    }
  }
  if (a.absmax) wave_absmax(a.absmax, mx);
  if (a.out_fp32) return;
  __syncthreads();
  const int cg = a.co >> 3;  // 8-channel groups per pixel (co is a multiple of 8)
  const int tot = 4 * R * 16 * cg;
  for (int e = tid; e < tot; e += 256) {
    const int g = e % cg, pix = e / cg;
    const int ty = pix >> 4, tx = pix & 15;
    const int y = y0 + ty, x = x0 + tx;
    if (y >= a.h || x >= a.w) continue;
    E::copy8(a.out + ((((int64_t)b * a.h + y) * a.w + x) * a.out_ch + g * 8) * E::kBytes,
             smem + ((size_t)pix * OS + g * 8) * E::kBytes);
  }
}

template <class E>
fv_status launch_conv(const ConvArgs& a, int nb, hipStream_t s);

}  // namespace net
}  // namespace fv
