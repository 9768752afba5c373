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
  static constexpr int kK = 32;          // K per MFMA (16x16x32)
  static constexpr int kFragBytes = 16;  // operand bytes per lane
  static constexpr int kSub = 1;         // 8-channel pixel reads per lane and chunk
  static constexpr bool kPrefetch = true;  // double-buffer the operands across chunks
  typedef bf16x8_t Frag;
  static __device__ __forceinline__ Frag frag(const uint8_t* p) { return *(const Frag*)p; }
  static __device__ __forceinline__ Frag bfrag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(Frag, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  }
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
  static __device__ __forceinline__ void store8_inrange(uint8_t* p, const float v[8]) {
    store8(p, v);
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
  static __device__ __forceinline__ void store4(uint8_t* p, const float v[4]) {
    *(uint2*)p = make_uint2(enc_bits(v[0]) | (enc_bits(v[1]) << 16),
                            enc_bits(v[2]) | (enc_bits(v[3]) << 16));
  }
  // the value as stored and read back
  static __device__ __forceinline__ float rnd(float v) { return bf16_bits_to_f(enc_bits(v)); }
  // ReLU (when relu) and the range of the stored type
  static __device__ __forceinline__ float act(float v, int relu) {
    return relu ? fmaxf(v, 0.0f) : v;
  }
  static __device__ __forceinline__ float rnd_act(float v) { return rnd(v); }
  static __device__ __forceinline__ void lstore4(uint8_t* p, const float v[4]) {
    *(uint2*)p = make_uint2(enc_bits(v[0]) | (enc_bits(v[1]) << 16),
                            enc_bits(v[2]) | (enc_bits(v[3]) << 16));
  }
  static __device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, int voff, int soff,
                                                 const float v[4]) {
    typedef __attribute__((__vector_size__(2 * sizeof(int)))) int i2;
    const i2 w = {(int)(enc_bits(v[0]) | (enc_bits(v[1]) << 16)),
                  (int)(enc_bits(v[2]) | (enc_bits(v[3]) << 16))};
    __builtin_amdgcn_raw_buffer_store_b64(w, r, voff, soff, 0);
  }
};

typedef int i32x8_t __attribute__((ext_vector_type(8)));

struct FP8 {
  static constexpr int kBytes = 1;
  static constexpr int kK = 128;         // K per MFMA (16x16x128, E4M3 operands)
  static constexpr int kFragBytes = 32;
  static constexpr int kSub = 4;
  static constexpr bool kPrefetch = false;
  // A lane's operand: 32 consecutive K positions (lane group g of a chunk
  // holds K = 32 g .. 32 g + 31); any order consistent between the two
  // operands gives the same dot product.
  typedef i32x8_t Frag;
  static __device__ __forceinline__ Frag frag(const uint8_t* p) { return *(const Frag*)p; }
  static __device__ __forceinline__ Frag bfrag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i4;
    const i4 lo = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    const i4 hi =
        __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + 16, 0));
    return Frag{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  }
  // the 32 bytes of a pixel operand from four 8-byte reads
  static __device__ __forceinline__ Frag frag4(const uint8_t* p, int4 o) {
    const uint2 a = *(const uint2*)(p + o.x), b = *(const uint2*)(p + o.y);
    const uint2 c = *(const uint2*)(p + o.z), d = *(const uint2*)(p + o.w);
    return Frag{(int)a.x, (int)a.y, (int)b.x, (int)b.y, (int)c.x, (int)c.y, (int)d.x, (int)d.y};
  }
  static __device__ __forceinline__ f32x4_t mma(Frag a, Frag b, f32x4_t c) {
    // unit block scales (E8M0 127 = 2^0)
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
  }
  static __device__ __forceinline__ void copy8(uint8_t* dst, const uint8_t* src) {
    *(uint2*)dst = *(const uint2*)src;
  }
  static __device__ __forceinline__ void zero8(uint8_t* dst) { *(uint2*)dst = make_uint2(0, 0); }
  static __device__ __forceinline__ float sat(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }
  static __device__ __forceinline__ uint8_t enc(float v) {
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(sat(v), 0.0f, 0, false) & 0xff);
  }
  // two bytes per conversion (bytes 0, 1 of the selected 16-bit word)
  static __device__ __forceinline__ void load8(const uint8_t* p, float v[8]) {
    const uint2 u = *(const uint2*)p;
    const auto a = __builtin_amdgcn_cvt_pk_f32_fp8((int)u.x, false);
    const auto b = __builtin_amdgcn_cvt_pk_f32_fp8((int)u.x, true);
    const auto c = __builtin_amdgcn_cvt_pk_f32_fp8((int)u.y, false);
    const auto d = __builtin_amdgcn_cvt_pk_f32_fp8((int)u.y, true);
    v[0] = a[0];
    v[1] = a[1];
    v[2] = b[0];
    v[3] = b[1];
    v[4] = c[0];
    v[5] = c[1];
    v[6] = d[0];
    v[7] = d[1];
  }
  // store8 for values known to lie in the E4M3 range (no clamp)
  static __device__ __forceinline__ void store8_inrange(uint8_t* p, const float v[8]) {
    int lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], hi, true);
    *(uint2*)p = make_uint2((uint32_t)lo, (uint32_t)hi);
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
  static __device__ __forceinline__ void store4(uint8_t* p, const float v[4]) {
    int w = 0;
    w = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[0]), sat(v[1]), w, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(sat(v[2]), sat(v[3]), w, true);
    *(uint32_t*)p = (uint32_t)w;
  }
  static __device__ __forceinline__ float rnd(float v) {
    return __builtin_amdgcn_cvt_f32_fp8(__builtin_amdgcn_cvt_pk_fp8_f32(sat(v), 0.0f, 0, false), 0);
  }
  // ReLU (when relu) and saturation to the E4M3 range in one clamp; values
  // from act() need no further clamp before conversion
  static __device__ __forceinline__ float act(float v, int relu) {
    return __builtin_amdgcn_fmed3f(v, relu ? 0.0f : -448.0f, 448.0f);
  }
  static __device__ __forceinline__ float rnd_act(float v) {
    return __builtin_amdgcn_cvt_f32_fp8(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false), 0);
  }
  static __device__ __forceinline__ void lstore4(uint8_t* p, const float v[4]) {
    int w = 0;
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], w, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
    *(int*)p = w;
  }
  // 4 values from act() packed to E4M3 and stored
  static __device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, int voff, int soff,
                                                 const float v[4]) {
    int w = 0;
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], w, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
    __builtin_amdgcn_raw_buffer_store_b32(w, r, voff, soff, 0);
  }
};

// Cross-lane partners without an LDS round trip.  The gfx950 lane-swap
// instructions (rows of 16 lanes, halves of 32) leave v[l] and v[l ^ 16]
// (resp. v[l ^ 32]) in their two results at every lane l, in an order that
// depends on the lane; the sum or maximum of the two is therefore what
// v + v[l ^ m] (resp. max) gives, since both operations are commutative.
__device__ __forceinline__ float pair_sum16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_max16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float pair_max32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
// v of lane l ^ 1 (a quad permutation [1, 0, 3, 2])
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

__device__ __forceinline__ void wave_absmax(float* dst, float m) {
  for (int off = 32; off; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.f) atomicMax((unsigned int*)dst, __float_as_uint(m));
}

// One 3x3 convolution as an implicit GEMM: M = output channels, N = output
// pixels, K = 9 taps x input channels.
struct ConvArgs {
  const uint8_t* src0;  // NHWC, c0 channels; half resolution if up0
  const uint8_t* src1;  // NHWC, c1 channels (concatenated after src0), or null
  const uint8_t* src2;  // NHWC, c2 channels (concatenated after src1), or null
  int c0, c1, c2, cip;  // cip = c0 + c1 + c2 rounded up to 8
  int up0;
  int n, h, w;          // output size
  const uint8_t* wsw;   // swizzled weight fragments [kc][nb][64 lanes][kFragBytes]
  int kc;
  const float* alpha;   // per-output-channel multiplier, or null (= 1)
  const float* bias;    // per-output-channel bias, or null
  int co, relu;
  uint8_t* out;         // NHWC, out_ch channel stride
  int out_ch, out_fp32;
  float* absmax;        // per-tensor running maximum (calibration), or null
  uint8_t* pool_out;    // 2x2 average of the stored output (half resolution,
                        // out_ch stride), or null
  // BF16 only: the stored value is v * [gate > 0], gate being a BF16 tensor
  // laid out as the output (out_ch stride): an input-gradient conv storing
  // the next layer's masked output gradient (the ReLU derivative of the
  // forward activation gate), or null
  const uint8_t* gate;
  uint32_t out_bytes, pool_bytes;  // set by launch_conv (buffer-store range checks)
  uint32_t src0_bytes, src1_bytes, src2_bytes;  // sizes for the buffer-load range checks
  // set by launch_conv: e / ng == umulhi(e, gmagic) for the ng fill-item
  // channel groups copied from memory (0: ng == 1); umagic likewise for the
  // groups of the low-resolution patch of an upsampled source 0
  uint32_t gmagic, umagic;
  uint32_t umagic8;  // same for the c0 / 8 groups of the upsampling pass
  int wide;   // set by launch_conv: fill items of 16 channels (FP8) instead of 8
  int b_lds;  // set by launch_conv: the weight fragments are staged in LDS
  // Fused first layer (inference, 2 output blocks, b_lds): the patch of this
  // conv is computed in the block from the frame instead of read from src0:
  // the packed input [M rgb, M, M depth / 2, O_d,prev rgb] (times f_inv, the
  // input tensor's inverse scale; zero outside the image; O_d,prev = 0 when
  // f_prev is null), then a 3x3 conv of its 8 channels to co0 = 32 channels
  // with scale/bias f_alpha/f_bias and ReLU, zero outside the image (the
  // padding of this conv).
  int fuse0;
  const float4* f_rgba;
  const uint8_t* f_mask;
  const float* f_depth;
  const float* f_prev;  // [n h w 3] or null
  float f_inv;
  const uint8_t* f_wsw;  // the first layer's weight fragments
  int f_kc;
  const float* f_alpha;  // or null (= 1)
  const float* f_bias;
  // FP8 conv with a BF16 first layer (the recurrent form, whose fed-back O_d
  // is a dense image): the packed input, the first layer's weight fragments
  // (f_wsw, f_kc) and its MFMA are BF16; its output is stored in the patch in
  // FP8 with f_alpha / f_bias folding the output scale
  int f_mixed;
};

template <class E>
struct Chunk8;  // 8 elements: 16 bytes (BF16) or 8 bytes (FP8)
template <>
struct Chunk8<BF16> {
  typedef uint4 T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, int off) {
    typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i4;
    const i4 v = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return make_uint4((uint32_t)v[0], (uint32_t)v[1], (uint32_t)v[2], (uint32_t)v[3]);
  }
};
template <>
struct Chunk8<FP8> {
  typedef uint2 T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, int off) {
    typedef __attribute__((__vector_size__(2 * sizeof(int)))) int i2;
    const i2 v = __builtin_bit_cast(i2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    return make_uint2((uint32_t)v[0], (uint32_t)v[1]);
  }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}

// Low-resolution staging for an upsampled source 0: the tile's output rows
// [y0-1, y0+4R] and columns [x0-1, x0+16] read low-resolution rows
// [y0/2-1, y0/2+2R] and columns [x0/2-1, x0/2+8] (half-pixel centres), so a
// (2R+2) x 10 patch of source-0 pixels (clamped to the image) is loaded once.
template <int R>
struct LowPatch {
  static constexpr int kRows = 2 * R + 2, kCols = 10;
};

// Patch pixel stride in elements (cip is a multiple of 8).  The 16 lanes of
// a fragment read 16 consecutive pixels; a stride of 8 mod 16 elements (FP8:
// 8 mod 16 bytes for 8-byte reads; BF16: 16 mod 32 bytes for 16-byte reads)
// spreads them over all LDS banks.
template <class E>
__host__ __device__ inline int patch_stride(int cip) {
  return cip + ((cip % 16) == 0 ? 8 : 0);
}

// Weight fragments of a layer are staged in LDS when they take at most this
// many bytes (the K loop then reads only LDS).
constexpr size_t kMaxLdsWeights = 48 * 1024;

// Bytes of dynamic LDS k_conv3x3<E, NB, R> needs: the input patch, the
// low-resolution source patch (upsampled source 0), the table of K-chunk
// patch offsets (4 kSub per chunk), the per-channel scale and bias and, when
// b_lds, the weight fragments.  Every
// region starts 16-byte aligned.
template <class E, int R>
__host__ __device__ inline size_t conv_lds_bytes(int cip, int c0, int up0, int kc, int nb,
                                                 int co, int b_lds) {
  size_t patch = (size_t)(4 * R + 2) * 18 * patch_stride<E>(cip) * E::kBytes;
  size_t low = up0 ? (size_t)LowPatch<R>::kRows * LowPatch<R>::kCols * c0 * E::kBytes : 0;
  size_t w = b_lds ? (size_t)kc * nb * 64 * E::kFragBytes : 0;
  return patch + low + (size_t)16 * E::kSub * kc + (size_t)2 * 4 * ((co + 3) & ~3) + w;
}

// Block = 4 waves; tile = (4 R) rows x 16 columns of one image; wave w owns
// rows [w R, w R + R), each row one 16-pixel N block.  Every global load a
// block needs before its K loop (the input patch: tile + 1-pixel halo, all
// cip channels; the weight fragments when they fit in LDS; the per-channel
// scale and bias) is issued at once, so a block waits for one memory round
// trip before its MFMAs.  Per 32- (BF16) or 128-wide (FP8) K chunk each lane
// reads its pixel operand (8 channels at one tap, or four such groups) from
// LDS.  With the weights as the A operand each lane's accumulator holds 4
// consecutive channels of one pixel, so the epilogue writes them straight to
// global memory as one packed store.
// Extra LDS of a fused first layer (after the regular regions): the packed
// input patch (4 R + 4) x 20 pixels x 8 channels, its K-chunk table, scale
// and bias of 32 channels, and its weight fragments (2 output blocks).
template <class E, int R>
__host__ __device__ inline size_t fuse0_lds_bytes(int f_kc) {
  return (size_t)(4 * R + 4) * 20 * 8 * E::kBytes + (size_t)16 * E::kSub * f_kc + 2 * 4 * 32 +
         (size_t)f_kc * 2 * 64 * E::kFragBytes;
}

// Fused first layer (see ConvArgs::fuse0): fills the block's patch (output
// tile + 1-pixel halo, 32 channels, stride S) by computing the first conv on
// it.  Also stages this conv's K-chunk table, scale/bias and weights (the
// regular fill does that otherwise) and ends with every LDS region written
// (the caller synchronises before its K loop).
template <class E, class F0, int R>
__device__ __forceinline__ void fuse0_fill(const ConvArgs& a, uint8_t* smem, int S, int* ktab,
                                        float* s_ab, uint8_t* wsm, int b, int y0, int x0) {
  constexpr int PR = 4 * R + 2, PC = 18;       // this conv's patch
  constexpr int IR = 4 * R + 4, IC = 20;       // the packed-input patch
  constexpr int NBLK = (PR * PC + 15) / 16;    // 16-pixel blocks of the patch
  typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int cpad = (a.co + 3) & ~3;
  uint8_t* in = smem + conv_lds_bytes<E, R>(a.cip, a.c0, 0, a.kc, 2, a.co, 1);
  int* ktab0 = (int*)(in + (size_t)IR * IC * 8 * F0::kBytes);
  float* s_ab0 = (float*)(ktab0 + 4 * F0::kSub * a.f_kc);
  uint8_t* wsm0 = (uint8_t*)(s_ab0 + 64);
  // 1. loads: packed-input pixels (at most 2 per thread), both layers' weights
  // and scale/bias
  float4 px_c[2];
  uint32_t px_m[2];
  float px_d[2];
  float px_p[2][3];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = tid + u * 256;
    px_m[u] = 0;
    px_p[u][0] = px_p[u][1] = px_p[u][2] = 0.0f;
    if (i < IR * IC) {
      const int r = i / IC, c = i - r * IC;
      const int y = y0 - 2 + r, x = x0 - 2 + c;
      if (y >= 0 && y < a.h && x >= 0 && x < a.w) {
        const int64_t p = ((int64_t)b * a.h + y) * a.w + x;
        px_m[u] = a.f_mask[p];
        px_c[u] = a.f_rgba[p];
        px_d[u] = a.f_depth ? a.f_depth[p] : 0.0f;
        if (a.f_prev) {
          px_p[u][0] = a.f_prev[p * 3 + 0];
          px_p[u][1] = a.f_prev[p * 3 + 1];
          px_p[u][2] = a.f_prev[p * 3 + 2];
        }
      }
    }
  }
  const int n16 = a.kc * 2 * 64 * E::kFragBytes / 16;
  const int n16f = a.f_kc * 2 * 64 * F0::kFragBytes / 16;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.wsw, (uint32_t)n16 * 16);
  const __amdgpu_buffer_rsrc_t rw0 = make_rsrc(a.f_wsw, (uint32_t)n16f * 16);
  for (int base = tid; base < n16 + n16f; base += 256 * 4) {
    i4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 256;
      if (e < n16)
        v[u] = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(rw, e * 16, 0, 0));
      else if (e < n16 + n16f)
        v[u] = __builtin_bit_cast(
            i4, __builtin_amdgcn_raw_buffer_load_b128(rw0, (e - n16) * 16, 0, 0));
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = base + u * 256;
      if (e < n16)
        *(i4*)(wsm + (size_t)e * 16) = v[u];
      else if (e < n16 + n16f)
        *(i4*)(wsm0 + (size_t)(e - n16) * 16) = v[u];
    }
  }
  if (tid < 64) {
    const int c = tid & 31;
    const bool is_bias = tid >= 32;
    const float* src = is_bias ? a.f_bias : a.f_alpha;
    s_ab0[tid] = src ? src[c] : (is_bias ? 0.0f : 1.0f);
  } else if (tid < 64 + 2 * a.co) {
    const int e = tid - 64;
    const float* src = e < a.co ? a.alpha : a.bias;
    s_ab[e < a.co ? e : cpad + e - a.co] =
        src ? src[e < a.co ? e : e - a.co] : (e < a.co ? 1.0f : 0.0f);
  }
  // K-chunk tables: this conv's (patch stride S, 18 wide) and the first
  // layer's (packed-input stride 8, 20 wide)
  for (int e = tid; e < 4 * E::kSub * a.kc; e += 256) {
    const int k = e * 8, tap = k / a.cip, ch = k - tap * a.cip;
    const int ky = tap / 3, kx = tap - 3 * ky;
    ktab[e] = tap < 9 ? ((ky * PC + kx) * S + ch) * E::kBytes : 0;
  }
  for (int e = tid; e < 4 * F0::kSub * a.f_kc; e += 256) {
    const int tap = e;  // 8 input channels: one tap per 8 K positions
    const int ky = tap / 3, kx = tap - 3 * ky;
    ktab0[e] = tap < 9 ? (ky * IC + kx) * 8 * F0::kBytes : 0;
  }
  // 2. packed input -> LDS (the k_pack arithmetic: values times f_inv)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = tid + u * 256;
    if (i >= IR * IC) continue;
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (px_m[u]) {
      v[0] = px_c[u].x;
      v[1] = px_c[u].y;
      v[2] = px_c[u].z;
      v[3] = 1.0f;
      v[4] = 0.5f * px_d[u];
    }
    v[5] = px_p[u][0];
    v[6] = px_p[u][1];
    v[7] = px_p[u][2];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] *= a.f_inv;
    F0::store8(in + (size_t)i * 8 * F0::kBytes, v);
  }
  __syncthreads();
  // 3. the first conv on the patch pixels, 16 consecutive patch pixels per
  // MFMA column block; ReLU'd, stored in the patch (zero outside the image)
  for (int blk = wave; blk < NBLK; blk += 4) {
    const int p = blk * 16 + col;
    const int pc = p < PR * PC ? p : 0;
    const int r = pc / PC, c = pc - r * PC;
    const uint8_t* pin = in + (size_t)(r * IC + c) * 8 * F0::kBytes;
    f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
    for (int ch = 0; ch < a.f_kc; ++ch) {
      typename F0::Frag af, bf[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        bf[nb] = F0::frag(wsm0 + lane * F0::kFragBytes + (ch * 2 + nb) * 64 * F0::kFragBytes);
      if constexpr (F0::kSub == 1)
        af = F0::frag(pin + ktab0[4 * ch + grp]);
      else
        af = F0::frag4(pin, ((const int4*)ktab0)[4 * ch + grp]);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[nb] = F0::mma(bf[nb], af, acc[nb]);
    }
    const int y = y0 - 1 + r, x = x0 - 1 + c;
    const bool inside = p < PR * PC && y >= 0 && y < a.h && x >= 0 && x < a.w;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int c4 = nb * 16 + 4 * grp;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v[i] = inside ? E::act(fmaf(acc[nb][i], s_ab0[c4 + i], s_ab0[32 + c4 + i]), 1) : 0.0f;
      if (p < PR * PC) E::lstore4(smem + ((size_t)pc * S + c4) * E::kBytes, v);
    }
  }
}

// Occupancy target (waves per SIMD) for the register allocator, out of 512
// registers: the accumulators (4 NB R) plus about 80 (FP8) or 96 (BF16,
// double-buffered operands) for the rest; at 5 or more N blocks the weight
// fragments alone need so many registers that two waves is the target.
template <class E, int NB, int R>
struct ConvWaves {
  static constexpr int kRegs = 4 * NB * R + (E::kBytes == 2 ? 96 : 80);
  static constexpr int v = NB >= 5 ? 2 : (512 / kRegs > 8 ? 8 : 512 / kRegs);
};

template <class E, int NB, int R>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(ConvWaves<E, NB, R>::v))) k_conv3x3(ConvArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  constexpr int PR = 4 * R + 2, PC = 18;
  constexpr int LR = LowPatch<R>::kRows, LC = LowPatch<R>::kCols;
  constexpr int kPF = E::kBytes == 1 ? 6 : 8;  // fill items per thread in the first batch
  constexpr int kPW = 6;                      // weight loads (16 B) per thread in flight
  constexpr int kOutside = (int)0x80000000u;  // beyond every source (< 2 GiB)
  using Item = uint4;  // 16 bytes: 16 FP8 channels (wide), else 8 channels
  typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i4;
  const int S = patch_stride<E>(a.cip);  // patch pixel stride in elements
  const int tid = threadIdx.x;
  // one block per tile: grid (tile columns, tile rows, images)
  const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 4 * R, b = blockIdx.z;
  uint8_t* low = smem + (size_t)PR * PC * S * E::kBytes;
  int* ktab = (int*)(low + (a.up0 ? (size_t)LR * LC * a.c0 * E::kBytes : 0));
  float* s_ab = (float*)(ktab + 4 * E::kSub * a.kc);  // alpha[co], bias[co]
  uint8_t* wsm = (uint8_t*)(s_ab + 2 * ((a.co + 3) & ~3));  // staged weights (b_lds)
  // LDS fill items: the first nlow are the low-resolution patch of an
  // upsampled source 0 (8 channels each, rows/columns clamped to the image,
  // which is what the clamped bilinear taps read at the borders), the rest
  // the channel groups copied from memory (all of them, or those of source 1
  // after an upsampled source 0).  Pixels outside the image and padding
  // channels load from an out-of-range offset, which the hardware reads as
  // zero.
  const int IW = E::kBytes == 1 && a.wide ? 16 : 8;  // channels per fill item
  const int groups = a.cip / IW, g0 = a.up0 ? a.c0 / IW : 0, ng = groups - g0;
  const int nlow = a.up0 ? LR * LC * g0 : 0;
  const int nitems = nlow + PR * PC * ng;
  const int hh = a.h >> 1, ww = a.w >> 1;
  const __amdgpu_buffer_rsrc_t r0 = make_rsrc(a.src0, a.src0_bytes);
  const __amdgpu_buffer_rsrc_t r1 =
      make_rsrc(a.src1 ? a.src1 : a.src0, a.src1 ? a.src1_bytes : 0u);
  const __amdgpu_buffer_rsrc_t r2 =
      make_rsrc(a.src2 ? a.src2 : a.src0, a.src2 ? a.src2_bytes : 0u);
  // a fill item's load: 16 bytes, or 8 (narrow FP8 items; the upper half
  // is unused)
  auto load16 = [&](__amdgpu_buffer_rsrc_t r, int off) -> Item {
    if (E::kBytes == 2 || IW == 16)
      return __builtin_bit_cast(Item, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const uint2 v = Chunk8<FP8>::load(r, off);
    return make_uint4(v.x, v.y, 0u, 0u);
  };
  auto load_item = [&](int i) -> Item {
    if (i < nlow) {
      const int pix = (int)__umulhi((uint32_t)i, a.umagic), g = i - pix * g0;
      const int r = pix / LC, c = pix - r * LC;
      const int ly = min(max((y0 >> 1) - 1 + r, 0), hh - 1);
      const int lx = min(max((x0 >> 1) - 1 + c, 0), ww - 1);
      const uint32_t p = ((uint32_t)b * (uint32_t)hh + (uint32_t)ly) * (uint32_t)ww + (uint32_t)lx;
      return load16(r0, (int)((p * (uint32_t)a.c0 + g * IW) * E::kBytes));
    }
    const int e = i - nlow;
    const int pix = a.gmagic ? (int)__umulhi((uint32_t)e, a.gmagic) : e;
    const int g = g0 + e - pix * ng;
    const int r = pix / PC, c = pix - r * PC;
    const int y = y0 - 1 + r, x = x0 - 1 + c, ch = g * IW;
    const bool in = y >= 0 && y < a.h && x >= 0 && x < a.w;
    const uint32_t p = ((uint32_t)b * (uint32_t)a.h + (uint32_t)y) * (uint32_t)a.w + (uint32_t)x;
    if (ch < a.c0)  // (never with an upsampled source 0: then g >= g0)
      return load16(r0, in ? (int)((p * (uint32_t)a.c0 + ch) * E::kBytes) : kOutside);
    const int c01 = a.c0 + a.c1;
    if (ch < c01 || !a.src2)
      return load16(r1, in && ch < c01 ? (int)((p * (uint32_t)a.c1 + (ch - a.c0)) * E::kBytes)
                                       : kOutside);
    return load16(r2, in && ch < c01 + a.c2
                          ? (int)((p * (uint32_t)a.c2 + (ch - c01)) * E::kBytes)
                          : kOutside);
  };
  auto store_item = [&](int i, const Item& v) {
    uint8_t* dst;
    if (i < nlow) {
      dst = low + (size_t)i * IW * E::kBytes;
    } else {
      const int e = i - nlow;
      const int pix = a.gmagic ? (int)__umulhi((uint32_t)e, a.gmagic) : e;
      const int g = g0 + e - pix * ng;
      dst = smem + ((size_t)pix * S + g * IW) * E::kBytes;
    }
    if (E::kBytes == 2) {
      *(Item*)dst = v;  // 16-byte aligned: the BF16 patch stride is 16 mod 32 bytes
    } else {
      // the FP8 patch stride is 8 mod 16 bytes: 8-byte stores
      *(uint2*)dst = make_uint2(v.x, v.y);
      if (IW == 16) *(uint2*)(dst + 8) = make_uint2(v.z, v.w);
    }
  };
  bool fused = false;
  if constexpr (NB == 2) fused = a.fuse0;
  if (fused) {
    if constexpr (NB == 2) {
      if constexpr (E::kBytes == 1) {
        if (a.f_mixed)
          fuse0_fill<E, BF16, R>(a, smem, S, ktab, s_ab, wsm, b, y0, x0);
        else
          fuse0_fill<E, E, R>(a, smem, S, ktab, s_ab, wsm, b, y0, x0);
      } else {
        fuse0_fill<E, E, R>(a, smem, S, ktab, s_ab, wsm, b, y0, x0);
      }
    }
  } else {
  // 1. every global load up front: patch items, weight fragments, scale/bias
  Item pf[kPF];
#pragma unroll
  for (int u = 0; u < kPF; ++u)
    if (tid + u * 256 < nitems) pf[u] = load_item(tid + u * 256);
  const int n16 = a.b_lds ? a.kc * NB * 64 * E::kFragBytes / 16 : 0;
  const __amdgpu_buffer_rsrc_t rw = make_rsrc(a.wsw, (uint32_t)a.kc * NB * 64 * E::kFragBytes);
  i4 wv[kPW];
#pragma unroll
  for (int u = 0; u < kPW; ++u)
    if (tid + u * 256 < n16)
      wv[u] = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(rw, (tid + u * 256) * 16,
                                                                           0, 0));
  // scale (entries 0 .. co-1) and bias (co .. 2 co - 1), two per thread
  // (co <= 256, checked by the launcher)
  float ab[2] = {0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * 256;
    if (e < 2 * a.co) {
      const float* src = e < a.co ? a.alpha : a.bias;
      ab[u] = src ? src[e < a.co ? e : e - a.co] : (e < a.co ? 1.0f : 0.0f);
    }
  }
  // 2. K-chunk table: entry e = (4 c + g) kSub + q = byte offset, from a
  // pixel's top-left halo pixel, of the 8 K positions 8 e .. 8 e + 7 (lane
  // group g's q-th read in chunk c; K is tap-major: tap = k / cip, channel =
  // k % cip).  Positions past the 9 taps carry zero weights; they point at
  // offset 0, a finite activation.
  for (int e = tid; e < 4 * E::kSub * a.kc; e += 256) {
    const int k = e * 8, tap = k / a.cip, ch = k - tap * a.cip;
    const int ky = tap / 3, kx = tap - 3 * ky;
    ktab[e] = tap < 9 ? ((ky * PC + kx) * S + ch) * E::kBytes : 0;
  }
  // 3. LDS stores (the rest of a large fill and of large weights in batches)
#pragma unroll
  for (int u = 0; u < kPF; ++u)
    if (tid + u * 256 < nitems) store_item(tid + u * 256, pf[u]);
#pragma unroll
  for (int u = 0; u < kPW; ++u)
    if (tid + u * 256 < n16) *(i4*)(wsm + (size_t)(tid + u * 256) * 16) = wv[u];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * 256;
    if (e < 2 * a.co) s_ab[e < a.co ? e : ((a.co + 3) & ~3) + e - a.co] = ab[u];
  }
  for (int base = tid + kPF * 256; base < nitems; base += 256 * 4) {
    Item v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < nitems) v[u] = load_item(base + u * 256);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < nitems) store_item(base + u * 256, v[u]);
  }
  for (int base = tid + kPW * 256; base < n16; base += 256 * 4) {
    i4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < n16)
        v[u] = __builtin_bit_cast(i4, __builtin_amdgcn_raw_buffer_load_b128(rw, (base + u * 256) * 16,
                                                                            0, 0));
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < n16) *(i4*)(wsm + (size_t)(base + u * 256) * 16) = v[u];
  }
  if (a.up0) {
    // 4. bilinear x2 (half-pixel centres) from the staged low patch.  Patch
    // rows 2i and 2i + 1 are output rows y0 - 1 + 2i (+1); both read staged
    // rows i and i + 1, with weight 0.25 (even row) or 0.75 (odd row) on the
    // second (columns alike): the same taps and weights as the clamped
    // formula, borders included.  One item = a 2 x 2 block of patch pixels
    // and 8 channels, computed from one 2 x 2 block of staged pixels.
    __syncthreads();
    constexpr int PB = PR / 2, CB = PC / 2;  // 2 x 2 blocks per patch column / row
    const int u8 = a.c0 >> 3;                 // 8-channel groups of source 0
    const int tot = PB * CB * u8;
    const int rs = LC * a.c0;
    for (int e = tid; e < tot; e += 256) {
      const int blk = (int)__umulhi((uint32_t)e, a.umagic8), g = e - blk * u8;
      const int i = blk / CB, j = blk - i * CB;
      const uint8_t* p = low + (i * rs + j * a.c0 + g * 8) * E::kBytes;
      float v00[8], v01[8], v10[8], v11[8];
      E::load8(p, v00);
      E::load8(p + a.c0 * E::kBytes, v01);
      E::load8(p + rs * E::kBytes, v10);
      E::load8(p + (rs + a.c0) * E::kBytes, v11);
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const float fx = dx ? 0.75f : 0.25f;
        float top[8], bot[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          top[k] = fmaf(fx, v01[k] - v00[k], v00[k]);
          bot[k] = fmaf(fx, v11[k] - v10[k], v10[k]);
        }
        const int c = 2 * j + dx, x = x0 - 1 + c;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const float fy = dy ? 0.75f : 0.25f;
          const int r = 2 * i + dy, y = y0 - 1 + r;
          uint8_t* dst = smem + ((size_t)(r * PC + c) * S + g * 8) * E::kBytes;
          if (y < 0 || y >= a.h || x < 0 || x >= a.w) {
            E::zero8(dst);
            continue;
          }
          float o[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) o[k] = fmaf(fy, bot[k] - top[k], top[k]);
          // a convex blend of stored values stays in the format's range
          E::store8_inrange(dst, o);
        }
      }
    }
  }
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, grp = lane >> 4;
  // weight fragments by buffer loads: per-lane offset in a VGPR, the chunk's
  // offset uniform (SGPR)
  const __amdgpu_buffer_rsrc_t wr =
      make_rsrc(a.wsw, (uint32_t)a.kc * NB * 64 * E::kFragBytes);
  const int wlane = lane * E::kFragBytes;
  auto load_b = [&](int c, typename E::Frag* bf) {
    if (a.b_lds) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = E::frag(wsm + wlane + (c * NB + nb) * 64 * E::kFragBytes);
    } else {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        bf[nb] = E::bfrag(wr, wlane, (c * NB + nb) * 64 * E::kFragBytes);
    }
  };
  // this lane's pixel (row wave R + rr, column col) in the patch, in bytes
  const uint8_t* prow = smem + (size_t)((wave * R) * PC + col) * S * E::kBytes;
  const int rstep = PC * S * E::kBytes;
  using Off = typename std::conditional<E::kSub == 1, int, int4>::type;
  auto load_a = [&](Off off, typename E::Frag* af) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      if constexpr (E::kSub == 1)
        af[rr] = E::frag(prow + rr * rstep + off);
      else
        af[rr] = E::frag4(prow + rr * rstep, off);
    }
  };
  auto koff = [&](int c) -> Off { return ((const Off*)ktab)[4 * c + grp]; };
  {
    f32x4_t acc[R][NB];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    if constexpr (!E::kPrefetch) {
      // 32-byte fragments: no register double buffering (it would double the
      // operand registers); the other waves on the SIMD cover the LDS latency
      for (int c = 0; c < a.kc; ++c) {
        typename E::Frag af[R], bf[NB];
        load_b(c, bf);
        load_a(koff(c), af);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int rr = 0; rr < R; ++rr) acc[rr][nb] = E::mma(bf[nb], af[rr], acc[rr][nb]);
      }
    } else {
      typename E::Frag acur[R], anext[R], bcur[NB], bnext[NB];
      load_a(koff(0), acur);
      load_b(0, bcur);
      Off offn = koff(a.kc > 1 ? 1 : 0);
      for (int c = 0; c < a.kc; ++c) {
        const bool more = c + 1 < a.kc;
        if (more) {
          load_b(c + 1, bnext);
          load_a(offn, anext);
          offn = koff(c + 2 < a.kc ? c + 2 : 0);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int rr = 0; rr < R; ++rr) acc[rr][nb] = E::mma(bcur[nb], acur[rr], acc[rr][nb]);
        if (more) {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) bcur[nb] = bnext[nb];
#pragma unroll
          for (int rr = 0; rr < R; ++rr) acur[rr] = anext[rr];
        }
      }
    }
    // epilogue: scale, bias, ReLU, one packed store per 4 channels; with
    // pool_out also the 2x2 average of the stored values (rows rr, rr + 1 of
    // this lane, columns of this lane and its neighbour lane ^ 1), summed in
    // the order (0,0), (0,1), (1,0), (1,1) like the stand-alone pooling
    // kernel.  Stores are buffer stores at a 32-bit offset (outputs < 2 GiB,
    // checked by the launcher): the lane's offset is computed once, the row
    // step is uniform; rows below the image are skipped (uniform test) and
    // columns past it or channels past co get an out-of-range offset, which
    // drops the store.
    const int x = x0 + col, yb = y0 + wave * R;
    const int ob = a.out_fp32 ? 4 : E::kBytes;
    const int cpad = (a.co + 3) & ~3;
    const __amdgpu_buffer_rsrc_t ro = make_rsrc(a.out, a.out_bytes);
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(a.gate ? a.gate : a.out, a.out_bytes);
    const int rowb = a.w * a.out_ch * ob;
    const int vo = x < a.w ? (((b * a.h + yb) * a.w + x) * a.out_ch + 4 * grp) * ob : kOutside;
    const bool pool = R >= 2 && a.pool_out;
    const __amdgpu_buffer_rsrc_t rp = make_rsrc(a.pool_out ? a.pool_out : a.out, a.pool_bytes);
    const int prow = (a.w >> 1) * a.out_ch * E::kBytes;
    const int vp = x < a.w && !(col & 1)
                       ? (((b * (a.h >> 1) + (yb >> 1)) * (a.w >> 1) + (x >> 1)) * a.out_ch +
                          4 * grp) * E::kBytes
                       : kOutside;
    float mx = 0.f;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c4 = nb * 16 + 4 * grp;
      const bool cok = c4 < a.co;  // co is a multiple of 8: c4 < co means c4 + 3 < co
      const int cl = cok ? c4 : 0;
      float al[4], bi[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        al[i] = s_ab[cl + i];
        bi[i] = s_ab[cpad + cl + i];
      }
      const int vn = cok ? vo + nb * 16 * ob : kOutside;
      float st[R][4];
#pragma unroll
      for (int rr = 0; rr < R; ++rr) {
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          v[i] = fmaf(acc[rr][nb][i], al[i], bi[i]);
          if (!a.out_fp32) v[i] = E::act(v[i], a.relu);
          st[rr][i] = v[i];
        }
        if (yb + rr >= a.h) continue;  // uniform across the wave
        if (a.absmax && cok && x < a.w)
#pragma unroll
          for (int i = 0; i < 4; ++i) mx = fmaxf(mx, fabsf(v[i]));
        if (a.out_fp32) {
          typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
          __builtin_amdgcn_raw_buffer_store_b128(
              __builtin_bit_cast(__attribute__((__vector_size__(4 * sizeof(int)))) int,
                                 f4{v[0], v[1], v[2], v[3]}),
              ro, vn, rr * rowb, 0);
        } else {
          if constexpr (E::kBytes == 2) {
            if (a.gate) {
              const uint2 gb = __builtin_bit_cast(
                  uint2, __builtin_amdgcn_raw_buffer_load_b64(rg, vn, rr * rowb, 0));
              const uint32_t gw[2] = {gb.x, gb.y};
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float y = bf16_bits_to_f(i & 1 ? gw[i >> 1] >> 16 : gw[i >> 1] & 0xffffu);
                v[i] = y > 0.f ? v[i] : 0.f;
              }
            }
          }
          E::bstore4(ro, vn, rr * rowb, v);
        }
      }
      if (pool) {
#pragma unroll
        for (int rr = 0; rr + 1 < R; rr += 2) {
          float pv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float t0 = E::rnd_act(st[rr][i]), t1 = E::rnd_act(st[rr + 1][i]);
            const float n0 = lane_xor1(t0), n1 = lane_xor1(t1);
            pv[i] = (((t0 + n0) + t1) + n1) * 0.25f;
          }
          if (yb + rr >= a.h) continue;
          E::bstore4(rp, cok ? vp + nb * 16 * E::kBytes : kOutside, (rr >> 1) * prow, pv);
        }
      }
    }
    if (a.absmax) wave_absmax(a.absmax, mx);
  }
}

template <class E>
fv_status launch_conv(const ConvArgs& a, int nb, hipStream_t s);

}  // namespace net
}  // namespace fv
