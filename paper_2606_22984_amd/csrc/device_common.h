// Device-side building blocks shared by the gfx950 kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvan {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kWave = 64;
constexpr float kLnEps = 1e-5f;

typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;

// 16-byte non-temporal load of row data that a kernel reads exactly once, so that
// the stream does not push the weights other workgroups re-read out of L2.
typedef float f32x4nt_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 load_nt4(const float* p) {
  const f32x4nt_t v = __builtin_nontemporal_load(reinterpret_cast<const f32x4nt_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// Precision modes (fvan_precision: 0 and 2).  KvT: K/V cache element; ActT: stored GEMM
// A operand (activations); WT: packed weight element; KC: K consumed per
// 16x16 MFMA fragment step; SPLIT: weights and activations are carried as
// bf16 hi + lo pairs and each step issues hi*hi + hi*lo + lo*hi.
template <int MODE> struct Mode;
template <> struct Mode<0> {            // FP32: FP32 MFMA, FP32 K/V
  typedef float KvT; typedef float ActT; typedef float WT;
  static constexpr int KC = 16; static constexpr bool SPLIT = false;
};
template <> struct Mode<2> {            // BF16 split-operand MFMA, FP16 K/V
  typedef _Float16 KvT; typedef float ActT; typedef __bf16 WT;
  static constexpr int KC = 32; static constexpr bool SPLIT = true;
};

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(__bf16 x) { return (float)x; }
__device__ __forceinline__ float to_f(_Float16 x) { return (float)x; }
template <typename T> __device__ __forceinline__ T from_f(float x);
template <> __device__ __forceinline__ float from_f<float>(float x) { return x; }
template <> __device__ __forceinline__ __bf16 from_f<__bf16>(float x) { return (__bf16)x; }        // RNE
template <> __device__ __forceinline__ _Float16 from_f<_Float16>(float x) { return (_Float16)x; }  // RNE

// A 16-byte chunk of K/V elements, unpacked to floats.
template <typename T> struct Chunk;
template <> struct Chunk<float> {
  static constexpr int N = 4;
  float v[4];
  __device__ __forceinline__ void unpack(const uint4& t) {
    v[0] = __uint_as_float(t.x); v[1] = __uint_as_float(t.y); v[2] = __uint_as_float(t.z); v[3] = __uint_as_float(t.w);
  }
  __device__ __forceinline__ void load(const float* p) { unpack(*reinterpret_cast<const uint4*>(p)); }
};
template <> struct Chunk<__bf16> {
  static constexpr int N = 8;
  float v[8];
  __device__ __forceinline__ void load(const __bf16* p) { unpack(*reinterpret_cast<const uint4*>(p)); }
  __device__ __forceinline__ void unpack(const uint4& t) {
    uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = __uint_as_float(w[i] << 16);
      v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
};
template <> struct Chunk<_Float16> {
  static constexpr int N = 8;
  float v[8];
  __device__ __forceinline__ void load(const _Float16* p) { unpack(*reinterpret_cast<const uint4*>(p)); }
  __device__ __forceinline__ void unpack(const uint4& t) {
    f16x8 h;
    __builtin_memcpy(&h, &t, 16);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (float)h[i];
  }
};

__device__ __forceinline__ floatx4 mfma_bf16(const uint4& a, const uint4& b, floatx4 acc) {
  bf16x8 av, bv;
  __builtin_memcpy(&av, &a, 16);
  __builtin_memcpy(&bv, &b, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
}

// Split 8 floats into bf16 hi and lo parts (x = hi + lo + O(2^-16 |x|)).
// Vector conversions round two floats per instruction (round-to-nearest-even,
// as the scalar cast); hi is widened back by shifting, not converted.
typedef float f32x8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void split8(const float* x, uint4& hi, uint4& lo) {
  const f32x8_t v = {x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7]};
  const bf16x8 h = __builtin_convertvector(v, bf16x8);
  __builtin_memcpy(&hi, &h, 16);
  const f32x8_t hf = {__uint_as_float(hi.x << 16), __uint_as_float(hi.x & 0xFFFF0000u),
                      __uint_as_float(hi.y << 16), __uint_as_float(hi.y & 0xFFFF0000u),
                      __uint_as_float(hi.z << 16), __uint_as_float(hi.z & 0xFFFF0000u),
                      __uint_as_float(hi.w << 16), __uint_as_float(hi.w & 0xFFFF0000u)};
  const bf16x8 l = __builtin_convertvector(v - hf, bf16x8);
  __builtin_memcpy(&lo, &l, 16);
}

// One 16x16 output tile step over a K chunk of Mode<MODE>::KC elements.
// Lane l supplies A elements of row l%16 and B elements of column l%16, both
// for the same K sub-range (l/16) of the chunk; whatever K permutation the
// hardware applies is the same for A and B, so the product is the chunk's dot
// product.  Output layout: lane l holds C[4*(l/16)+i][l%16], i = 0..3.
// a: the lane's A elements (ActT); b / blo: the lane's 16-byte packed weight
// fragment(s).
template <int MODE> struct Frag;
template <> struct Frag<0> {
  static __device__ __forceinline__ floatx4 step(const float* a, const uint4* b, const uint4*, floatx4 acc) {
    const float4 av = *reinterpret_cast<const float4*>(a);
    const uint4 bv = *b;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, __uint_as_float(bv.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, __uint_as_float(bv.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, __uint_as_float(bv.z), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, __uint_as_float(bv.w), acc, 0, 0, 0);
    return acc;
  }
  // two 16-row A tiles against one B fragment (loaded once)
  static __device__ __forceinline__ void step2(const float* a0, const float* a1, const uint4* b, const uint4*,
                                               floatx4& acc0, floatx4& acc1) {
    step2v(a0, a1, *b, *b, acc0, acc1);
  }
  // one 16-row A tile against a B fragment already in registers
  static __device__ __forceinline__ void step1v(const float* a0, const uint4 bv, const uint4, floatx4& acc0) {
    const float4 x = *reinterpret_cast<const float4*>(a0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, __uint_as_float(bv.x), acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, __uint_as_float(bv.y), acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, __uint_as_float(bv.z), acc0, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, __uint_as_float(bv.w), acc0, 0, 0, 0);
  }
  // the same with the B fragment already in registers
  static __device__ __forceinline__ void step2v(const float* a0, const float* a1, const uint4 bv, const uint4,
                                                floatx4& acc0, floatx4& acc1) {
    const float4 x = *reinterpret_cast<const float4*>(a0), y = *reinterpret_cast<const float4*>(a1);
    const float b0 = __uint_as_float(bv.x), b1 = __uint_as_float(bv.y), b2 = __uint_as_float(bv.z),
                b3 = __uint_as_float(bv.w);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(y.x, b0, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, b1, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(y.y, b1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, b2, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(y.z, b2, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, b3, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(y.w, b3, acc1, 0, 0, 0);
  }
};
template <> struct Frag<2> {
  static __device__ __forceinline__ floatx4 step(const float* a, const uint4* b, const uint4* blo, floatx4 acc) {
    float x[8];
    const float4 a0 = *reinterpret_cast<const float4*>(a);
    const float4 a1 = *reinterpret_cast<const float4*>(a + 4);
    x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w; x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
    uint4 ah, al;
    split8(x, ah, al);
    const uint4 bh = *b, bl = *blo;
    acc = mfma_bf16(al, bh, acc);
    acc = mfma_bf16(ah, bl, acc);
    return mfma_bf16(ah, bh, acc);
  }
  static __device__ __forceinline__ void split_a(const float* a, uint4& ah, uint4& al) {
    float x[8];
    const float4 a0 = *reinterpret_cast<const float4*>(a);
    const float4 a1 = *reinterpret_cast<const float4*>(a + 4);
    x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w; x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
    split8(x, ah, al);
  }
  static __device__ __forceinline__ void step2(const float* a0, const float* a1, const uint4* b, const uint4* blo,
                                               floatx4& acc0, floatx4& acc1) {
    step2v(a0, a1, *b, *blo, acc0, acc1);
  }
  static __device__ __forceinline__ void step1v(const float* a0, const uint4 bh, const uint4 bl, floatx4& acc0) {
    uint4 xh, xl;
    split_a(a0, xh, xl);
    acc0 = mfma_bf16(xl, bh, acc0);
    acc0 = mfma_bf16(xh, bl, acc0);
    acc0 = mfma_bf16(xh, bh, acc0);
  }
  static __device__ __forceinline__ void step2v(const float* a0, const float* a1, const uint4 bh, const uint4 bl,
                                                floatx4& acc0, floatx4& acc1) {
    uint4 xh, xl, yh, yl;
    split_a(a0, xh, xl);
    split_a(a1, yh, yl);
    acc0 = mfma_bf16(xl, bh, acc0);
    acc1 = mfma_bf16(yl, bh, acc1);
    acc0 = mfma_bf16(xh, bl, acc0);
    acc1 = mfma_bf16(yh, bl, acc1);
    acc0 = mfma_bf16(xh, bh, acc0);
    acc1 = mfma_bf16(yh, bh, acc1);
  }
};

// An A fragment held in MFMA-ready form, for reuse against many B fragments:
// load() reads the lane's LK elements (splitting them once in split mode) and
// mma() multiplies by one B fragment (hi at b, lo at blo in split mode), with
// the same products as Frag<MODE>::step.
template <int MODE> struct FragA;
template <> struct FragA<0> {
  float4 v;
  __device__ __forceinline__ void load(const float* a) { v = *reinterpret_cast<const float4*>(a); }
  __device__ __forceinline__ floatx4 mma(const uint4* b, const uint4*, floatx4 acc) const {
    const uint4 bv = *b;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.x, __uint_as_float(bv.x), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.y, __uint_as_float(bv.y), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v.z, __uint_as_float(bv.z), acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x4f32(v.w, __uint_as_float(bv.w), acc, 0, 0, 0);
  }
};
template <> struct FragA<2> {
  uint4 h, l;
  __device__ __forceinline__ void load(const float* a) { Frag<2>::split_a(a, h, l); }
  __device__ __forceinline__ floatx4 mma(const uint4* b, const uint4* blo, floatx4 acc) const {
    const uint4 bh = *b, bl = *blo;
    acc = mfma_bf16(l, bh, acc);
    acc = mfma_bf16(h, bl, acc);
    return mfma_bf16(h, bh, acc);
  }
};

// Reductions over the lane pairs (l, l ^ 16) and (l, l ^ 32) through the gfx950
// lane-swap instructions (VALU, no LDS round trip): each swap returns the lane's
// own value and its partner's, in an order that depends on the lane, so only
// order-free combinations (sum, max) are formed.
__device__ __forceinline__ float sum_xor16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float sum_xor32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float max_xor16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float max_xor32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// v from lane l ^ off, without an LDS round trip where the hardware allows:
// DPP quad permutes (off 1, 2) and row rotation by 8 (= xor 8 inside a 16-lane
// row), the lane swaps for off 16 and 32; other offsets use ds_bpermute.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_xor(float v, int off) {
  switch (off) {
    case 1: return dpp<0xB1>(v);             // quad_perm(1, 0, 3, 2)
    case 2: return dpp<0x4E>(v);             // quad_perm(2, 3, 0, 1)
    case 8: return dpp<0x128>(v);            // row_ror:8
    case 16: {
      const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
      return __uint_as_float((threadIdx.x & 16) ? r[0] : r[1]);
    }
    case 32: {
      const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
      return __uint_as_float((threadIdx.x & 32) ? r[0] : r[1]);
    }
    default: return __shfl_xor(v, off);
  }
}
// Sum over the 16 lanes of a row, the same in every lane of it (row rotations by
// 8 and 4 pair lanes symmetrically within the rotation classes, then the quads).
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp<0x128>(v);                        // row_ror:8
  v += dpp<0x124>(v);                        // row_ror:4
  v += dpp<0x4E>(v);
  v += dpp<0xB1>(v);
  return v;
}

// Maximum over the 16 lanes of a row, the same in every lane of it.
__device__ __forceinline__ float row_max16(float v) {
  v = fmaxf(v, dpp<0x128>(v));               // row_ror:8
  v = fmaxf(v, dpp<0x124>(v));               // row_ror:4
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0xB1>(v));
  return v;
}

// Normal CDF Phi(x) = (1 + erf(x / sqrt 2)) / 2 and the Gaussian factor exp(-x^2 / 2),
// branch-free: erfc(z) for z = |x| / sqrt 2 >= 0 from the rational-times-Gaussian
// form of Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26
// (Hastings), whose absolute error in erf is at most 1.5e-7; the Gaussian factor
// exp(-z^2) is the same exp(-x^2 / 2) that GELU's derivative needs.
__device__ __forceinline__ void phi_gauss(float x, float& cdf, float& gauss) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  gauss = __expf(-0.5f * x * x);
  const float half_erfc = 0.5f * poly * gauss;        // (1 - erf(z)) / 2
  cdf = x >= 0.f ? 1.0f - half_erfc : half_erfc;
}
__device__ __forceinline__ float gelu(float x) {
  float cdf, gauss;
  phi_gauss(x, cdf, gauss);
  return x * cdf;
}
// GELU(x) = x Phi(x) and its derivative Phi(x) + x phi(x), phi(x) = exp(-x^2/2) / sqrt(2 pi).
__device__ __forceinline__ void gelu_and_grad(float x, float& g, float& gp) {
  float cdf, gauss;
  phi_gauss(x, cdf, gauss);
  g = x * cdf;
  gp = fmaf(x * 0.39894228040143268f, gauss, cdf);
}
__device__ __forceinline__ float gelu_grad(float x) {
  float g, gp;
  gelu_and_grad(x, g, gp);
  return gp;
}

// log(1 + exp(x)) without overflow.
__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.0f) + log1pf(__expf(-fabsf(x))); }

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-8f; }


// Index v of the work item a workgroup runs, for a 1-D grid of T workgroups
// whose work items are numbered so that items sharing data are adjacent.  The
// hardware deals workgroups to the 8 XCDs round-robin by id (XCD x runs ids
// x, x+8, ...); this gives XCD x the contiguous range of items starting at
// x * floor(T/8) + min(x, T mod 8), so adjacent items run on one XCD, close in
// time, and share its L2.  A bijection of [0, T).
__device__ __forceinline__ int xcd_contiguous(int L, int T) {
  const int x = L & 7, slot = L >> 3, q = T >> 3, r = T & 7;
  return x * q + min(x, r) + slot;
}

}  // namespace fvan
