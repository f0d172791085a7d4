// Band+prefix masked attention (forward and backward) for the split-precision
// mode (d_head = 16), on the FP16 Q, K and V that mode stores.
//
// A product of two FP16 numbers is exact in FP32, so the scores S^T = K Q^T
// come from one 16x16x16 FP16 MFMA per 16x16 tile with FP32 accumulation, and
// the scale 1/sqrt(16) * log2(e) is applied in FP32 afterwards.  For O^T = V^T P^T
// the probabilities are split into FP16 hi + lo (P - hi is exact in FP32, its
// rounding to FP16 leaves a relative error near 2^-22 of P) and one 16x16x32
// FP16 MFMA forms V^T [P_hi ; P_lo] with V^T given twice along the contraction.
//
// Tiles of 16 keys x 16 queries are classed per wave from scalars: empty (no
// query of the wave sees a key of the tile: skipped), full (every query sees
// every key: no per-element mask) or partial (per-element mask).  Only the tiles
// on the diagonal, on the band's far edge and on the prefix / band seam are
// partial.  The running maximum starts from a finite floor, so fully masked
// rows need no guards in the exponentials.
//
// The backward keeps the BF16 hi/lo split for every product with a gradient
// operand (dO, dP, dS: FP16's exponent range is too narrow for them), arranged so
// that no operand is shuffled in registers: with the 16x16x32 contraction index
// over (part, dim), a product a.b is
//   [a_h | a_l] . [b_h ; b_h]  +  [a_h | a_l] . [b_l ; 0]
// (a_h b_h + a_l b_h + a_h b_l; the dropped a_l b_l is below 2^-16 relative), where
// [a_h | a_l] is the layout staged in LDS and {[b_h | b_h], [b_l | 0]} is built once
// in registers (SplitDup), for a loop-invariant operand or one formed per tile.
//
// The 16x16x16 and 16x16x32 products never feed each other's accumulators: a
// 16x16x32 result fed straight into a dependent 16x16x16 MFMA came out wrong with
// this toolchain, so every score tile starts from a zero accumulator and every
// accumulator chain uses one opcode.
#pragma once

#include "attn_mfma.h"

namespace fvan {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// FP16 hi/lo split of four FP32 values as the 8-element B operand [hi ; lo].
__device__ __forceinline__ half2_t pkrtz(float a, float b) {
  return __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(a, b));
}
__device__ __forceinline__ half8_t split_f16x4(float a, float b, float c, float d) {
  const half2_t h0 = pkrtz(a, b), h1 = pkrtz(c, d);
  const half2_t l0 = pkrtz(a - (float)h0.x, b - (float)h0.y);
  const half2_t l1 = pkrtz(c - (float)h1.x, d - (float)h1.y);
  return half8_t{h0.x, h0.y, h1.x, h1.y, l0.x, l0.y, l1.x, l1.y};
}

// {[x_h | x_h], [x_l | 0]} of four FP32 values (the register side of a split product).
struct SplitDup {
  bf16x8 hh, l0;
};
__device__ __forceinline__ SplitDup split_dup(float a, float b, float c, float d) {
  const SplitBf16x4 t = AOp<2>::make(a, b, c, d);
  const bf16x4 z = {(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
  return SplitDup{__builtin_shufflevector(t.h, t.h, 0, 1, 2, 3, 4, 5, 6, 7),
                  __builtin_shufflevector(t.l, z, 0, 1, 2, 3, 4, 5, 6, 7)};
}
__device__ __forceinline__ bf16x8 as_hl(const SplitBf16x4& t) {
  return __builtin_shufflevector(t.h, t.l, 0, 1, 2, 3, 4, 5, 6, 7);
}
// acc += A B with A staged as [a_h | a_l] and B = split_dup(b)
__device__ __forceinline__ floatx4 mma_hl_dup(const SplitBf16x4& a, const SplitDup& b, floatx4 acc) {
  const bf16x8 a8 = as_hl(a);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b.hh, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a8, b.l0, acc, 0, 0, 0);
}
// acc += A B with A = split_dup(a) and B staged as [b_h ; b_l]
__device__ __forceinline__ floatx4 mma_dup_hl(const SplitDup& a, const SplitBf16x4& b, floatx4 acc) {
  const bf16x8 b8 = as_hl(b);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hh, b8, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l0, b8, acc, 0, 0, 0);
}

constexpr float kMaxFloor = -1e30f;   // finite start of the running maximum (unscaled score units)
constexpr int kKhStride = 20;         // K rows in LDS: 16 halves + 4 (40 bytes)
constexpr int kVtStride = kKeyChunk + 8;   // V^T rows in LDS: one per dim

// One workgroup = (64 queries, head, sample), wave w owns queries t0+16w..+15, as
// in the FP32 kernel; writes XM = X + O and LSE (log2 units, scaled scores).
static __global__ __launch_bounds__(kFwdThreads) void attn_fwd_f16(const _Float16* __restrict__ QKV,
                                                            const float* __restrict__ X, float* __restrict__ XM,
                                                            float* __restrict__ LSE, int N, int D, int H, int W,
                                                            int P) {
  __shared__ __align__(16) _Float16 Kh[kKeyChunk][kKhStride];   // K, A layout rows
  __shared__ __align__(16) _Float16 Vt[16][kVtStride];          // V^T: [dim][key]
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the tile classes below are scalar
  constexpr int R = attn_rows(kFwdThreads);
  const AttnItem it = attn_item((N + R - 1) / R, H);
  const int t0 = it.tile * R, h = it.h, b = it.b;
  const int t1 = min(t0 + R, N);
  const int64_t rowbase = (int64_t)b * N;
  const int tq = t0 + 16 * wave + c;
  const bool qok = tq < N;
  half4_t qh = {0, 0, 0, 0};               // B operand Q^T[dim 4g..4g+3][query c]
  if (qok) qh = *reinterpret_cast<const half4_t*>(QKV + (rowbase + tq) * 3 * D + h * 16 + 4 * g);
  const KeyRange kr(t0, t1, W, P);
  const QueryVis vis(kr, tq, W, qok);
  // the wave's queries tw0..tw1 and the virtual keys any of them sees: [0, wa1), [wb0, wb1)
  const int tw0 = t0 + 16 * wave, tw1 = min(tw0 + 15, N - 1);
  const int wa1 = tw0 < N ? min(kr.pend, tw1 + 1) : 0;
  const int wb0 = kr.pend + max(0, tw0 - W - kr.bstart);
  const int wb1 = tw0 < N ? kr.pend + tw1 - kr.bstart + 1 : 0;
  // staging: thread -> (key tid / 2, dims 8 (tid & 1) ..), 16 bytes of K and of V
  const int skey = tid >> 1, sch = (tid & 1) * 8;
  static_assert(kKeyChunk * 2 == kFwdThreads, "one K and one V chunk per thread");
  uint4 kraw = make_uint4(0u, 0u, 0u, 0u), vraw = kraw;
  auto fetch = [&](int v0) {
    kraw = make_uint4(0u, 0u, 0u, 0u);
    vraw = kraw;
    if (skey < kr.nk - v0) {
      const _Float16* kp = QKV + (rowbase + kr.pos(v0 + skey)) * 3 * D + D + h * 16 + sch;
      kraw = *reinterpret_cast<const uint4*>(kp);
      vraw = *reinterpret_cast<const uint4*>(kp + D);
    }
  };
  fetch(0);
  float mx = kMaxFloor, l = 0.f;
  floatx4 o = {0.f, 0.f, 0.f, 0.f};        // O^T[dim 4g+i][query c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();                        // the previous chunk's reads are done
    {
      uint2* kd = reinterpret_cast<uint2*>(&Kh[skey][sch]);
      kd[0] = make_uint2(kraw.x, kraw.y);
      kd[1] = make_uint2(kraw.z, kraw.w);
      const uint32_t vw[4] = {vraw.x, vraw.y, vraw.z, vraw.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        Vt[sch + 2 * e][skey] = __builtin_bit_cast(half2_t, vw[e]).x;
        Vt[sch + 2 * e + 1][skey] = __builtin_bit_cast(half2_t, vw[e]).y;
      }
    }
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) fetch(v0 + kKeyChunk);
    for (int kt0 = 0; kt0 < nv; kt0 += 64) {
      // class of each 16-key tile for this wave: 0 empty, 1 partial, 2 full
      int cls[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kl = kt0 + 16 * u, vb = v0 + kl;
        const bool any = (kl < nv) & ((vb < wa1) | ((vb + 16 > wb0) & (vb < wb1)));
        bool full = false;
        if (kl + 16 <= nv) {
          if (vb + 16 <= kr.pend) {
            full = vb + 15 <= tw0;                                        // prefix keys j <= t
          } else if (vb >= kr.pend) {
            const int p0 = kr.bstart + (vb - kr.pend);
            full = (p0 + 15 <= tw0) & (tw1 - p0 <= W);                    // band keys t - W <= j <= t
          }
        }
        cls[u] = any ? (full ? 2 : 1) : 0;
      }
      if ((cls[0] | cls[1] | cls[2] | cls[3]) == 0) continue;
      float s[16];
      float bmax = kMaxFloor;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kl = kt0 + 16 * u;
        if (cls[u] == 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i) s[4 * u + i] = -INFINITY;
          continue;
        }
        const half4_t ka = *reinterpret_cast<const half4_t*>(&Kh[kl + c][4 * g]);
        const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x16f16(ka, qh, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        if (cls[u] == 2) {
#pragma unroll
          for (int i = 0; i < 4; ++i) s[4 * u + i] = acc[i];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) s[4 * u + i] = vis(v0 + kl + 4 * g + i) ? acc[i] : -INFINITY;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) bmax = fmaxf(bmax, s[4 * u + i]);
      }
      bmax = max_xor32(max_xor16(bmax));
      const float mn = fmaxf(mx, bmax);
      const float ms = mn * kScaleLog2;
      const float corr = __builtin_amdgcn_exp2f((mx - mn) * kScaleLog2);
      float ps = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        s[i] = __builtin_amdgcn_exp2f(fmaf(s[i], kScaleLog2, -ms));   // masked: exp2(-inf) = 0
        ps += s[i];
      }
      ps = sum_xor32(sum_xor16(ps));
      l = l * corr + ps;
      mx = mn;
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] *= corr;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (cls[u] == 0) continue;
        const int kl = kt0 + 16 * u;
        // A = V^T[dim c][keys kl+4g..+3] twice along k, B = [P_hi ; P_lo] of those keys, query c
        const half4_t va = *reinterpret_cast<const half4_t*>(&Vt[c][kl + 4 * g]);
        const half8_t a8 = __builtin_shufflevector(va, va, 0, 1, 2, 3, 0, 1, 2, 3);
        o = __builtin_amdgcn_mfma_f32_16x16x32_f16(a8, split_f16x4(s[4 * u], s[4 * u + 1], s[4 * u + 2], s[4 * u + 3]),
                                                  o, 0, 0, 0);
      }
    }
  }
  if (qok) {
    const float inv = 1.0f / l;
    const int64_t r = rowbase + tq;
    const float4 xv = *reinterpret_cast<const float4*>(X + r * D + h * 16 + 4 * g);
    *reinterpret_cast<float4*>(XM + r * D + h * 16 + 4 * g) =
        make_float4(xv.x + o[0] * inv, xv.y + o[1] * inv, xv.z + o[2] * inv, xv.w + o[3] * inv);
    if (g == 0) LSE[r * H + h] = mx * kScaleLog2 + __log2f(l);
  }
}

// ---------------------------------------------------------------- backward: dQ
// One workgroup = (128 queries, head, sample), as in the FP32 kernel.  O is
// recovered as XM - X.  Writes DELTA = dO . O, dQ (scaled) into dQKV and the
// feature-major copy T.
static __global__ __launch_bounds__(kDqThreads) void attn_bwd_dq_f16(const _Float16* __restrict__ QKV,
                                                              const float* __restrict__ X,
                                                              const float* __restrict__ XM,
                                                              const float* __restrict__ dO,
                                                              const float* __restrict__ LSE,
                                                              float* __restrict__ DELTA, float* __restrict__ dQKV,
                                                              float* __restrict__ T, int64_t ldT, int N, int D, int H,
                                                              int W, int P) {
  typedef SplitBf16x4 OT;
  __shared__ __align__(16) _Float16 Kh[kKeyChunk][kKhStride];   // K rows (S^T = K Q^T)
  __shared__ __align__(16) float Kf[kKeyChunk][20];             // K as floats, for Kb
  __shared__ __align__(16) OT Va[kKeyChunk][kAStride];          // V, A layout (dP^T = V dO^T)
  __shared__ __align__(16) OT Kb[16][kKeyChunk / 4 + 1];        // K, B layout (dQ = dS K)
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the tile classes below are scalar
  constexpr int R = attn_rows(kDqThreads);
  const AttnItem it = attn_item((N + R - 1) / R, H);
  const int t0 = it.tile * R, h = it.h, b = it.b;
  const int t1 = min(t0 + R, N);
  const int64_t rowbase = (int64_t)b * N;
  const KeyRange kr(t0, t1, W, P);
  // staging: threads [0, 256) take 16 bytes of K, threads [256, 512) 16 bytes of V,
  // of key (tid % 256) / 2, dims 8 (tid & 1) ..
  static_assert(kKeyChunk * 4 == kDqThreads, "one K or V chunk per thread");
  const bool isv = tid >= 2 * kKeyChunk;
  const int skey = (tid & (2 * kKeyChunk - 1)) >> 1, sch = (tid & 1) * 8;
  uint4 raw = make_uint4(0u, 0u, 0u, 0u);
  auto fetch = [&](int v0) {
    raw = make_uint4(0u, 0u, 0u, 0u);
    if (skey < kr.nk - v0)
      raw = *reinterpret_cast<const uint4*>(QKV + (rowbase + kr.pos(v0 + skey)) * 3 * D + (isv ? 2 : 1) * D + h * 16 +
                                            sch);
  };
  fetch(0);
  const int tq = t0 + 16 * wave + c;
  const bool qok = tq < N;
  const QueryVis vis(kr, tq, W, qok);
  const int tw0 = t0 + 16 * wave, tw1 = min(tw0 + 15, N - 1);
  const int wa1 = tw0 < N ? min(kr.pend, tw1 + 1) : 0;
  const int wb0 = kr.pend + max(0, tw0 - W - kr.bstart);
  const int wb1 = tw0 < N ? kr.pend + tw1 - kr.bstart + 1 : 0;
  const int64_t r = rowbase + tq;
  half4_t qh = {0, 0, 0, 0};
  float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float lse = 0.f, delta = 0.f;
  if (qok) {
    qh = *reinterpret_cast<const half4_t*>(QKV + r * 3 * D + h * 16 + 4 * g);
    g4 = *reinterpret_cast<const float4*>(dO + r * D + h * 16 + 4 * g);
    const float4 xm = *reinterpret_cast<const float4*>(XM + r * D + h * 16 + 4 * g);
    const float4 xx = *reinterpret_cast<const float4*>(X + r * D + h * 16 + 4 * g);
    delta = g4.x * (xm.x - xx.x) + g4.y * (xm.y - xx.y) + g4.z * (xm.z - xx.z) + g4.w * (xm.w - xx.w);
    lse = LSE[r * H + h];
  }
  delta = sum_xor32(sum_xor16(delta));
  if (qok && g == 0) DELTA[r * H + h] = delta;
  const SplitDup gB = split_dup(g4.x, g4.y, g4.z, g4.w);   // dO^T[dim 4g..][query c]
  floatx4 dq = {0.f, 0.f, 0.f, 0.f};                       // dQ[query 16w+4g+i][dim c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();
    {
      Chunk<_Float16> ch;
      ch.unpack(raw);
      if (isv) {
        Va[skey][sch / 4] = AOp<2>::make(ch.v[0], ch.v[1], ch.v[2], ch.v[3]);
        Va[skey][sch / 4 + 1] = AOp<2>::make(ch.v[4], ch.v[5], ch.v[6], ch.v[7]);
      } else {
        uint2* kd = reinterpret_cast<uint2*>(&Kh[skey][sch]);
        kd[0] = make_uint2(raw.x, raw.y);
        kd[1] = make_uint2(raw.z, raw.w);
        *reinterpret_cast<float4*>(&Kf[skey][sch]) = make_float4(ch.v[0], ch.v[1], ch.v[2], ch.v[3]);
        *reinterpret_cast<float4*>(&Kf[skey][sch + 4]) = make_float4(ch.v[4], ch.v[5], ch.v[6], ch.v[7]);
      }
    }
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) fetch(v0 + kKeyChunk);
    build_b<2, kKeyChunk, kDqThreads>(Kf, Kb);
    __syncthreads();
    for (int kb = 0; kb < nv; kb += 16) {
      const int vb = v0 + kb;
      if ((vb >= wa1) & ((vb + 16 <= wb0) | (vb >= wb1))) continue;   // no query of the wave sees these keys
      bool full = false;
      if (kb + 16 <= nv) {
        if (vb + 16 <= kr.pend) {
          full = vb + 15 <= tw0;
        } else if (vb >= kr.pend) {
          const int p0 = kr.bstart + (vb - kr.pend);
          full = (p0 + 15 <= tw0) & (tw1 - p0 <= W);
        }
      }
      const half4_t ka = *reinterpret_cast<const half4_t*>(&Kh[kb + c][4 * g]);
      const floatx4 sa = __builtin_amdgcn_mfma_f32_16x16x16f16(ka, qh, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const floatx4 pa = mma_hl_dup(Va[kb + c][g], gB, floatx4{0.f, 0.f, 0.f, 0.f});   // dP^T[key 4g+i][query c]
      float p[4], ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) p[i] = __builtin_amdgcn_exp2f(fmaf(sa[i], kScaleLog2, -lse));
      // one branch on the wave-uniform class around all four masks: per element the
      // compiler would turn the test into selects computed for full tiles too
      if (!full) {
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] = vis(vb + 4 * g + i) ? p[i] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) ds[i] = p[i] * (pa[i] - delta);
      // dQ[query][dim] += dS[query][key] K[key][dim]; the lane's dS is the A layout of dS
      dq = mma_dup_hl(split_dup(ds[0], ds[1], ds[2], ds[3]), Kb[c][kb / 4 + g], dq);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int tqi = t0 + 16 * wave + 4 * g + i;
    if (tqi < N) {
      const int64_t ri = rowbase + tqi;
      const float v = dq[i] * 0.25f;
      dQKV[ri * 3 * D + h * 16 + c] = v;
      T[(int64_t)(h * 16 + c) * ldT + ri] = v;
    }
  }
}

// ---------------------------------------------------------------- backward: dK, dV
// One workgroup = (head, 64 keys, sample), wave w owns keys j0+16w..+15 and loops
// over the 64-query blocks that can see the tile, as in the FP32 kernel.
static __global__ __launch_bounds__(kDkvThreads) void attn_bwd_dkv_f16(const _Float16* __restrict__ QKV,
                                                                const float* __restrict__ dO,
                                                                const float* __restrict__ LSE,
                                                                const float* __restrict__ DELTA,
                                                                float* __restrict__ dQKV, float* __restrict__ T,
                                                                int64_t ldT, int N, int D, int H, int W, int P) {
  typedef SplitBf16x4 OT;
  constexpr int QB = attn_rows(kDkvThreads);
  __shared__ __align__(16) _Float16 Qh[QB][kKhStride];   // Q rows (S = Q K^T)
  __shared__ __align__(16) float Qf[QB][20];
  __shared__ __align__(16) float Gf[QB][20];
  __shared__ __align__(16) OT Ga[QB][kAStride];          // dO, A layout (dP = dO V^T)
  __shared__ __align__(16) OT Qb[16][QB / 4 + 1];        // Q, B layout (dK += dS^T Q)
  __shared__ __align__(16) OT Gb[16][QB / 4 + 1];        // dO, B layout (dV += P^T dO)
  __shared__ __align__(16) float Ls[QB];
  __shared__ __align__(16) float Ds[QB];
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the tile classes below are scalar
  const AttnItem it = attn_item((N + QB - 1) / QB, H);
  const int h = it.h, j0 = it.tile * QB, b = it.b;
  const int j1 = min(j0 + QB, N);
  const int64_t rowbase = (int64_t)b * N;
  const int jk = j0 + 16 * wave + c;               // this lane's key (B-operand column)
  const bool kok = jk < N;
  half4_t kh = {0, 0, 0, 0};
  float4 v4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (kok) {
    const _Float16* kp = QKV + (rowbase + jk) * 3 * D + D + h * 16 + 4 * g;
    kh = *reinterpret_cast<const half4_t*>(kp);
    const half4_t vh = *reinterpret_cast<const half4_t*>(kp + D);
    v4 = make_float4((float)vh.x, (float)vh.y, (float)vh.z, (float)vh.w);
  }
  const SplitDup vB = split_dup(v4.x, v4.y, v4.z, v4.w);   // V^T[dim 4g..][key c]
  const int qend = j0 < P ? N : min(N, j1 + W);
  const int qw = kok ? max(0, min(jk < P ? N : jk + W + 1, qend) - jk) : 0;
  const int jw0 = j0 + 16 * wave;
  const int qhi_w = jw0 >= N ? jw0 : (jw0 < P ? qend : min(qend, min(N - 1, jw0 + 15) + W + 1));
  // the wave's keys all lie in the prefix, or all in the band (else its tiles are partial)
  const bool wpre = jw0 + 15 < P, wband = jw0 >= P, wkeys = jw0 + 15 < N;
  // staging roles as in the FP32 kernel: dO row tid/4, quarter tid%4; Q row tid/2,
  // dims 8 (tid & 1) .. (tid < 2 QB); LSE (tid < QB) or DELTA (QB <= tid < 2 QB)
  static_assert(QB * 4 == kDkvThreads, "dK/dV staging: one dO quarter-row per thread");
  const int gr = tid >> 2, gc = (tid & 3) * 4;
  const int qr = tid >> 1, qc = (tid & 1) * 8;
  const bool qthr = tid < 2 * QB;
  const int sr = tid % QB;
  float4 graw = make_float4(0.f, 0.f, 0.f, 0.f);
  uint4 qraw = make_uint4(0u, 0u, 0u, 0u);
  float sraw = 0.f;
  auto fetch = [&](int i0) {
    const int nq = min(QB, qend - i0);
    graw = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gr < nq) graw = *reinterpret_cast<const float4*>(dO + (rowbase + i0 + gr) * D + h * 16 + gc);
    qraw = make_uint4(0u, 0u, 0u, 0u);
    if (qthr & (qr < nq)) qraw = *reinterpret_cast<const uint4*>(QKV + (rowbase + i0 + qr) * 3 * D + h * 16 + qc);
    sraw = 0.f;
    if ((tid < 2 * QB) & (sr < nq)) sraw = (tid < QB ? LSE : DELTA)[(rowbase + i0 + sr) * H + h];
  };
  fetch(j0);
  floatx4 dk = {0.f, 0.f, 0.f, 0.f}, dv = {0.f, 0.f, 0.f, 0.f};   // [key 16w+4g+i][dim c]
  for (int i0 = j0; i0 < qend; i0 += QB) {
    const int nq = min(QB, qend - i0);
    __syncthreads();                                 // the previous block's reads are done
    *reinterpret_cast<float4*>(&Gf[gr][gc]) = graw;
    if (qthr) {
      uint2* qd = reinterpret_cast<uint2*>(&Qh[qr][qc]);
      qd[0] = make_uint2(qraw.x, qraw.y);
      qd[1] = make_uint2(qraw.z, qraw.w);
      Chunk<_Float16> ch;
      ch.unpack(qraw);
      *reinterpret_cast<float4*>(&Qf[qr][qc]) = make_float4(ch.v[0], ch.v[1], ch.v[2], ch.v[3]);
      *reinterpret_cast<float4*>(&Qf[qr][qc + 4]) = make_float4(ch.v[4], ch.v[5], ch.v[6], ch.v[7]);
    }
    if (tid < QB) Ls[sr] = sraw;
    else if (tid < 2 * QB) Ds[sr] = sraw;
    __syncthreads();
    if (i0 + QB < qend) fetch(i0 + QB);
    build_a<2, QB, kDkvThreads>(Gf, Ga);
    build_b<2, QB, kDkvThreads>(Qf, Qb);
    build_b<2, QB, kDkvThreads>(Gf, Gb);
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += 16) {
      const int iq0 = i0 + q0;
      if ((iq0 + 16 <= jw0) | (iq0 >= qhi_w)) continue;   // no key of the wave sees these queries
      // every (query, key) pair of the tile visible: keys before every query, and
      // within the band of every query unless all are prefix keys
      const bool full = wkeys & (iq0 + 16 <= qend) & (jw0 + 15 <= iq0) & (wpre | (wband & (iq0 + 15 - jw0 <= W)));
      const half4_t qa = *reinterpret_cast<const half4_t*>(&Qh[q0 + c][4 * g]);
      const floatx4 sa = __builtin_amdgcn_mfma_f32_16x16x16f16(qa, kh, floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const floatx4 pa = mma_hl_dup(Ga[q0 + c][g], vB, floatx4{0.f, 0.f, 0.f, 0.f});   // dP[q 4g+i][key c]
      const float4 l4 = *reinterpret_cast<const float4*>(&Ls[q0 + 4 * g]);
      const float4 d4 = *reinterpret_cast<const float4*>(&Ds[q0 + 4 * g]);
      const float lq[4] = {l4.x, l4.y, l4.z, l4.w}, dl[4] = {d4.x, d4.y, d4.z, d4.w};
      float p[4], ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) p[i] = __builtin_amdgcn_exp2f(fmaf(sa[i], kScaleLog2, -lq[i]));
      if (!full) {   // one uniform branch around all four masks, as in the dQ kernel
#pragma unroll
        for (int i = 0; i < 4; ++i) p[i] = (unsigned)(iq0 + 4 * g + i - jk) < (unsigned)qw ? p[i] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) ds[i] = p[i] * (pa[i] - dl[i]);
      dv = mma_dup_hl(split_dup(p[0], p[1], p[2], p[3]), Gb[c][q0 / 4 + g], dv);      // dV += P^T dO
      dk = mma_dup_hl(split_dup(ds[0], ds[1], ds[2], ds[3]), Qb[c][q0 / 4 + g], dk);  // dK += dS^T Q
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int jj = j0 + 16 * wave + 4 * g + i;
    if (jj < N) {
      const int64_t rj = rowbase + jj;
      const float kvv = dk[i] * 0.25f;
      const float vvv = dv[i];
      dQKV[rj * 3 * D + D + h * 16 + c] = kvv;
      dQKV[rj * 3 * D + 2 * D + h * 16 + c] = vvv;
      T[(int64_t)(D + h * 16 + c) * ldT + rj] = kvv;
      T[(int64_t)(2 * D + h * 16 + c) * ldT + rj] = vvv;
    }
  }
}

}  // namespace fvan
