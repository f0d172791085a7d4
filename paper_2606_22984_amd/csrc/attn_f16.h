// Band+prefix masked attention forward for the split-precision mode (d_head = 16),
// on the FP16 Q, K and V that mode stores.
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

constexpr float kMaxFloor = -1e30f;   // finite start of the running maximum (unscaled score units)
constexpr int kKhStride = 20;         // K rows in LDS: 16 halves + 4 (40 bytes)
constexpr int kVtStride = kKeyChunk + 8;   // V^T rows in LDS: one per dim

// One workgroup = (64 queries, head, sample), wave w owns queries t0+16w..+15, as
// in the FP32 kernel; writes XM = X + O and LSE (log2 units, scaled scores).
__global__ __launch_bounds__(kFwdThreads) void attn_fwd_f16(const _Float16* __restrict__ QKV,
                                                            const float* __restrict__ X, float* __restrict__ XM,
                                                            float* __restrict__ LSE, int N, int D, int H, int W,
                                                            int P) {
  __shared__ __align__(16) _Float16 Kh[kKeyChunk][kKhStride];   // K, A layout rows
  __shared__ __align__(16) _Float16 Vt[16][kVtStride];          // V^T: [dim][key]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
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

}  // namespace fvan
