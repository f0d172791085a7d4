// Band+prefix masked attention for head widths 32 and 64 (the teacher-forced
// pass and its backward), in FP32 arithmetic on the stored Q/K/V.  The 16-wide
// heads take the MFMA kernels of attn_mfma.h; these kernels serve the wider
// heads of the patch-token models (SI, 3D EA settings: two heads at
// d_model 128), whose sequences are short, so their attention is a small part
// of the pass.  Inputs and outputs are those of the MFMA kernels:
//   forward: XM = X + O, LSE (log2 units of the scaled scores);
//   dQ:      DELTA = dO . O, dQ into dQKV and the feature-major copy T;
//   dK/dV:   dK, dV into dQKV and T.
// Thread layout: 4 lanes per row (query or key), each holding DH/4 consecutive
// dims of the head; dot products are summed over the 4 lanes with DPP quad
// permutes.  The other side's rows (keys, or queries for dK/dV) are staged in
// LDS 64 at a time as floats.
#pragma once

#include "attn_mfma.h"

namespace fvan {

constexpr int kGenThreads = 256;
constexpr int kGenRows = kGenThreads / 4;   // queries (keys) per workgroup
constexpr int kGenStage = 64;               // rows of the other side staged at a time

template <int DH>
__host__ __device__ constexpr float gen_inv_sqrt() {
  return DH == 16 ? 0.25f : DH == 32 ? 0.17677669529663688f : 0.125f;
}
template <int DH>
__host__ __device__ constexpr float gen_scale_log2() {
  return gen_inv_sqrt<DH>() * 1.4426950408889634f;
}

// Sum over the 4 lanes of a quad, the same in each of them.
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  return v;
}

// The DH/4 elements of a lane's slice of row r, head h, from a [rows][stride] array.
template <int Q4, typename T>
__device__ __forceinline__ void load_slice(const T* __restrict__ p, float* out) {
#pragma unroll
  for (int i = 0; i < Q4; ++i) out[i] = to_f(p[i]);
}

// ---------------------------------------------------------------- forward
// One workgroup = (64 queries, head, sample).
template <typename KT, int DH>
__global__ __launch_bounds__(kGenThreads) void attn_fwd_gen(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                            float* __restrict__ XM, float* __restrict__ LSE, int N,
                                                            int D, int H, int W, int P) {
  constexpr int Q4 = DH / 4;
  __shared__ __align__(16) float Ks[kGenStage][DH + 4];
  __shared__ __align__(16) float Vs[kGenStage][DH + 4];
  const AttnItem it = attn_item((N + kGenRows - 1) / kGenRows, H);
  const int t0 = it.tile * kGenRows, h = it.h, b = it.b;
  const int t1 = min(t0 + kGenRows, N);
  const int64_t rowbase = (int64_t)b * N;
  const int part = threadIdx.x & 3, tq = t0 + (threadIdx.x >> 2);
  const bool qok = tq < N;
  const int c0 = h * DH + part * Q4;                 // first column of this lane's slice
  float q[Q4], o[Q4];
#pragma unroll
  for (int i = 0; i < Q4; ++i) { q[i] = 0.f; o[i] = 0.f; }
  if (qok) {
    load_slice<Q4>(QKV + (rowbase + tq) * 3 * D + c0, q);
#pragma unroll
    for (int i = 0; i < Q4; ++i) q[i] *= gen_scale_log2<DH>();
  }
  const KeyRange kr(t0, t1, W, P);
  const QueryVis vis(kr, tq, W, qok);
  float mx = -INFINITY, l = 0.f;
  for (int v0 = 0; v0 < kr.nk; v0 += kGenStage) {
    const int nv = min(kGenStage, kr.nk - v0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv * DH; idx += kGenThreads) {
      const int key = idx / DH, d = idx % DH;
      const KT* kp = QKV + (rowbase + kr.pos(v0 + key)) * 3 * D + D + h * DH + d;
      Ks[key][d] = to_f(kp[0]);
      Vs[key][d] = to_f(kp[D]);
    }
    __syncthreads();
    for (int k0 = 0; k0 < nv; k0 += 16) {
      float s[16];
      float mnew = mx;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int key = k0 + u;
        float d = 0.f;
        if (key < nv) {
#pragma unroll
          for (int i = 0; i < Q4; ++i) d += q[i] * Ks[key][part * Q4 + i];
        }
        d = quad_sum(d);
        s[u] = (key < nv) && vis(v0 + key) ? d : -INFINITY;
        mnew = fmaxf(mnew, s[u]);
      }
      const float corr = mnew == -INFINITY ? 1.f : __builtin_amdgcn_exp2f(mx - mnew);
      l *= corr;
#pragma unroll
      for (int i = 0; i < Q4; ++i) o[i] *= corr;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (s[u] == -INFINITY) continue;
        const float p = __builtin_amdgcn_exp2f(s[u] - mnew);
        l += p;
#pragma unroll
        for (int i = 0; i < Q4; ++i) o[i] += p * Vs[k0 + u][part * Q4 + i];
      }
      mx = mnew;
    }
  }
  if (qok) {
    const int64_t r = rowbase + tq;
    const float inv = 1.0f / l;
#pragma unroll
    for (int i = 0; i < Q4; ++i) XM[r * D + c0 + i] = X[r * D + c0 + i] + o[i] * inv;
    if (part == 0) LSE[r * H + h] = mx + __log2f(l);
  }
}

// ---------------------------------------------------------------- backward: dQ
// One workgroup = (64 queries, head, sample).  O is recovered as XM - X.
template <typename KT, typename AT, int DH>
__global__ __launch_bounds__(kGenThreads) void attn_bwd_dq_gen(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                               const float* __restrict__ XM,
                                                               const float* __restrict__ dO,
                                                               const float* __restrict__ LSE,
                                                               float* __restrict__ DELTA, AT* __restrict__ dQKV,
                                                               AT* __restrict__ T, int64_t ldT, int N, int D, int H,
                                                               int W, int P) {
  constexpr int Q4 = DH / 4;
  __shared__ __align__(16) float Ks[kGenStage][DH + 4];
  __shared__ __align__(16) float Vs[kGenStage][DH + 4];
  const AttnItem it = attn_item((N + kGenRows - 1) / kGenRows, H);
  const int t0 = it.tile * kGenRows, h = it.h, b = it.b;
  const int t1 = min(t0 + kGenRows, N);
  const int64_t rowbase = (int64_t)b * N;
  const int part = threadIdx.x & 3, tq = t0 + (threadIdx.x >> 2);
  const bool qok = tq < N;
  const int c0 = h * DH + part * Q4;
  const int64_t r = rowbase + tq;
  float q[Q4], g[Q4], dq[Q4];
  float delta = 0.f, lse = 0.f;
#pragma unroll
  for (int i = 0; i < Q4; ++i) { q[i] = 0.f; g[i] = 0.f; dq[i] = 0.f; }
  if (qok) {
    load_slice<Q4>(QKV + r * 3 * D + c0, q);
#pragma unroll
    for (int i = 0; i < Q4; ++i) {
      q[i] *= gen_scale_log2<DH>();
      g[i] = dO[r * D + c0 + i];
      delta += g[i] * (XM[r * D + c0 + i] - X[r * D + c0 + i]);
    }
    lse = LSE[r * H + h];
  }
  delta = quad_sum(delta);
  if (qok && part == 0) DELTA[r * H + h] = delta;
  const KeyRange kr(t0, t1, W, P);
  const QueryVis vis(kr, tq, W, qok);
  for (int v0 = 0; v0 < kr.nk; v0 += kGenStage) {
    const int nv = min(kGenStage, kr.nk - v0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nv * DH; idx += kGenThreads) {
      const int key = idx / DH, d = idx % DH;
      const KT* kp = QKV + (rowbase + kr.pos(v0 + key)) * 3 * D + D + h * DH + d;
      Ks[key][d] = to_f(kp[0]);
      Vs[key][d] = to_f(kp[D]);
    }
    __syncthreads();
    for (int key = 0; key < nv; ++key) {
      float s = 0.f, dp = 0.f;
#pragma unroll
      for (int i = 0; i < Q4; ++i) {
        s += q[i] * Ks[key][part * Q4 + i];
        dp += g[i] * Vs[key][part * Q4 + i];
      }
      s = quad_sum(s);
      dp = quad_sum(dp);
      const float p = vis(v0 + key) ? __builtin_amdgcn_exp2f(s - lse) : 0.f;
      const float ds = p * (dp - delta);
#pragma unroll
      for (int i = 0; i < Q4; ++i) dq[i] += ds * Ks[key][part * Q4 + i];
    }
  }
  if (qok) {
#pragma unroll
    for (int i = 0; i < Q4; ++i) {
      const AT v = from_f<AT>(dq[i] * gen_inv_sqrt<DH>());
      dQKV[r * 3 * D + c0 + i] = v;
      T[(int64_t)(c0 + i) * ldT + r] = v;
    }
  }
}

// ---------------------------------------------------------------- backward: dK, dV
// One workgroup = (64 keys, head, sample).  The queries that see key j are
// i >= j with i - j <= W, or every i >= j when j < P.
template <typename KT, typename AT, int DH>
__global__ __launch_bounds__(kGenThreads) void attn_bwd_dkv_gen(const KT* __restrict__ QKV,
                                                                const float* __restrict__ dO,
                                                                const float* __restrict__ LSE,
                                                                const float* __restrict__ DELTA,
                                                                AT* __restrict__ dQKV, AT* __restrict__ T, int64_t ldT,
                                                                int N, int D, int H, int W, int P) {
  constexpr int Q4 = DH / 4;
  __shared__ __align__(16) float Qs[kGenStage][DH + 4];
  __shared__ __align__(16) float Gs[kGenStage][DH + 4];
  __shared__ float Ls[kGenStage], Ds[kGenStage];
  const AttnItem it = attn_item((N + kGenRows - 1) / kGenRows, H);
  const int j0 = it.tile * kGenRows, h = it.h, b = it.b;
  const int j1 = min(j0 + kGenRows, N);
  const int64_t rowbase = (int64_t)b * N;
  const int part = threadIdx.x & 3, j = j0 + (threadIdx.x >> 2);
  const bool kok = j < N;
  const int c0 = h * DH + part * Q4;
  float k[Q4], v[Q4], dk[Q4], dv[Q4];
#pragma unroll
  for (int i = 0; i < Q4; ++i) { k[i] = 0.f; v[i] = 0.f; dk[i] = 0.f; dv[i] = 0.f; }
  if (kok) {
    load_slice<Q4>(QKV + (rowbase + j) * 3 * D + D + c0, k);
    load_slice<Q4>(QKV + (rowbase + j) * 3 * D + 2 * D + c0, v);
  }
  // queries of the tile's keys: [j0, i_end)
  const int i_end = j0 < P ? N : min(N, j1 - 1 + W + 1);
  for (int i0 = j0; i0 < i_end; i0 += kGenStage) {
    const int nq = min(kGenStage, i_end - i0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nq * DH; idx += kGenThreads) {
      const int qi = idx / DH, d = idx % DH;
      const int64_t rq = rowbase + i0 + qi;
      Qs[qi][d] = to_f(QKV[rq * 3 * D + h * DH + d]);
      Gs[qi][d] = dO[rq * D + h * DH + d];
    }
    for (int qi = threadIdx.x; qi < nq; qi += kGenThreads) {
      Ls[qi] = LSE[(rowbase + i0 + qi) * H + h];
      Ds[qi] = DELTA[(rowbase + i0 + qi) * H + h];
    }
    __syncthreads();
    for (int qi = 0; qi < nq; ++qi) {
      float s = 0.f, dp = 0.f;
#pragma unroll
      for (int i = 0; i < Q4; ++i) {
        s += Qs[qi][part * Q4 + i] * k[i];
        dp += Gs[qi][part * Q4 + i] * v[i];
      }
      s = quad_sum(s) * gen_scale_log2<DH>();
      dp = quad_sum(dp);
      const float p = kok && visible(i0 + qi, j, W, P) ? __builtin_amdgcn_exp2f(s - Ls[qi]) : 0.f;
      const float ds = p * (dp - Ds[qi]);
#pragma unroll
      for (int i = 0; i < Q4; ++i) {
        dk[i] += ds * Qs[qi][part * Q4 + i];
        dv[i] += p * Gs[qi][part * Q4 + i];
      }
    }
  }
  if (kok) {
    const int64_t r = rowbase + j;
#pragma unroll
    for (int i = 0; i < Q4; ++i) {
      const AT kv = from_f<AT>(dk[i] * gen_inv_sqrt<DH>()), vv = from_f<AT>(dv[i]);
      dQKV[r * 3 * D + D + c0 + i] = kv;
      dQKV[r * 3 * D + 2 * D + c0 + i] = vv;
      T[(int64_t)(D + c0 + i) * ldT + r] = kv;
      T[(int64_t)(2 * D + c0 + i) * ldT + r] = vv;
    }
  }
}

}  // namespace fvan
