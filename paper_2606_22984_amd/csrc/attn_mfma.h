// Band+prefix masked attention on MFMA for the teacher-forced pass and its
// backward (d_head = 16 = one 16x16 MFMA tile of K).
//
// Notation per (sample, head): S = Q K^T / sqrt(16) in log2 units (the scale
// and log2(e) are folded into Q or K), P = 2^(S - LSE), O = P V.
// Lane layouts of a 16x16 tile (l = lane): the A operand holds A[l%16][4g..4g+3]
// and the B operand B[4g..4g+3][l%16] with g = l/16; the accumulator holds
// C[4g+i][l%16].  Computing S^T = K Q^T therefore leaves lane l with keys 4g+i
// of query l%16, which is the B layout P^T needs in O^T = V^T P^T and the A
// layout dS needs in dQ = dS K; the dK/dV kernel forms S = Q K^T instead, which
// leaves P^T and dS^T in the A layout of dV and dK.
//
// Precision of the tile products (mode = fvan_precision): FP32 MFMA
// (16x16x4, four per tile) for FVAN_FP32, BF16 MFMA (16x16x16) for FVAN_BF16,
// and for FVAN_BF16_SPLIT three BF16 MFMAs on hi/lo operand splits
// (lo*hi + hi*lo + hi*hi; the dropped lo*lo term is below 2^-16 relative).
#pragma once

#include <algorithm>

#include "device_common.h"

namespace fvan {

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

__device__ __forceinline__ bf16x4 bf4(float a, float b, float c, float d) {
  bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
  return v;
}

template <int MODE>
__device__ __forceinline__ floatx4 mfma16(const float4& a, const float4& b, floatx4 acc) {
  if constexpr (MODE == 1) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bf4(a.x, a.y, a.z, a.w), bf4(b.x, b.y, b.z, b.w), acc, 0, 0, 0);
  } else if constexpr (MODE == 2) {
    const bf16x4 ah = bf4(a.x, a.y, a.z, a.w), bh = bf4(b.x, b.y, b.z, b.w);
    const bf16x4 al = bf4(a.x - (float)ah[0], a.y - (float)ah[1], a.z - (float)ah[2], a.w - (float)ah[3]);
    const bf16x4 bl = bf4(b.x - (float)bh[0], b.y - (float)bh[1], b.z - (float)bh[2], b.w - (float)bh[3]);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
  }
}

// 16 consecutive elements (one head's slice of a row) as floats.
template <typename T>
__device__ __forceinline__ void load16(const T* p, float* out) {
  Chunk<T> a, b;
  a.unpack(*reinterpret_cast<const uint4*>(p));
  b.unpack(*reinterpret_cast<const uint4*>(p + 8));
#pragma unroll
  for (int i = 0; i < 8; ++i) { out[i] = a.v[i]; out[8 + i] = b.v[i]; }
}
template <>
__device__ __forceinline__ void load16<float>(const float* p, float* out) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float4 t = reinterpret_cast<const float4*>(p)[i];
    out[4 * i] = t.x; out[4 * i + 1] = t.y; out[4 * i + 2] = t.z; out[4 * i + 3] = t.w;
  }
}

template <typename T>
__device__ __forceinline__ float4 load4(const T* p) {
  return make_float4(to_f(p[0]), to_f(p[1]), to_f(p[2]), to_f(p[3]));
}
__device__ __forceinline__ float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// Branch-free mask test (bitwise, so no divergent control flow in the tile loops).
__device__ __forceinline__ bool visible(int t, int j, int W, int P) {
  return (j <= t) & ((t - j <= W) | (j < P));
}

constexpr float kScaleLog2 = 0.25f * 1.4426950408889634f;   // 1/sqrt(16) * log2(e)

constexpr int kKeyChunk = 128;                               // keys staged in LDS at a time

// The keys a query tile [t0, t1) can see: [0, pend) then [bstart, t1), as one
// virtual index v -> position.
struct KeyRange {
  int pend, bstart, nk;
  __device__ KeyRange(int t0, int t1, int W, int P) {
    pend = min(P, t1);
    bstart = max(P, t0 - W);
    nk = pend + max(0, t1 - bstart);
  }
  __device__ __forceinline__ int pos(int v) const { return v < pend ? v : bstart + (v - pend); }
};

// Stages kKeyChunk keys (one head's K and V slices) of a query tile's visible
// range into LDS as floats, [key][dim] with rows padded to 20.  Every thread
// loads 16-byte chunks; the next chunk is fetched into registers while the
// current one is processed.
template <typename KT>
struct KeyStager {
  static constexpr int QE = 16 / (int)sizeof(KT);            // elements per 16-byte chunk
  static constexpr int QC = 16 / QE;                         // chunks per key slice
  static constexpr int NLD = kKeyChunk * QC / 256;           // chunks per thread (1 or 2)
  uint4 kraw[NLD], vraw[NLD];
  __device__ __forceinline__ void fetch(const KT* __restrict__ QKV, int64_t rowbase, int D, int h,
                                        const KeyRange& kr, int v0) {
    const int nv = min(kKeyChunk, kr.nk - v0);
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int idx = threadIdx.x + 256 * u, key = idx / QC, ch = (idx % QC) * QE;
      kraw[u] = make_uint4(0u, 0u, 0u, 0u);
      vraw[u] = kraw[u];
      if (key < nv) {
        const KT* kp = QKV + (rowbase + kr.pos(v0 + key)) * 3 * D + D + h * 16 + ch;
        kraw[u] = *reinterpret_cast<const uint4*>(kp);
        vraw[u] = *reinterpret_cast<const uint4*>(kp + D);
      }
    }
  }
  __device__ __forceinline__ void commit(float (*Ks)[20], float (*Vs)[20]) const {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int idx = threadIdx.x + 256 * u, key = idx / QC, ch = (idx % QC) * QE;
      Chunk<KT> kc, vc;
      kc.unpack(kraw[u]);
      vc.unpack(vraw[u]);
#pragma unroll
      for (int e = 0; e < QE; e += 4) {
        *reinterpret_cast<float4*>(&Ks[key][ch + e]) = make_float4(kc.v[e], kc.v[e + 1], kc.v[e + 2], kc.v[e + 3]);
        *reinterpret_cast<float4*>(&Vs[key][ch + e]) = make_float4(vc.v[e], vc.v[e + 1], vc.v[e + 2], vc.v[e + 3]);
      }
    }
  }
};

// ---------------------------------------------------------------- forward
// One workgroup = (64 queries, head, sample); wave w owns queries t0+16w..+15.
// Writes XM = X + O, and LSE (log2 units).
template <typename KT, int MODE>
__global__ __launch_bounds__(256) void attn_fwd_mfma(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                     float* __restrict__ XM, float* __restrict__ LSE, int N, int D,
                                                     int H, int W, int P) {
  __shared__ __align__(16) float Ks[kKeyChunk][20];   // [key][dim] (padded)
  __shared__ __align__(16) float Vs[kKeyChunk][20];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int t0 = blockIdx.x * 64, h = blockIdx.y, b = blockIdx.z;
  const int t1 = min(t0 + 64, N);
  const int64_t rowbase = (int64_t)b * N;
  const int tq = t0 + 16 * wave + c;                 // this lane's query
  const bool qok = tq < N;
  float4 q4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (qok) {
    q4 = load4(QKV + (rowbase + tq) * 3 * D + h * 16 + 4 * g);
    q4.x *= kScaleLog2; q4.y *= kScaleLog2; q4.z *= kScaleLog2; q4.w *= kScaleLog2;
  }
  const KeyRange kr(t0, t1, W, P);
  KeyStager<KT> st;
  st.fetch(QKV, rowbase, D, h, kr, 0);
  float mx = -INFINITY, l = 0.f;
  floatx4 o = {0.f, 0.f, 0.f, 0.f};                 // O^T[dim 4g+i][query c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();
    st.commit(Ks, Vs);
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) st.fetch(QKV, rowbase, D, h, kr, v0 + kKeyChunk);
    for (int kt0 = 0; kt0 < nv; kt0 += 64) {         // 4 key tiles of 16 per softmax update
      float s[16];
      float bmax = -INFINITY;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kb = kt0 + 16 * u;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        if (kb < nv) acc = mfma16<MODE>(load4(&Ks[kb + c][4 * g]), q4, acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int kv = kb + 4 * g + i;
          const bool ok = (kv < nv) & qok & visible(tq, kr.pos(v0 + kv), W, P);
          s[4 * u + i] = ok ? acc[i] : -INFINITY;
          bmax = fmaxf(bmax, s[4 * u + i]);
        }
      }
      bmax = fmaxf(bmax, __shfl_xor(bmax, 16));
      bmax = fmaxf(bmax, __shfl_xor(bmax, 32));
      const float mn = fmaxf(mx, bmax);
      const float corr = mn == -INFINITY ? 1.f : __builtin_amdgcn_exp2f(mx - mn);
      float ps = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float e = __builtin_amdgcn_exp2f(s[i] - mn);   // -inf - finite -> 0; guarded below for mn = -inf
        s[i] = mn == -INFINITY ? 0.f : e;
        ps += s[i];
      }
      ps += __shfl_xor(ps, 16);
      ps += __shfl_xor(ps, 32);
      l = l * corr + ps;
      mx = mn;
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] *= corr;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kb = kt0 + 16 * u;
        if (kb < nv) {
          const int r0 = kb + 4 * g;                  // A = V^T[dim c][keys r0..r0+3]
          const float4 vt = make_float4(Vs[r0][c], Vs[r0 + 1][c], Vs[r0 + 2][c], Vs[r0 + 3][c]);
          o = mfma16<MODE>(vt, make_float4(s[4 * u], s[4 * u + 1], s[4 * u + 2], s[4 * u + 3]), o);
        }
      }
    }
  }
  // lane (g, c) holds O^T[dim 4g+i][query c]: query tq, dims 4g..4g+3
  if (qok) {
    const float inv = 1.0f / l;
    const int64_t r = rowbase + tq;
    const float4 xv = *reinterpret_cast<const float4*>(X + r * D + h * 16 + 4 * g);
    float4 out = make_float4(xv.x + o[0] * inv, xv.y + o[1] * inv, xv.z + o[2] * inv, xv.w + o[3] * inv);
    *reinterpret_cast<float4*>(XM + r * D + h * 16 + 4 * g) = out;
    if (g == 0) LSE[r * H + h] = mx + __log2f(l);
  }
}

// ---------------------------------------------------------------- backward: dQ
// One workgroup = (64 queries, head, sample).  O is recovered as XM - X.
// Writes DELTA = dO . O, dQ (scaled) into dQKV and the feature-major copy T.
template <typename KT, typename AT, int MODE>
__global__ __launch_bounds__(256) void attn_bwd_dq_mfma(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                        const float* __restrict__ XM, const float* __restrict__ dO,
                                                        const float* __restrict__ LSE, float* __restrict__ DELTA,
                                                        AT* __restrict__ dQKV, AT* __restrict__ T, int64_t ldT, int N,
                                                        int D, int H, int W, int P) {
  __shared__ __align__(16) float Ks[kKeyChunk][20];
  __shared__ __align__(16) float Vs[kKeyChunk][20];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int t0 = blockIdx.x * 64, h = blockIdx.y, b = blockIdx.z;
  const int t1 = min(t0 + 64, N);
  const int64_t rowbase = (int64_t)b * N;
  const KeyRange kr(t0, t1, W, P);
  KeyStager<KT> st;
  st.fetch(QKV, rowbase, D, h, kr, 0);
  const int tq = t0 + 16 * wave + c;
  const bool qok = tq < N;
  const int64_t r = rowbase + tq;
  float4 q4 = make_float4(0.f, 0.f, 0.f, 0.f), g4 = q4;
  float lse = 0.f, delta = 0.f;
  if (qok) {
    q4 = load4(QKV + r * 3 * D + h * 16 + 4 * g);
    q4.x *= kScaleLog2; q4.y *= kScaleLog2; q4.z *= kScaleLog2; q4.w *= kScaleLog2;
    g4 = *reinterpret_cast<const float4*>(dO + r * D + h * 16 + 4 * g);
    const float4 xm = *reinterpret_cast<const float4*>(XM + r * D + h * 16 + 4 * g);
    const float4 xx = *reinterpret_cast<const float4*>(X + r * D + h * 16 + 4 * g);
    delta = g4.x * (xm.x - xx.x) + g4.y * (xm.y - xx.y) + g4.z * (xm.z - xx.z) + g4.w * (xm.w - xx.w);
    lse = LSE[r * H + h];
  }
  delta += __shfl_xor(delta, 16);
  delta += __shfl_xor(delta, 32);
  if (qok && g == 0) DELTA[r * H + h] = delta;
  floatx4 dq = {0.f, 0.f, 0.f, 0.f};               // dQ[query 16w+4g+i][dim c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();
    st.commit(Ks, Vs);
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) st.fetch(QKV, rowbase, D, h, kr, v0 + kKeyChunk);
    for (int kb = 0; kb < nv; kb += 16) {
      floatx4 sa = {0.f, 0.f, 0.f, 0.f}, pa = {0.f, 0.f, 0.f, 0.f};
      sa = mfma16<MODE>(load4(&Ks[kb + c][4 * g]), q4, sa);     // S^T[key 4g+i][query c]
      pa = mfma16<MODE>(load4(&Vs[kb + c][4 * g]), g4, pa);     // dP^T[key 4g+i][query c]
      float ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int kv = kb + 4 * g + i;
        const bool ok = (kv < nv) & qok & visible(tq, kr.pos(v0 + kv), W, P);
        const float e = __builtin_amdgcn_exp2f(sa[i] - lse);
        const float p = ok ? e : 0.f;
        ds[i] = p * (pa[i] - delta);
      }
      // dQ[query][dim] += dS[query][key] K[key][dim]; lane's dS = A layout of dS
      const int r0 = kb + 4 * g;
      const float4 kt = make_float4(Ks[r0][c], Ks[r0 + 1][c], Ks[r0 + 2][c], Ks[r0 + 3][c]);
      dq = mfma16<MODE>(make_float4(ds[0], ds[1], ds[2], ds[3]), kt, dq);
    }
  }
  // dq[i] = dQ[query 16w + 4g + i][dim c]
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int tqi = t0 + 16 * wave + 4 * g + i;
    if (tqi < N) {
      const int64_t ri = rowbase + tqi;
      const AT v = from_f<AT>(dq[i] * 0.25f);
      dQKV[ri * 3 * D + h * 16 + c] = v;
      T[(int64_t)(h * 16 + c) * ldT + ri] = v;
    }
  }
}

// ---------------------------------------------------------------- backward: dK, dV
// One workgroup = (head, 64 keys, sample) with the head as the fastest grid index:
// workgroups go to the eight XCDs round-robin by linear index, so each XCD gets
// one head's tiles and the long prefix tiles are spread evenly (with the tile
// index fastest, every prefix tile would land on the same two XCDs).  Wave w
// owns keys j0+16w..+15 and loops over the 64-query blocks that can see the tile
// ([j0, j1 + W), or [j0, N) when the tile holds prefix keys).  Scores are formed as S = Q K^T (A = staged query
// rows, B = the wave's fixed keys), so lane l holds S[4g+i][key l%16]: exactly the
// A layout of P^T and dS^T in dV += P^T dO and dK += dS^T Q, with no transpose.
// The next query block is fetched into registers while the current one is
// processed; every thread issues at most three 16-byte (or 4-byte) loads per block.
template <typename KT, typename AT, int MODE>
__global__ __launch_bounds__(256) void attn_bwd_dkv_mfma(const KT* __restrict__ QKV, const float* __restrict__ dO,
                                                         const float* __restrict__ LSE, const float* __restrict__ DELTA,
                                                         AT* __restrict__ dQKV, AT* __restrict__ T, int64_t ldT, int N,
                                                         int D, int H, int W, int P) {
  constexpr int QB = 64;
  constexpr int QE = 16 / (int)sizeof(KT);          // Q elements per 16-byte chunk
  constexpr int QC = 16 / QE;                       // 16-byte chunks per query row slice
  __shared__ __align__(16) float Qs[QB][20];
  __shared__ __align__(16) float Gs[QB][20];
  __shared__ __align__(16) float Ls[QB];
  __shared__ __align__(16) float Ds[QB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
  const int h = blockIdx.x, j0 = blockIdx.y * 64, b = blockIdx.z;
  const int j1 = min(j0 + 64, N);
  const int64_t rowbase = (int64_t)b * N;
  const int jk = j0 + 16 * wave + c;               // this lane's key (B-operand column)
  const bool kok = jk < N;
  float4 k4 = make_float4(0.f, 0.f, 0.f, 0.f), v4 = k4;
  if (kok) {
    const KT* kp = QKV + (rowbase + jk) * 3 * D + D + h * 16 + 4 * g;
    k4 = load4(kp);
    k4.x *= kScaleLog2; k4.y *= kScaleLog2; k4.z *= kScaleLog2; k4.w *= kScaleLog2;
    v4 = load4(kp + D);
  }
  const int qend = j0 < P ? N : min(N, j1 + W);
  // staging roles: dO row tid/4, quarter tid%4; Q row tid/QC, chunk tid%QC (tid < 64*QC);
  // LSE (tid < 64) or DELTA (64 <= tid < 128) of row tid%64
  const int gr = tid >> 2, gc = (tid & 3) * 4;
  const int qr = tid / QC, qc = (tid % QC) * QE;
  const bool qthr = tid < 64 * QC;
  const int sr = tid & 63;
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
    if ((tid < 128) & (sr < nq)) sraw = (tid < 64 ? LSE : DELTA)[(rowbase + i0 + sr) * H + h];
  };
  fetch(j0);
  floatx4 dk = {0.f, 0.f, 0.f, 0.f}, dv = {0.f, 0.f, 0.f, 0.f};   // [key 16w+4g+i][dim c]
  for (int i0 = j0; i0 < qend; i0 += QB) {
    const int nq = min(QB, qend - i0);
    __syncthreads();                                 // the previous block's reads are done
    *reinterpret_cast<float4*>(&Gs[gr][gc]) = graw;
    if (qthr) {
      Chunk<KT> ch;
      ch.unpack(qraw);
#pragma unroll
      for (int e = 0; e < QE; ++e) Qs[qr][qc + e] = ch.v[e];
    }
    if (tid < 64) Ls[sr] = sraw;
    else if (tid < 128) Ds[sr] = sraw;
    __syncthreads();
    if (i0 + QB < qend) fetch(i0 + QB);
    for (int qb = 0; qb < nq; qb += 16) {
      const floatx4 z = {0.f, 0.f, 0.f, 0.f};
      const floatx4 sa = mfma16<MODE>(*reinterpret_cast<const float4*>(&Qs[qb + c][4 * g]), k4, z);  // S[q 4g+i][key c]
      const floatx4 pa = mfma16<MODE>(*reinterpret_cast<const float4*>(&Gs[qb + c][4 * g]), v4, z);  // dP[q 4g+i][key c]
      const float4 l4 = *reinterpret_cast<const float4*>(&Ls[qb + 4 * g]);
      const float4 d4 = *reinterpret_cast<const float4*>(&Ds[qb + 4 * g]);
      const float lq[4] = {l4.x, l4.y, l4.z, l4.w}, dq[4] = {d4.x, d4.y, d4.z, d4.w};
      float p[4], ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = qb + 4 * g + i;
        const bool ok = (q < nq) & kok & visible(i0 + q, jk, W, P);
        const float e = __builtin_amdgcn_exp2f(sa[i] - lq[i]);
        p[i] = ok ? e : 0.f;
        ds[i] = p[i] * (pa[i] - dq[i]);
      }
      const int r0 = qb + 4 * g;
      const float4 go = make_float4(Gs[r0][c], Gs[r0 + 1][c], Gs[r0 + 2][c], Gs[r0 + 3][c]);
      const float4 qo = make_float4(Qs[r0][c], Qs[r0 + 1][c], Qs[r0 + 2][c], Qs[r0 + 3][c]);
      dv = mfma16<MODE>(make_float4(p[0], p[1], p[2], p[3]), go, dv);     // dV[key][dim] += P^T[key][q] dO[q][dim]
      dk = mfma16<MODE>(make_float4(ds[0], ds[1], ds[2], ds[3]), qo, dk); // dK[key][dim] += dS^T[key][q] Q[q][dim]
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int jj = j0 + 16 * wave + 4 * g + i;
    if (jj < N) {
      const int64_t rj = rowbase + jj;
      const AT kvv = from_f<AT>(dk[i] * 0.25f);
      const AT vvv = from_f<AT>(dv[i]);
      dQKV[rj * 3 * D + D + h * 16 + c] = kvv;
      dQKV[rj * 3 * D + 2 * D + h * 16 + c] = vvv;
      T[(int64_t)(D + h * 16 + c) * ldT + rj] = kvv;
      T[(int64_t)(2 * D + h * 16 + c) * ldT + rj] = vvv;
    }
  }
}

}  // namespace fvan
