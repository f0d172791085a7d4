// Band+prefix masked attention on MFMA for the teacher-forced pass and its
// backward (d_head = 16 = one 16x16 MFMA tile of K).
//
// Notation per (sample, head): S = Q K^T / sqrt(16) in log2 units (the scale
// and log2(e) are folded into Q or K), P = 2^(S - LSE), O = P V.
// Lane layouts of a 16x16 tile (l = lane, g = l/16, c = l%16): the A operand
// holds A[c][4g..4g+3], the B operand B[4g..4g+3][c] and the accumulator
// C[4g+i][c].  Computing S^T = K Q^T leaves lane l with keys 4g+i of query c,
// which is the B layout P^T needs in O^T = V^T P^T and the A layout dS needs in
// dQ = dS K; the dK/dV kernel forms S = Q K^T instead, which leaves P^T and dS^T
// in the A layout of dV and dK.
//
// Operands are converted once, when a block of rows is staged in LDS, into the
// MFMA operand type of the precision mode (AOp below), in both the A layout
// ([row][g]: four consecutive dims of a row) and the B layout ([dim][row group]:
// four consecutive rows of a dim), so the tile loops only load and multiply.
//
// These kernels run the FP32 mode (FP32 MFMA, 16x16x4, four per tile); split mode
// runs the FP16-MFMA kernels of attn_f16.h, which reuse the staging helpers, work
// orders and masks defined here.  AOp<2> below is the BF16 hi/lo operand split
// those kernels stage in LDS.
#pragma once

#include <algorithm>

#include "device_common.h"

namespace fvan {

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Round-to-nearest-even to bf16, two floats per conversion instruction.
__device__ __forceinline__ bf16x4 bf4(float a, float b, float c, float d) {
  const f32x4_t v = {a, b, c, d};
  return __builtin_convertvector(v, bf16x4);
}

// MFMA operand of one lane (four k values) per precision mode.
template <int MODE> struct AOp;
template <> struct AOp<0> {
  typedef float4 T;
  static __device__ __forceinline__ T make(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
  static __device__ __forceinline__ floatx4 mma(const T& a, const T& b, floatx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
  }
};
struct SplitBf16x4 {
  bf16x4 h, l;
};
template <> struct AOp<2> {
  typedef SplitBf16x4 T;
  // hi = bf16(x), lo = bf16(x - hi); hi is widened back by shifting, not converted
  static __device__ __forceinline__ T make(float a, float b, float c, float d) {
    const f32x4_t v = {a, b, c, d};
    T t;
    t.h = __builtin_convertvector(v, bf16x4);
    uint2 hw;
    __builtin_memcpy(&hw, &t.h, 8);
    const f32x4_t hf = {__uint_as_float(hw.x << 16), __uint_as_float(hw.x & 0xFFFF0000u),
                        __uint_as_float(hw.y << 16), __uint_as_float(hw.y & 0xFFFF0000u)};
    t.l = __builtin_convertvector(v - hf, bf16x4);
    return t;
  }
};

template <int MODE>
__device__ __forceinline__ typename AOp<MODE>::T aop(const float4& v) {
  return AOp<MODE>::make(v.x, v.y, v.z, v.w);
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
// A-layout operand tiles hold 4 operands per row padded to 5: an MFMA read of
// rows r..r+15 at one g then starts every lane's 8- or 16-byte access at a
// different bank offset (row strides of 4 operands put 16 lanes on 4 offsets).
constexpr int kAStride = 5;
constexpr int kKeyChunk = 128;                               // keys staged in LDS at a time
// Workgroup shapes, measured per kernel at the 3D workload: the forward and the
// dK/dV kernels run 4 waves x 16 rows, the dQ kernel 8 waves x 16 rows (its key
// staging is then shared by 128 queries).
constexpr int kFwdThreads = 256, kDqThreads = 512, kDkvThreads = 256;
__host__ __device__ constexpr int attn_rows(int threads) { return threads / 4; }   // 16 rows per wave

// Work item of a 1-D attention grid of ntile * H * nsamp workgroups, in (head
// fastest, then tile, then sample) order dealt to the XCDs in contiguous
// ranges: the heads and neighbouring tiles of a sample run on one XCD and share
// its L2 (a head's 16 dims fill only part of a cache line of Q, K, V or dO),
// and every XCD gets the same mix of prefix and band tiles.
struct AttnItem {
  int tile, h, b;
};
__device__ __forceinline__ AttnItem attn_item(int ntile, int H) {
  const int v = xcd_contiguous(blockIdx.x, gridDim.x);
  AttnItem it;
  it.h = v % H;
  const int rest = v / H;
  it.tile = rest % ntile;
  it.b = rest / ntile;
  return it;
}

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

// The virtual key indices (KeyRange order) that query t of the tile sees, as two
// intervals [0, a1) and [b0, b0 + bw): the prefix keys j <= t, then the band keys
// t - W <= j <= t (band keys are >= P by construction).  Equivalent to visible()
// on every key of the range, at two compares per key instead of a select and five.
struct QueryVis {
  int a1, b0, bw;
  __device__ QueryVis(const KeyRange& kr, int t, int W, bool ok) {
    a1 = ok ? min(kr.pend, t + 1) : 0;
    b0 = kr.pend + max(0, t - W - kr.bstart);
    bw = ok ? max(0, kr.pend + t - kr.bstart + 1 - b0) : 0;
  }
  __device__ __forceinline__ bool operator()(int v) const {
    return (v < a1) | ((unsigned)(v - b0) < (unsigned)bw);
  }
};

// Stages kKeyChunk keys (one head's K and V slices) of a query tile's visible
// range: every thread loads 16-byte chunks of K and V into registers (the next
// chunk is fetched while the current one is processed), commit() writes them to
// float tiles [key][dim] with rows padded to 20.
template <typename KT, int NTHREADS>
struct KeyStager {
  static constexpr int QE = 16 / (int)sizeof(KT);            // elements per 16-byte chunk
  static constexpr int QC = 16 / QE;                         // chunks per key slice
  static constexpr int NPC = kKeyChunk * QC;                 // 16-byte chunks per staged block
  static constexpr int NLD = (NPC + NTHREADS - 1) / NTHREADS;   // per thread
  uint4 kraw[NLD], vraw[NLD];
  __device__ __forceinline__ void fetch(const KT* __restrict__ QKV, int64_t rowbase, int D, int h,
                                        const KeyRange& kr, int v0) {
    const int nv = min(kKeyChunk, kr.nk - v0);
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int idx = threadIdx.x + NTHREADS * u, key = idx / QC, ch = (idx % QC) * QE;
      kraw[u] = make_uint4(0u, 0u, 0u, 0u);
      vraw[u] = kraw[u];
      if ((idx < NPC) & (key < nv)) {
        const KT* kp = QKV + (rowbase + kr.pos(v0 + key)) * 3 * D + D + h * 16 + ch;
        kraw[u] = *reinterpret_cast<const uint4*>(kp);
        vraw[u] = *reinterpret_cast<const uint4*>(kp + D);
      }
    }
  }
  __device__ __forceinline__ void commit(float (*Kf)[20], float (*Vf)[20]) const {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int idx = threadIdx.x + NTHREADS * u, key = idx / QC, ch = (idx % QC) * QE;
      if (idx >= NPC) break;
      Chunk<KT> kc, vc;
      kc.unpack(kraw[u]);
      vc.unpack(vraw[u]);
#pragma unroll
      for (int e = 0; e < QE; e += 4) {
        *reinterpret_cast<float4*>(&Kf[key][ch + e]) = make_float4(kc.v[e], kc.v[e + 1], kc.v[e + 2], kc.v[e + 3]);
        *reinterpret_cast<float4*>(&Vf[key][ch + e]) = make_float4(vc.v[e], vc.v[e + 1], vc.v[e + 2], vc.v[e + 3]);
      }
    }
  }
};

// Operand tiles of R staged rows (R = 64 or 128) of one head: A layout [row][g]
// (dims 4g..4g+3 of the row) and B layout [dim][row group] (rows 4j..4j+3 of
// the dim; one padding column against bank conflicts).  Built by all the
// workgroup's threads from a float tile [row][dim].
template <int MODE, int R, int NTHREADS>
__device__ __forceinline__ void build_a(const float (*F)[20], typename AOp<MODE>::T (*A)[kAStride]) {
#pragma unroll
  for (int idx = threadIdx.x; idx < R * 4; idx += NTHREADS) {
    // consecutive lanes take consecutive rows at one g: the padded stride of 5
    // operands and the 80-byte float rows put them on distinct banks
    const int row = idx % R, g = idx / R;
    A[row][g] = aop<MODE>(*reinterpret_cast<const float4*>(&F[row][4 * g]));
  }
}
template <int MODE, int R, int NTHREADS>
__device__ __forceinline__ void build_b(const float (*F)[20], typename AOp<MODE>::T (*B)[R / 4 + 1]) {
#pragma unroll
  for (int idx = threadIdx.x; idx < R * 4; idx += NTHREADS) {
    // consecutive lanes take consecutive dims: the column reads F[4j + r][dim] of a
    // wave then hit 64 distinct banks (rows are 80 bytes apart)
    const int dim = idx & 15, j = idx >> 4;
    B[dim][j] = AOp<MODE>::make(F[4 * j][dim], F[4 * j + 1][dim], F[4 * j + 2][dim], F[4 * j + 3][dim]);
  }
}

// ---------------------------------------------------------------- forward
// One workgroup = (64 queries, head, sample); wave w owns queries t0+16w..+15.
// Writes XM = X + O, and LSE (log2 units).
template <typename KT, int MODE>
__global__ __launch_bounds__(kFwdThreads) void attn_fwd_mfma(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                     float* __restrict__ XM, float* __restrict__ LSE, int N, int D,
                                                     int H, int W, int P) {
  typedef AOp<MODE> Op;
  typedef typename Op::T OT;
  __shared__ __align__(16) float Kf[kKeyChunk][20];
  __shared__ __align__(16) float Vf[kKeyChunk][20];
  __shared__ __align__(16) OT Ka[kKeyChunk][kAStride];        // K, A layout
  __shared__ __align__(16) OT Vb[16][kKeyChunk / 4 + 1];      // V^T as the A operand: [dim][key group]
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
  constexpr int R = attn_rows(kFwdThreads);
  const AttnItem it = attn_item((N + R - 1) / R, H);
  const int t0 = it.tile * R, h = it.h, b = it.b;
  const int t1 = min(t0 + attn_rows(kFwdThreads), N);
  const int64_t rowbase = (int64_t)b * N;
  const int tq = t0 + 16 * wave + c;                 // this lane's query
  const bool qok = tq < N;
  float4 q4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (qok) {
    q4 = load4(QKV + (rowbase + tq) * 3 * D + h * 16 + 4 * g);
    q4.x *= kScaleLog2; q4.y *= kScaleLog2; q4.z *= kScaleLog2; q4.w *= kScaleLog2;
  }
  const OT qb = aop<MODE>(q4);                       // B operand Q^T[dim 4g..][query c]
  const KeyRange kr(t0, t1, W, P);
  const QueryVis vis(kr, tq, W, qok);
  // virtual keys seen by any query of the wave: [0, wa1) and [wb0, wb1) (as in the dQ kernel)
  const int tw0 = t0 + 16 * wave, tw1 = min(tw0 + 15, N - 1);
  const int wa1 = tw0 < N ? min(kr.pend, tw1 + 1) : 0;
  const int wb0 = kr.pend + max(0, tw0 - W - kr.bstart);
  const int wb1 = tw0 < N ? kr.pend + tw1 - kr.bstart + 1 : 0;
  auto wave_sees = [&](int v) { return (v < wa1) | ((v + 16 > wb0) & (v < wb1)); };   // a 16-key group
  KeyStager<KT, kFwdThreads> st;
  st.fetch(QKV, rowbase, D, h, kr, 0);
  float mx = -INFINITY, l = 0.f;
  floatx4 o = {0.f, 0.f, 0.f, 0.f};                 // O^T[dim 4g+i][query c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();
    st.commit(Kf, Vf);
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) st.fetch(QKV, rowbase, D, h, kr, v0 + kKeyChunk);
    build_a<MODE, kKeyChunk, kFwdThreads>(Kf, Ka);
    build_b<MODE, kKeyChunk, kFwdThreads>(Vf, Vb);
    __syncthreads();
    for (int kt0 = 0; kt0 < nv; kt0 += 64) {         // 4 key tiles of 16 per softmax update
      bool used[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) used[u] = (kt0 + 16 * u < nv) && wave_sees(v0 + kt0 + 16 * u);
      if (!(used[0] | used[1] | used[2] | used[3])) continue;   // no query of the wave sees these keys
      float s[16];
      float bmax = -INFINITY;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kb = kt0 + 16 * u;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        if (used[u]) acc = Op::mma(Ka[kb + c][g], qb, acc);   // S^T[key 4g+i][query c]
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool ok = vis(v0 + kb + 4 * g + i);   // keys past nv lie beyond kr.nk: never visible
          s[4 * u + i] = ok ? acc[i] : -INFINITY;
          bmax = fmaxf(bmax, s[4 * u + i]);
        }
      }
      bmax = max_xor32(max_xor16(bmax));
      const float mn = fmaxf(mx, bmax);
      const float corr = mn == -INFINITY ? 1.f : __builtin_amdgcn_exp2f(mx - mn);
      float ps = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float e = __builtin_amdgcn_exp2f(s[i] - mn);   // -inf - finite -> 0; guarded below for mn = -inf
        s[i] = mn == -INFINITY ? 0.f : e;
        ps += s[i];
      }
      ps = sum_xor32(sum_xor16(ps));
      l = l * corr + ps;
      mx = mn;
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] *= corr;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kb = kt0 + 16 * u;
        if (used[u])   // A = V^T[dim c][keys kb+4g..+3], B = P^T[keys][query c]
          o = Op::mma(Vb[c][kb / 4 + g], Op::make(s[4 * u], s[4 * u + 1], s[4 * u + 2], s[4 * u + 3]), o);
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
// One workgroup = (128 queries, head, sample).  O is recovered as XM - X.
// Writes DELTA = dO . O, dQ (scaled) into dQKV and the feature-major copy T.
template <typename KT, typename AT, int MODE>
__global__ __launch_bounds__(kDqThreads) void attn_bwd_dq_mfma(const KT* __restrict__ QKV, const float* __restrict__ X,
                                                        const float* __restrict__ XM, const float* __restrict__ dO,
                                                        const float* __restrict__ LSE, float* __restrict__ DELTA,
                                                        AT* __restrict__ dQKV, AT* __restrict__ T, int64_t ldT, int N,
                                                        int D, int H, int W, int P) {
  typedef AOp<MODE> Op;
  typedef typename Op::T OT;
  __shared__ __align__(16) float Kf[kKeyChunk][20];
  __shared__ __align__(16) float Vf[kKeyChunk][20];
  __shared__ __align__(16) OT Ka[kKeyChunk][kAStride];
  __shared__ __align__(16) OT Va[kKeyChunk][kAStride];
  __shared__ __align__(16) OT Kb[16][kKeyChunk / 4 + 1];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
  constexpr int R = attn_rows(kDqThreads);
  const AttnItem it = attn_item((N + R - 1) / R, H);
  const int t0 = it.tile * R, h = it.h, b = it.b;
  const int t1 = min(t0 + attn_rows(kDqThreads), N);
  const int64_t rowbase = (int64_t)b * N;
  const KeyRange kr(t0, t1, W, P);
  KeyStager<KT, kDqThreads> st;
  st.fetch(QKV, rowbase, D, h, kr, 0);
  const int tq = t0 + 16 * wave + c;
  const bool qok = tq < N;
  const QueryVis vis(kr, tq, W, qok);
  // the virtual keys seen by any query of the wave (queries tw0..tw1, in order):
  // [0, wa1) and [wb0, wb1); a 16-key step outside both is skipped by the whole wave
  const int tw0 = t0 + 16 * wave, tw1 = min(tw0 + 15, N - 1);
  const int wa1 = tw0 < N ? min(kr.pend, tw1 + 1) : 0;
  const int wb0 = kr.pend + max(0, tw0 - W - kr.bstart);
  const int wb1 = tw0 < N ? kr.pend + tw1 - kr.bstart + 1 : 0;
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
  delta = sum_xor32(sum_xor16(delta));
  if (qok && g == 0) DELTA[r * H + h] = delta;
  const OT qb = aop<MODE>(q4), gb = aop<MODE>(g4);   // B operands Q^T, dO^T [dim 4g..][query c]
  floatx4 dq = {0.f, 0.f, 0.f, 0.f};               // dQ[query 16w+4g+i][dim c]
  for (int v0 = 0; v0 < kr.nk; v0 += kKeyChunk) {
    const int nv = min(kKeyChunk, kr.nk - v0);
    __syncthreads();
    st.commit(Kf, Vf);
    __syncthreads();
    if (v0 + kKeyChunk < kr.nk) st.fetch(QKV, rowbase, D, h, kr, v0 + kKeyChunk);
    build_a<MODE, kKeyChunk, kDqThreads>(Kf, Ka);
    build_a<MODE, kKeyChunk, kDqThreads>(Vf, Va);
    build_b<MODE, kKeyChunk, kDqThreads>(Kf, Kb);
    __syncthreads();
    for (int kb = 0; kb < nv; kb += 16) {
      const int vb = v0 + kb;
      if ((vb >= wa1) & ((vb + 16 <= wb0) | (vb >= wb1))) continue;   // no query of the wave sees these keys
      const floatx4 z = {0.f, 0.f, 0.f, 0.f};
      const floatx4 sa = Op::mma(Ka[kb + c][g], qb, z);     // S^T[key 4g+i][query c]
      const floatx4 pa = Op::mma(Va[kb + c][g], gb, z);     // dP^T[key 4g+i][query c]
      float ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool ok = vis(v0 + kb + 4 * g + i);
        const float e = __builtin_amdgcn_exp2f(sa[i] - lse);
        const float p = ok ? e : 0.f;
        ds[i] = p * (pa[i] - delta);
      }
      // dQ[query][dim] += dS[query][key] K[key][dim]; lane's dS = A layout of dS
      dq = Op::mma(Op::make(ds[0], ds[1], ds[2], ds[3]), Kb[c][kb / 4 + g], dq);
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
// ([j0, j1 + W), or [j0, N) when the tile holds prefix keys).  The next query
// block is fetched into registers while the current one is processed.
template <typename KT, typename AT, int MODE>
__global__ __launch_bounds__(kDkvThreads) void attn_bwd_dkv_mfma(const KT* __restrict__ QKV, const float* __restrict__ dO,
                                                         const float* __restrict__ LSE, const float* __restrict__ DELTA,
                                                         AT* __restrict__ dQKV, AT* __restrict__ T, int64_t ldT, int N,
                                                         int D, int H, int W, int P) {
  typedef AOp<MODE> Op;
  typedef typename Op::T OT;
  constexpr int QB = attn_rows(kDkvThreads);
  constexpr int QE = 16 / (int)sizeof(KT);          // Q elements per 16-byte chunk
  constexpr int QC = 16 / QE;                       // 16-byte chunks per query row slice
  __shared__ __align__(16) float Qf[QB][20];
  __shared__ __align__(16) float Gf[QB][20];
  __shared__ __align__(16) OT Qa[QB][kAStride];     // Q, A layout (S = Q K^T)
  __shared__ __align__(16) OT Ga[QB][kAStride];     // dO, A layout (dP = dO V^T)
  __shared__ __align__(16) OT Qb[16][QB / 4 + 1];   // Q, B layout (dK += dS^T Q)
  __shared__ __align__(16) OT Gb[16][QB / 4 + 1];   // dO, B layout (dV += P^T dO)
  __shared__ __align__(16) float Ls[QB];
  __shared__ __align__(16) float Ds[QB];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, c = lane & 15;
  const AttnItem it = attn_item((N + QB - 1) / QB, H);
  const int h = it.h, j0 = it.tile * QB, b = it.b;
  const int j1 = min(j0 + QB, N);
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
  const OT kb = aop<MODE>(k4), vb = aop<MODE>(v4);  // B operands K^T, V^T [dim 4g..][key c]
  const int qend = j0 < P ? N : min(N, j1 + W);
  // queries that see this lane's key: jk <= iq < qhi (any later query for a prefix key)
  const int qw = kok ? max(0, min(jk < P ? N : jk + W + 1, qend) - jk) : 0;
  // and the queries that see any key of the wave (keys jw0..jw0+15, in order): a
  // 16-query step outside [jw0, qhi_w) is skipped by the whole wave
  const int jw0 = j0 + 16 * wave;
  const int qhi_w = jw0 >= N ? jw0 : (jw0 < P ? qend : min(qend, min(N - 1, jw0 + 15) + W + 1));
  // staging roles (QB rows): dO row tid/4, quarter tid%4; Q row tid/QC, chunk
  // tid%QC (tid < QB*QC); LSE (tid < QB) or DELTA (QB <= tid < 2 QB) of row tid%QB
  static_assert(QB * 4 == kDkvThreads, "dK/dV staging: one dO quarter-row per thread");
  const int gr = tid >> 2, gc = (tid & 3) * 4;
  const int qr = tid / QC, qc = (tid % QC) * QE;
  const bool qthr = tid < QB * QC;
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
      Chunk<KT> ch;
      ch.unpack(qraw);
#pragma unroll
      for (int e = 0; e < QE; ++e) Qf[qr][qc + e] = ch.v[e];
    }
    if (tid < QB) Ls[sr] = sraw;
    else if (tid < 2 * QB) Ds[sr] = sraw;
    __syncthreads();
    if (i0 + QB < qend) fetch(i0 + QB);
    build_a<MODE, QB, kDkvThreads>(Qf, Qa);
    build_a<MODE, QB, kDkvThreads>(Gf, Ga);
    build_b<MODE, QB, kDkvThreads>(Qf, Qb);
    build_b<MODE, QB, kDkvThreads>(Gf, Gb);
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += 16) {
      if ((i0 + q0 + 16 <= jw0) | (i0 + q0 >= qhi_w)) continue;   // no key of the wave sees these queries
      const floatx4 z = {0.f, 0.f, 0.f, 0.f};
      const floatx4 sa = Op::mma(Qa[q0 + c][g], kb, z);   // S[q 4g+i][key c]
      const floatx4 pa = Op::mma(Ga[q0 + c][g], vb, z);   // dP[q 4g+i][key c]
      const float4 l4 = *reinterpret_cast<const float4*>(&Ls[q0 + 4 * g]);
      const float4 d4 = *reinterpret_cast<const float4*>(&Ds[q0 + 4 * g]);
      const float lq[4] = {l4.x, l4.y, l4.z, l4.w}, dq[4] = {d4.x, d4.y, d4.z, d4.w};
      float p[4], ds[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool ok = (unsigned)(i0 + q0 + 4 * g + i - jk) < (unsigned)qw;   // also excludes iq >= qend
        const float e = __builtin_amdgcn_exp2f(sa[i] - lq[i]);
        p[i] = ok ? e : 0.f;
        ds[i] = p[i] * (pa[i] - dq[i]);
      }
      dv = Op::mma(Op::make(p[0], p[1], p[2], p[3]), Gb[c][q0 / 4 + g], dv);      // dV += P^T dO
      dk = Op::mma(Op::make(ds[0], ds[1], ds[2], ds[3]), Qb[c][q0 / 4 + g], dk);  // dK += dS^T Q
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
