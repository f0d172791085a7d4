// KV-cached ancestral sampling (Alg. 2 of the paper) for gfx950.
//
// One workgroup (8 waves) owns a tile of KM = 32 (or 16) samples and runs every step
// t = 0..N-1 and every layer without leaving the kernel: samples are
// independent, so no grid-wide synchronisation is ever needed.  Per layer step:
//   LN1 (16 lanes per sample, shuffle reductions)
//   QKV = LN1(h) W^T + b on MFMA (32 samples x 3d: every weight fragment a wave
//        loads feeds both 16-sample row tiles, which halves the weight traffic
//        per sample), k_t and v_t go straight from the MFMA accumulators to the
//        sample's KV cache slot
//   attention: one wave per sample, K/V rows streamed with 16-byte coalesced
//        loads, per-head dot products and an online softmax reduced with lane
//        shuffles; the heads' concatenation is added to h (no W_O)
//   LN2 + FFN (4d hidden kept in LDS) on MFMA, residual added in place
// then the head, the Philox draw and the decision.  The KV cache of a sample
// and layer holds the prefix positions [0, P) and a ring of the last R band
// positions, so the visible keys of step t are always slots [0, nvis).
//
// Template parameters: D = d_model, MODE = precision, DH = head width (16, 32
// or 64), TOK = a model over 2^D-spin patch tokens: the head has `vocab`
// outputs, the token is drawn from the V-way softmax by one uniform (walking
// the vocabulary from the top, so V = 2 is the binary rule) and fed to the token
// embedding of the next position; the token, not a spin, is written out.
//
// The kernel templates are instantiated in decode.hip (the single-spin kernels
// with 16-wide heads) and decode_ext.hip (other head widths and token models).
#pragma once

#include "device_common.h"
#include "fvan_model.h"

namespace fvan {

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxVocab = 256;

// KM: samples per workgroup, 32 (two 16-row MFMA tiles: every weight fragment
// feeds both) or 16 (one tile; twice the workgroups for a batch).
template <int D, int MODE, bool TOK, int KM>
struct DecodeSmem {
  typedef typename Mode<MODE>::ActT A;
  static constexpr int PAD = 16 / (int)sizeof(A);
  static constexpr int LDA = D + PAD;
  static constexpr int LDH = 4 * D + PAD;
  static constexpr int LDZ = kMaxVocab + 1;
  __align__(16) float h[KM][D];
  A a[KM][LDA];
  union {
    float q[KM][D];
    A hid[KM][LDH];
    float z[TOK ? KM : 1][TOK ? LDZ : 1];   // logits of the vocab-way head
  } u;
  int tok[KM];
  int8_t sbuf[KM][64];
  // FFN2 partial sums of the waves that take the upper K ranges in split mode
  // when d < 128 (fewer output tiles than waves; FP32 mode measured no gain)
  static constexpr int KP = Mode<MODE>::SPLIT && D / 16 < kWaves ? kWaves / (D / 16) - 1 : 0;
  float kpart[KP > 0 ? KP : 1][KP > 0 ? KM : 1][KP > 0 ? D : 1];
};


__device__ __forceinline__ float reduce16(float v) { return row_sum16(v); }

// 16-byte load of the K/V stream, marked non-temporal so that it does not push
// the layer weights out of L2
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ uint4 stream_load16(const T* p) {
  const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// LayerNorm of the KM residual rows into the MFMA operand buffer (16 lanes per row).
// In split mode the output is written already split, once: each group of 8
// consecutive elements of a row is a BF16 hi uint4 followed by its lo uint4 (the
// same hi/lo as the GEMMs' own split of FP32 operands), so the QKV and FFN1
// products read their A fragments without converting them per output tile.
template <int D, int MODE, bool TOK, int KM>
__device__ __forceinline__ void ln_rows(DecodeSmem<D, MODE, TOK, KM>& sm, const float* __restrict__ g,
                                        const float* __restrict__ b) {
  typedef typename Mode<MODE>::ActT T;
  constexpr int PER = D / 16;
  constexpr bool SPLIT = Mode<MODE>::SPLIT;
  const int m = threadIdx.x >> 4, part = threadIdx.x & 15;
  if (m >= KM) return;
  float x[PER];
  float s = 0.f;
  // split mode: PER consecutive elements per lane; otherwise strided by 16
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    x[i] = sm.h[m][SPLIT ? part * PER + i : part + 16 * i];
    s += x[i];
  }
  const float mean = reduce16(s) * (1.0f / D);
  float v = 0.f;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    x[i] -= mean;
    v += x[i] * x[i];
  }
  const float rstd = rsqrtf(reduce16(v) * (1.0f / D) + kLnEps);
  if constexpr (SPLIT) {
    static_assert(PER % 2 == 0 && 8 % PER == 0, "a lane's elements lie in one 8-element group");
    float y[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = part * PER + i;
      y[i] = x[i] * rstd * g[k] + b[k];
    }
    // hi = bf16(y), lo = bf16(y - hi), two elements per 32-bit word
    uint32_t hw[PER / 2], lw[PER / 2];
#pragma unroll
    for (int i = 0; i < PER; i += 2) {
      const f32x2_t v2 = {y[i], y[i + 1]};
      const bf16x2_t h2 = __builtin_convertvector(v2, bf16x2_t);
      uint32_t hb;
      __builtin_memcpy(&hb, &h2, 4);
      const f32x2_t r2 = {y[i] - __uint_as_float(hb << 16), y[i + 1] - __uint_as_float(hb & 0xFFFF0000u)};
      const bf16x2_t l2 = __builtin_convertvector(r2, bf16x2_t);
      hw[i / 2] = hb;
      __builtin_memcpy(&lw[i / 2], &l2, 4);
    }
    uint32_t* row = reinterpret_cast<uint32_t*>(&sm.a[m][0]);
    const int j = part * PER / 8, o = (part * PER % 8) / 2;   // group, 32-bit word inside the group's uint4
#pragma unroll
    for (int w = 0; w < PER / 2; ++w) {
      row[8 * j + o + w] = hw[w];
      row[8 * j + 4 + o + w] = lw[w];
    }
  } else {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = part + 16 * i;
      sm.a[m][k] = from_f<T>(x[i] * rstd * g[k] + b[k]);
    }
  }
}

// The output tiles nt = nt0, nt0 + step, ... < ntn of A[16 NRT x K] (LDS, row
// stride lda) . pack, each finished tile handed to epi(nt, acc0, acc1).  The
// weight fragments come G chunks per round, and the next round's (of this tile
// or of the wave's next tile) are loaded while the current round multiplies, so
// a phase exposes one L2 latency instead of one per round.  Per tile the chunks
// are summed in order, as a single pass over the tile would; acc1 stays zero
// when NRT = 1.
// PRE: A holds split-mode operands written by ln_rows (per 8-element group a hi
// uint4, then its lo uint4; row stride lda elements of Mode<2>::ActT).
template <int MODE, int K, int NRT, typename Epi, bool PRE = false>
__device__ __forceinline__ void mfma_tiles(const typename Mode<MODE>::ActT* A, int lda,
                                           const uint4* __restrict__ pack, size_t lo_u4, int nt0, int ntn, int step,
                                           int lane, Epi&& epi) {
  constexpr int KC = Mode<MODE>::KC;
  constexpr int NC = K / KC;
  constexpr int GM = Mode<MODE>::SPLIT ? 2 : 4;
  constexpr int G = NC < GM ? NC : GM;
  static_assert(NC % G == 0, "K chunks in groups of G");
  constexpr int R = NC / G;                 // rounds per tile
  if (nt0 >= ntn) return;
  static_assert(!PRE || Mode<MODE>::SPLIT, "pre-split operands in split mode only");
  const typename Mode<MODE>::ActT* arow = A + (lane & 15) * lda + (lane >> 4) * (KC / 4);
  const typename Mode<MODE>::ActT* arow1 = arow + 16 * lda;
  // pre-split: lane (g, c) takes group 4 kc + g of row c: uint4s 2 (4 kc + g) and + 1
  const uint4* prow = reinterpret_cast<const uint4*>(A) + (lane & 15) * (lda * (int)sizeof(*A) / 16) + 2 * (lane >> 4);
  const uint4* prow1 = prow + 16 * (lda * (int)sizeof(*A) / 16);
  uint4 bh[G], bl[G], nh[G], nl[G];
#define FVAN_DT_LOAD(T, RR, H, L)                                                              \
  _Pragma("unroll") for (int u = 0; u < G; ++u) {                                            \
    const uint4* bp_ = pack + (size_t)(T) * NC * 64 + (size_t)((RR) * G + u) * 64 + lane;    \
    H[u] = bp_[0];                                                                           \
    L[u] = Mode<MODE>::SPLIT ? bp_[lo_u4] : H[u];                                            \
  }
  // rounds are consumed in order; the loads of the next two rounds are in flight
  // while a round multiplies
  auto advance = [&](int& t, int& rr) {
    if (++rr == R) {
      rr = 0;
      t += step;
    }
  };
  uint4 mh[G], ml[G];
  FVAN_DT_LOAD(nt0, 0, bh, bl);
  int nt1 = nt0, r1 = 0;
  advance(nt1, r1);
  bool more1 = nt1 < ntn;
  if (more1) {
    FVAN_DT_LOAD(nt1, r1, nh, nl);
  }
  floatx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
  int nt = nt0, r = 0;
  for (;;) {
    int nt2 = nt1, r2 = r1;
    advance(nt2, r2);
    const bool more2 = more1 && nt2 < ntn;
    if (more2) {
      FVAN_DT_LOAD(nt2, r2, mh, ml);
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int kc = r * G + u;
      if constexpr (PRE) {
        // the same three products in the same order as Frag<2>::step1v / step2v
        static_assert(KC == 32, "four 8-element groups per K chunk");
        const uint4 xh = prow[8 * kc], xl = prow[8 * kc + 1];
        if constexpr (NRT == 2) {
          const uint4 yh = prow1[8 * kc], yl = prow1[8 * kc + 1];
          acc0 = mfma_bf16(xl, bh[u], acc0);
          acc1 = mfma_bf16(yl, bh[u], acc1);
          acc0 = mfma_bf16(xh, bl[u], acc0);
          acc1 = mfma_bf16(yh, bl[u], acc1);
          acc0 = mfma_bf16(xh, bh[u], acc0);
          acc1 = mfma_bf16(yh, bh[u], acc1);
        } else {
          acc0 = mfma_bf16(xl, bh[u], acc0);
          acc0 = mfma_bf16(xh, bl[u], acc0);
          acc0 = mfma_bf16(xh, bh[u], acc0);
        }
      } else {
        const int k = kc * KC;
        if constexpr (NRT == 2)
          Frag<MODE>::step2v(arow + k, arow1 + k, bh[u], bl[u], acc0, acc1);
        else
          Frag<MODE>::step1v(arow + k, bh[u], bl[u], acc0);
      }
    }
    if (r == R - 1) {
      epi(nt, acc0, acc1);
      acc0 = floatx4{0.f, 0.f, 0.f, 0.f};
      acc1 = acc0;
    }
    if (!more1) break;
    nt = nt1;
    r = r1;
    nt1 = nt2;
    r1 = r2;
    more1 = more2;
#pragma unroll
    for (int u = 0; u < G; ++u) {
      bh[u] = nh[u];
      bl[u] = nl[u];
      nh[u] = mh[u];
      nl[u] = ml[u];
    }
  }
#undef FVAN_DT_LOAD
}

template <int D, int MODE, int DH, bool TOK, int KM>
__device__ void decode_tile(DecodeSmem<D, MODE, TOK, KM>& sm, const DecodeUnit& U, int local_tile) {
  typedef typename Mode<MODE>::KvT T;
  typedef DecodeSmem<D, MODE, TOK, KM> Sm;
  constexpr int NRT = KM / 16;          // 16-row MFMA tiles
  static_assert(KM == 16 || KM == 32, "16 or 32 samples per workgroup");
  constexpr int VEC = Chunk<T>::N;
  constexpr int LPR = D / VEC;          // lanes per K/V row
  constexpr int RPL = 64 / LPR;         // rows per wave load
  constexpr int LPH = DH / VEC;         // lanes per head
  // rows per lane in flight: 5 at d = 64 (40-row batches: a 2D lattice step's
  // visible keys, up to 2L + 2, take one or two batches instead of two or three;
  // measured 11% faster at L = 16), 4 otherwise (at d = 128 a fifth row spills
  // registers and gains nothing)
  constexpr int UNR = D == 64 ? 5 : 4;
  static_assert(DH == 16 || DH == 32 || DH == 64, "head width 16, 32 or 64");
  static_assert(LPH >= 2 && LPH <= LPR, "a head spans 2 .. LPR lanes of a row");
  // 1/sqrt(DH) * log2(e)
  constexpr float kScaleLog2 = (DH == 16 ? 0.25f : DH == 32 ? 0.17677669529663688f : 0.125f) * 1.4426950408889634f;

  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b0 = local_tile * KM;
  const int nb = min(KM, U.B - b0);
  const int N = U.N, P = U.P, R = U.R, S = U.S, nl = U.n_layers, dt = U.d_token;
  const float* __restrict__ theta = U.theta;
  const char* wbase = reinterpret_cast<const char*>(U.wpack);
  T* kvbase = reinterpret_cast<T*>(U.kv);
  const size_t plane = (size_t)S * D;   // elements of one K (or V) block

  // head-phase ownership: thread 16*m handles sample row m
  const int hm = tid >> 4, hpart = tid & 15;
  float lq = 0.f;
  float ur[4] = {0.f, 0.f, 0.f, 0.f};
  if (tid < KM) sm.tok[tid] = 0;   // start token
  __syncthreads();

  for (int t = 0; t < N; ++t) {
    // ---- concatenated embedding [tok_emb[tok]; pos_emb[t]] ----
    for (int i = tid; i < KM * D; i += kThreads) {
      const int m = i / D, k = i % D;
      sm.h[m][k] = k < dt ? theta[sm.tok[m] * dt + k] : theta[U.pos_off + (size_t)t * (D - dt) + (k - dt)];
    }
    const int slot = t < P ? t : P + (t - P) % R;
    const int nvis = t < P ? t + 1 : P + min(t - P + 1, R);
    __syncthreads();

    for (int l = 0; l < nl; ++l) {
      const float* lp = theta + U.layer0 + (size_t)l * U.layer_stride;
      const char* wl = wbase + (size_t)l * U.p_layer_stride;
      ln_rows<D, MODE, TOK, KM>(sm, lp + U.o_ln1_g, lp + U.o_ln1_b);
      __syncthreads();

      // ---- QKV projection; k_t, v_t appended to the cache ----
      {
        const uint4* pk = reinterpret_cast<const uint4*>(wl + U.p_qkv);
        auto qkv_epi = [&](int nt, const floatx4& a0, const floatx4& a1) {
          const floatx4 acc[2] = {a0, a1};
          const int n = nt * 16 + (lane & 15);
          const float bias = lp[U.o_qkv_b + n];
#pragma unroll
          for (int ri = 0; ri < 4 * NRT; ++ri) {
            const int row = 16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3);
            const float val = acc[ri >> 2][ri & 3] + bias;
            if (n < D) {
              sm.u.q[row][n] = val;
            } else if (row < nb) {
              const int which = n >= 2 * D ? 1 : 0;
              const int col = n - D - which * D;
              T* dst = kvbase + ((size_t)(b0 + row) * nl + l) * 2 * plane + which * plane + (size_t)slot * D + col;
              *dst = from_f<T>(val);
            }
          }
        };
        mfma_tiles<MODE, D, NRT, decltype(qkv_epi)&, Mode<MODE>::SPLIT>(&sm.a[0][0], Sm::LDA, pk, (size_t)3 * D * D / 8,
                                                                       wave, 3 * D / 16, kWaves, lane, qkv_epi);
      }
      __threadfence_block();
      __syncthreads();

      // ---- masked attention over slots [0, nvis), one wave per sample ----
      // The wave's samples are walked as one stream of row batches (UNR rows per
      // lane, RPL rows per wave load); the next batch's raw 16-byte K/V loads are
      // issued before the current batch is reduced, across sample boundaries too.
      {
        const int lrow = lane / LPR;
        const int lcol = (lane % LPR) * VEC;
        const int per = (nvis + RPL * UNR - 1) / (RPL * UNR);   // batches per sample
        const int nsw = nb > wave ? (nb - wave + kWaves - 1) / kWaves : 0;   // samples of this wave
        const int total = per * nsw;
        uint4 kr[UNR], vr[UNR];
        auto issue = [&](int bi, uint4* kk, uint4* vv) {
          const int m = wave + kWaves * (bi / per);
          const int s0 = (bi % per) * RPL * UNR;
          const T* Kb = kvbase + ((size_t)(b0 + m) * nl + l) * 2 * plane;
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const int s = s0 + u * RPL + lrow;
            // rows past the visible keys are zero, so their (zero) probabilities
            // multiply zeros, not stale register contents
            kk[u] = make_uint4(0u, 0u, 0u, 0u);
            vv[u] = kk[u];
            if (s < nvis) {
              kk[u] = stream_load16(Kb + (size_t)s * D + lcol);
              vv[u] = stream_load16(Kb + plane + (size_t)s * D + lcol);
            }
          }
        };
        if (total > 0) issue(0, kr, vr);
        float qv[VEC], o[VEC];
        float mx = -INFINITY, sum = 0.f;
        for (int bi = 0; bi < total; ++bi) {
          uint4 kn[UNR], vn[UNR];
          if (bi + 1 < total) issue(bi + 1, kn, vn);
          const int m = wave + kWaves * (bi / per);
          const int part = bi % per;
          if (part == 0) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) { qv[i] = sm.u.q[m][lcol + i] * kScaleLog2; o[i] = 0.f; }
            mx = -INFINITY;
            sum = 0.f;
          }
          const int s0 = part * RPL * UNR;
          float sc[UNR];
          float mnew = mx;
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            Chunk<T> kc;
            kc.unpack(kr[u]);
            float d = 0.f;
#pragma unroll
            for (int i = 0; i < VEC; ++i) d += qv[i] * kc.v[i];
            if (LPH >= 2) d += lane_xor(d, 1);
            if (LPH >= 4) d += lane_xor(d, 2);
            if (LPH >= 8) d += lane_xor(d, 4);
            if (LPH >= 16) d += lane_xor(d, 8);
            sc[u] = s0 + u * RPL + lrow < nvis ? d : -INFINITY;
            mnew = fmaxf(mnew, sc[u]);
          }
          const float corr = mnew != -INFINITY ? __builtin_amdgcn_exp2f(mx - mnew) : 1.f;
          sum *= corr;
#pragma unroll
          for (int i = 0; i < VEC; ++i) o[i] *= corr;
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const bool ok = sc[u] != -INFINITY;
            const float p = ok ? __builtin_amdgcn_exp2f(sc[u] - mnew) : 0.f;
            Chunk<T> vc;
            vc.unpack(vr[u]);
            sum += p;
#pragma unroll
            for (int i = 0; i < VEC; ++i) o[i] += p * vc.v[i];
          }
          mx = mnew;
          if (part == per - 1) {
            // merge the RPL row groups of the wave, then add the heads' outputs to h
#pragma unroll
            for (int off = LPR; off < 64; off <<= 1) {
              const float m2 = lane_xor(mx, off);
              const float s2 = lane_xor(sum, off);
              const float mn = fmaxf(mx, m2);
              const float c1 = mx == -INFINITY ? 0.f : __builtin_amdgcn_exp2f(mx - mn);
              const float c2 = m2 == -INFINITY ? 0.f : __builtin_amdgcn_exp2f(m2 - mn);
              sum = sum * c1 + s2 * c2;
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                const float o2 = lane_xor(o[i], off);
                o[i] = o[i] * c1 + o2 * c2;
              }
              mx = mn;
            }
            if (lrow == 0) {
              const float inv = 1.0f / sum;
#pragma unroll
              for (int i = 0; i < VEC; ++i) sm.h[m][lcol + i] += o[i] * inv;
            }
          }
#pragma unroll
          for (int u = 0; u < UNR; ++u) { kr[u] = kn[u]; vr[u] = vn[u]; }
        }
      }
      __syncthreads();

      // ---- feed-forward block ----
      ln_rows<D, MODE, TOK, KM>(sm, lp + U.o_ln2_g, lp + U.o_ln2_b);
      __syncthreads();
      {
        const uint4* p1 = reinterpret_cast<const uint4*>(wl + U.p_ffn1);
        // split mode: GELU(h) goes to LDS already split, in the layout ln_rows
        // writes (per 8-element group of a row: 8 hi BF16, then 8 lo), for FFN2
        auto ffn1_epi = [&](int nt, const floatx4& a0, const floatx4& a1) {
          const floatx4 acc[2] = {a0, a1};
          const int n = nt * 16 + (lane & 15);
          const float bias = lp[U.o_ffn1_b + n];
#pragma unroll
          for (int ri = 0; ri < 4 * NRT; ++ri) {
            const int row = 16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3);
            const float gv = gelu(acc[ri >> 2][ri & 3] + bias);
            if constexpr (Mode<MODE>::SPLIT) {
              const __bf16 hb = (__bf16)gv;
              const __bf16 lb = (__bf16)(gv - (float)hb);
              __bf16* hr = reinterpret_cast<__bf16*>(&sm.u.hid[row][0]) + (n >> 3) * 16 + (n & 7);
              hr[0] = hb;
              hr[8] = lb;
            } else {
              sm.u.hid[row][n] = from_f<typename Mode<MODE>::ActT>(gv);
            }
          }
        };
        mfma_tiles<MODE, D, NRT, decltype(ffn1_epi)&, Mode<MODE>::SPLIT>(&sm.a[0][0], Sm::LDA, p1, (size_t)4 * D * D / 8,
                                                                        wave, 4 * D / 16, kWaves, lane, ffn1_epi);
      }
      __syncthreads();
      {
        const uint4* p2 = reinterpret_cast<const uint4*>(wl + U.p_ffn2);
        constexpr int NT2 = D / 16;         // output tiles
        if constexpr (Sm::KP == 0) {
          auto ffn2_epi = [&](int nt, const floatx4& a0, const floatx4& a1) {
            const floatx4 acc[2] = {a0, a1};
            const int n = nt * 16 + (lane & 15);
            const float bias = lp[U.o_ffn2_b + n];
#pragma unroll
            for (int ri = 0; ri < 4 * NRT; ++ri)
              sm.h[16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3)][n] += acc[ri >> 2][ri & 3] + bias;
          };
          mfma_tiles<MODE, 4 * D, NRT, decltype(ffn2_epi)&, Mode<MODE>::SPLIT>(&sm.u.hid[0][0], Sm::LDH, p2,
                                                                              (size_t)4 * D * D / 8, wave, NT2,
                                                                              kWaves, lane, ffn2_epi);
        } else {
          // fewer output tiles than waves: the SK waves of a tile take consecutive
          // K ranges; the upper ranges' sums meet the lowest one's through LDS and
          // are added in range order
          constexpr int SK = Sm::KP + 1;
          constexpr int KC = Mode<MODE>::KC;
          constexpr int NC2 = 4 * D / KC, NCS = NC2 / SK;
          static_assert(NC2 % SK == 0, "whole K chunks per range");
          const int tile = wave % NT2, part = wave / NT2;
          const int n = tile * 16 + (lane & 15);
          floatx4 r[2];
          auto keep = [&](int, const floatx4& a0, const floatx4& a1) {
            r[0] = a0;
            r[1] = a1;
          };
          mfma_tiles<MODE, 4 * D / SK, NRT, decltype(keep)&, Mode<MODE>::SPLIT>(
              &sm.u.hid[0][0] + part * NCS * KC, Sm::LDH, p2 + ((size_t)tile * NC2 + (size_t)part * NCS) * 64,
              (size_t)4 * D * D / 8, 0, 1, 1, lane, keep);
          if (part > 0) {
#pragma unroll
            for (int ri = 0; ri < 4 * NRT; ++ri)
              sm.kpart[part - 1][16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3)][n] = r[ri >> 2][ri & 3];
          }
          __syncthreads();
          if (part == 0) {
            const float bias = lp[U.o_ffn2_b + n];
#pragma unroll
            for (int ri = 0; ri < 4 * NRT; ++ri) {
              const int row = 16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3);
              float v = r[ri >> 2][ri & 3];
#pragma unroll
              for (int q = 0; q < Sm::KP; ++q) v += sm.kpart[q][row][n];
              sm.h[row][n] += v + bias;
            }
          }
        }
      }
      __syncthreads();
    }

    // ---- head, Philox draw, decision ----
    if constexpr (TOK) {
      // logits z[m][v] = W_h[v] . h[m] + b[v]: thread (v, half) for samples 16 half .. 16 half + 15
      {
        const int v = tid & (kMaxVocab - 1), half = tid / kMaxVocab;
        if (v < U.vocab && 16 * half < KM) {
          const float* wr = theta + U.head_w + (size_t)v * D;
          float acc[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll 2
          for (int k = 0; k < D; k += 4) {
            const float w0 = wr[k], w1 = wr[k + 1], w2 = wr[k + 2], w3 = wr[k + 3];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              const float4 x = *reinterpret_cast<const float4*>(&sm.h[16 * half + i][k]);
              acc[i] += w0 * x.x + w1 * x.y + w2 * x.z + w3 * x.w;
            }
          }
          const float bias = theta[U.head_b + v];
#pragma unroll
          for (int i = 0; i < 16; ++i) sm.u.z[16 * half + i][v] = acc[i] + bias;
        }
      }
      __syncthreads();
      // softmax and draw: 16 lanes per sample, lane hpart holds logits 16 hpart .. 16 hpart + 15.
      // The token is the largest k >= 1 with u < sum_{j >= k} p_j (else 0), decided as
      // u * total < sum_{j >= k} e_j with e_j = exp(z_j - max), total = sum_j e_j.
      if (hm < KM) {
        const int V = U.vocab, v0 = 16 * hpart;
        float zl[16];
        float mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          zl[j] = v0 + j < V ? sm.u.z[hm][v0 + j] : -INFINITY;
          mx = fmaxf(mx, zl[j]);
        }
        mx = row_max16(mx);
        float e[16], bs = 0.f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          e[j] = v0 + j < V ? expf(zl[j] - mx) : 0.f;
          bs += e[j];
        }
        // suffix sums over the lanes of the row: suf = sum of the block sums of lanes >= hpart
        float suf = bs;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          const float o = __shfl_down(suf, off, 16);
          if (hpart + off < 16) suf += o;
        }
        const float total = __shfl(suf, 0, 16);
        if ((t & 3) == 0) {
          const uint4 w = philox4x32_10(make_uint4((uint32_t)(t >> 2), (uint32_t)(b0 + hm), U.stream_lo, U.stream_hi),
                                        U.seed_lo, U.seed_hi);
          ur[0] = u24(w.x); ur[1] = u24(w.y); ur[2] = u24(w.z); ur[3] = u24(w.w);
        }
        const float ut = ur[t & 3] * total;
        float run = suf - bs;   // the blocks above this lane's
        float cand = -1.f;
#pragma unroll
        for (int j = 15; j >= 0; --j) {
          run += e[j];
          if (cand < 0.f && v0 + j >= 1 && v0 + j < V && ut < run) cand = (float)(v0 + j);
        }
        const int tk = max(0, (int)row_max16(cand));
        float zt = 0.f;
#pragma unroll
        for (int j = 0; j < 16; ++j) zt = v0 + j == tk ? zl[j] : zt;
        zt = row_sum16(zt);
        if (hpart == 0) {
          lq += zt - (mx + logf(total));
          sm.tok[hm] = tk;
          sm.sbuf[hm][t & 63] = (int8_t)(uint8_t)tk;
        }
      }
    } else {
      if (hm < KM) {
        const float* hw = theta + U.head_w;
        float z0 = 0.f, z1 = 0.f;
#pragma unroll
        for (int i = 0; i < D / 16; ++i) {
          const int k = hpart + 16 * i;
          const float x = sm.h[hm][k];
          z0 += x * hw[k];
          z1 += x * hw[D + k];
        }
        z0 = reduce16(z0);
        z1 = reduce16(z1);
        if (hpart == 0) {
          if ((t & 3) == 0) {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)(t >> 2), (uint32_t)(b0 + hm), U.stream_lo, U.stream_hi),
                                          U.seed_lo, U.seed_hi);
            ur[0] = u24(w.x); ur[1] = u24(w.y); ur[2] = u24(w.z); ur[3] = u24(w.w);
          }
          const float d = (z1 + theta[U.head_b + 1]) - (z0 + theta[U.head_b]);
          const float e = expf(-fabsf(d));
          const float pplus = d >= 0.f ? 1.0f / (1.0f + e) : e / (1.0f + e);
          const float u = ur[t & 3];
          const int s = u < pplus ? 1 : 0;
          lq += s ? -softplus(-d) : -softplus(d);
          sm.tok[hm] = s;
          sm.sbuf[hm][t & 63] = s ? (int8_t)1 : (int8_t)-1;
        }
      }
    }
    __syncthreads();
    if ((t & 63) == 63 || t == N - 1) {
      const int base = t & ~63;
      for (int i = tid; i < KM * 64; i += kThreads) {
        const int m = i >> 6, j = i & 63;
        if (m < nb && base + j <= t) U.spins[(size_t)(b0 + m) * N + base + j] = sm.sbuf[m][j];
      }
    }
  }
  if (hpart == 0 && hm < nb) U.logq[b0 + hm] = lq;
  __syncthreads();
}

template <int D, int MODE, int DH, bool TOK, int KM>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeUnit u0, const DecodeUnit* __restrict__ table,
                                                          int n_units, int total_tiles, int* queue) {
  __shared__ DecodeSmem<D, MODE, TOK, KM> sm;
  __shared__ int s_tile;
  bool first = true;
  for (;;) {
    if (threadIdx.x == 0) {
      if (queue) s_tile = atomicAdd(queue, 1);
      else s_tile = first ? (int)blockIdx.x : total_tiles;
    }
    __syncthreads();
    const int tile = s_tile;
    __syncthreads();
    first = false;
    if (tile >= total_tiles) break;
    if (table) {
      int lo = 0, hi = n_units - 1;        // last unit with tile0 <= tile
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
      }
      const DecodeUnit U = table[lo];
      decode_tile<D, MODE, DH, TOK, KM>(sm, U, tile - U.tile0);
    } else {
      decode_tile<D, MODE, DH, TOK, KM>(sm, u0, tile);
    }
  }
}

template <int D, int MODE, int DH, bool TOK, int KM>
hipError_t launch_d(const DecodeUnit& u0, const DecodeUnit* table, int n_units, int total_tiles, int* queue, int grid,
                    hipStream_t s) {
  hipLaunchKernelGGL((decode_kernel<D, MODE, DH, TOK, KM>), dim3(grid), dim3(kThreads), 0, s, u0, table, n_units,
                     total_tiles, queue);
  return hipGetLastError();
}

// The instantiations decode_ext.hip holds (X(D, MODE, DH, TOK, KM)): other head
// widths and token models with 32-sample tiles, and 16-sample tiles of the
// single-spin 16-wide-head kernels (batched launches) and of the patched 3D
// model's kernels.
#define FVAN_DECODE_EXT_LIST(X)                                                                                \
  X(32, 0, 32, false, 32) X(32, 2, 32, false, 32) X(64, 0, 32, false, 32) X(64, 2, 32, false, 32)             \
  X(64, 0, 64, false, 32) X(64, 2, 64, false, 32) X(128, 0, 32, false, 32) X(128, 2, 32, false, 32)           \
  X(128, 0, 64, false, 32) X(128, 2, 64, false, 32) X(32, 0, 16, true, 32) X(32, 2, 16, true, 32)             \
  X(32, 0, 32, true, 32) X(32, 2, 32, true, 32) X(64, 0, 16, true, 32) X(64, 2, 16, true, 32)                 \
  X(64, 0, 32, true, 32) X(64, 2, 32, true, 32) X(64, 0, 64, true, 32) X(64, 2, 64, true, 32)                 \
  X(128, 0, 16, true, 32) X(128, 2, 16, true, 32) X(128, 0, 32, true, 32) X(128, 2, 32, true, 32)             \
  X(128, 0, 64, true, 32) X(128, 2, 64, true, 32)                                                             \
  X(32, 0, 16, false, 16) X(32, 2, 16, false, 16) X(64, 0, 16, false, 16) X(64, 2, 16, false, 16)             \
  X(128, 0, 16, false, 16) X(128, 2, 16, false, 16) X(128, 0, 64, true, 16) X(128, 2, 64, true, 16)
#define FVAN_DECODE_INST(D, MODE, DH, TOK, KM)                                                         \
  template hipError_t launch_d<D, MODE, DH, TOK, KM>(const DecodeUnit&, const DecodeUnit*, int, int, int*, int, \
                                                      hipStream_t);
#define FVAN_DECODE_EXTERN(D, MODE, DH, TOK, KM) extern FVAN_DECODE_INST(D, MODE, DH, TOK, KM)

}  // namespace fvan
