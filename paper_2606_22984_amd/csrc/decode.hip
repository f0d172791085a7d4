// KV-cached ancestral sampling (Alg. 2 of the paper) for gfx950.
//
// One workgroup (8 waves) owns a tile of kM = 32 samples and runs every step
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
#include "device_common.h"
#include "fvan_model.h"

namespace fvan {

constexpr int kM = 32;                 // samples per workgroup (two 16-row MFMA tiles)
constexpr int kThreads = 512;
constexpr int kWaves = kThreads / 64;

int decode_tile_samples() { return kM; }

template <int D, int MODE>
struct DecodeSmem {
  typedef typename Mode<MODE>::ActT A;
  static constexpr int PAD = 16 / (int)sizeof(A);
  static constexpr int LDA = D + PAD;
  static constexpr int LDH = 4 * D + PAD;
  float h[kM][D];
  A a[kM][LDA];
  union {
    float q[kM][D];
    A hid[kM][LDH];
  } u;
  int tok[kM];
  int8_t sbuf[kM][64];
};

__device__ __forceinline__ float reduce16(float v) { return row_sum16(v); }

// LayerNorm of the kM residual rows into the MFMA operand buffer.
template <int D, int MODE>
__device__ __forceinline__ void ln_rows(DecodeSmem<D, MODE>& sm, const float* __restrict__ g,
                                        const float* __restrict__ b) {
  typedef typename Mode<MODE>::ActT T;
  constexpr int PER = D / 16;
  const int m = threadIdx.x >> 4, part = threadIdx.x & 15;
  float x[PER];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    x[i] = sm.h[m][part + 16 * i];
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
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k = part + 16 * i;
    sm.a[m][k] = from_f<T>(x[i] * rstd * g[k] + b[k]);
  }
}

// acc0, acc1 (16 x 16 tile nt of rows 0..15 and 16..31) = A[32 x K] (LDS, row
// stride lda elements) . pack tile nt; each weight fragment is loaded once.
// lo_u4: distance (in 16-byte units) from a split pack's hi part to its lo part.
template <int MODE, int K>
__device__ __forceinline__ void mfma_rowtiles(const typename Mode<MODE>::ActT* A, int lda,
                                              const uint4* __restrict__ pack, size_t lo_u4, int nt, int lane,
                                              floatx4& acc0, floatx4& acc1) {
  constexpr int KC = Mode<MODE>::KC;
  constexpr int NC = K / KC;
  acc0 = floatx4{0.f, 0.f, 0.f, 0.f};
  acc1 = acc0;
  const typename Mode<MODE>::ActT* arow = A + (lane & 15) * lda + (lane >> 4) * (KC / 4);
  const typename Mode<MODE>::ActT* arow1 = arow + 16 * lda;
  const uint4* bp = pack + (size_t)nt * NC * 64 + lane;
  // the weight fragments of G chunks are loaded together, so one L2 latency
  // is exposed per G chunks instead of per chunk
  constexpr int GM = Mode<MODE>::SPLIT ? 2 : 4;
  constexpr int G = NC < GM ? NC : GM;
  static_assert(NC % G == 0, "K chunks in groups of G");
#pragma unroll 1
  for (int c0 = 0; c0 < NC; c0 += G) {
    uint4 bh[G], bl[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      bh[u] = bp[(c0 + u) * 64];
      bl[u] = Mode<MODE>::SPLIT ? bp[(c0 + u) * 64 + lo_u4] : bh[u];
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
      Frag<MODE>::step2v(arow + (c0 + u) * KC, arow1 + (c0 + u) * KC, bh[u], bl[u], acc0, acc1);
  }
}

template <int D, int MODE>
__device__ void decode_tile(DecodeSmem<D, MODE>& sm, const DecodeUnit& U, int local_tile) {
  typedef typename Mode<MODE>::KvT T;
  typedef DecodeSmem<D, MODE> Sm;
  constexpr int VEC = Chunk<T>::N;
  constexpr int LPR = D / VEC;          // lanes per K/V row
  constexpr int RPL = 64 / LPR;         // rows per wave load
  constexpr int LPH = kHeadDim / VEC;   // lanes per head
  constexpr int UNR = 4;                // rows per lane in flight
  constexpr float kScaleLog2 = 0.25f * 1.4426950408889634f;   // 1/sqrt(16) * log2(e)

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int b0 = local_tile * kM;
  const int nb = min(kM, U.B - b0);
  const int N = U.N, P = U.P, R = U.R, S = U.S, nl = U.n_layers, dt = U.d_token;
  const float* __restrict__ theta = U.theta;
  const char* wbase = reinterpret_cast<const char*>(U.wpack);
  T* kvbase = reinterpret_cast<T*>(U.kv);
  const size_t plane = (size_t)S * D;   // elements of one K (or V) block

  // head-phase ownership: thread 16*m handles sample row m
  const int hm = tid >> 4, hpart = tid & 15;
  float lq = 0.f;
  float ur[4] = {0.f, 0.f, 0.f, 0.f};
  if (tid < kM) sm.tok[tid] = 0;   // start token
  __syncthreads();

  for (int t = 0; t < N; ++t) {
    // ---- concatenated embedding [tok_emb[tok]; pos_emb[t]] ----
    for (int i = tid; i < kM * D; i += kThreads) {
      const int m = i / D, k = i % D;
      sm.h[m][k] = k < dt ? theta[sm.tok[m] * dt + k] : theta[U.pos_off + (size_t)t * (D - dt) + (k - dt)];
    }
    const int slot = t < P ? t : P + (t - P) % R;
    const int nvis = t < P ? t + 1 : P + min(t - P + 1, R);
    __syncthreads();

    for (int l = 0; l < nl; ++l) {
      const float* lp = theta + U.layer0 + (size_t)l * U.layer_stride;
      const char* wl = wbase + (size_t)l * U.p_layer_stride;
      ln_rows<D, MODE>(sm, lp + U.o_ln1_g, lp + U.o_ln1_b);
      __syncthreads();

      // ---- QKV projection; k_t, v_t appended to the cache ----
      {
        const uint4* pk = reinterpret_cast<const uint4*>(wl + U.p_qkv);
        for (int nt = wave; nt < 3 * D / 16; nt += kWaves) {
          floatx4 acc[2];
          mfma_rowtiles<MODE, D>(&sm.a[0][0], Sm::LDA, pk, (size_t)3 * D * D / 8, nt, lane, acc[0], acc[1]);
          const int n = nt * 16 + (lane & 15);
          const float bias = lp[U.o_qkv_b + n];
#pragma unroll
          for (int ri = 0; ri < 8; ++ri) {
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
        }
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
              kk[u] = *reinterpret_cast<const uint4*>(Kb + (size_t)s * D + lcol);
              vv[u] = *reinterpret_cast<const uint4*>(Kb + plane + (size_t)s * D + lcol);
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
      ln_rows<D, MODE>(sm, lp + U.o_ln2_g, lp + U.o_ln2_b);
      __syncthreads();
      {
        const uint4* p1 = reinterpret_cast<const uint4*>(wl + U.p_ffn1);
        for (int nt = wave; nt < 4 * D / 16; nt += kWaves) {
          floatx4 acc[2];
          mfma_rowtiles<MODE, D>(&sm.a[0][0], Sm::LDA, p1, (size_t)4 * D * D / 8, nt, lane, acc[0], acc[1]);
          const int n = nt * 16 + (lane & 15);
          const float bias = lp[U.o_ffn1_b + n];
#pragma unroll
          for (int ri = 0; ri < 8; ++ri)
            sm.u.hid[16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3)][n] =
                from_f<typename Mode<MODE>::ActT>(gelu(acc[ri >> 2][ri & 3] + bias));
        }
      }
      __syncthreads();
      {
        const uint4* p2 = reinterpret_cast<const uint4*>(wl + U.p_ffn2);
        for (int nt = wave; nt < D / 16; nt += kWaves) {
          floatx4 acc[2];
          mfma_rowtiles<MODE, 4 * D>(&sm.u.hid[0][0], Sm::LDH, p2, (size_t)4 * D * D / 8, nt, lane, acc[0], acc[1]);
          const int n = nt * 16 + (lane & 15);
          const float bias = lp[U.o_ffn2_b + n];
#pragma unroll
          for (int ri = 0; ri < 8; ++ri) sm.h[16 * (ri >> 2) + 4 * (lane >> 4) + (ri & 3)][n] += acc[ri >> 2][ri & 3] + bias;
        }
      }
      __syncthreads();
    }

    // ---- head, Philox draw, decision ----
    {
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
    __syncthreads();
    if ((t & 63) == 63 || t == N - 1) {
      const int base = t & ~63;
      for (int i = tid; i < kM * 64; i += kThreads) {
        const int m = i >> 6, j = i & 63;
        if (m < nb && base + j <= t) U.spins[(size_t)(b0 + m) * N + base + j] = sm.sbuf[m][j];
      }
    }
  }
  if (hpart == 0 && hm < nb) U.logq[b0 + hm] = lq;
  __syncthreads();
}

template <int D, int MODE>
__global__ __launch_bounds__(kThreads) void decode_kernel(DecodeUnit u0, const DecodeUnit* __restrict__ table,
                                                          int n_units, int total_tiles, int* queue) {
  __shared__ DecodeSmem<D, MODE> sm;
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
      decode_tile<D, MODE>(sm, U, tile - U.tile0);
    } else {
      decode_tile<D, MODE>(sm, u0, tile);
    }
  }
}

template <int D, int MODE>
static hipError_t launch_d(const DecodeUnit& u0, const DecodeUnit* table, int n_units, int total_tiles, int* queue,
                           int grid, hipStream_t s) {
  hipLaunchKernelGGL((decode_kernel<D, MODE>), dim3(grid), dim3(kThreads), 0, s, u0, table, n_units, total_tiles,
                     queue);
  return hipGetLastError();
}

template <int D>
static hipError_t dispatch_mode(int precision, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                                int total_tiles, int* queue, int grid, hipStream_t s) {
  switch (precision) {
    case FVAN_FP32: return launch_d<D, 0>(u0, table, n_units, total_tiles, queue, grid, s);
    case FVAN_BF16_SPLIT: return launch_d<D, 2>(u0, table, n_units, total_tiles, queue, grid, s);
    default: return hipErrorInvalidValue;
  }
}

static hipError_t dispatch(int d_model, int precision, const DecodeUnit& u0, const DecodeUnit* table, int n_units,
                           int total_tiles, int* queue, int grid, hipStream_t s) {
  switch (d_model) {
    case 32: return dispatch_mode<32>(precision, u0, table, n_units, total_tiles, queue, grid, s);
    case 64: return dispatch_mode<64>(precision, u0, table, n_units, total_tiles, queue, grid, s);
    case 128: return dispatch_mode<128>(precision, u0, table, n_units, total_tiles, queue, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_decode(int d_model, int precision, const DecodeUnit* units_dev, int n_units, int total_tiles,
                         int* queue_counter, int grid, hipStream_t s) {
  DecodeUnit dummy{};
  return dispatch(d_model, precision, dummy, units_dev, n_units, total_tiles, queue_counter, grid, s);
}

hipError_t launch_decode_single(int d_model, int precision, const DecodeUnit& u, int tiles, hipStream_t s) {
  return dispatch(d_model, precision, u, nullptr, 1, tiles, nullptr, tiles, s);
}

}  // namespace fvan
