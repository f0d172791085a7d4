// Row-parallel kernels shared by the teacher-forced forward and the backward
// pass (which recomputes each layer's forward): LayerNorm, the row GEMM on
// packed weights with fused epilogues.
#pragma once

#include <type_traits>

#include <algorithm>

#include "device_common.h"
#include "passes.h"

namespace fvan {

// ---------------------------------------------------------------- LayerNorm
// 64 rows per workgroup, 16 lanes per row.  Optional outputs: row-major `out`
// [rows x D] and feature-major `outT` [D x ldT] (element (r, k) at k*ldT + r).
template <int D, typename OT, typename TT>
__global__ __launch_bounds__(256) void ln_kernel(const float* __restrict__ X, int64_t rows,
                                                 const float* __restrict__ g, const float* __restrict__ b,
                                                 OT* __restrict__ out, TT* __restrict__ outT, int64_t ldT) {
  constexpr int PER = D / 16;
  __shared__ float tile[64][D + 1];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int grp = threadIdx.x >> 4, part = threadIdx.x & 15;
  for (int rr = grp; rr < 64; rr += 16) {
    const int64_t r = r0 + rr;
    if (r >= rows) break;
    const float* x = X + r * D;
    float v[PER];
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) { v[i] = x[part + 16 * i]; s += v[i]; }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    const float mean = s * (1.0f / D);
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) { v[i] -= mean; q += v[i] * v[i]; }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) q += __shfl_xor(q, o, 16);
    const float rstd = rsqrtf(q * (1.0f / D) + kLnEps);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = part + 16 * i;
      const float y = v[i] * rstd * g[k] + b[k];
      if (out) out[r * D + k] = from_f<OT>(y);
      tile[rr][k] = y;
    }
  }
  if (outT) {
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * D; i += 256) {
      const int k = i >> 6, rr = i & 63;
      if (r0 + rr < rows) outT[(int64_t)k * ldT + r0 + rr] = from_f<TT>(tile[rr][k]);
    }
  }
}

// A fragments of one 16-row tile computed as LayerNorm(X row) (affine g, b;
// population variance, eps kLnEps): lane (g, c) holds row c's elements
// cc*KC + g*LK .. +LK for every chunk cc, so the four lanes of a row together
// hold it whole and the row statistics are two pair reductions.  NT: the rows are
// read with non-temporal loads (for a kernel that reads each row once, long after
// it was written, while L2 serves it re-read weights).
template <int MODE, int K, bool NT = false>
__device__ __forceinline__ void load_ln_frags(const float* __restrict__ X, int64_t row,
                                              const float* __restrict__ gam, const float* __restrict__ bet, int g,
                                              FragA<MODE>* fa) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int KC = Mode<MODE>::KC, LK = KC / 4, NC = K / KC;
  float x[NC][LK];
  float s = 0.f;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc)
#pragma unroll
    for (int i = 0; i < LK; i += 4) {
      const float* xp = X + row * K + cc * KC + g * LK + i;
      const float4 v = NT ? load_nt4(xp) : *reinterpret_cast<const float4*>(xp);
      x[cc][i] = v.x; x[cc][i + 1] = v.y; x[cc][i + 2] = v.z; x[cc][i + 3] = v.w;
      s += (v.x + v.y) + (v.z + v.w);
    }
  const float mean = sum_xor32(sum_xor16(s)) * (1.0f / K);
  float q = 0.f;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc)
#pragma unroll
    for (int i = 0; i < LK; ++i) { x[cc][i] -= mean; q += x[cc][i] * x[cc][i]; }
  const float rstd = rsqrtf(sum_xor32(sum_xor16(q)) * (1.0f / K) + kLnEps);
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    alignas(16) AT af[LK];
#pragma unroll
    for (int i = 0; i < LK; ++i) {
      const int k = cc * KC + g * LK + i;
      af[i] = from_f<AT>(x[cc][i] * rstd * gam[k] + bet[k]);
    }
    fa[cc].load(af);
  }
}

// ---------------------------------------------------------------- row GEMM
// C[r][n] = sum_k A[r][k] W[n][k] over a packed W [NOUT x K]; 128 rows per
// workgroup, one wave per 32 rows (two 16-row MFMA tiles: every weight fragment
// a wave loads from L2 feeds both).  A is read from HBM once: for K <= 128 the
// wave's A fragments stay in registers across all output tiles; for larger K
// (NOUT <= 128) the loop runs K-outer with every output tile's accumulator live.
constexpr int kGemmRows = 128;

template <int MODE, int K, int NOUT, int EPI>
__global__ __launch_bounds__(256) void gemm_rows_kernel(const typename Mode<MODE>::ActT* __restrict__ A,
                                                        int64_t rows, const uint4* __restrict__ pack,
                                                        EpiArgs e) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;                 // A elements per lane per chunk
  constexpr int NC = K / KC;
  constexpr int NT = NOUT / 16;
  constexpr size_t LO = (size_t)NOUT * K / 8;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kGemmRows + wave * 32;
  if (rbase >= rows) return;
  // clamp the A rows; stores are guarded (A is not read when the rows come from ln_x)
  const AT* arow[2] = {A + std::min<int64_t>(rbase + c, rows - 1) * K + g * LK,
                       A + std::min<int64_t>(rbase + 16 + c, rows - 1) * K + g * LK};
  auto load_frag = [&](FragA<MODE>& fa, int rt, int cc) {
    alignas(16) AT af[LK];
#pragma unroll
    for (int i = 0; i < LK; i += 16 / (int)sizeof(AT))
      *reinterpret_cast<uint4*>(&af[i]) = *reinterpret_cast<const uint4*>(arow[rt] + cc * KC + i);
    fa.load(af);
  };
  auto epilogue = [&](int nt, const floatx4& a0, const floatx4& a1) {
    const int n = nt * 16 + c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rbase + 4 * g + i;
      if (r < rows) Epi<MODE, EPI>::apply(e, r, n, NOUT, a0[i]);
      if (r + 16 < rows) Epi<MODE, EPI>::apply(e, r + 16, n, NOUT, a1[i]);
    }
  };
  if constexpr (K <= 128) {
    FragA<MODE> fa[2][NC];                   // the wave's A fragments, converted once
    if (e.ln_x) {                            // A = LayerNorm(ln_x rows), computed here
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
        load_ln_frags<MODE, K>(e.ln_x, std::min<int64_t>(rbase + 16 * rt + c, rows - 1), e.ln_g, e.ln_b, g, fa[rt]);
    } else {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) { load_frag(fa[0][cc], 0, cc); load_frag(fa[1][cc], 1, cc); }
    }
    for (int nt = 0; nt < NT; ++nt) {
      floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
      const uint4* bp = pack + (size_t)nt * NC * 64 + lane;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        a0 = fa[0][cc].mma(bp + cc * 64, bp + cc * 64 + LO, a0);
        a1 = fa[1][cc].mma(bp + cc * 64, bp + cc * 64 + LO, a1);
      }
      epilogue(nt, a0, a1);
    }
  } else {
    static_assert(NT <= 8, "K-outer row GEMM keeps at most 8 output tiles live");
    floatx4 acc[2][NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) { acc[0][nt] = floatx4{0.f, 0.f, 0.f, 0.f}; acc[1][nt] = acc[0][nt]; }
    const uint4* bp = pack + lane;
    for (int cc = 0; cc < NC; ++cc) {
      FragA<MODE> f0, f1;
      load_frag(f0, 0, cc);
      load_frag(f1, 1, cc);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const uint4* b = bp + ((size_t)nt * NC + cc) * 64;
        acc[0][nt] = f0.mma(b, b + LO, acc[0][nt]);
        acc[1][nt] = f1.mma(b, b + LO, acc[1][nt]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) epilogue(nt, acc[0][nt], acc[1][nt]);
  }
}

// Row GEMM with an LDS-staged epilogue for the wide outputs (K <= 128: the QKV
// projection and FFN1 with their GELU / GELU' epilogues).  Each group of four
// 16-column tiles is computed into an R x 64 tile in LDS (R = 64 or 128 rows);
// the workgroup then writes the row-major outputs as 256-byte row segments and
// the feature-major copy as R*4-byte column segments (16-byte stores), instead
// of one scattered element per lane.
//   EPI_GELU : h = acc + bias; hpre_out[r][n] = h, out[r][n] = GELU(h), outT[n][r] = GELU(h)
//   EPI_DGELU: d = acc * GELU'(hpre_in[r][n]); out[r][n] = d, outT[n][r] = d
//   EPI_STORE_KV: out[r][n] = acc + bias[n] in the K/V element type
// (each output only if its pointer is set).
template <typename T>
__device__ __forceinline__ void store4(T* p, float a, float b, float c, float d) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
  } else {
    typedef __attribute__((__vector_size__(4 * sizeof(T)))) T v4;
    v4 v = {from_f<T>(a), from_f<T>(b), from_f<T>(c), from_f<T>(d)};
    *reinterpret_cast<v4*>(p) = v;
  }
}

// 16-row tiles per wave of the staged kernel: two for the QKV projection (each
// weight fragment feeds both; measured faster), one for the HBM-bound 512-wide
// GELU / GELU' epilogues, where the larger tile halves the occupancy.
template <int EPI> struct StagedRowTiles { static constexpr int value = EPI == EPI_STORE_KV ? 2 : 1; };

template <int MODE, int K, int NOUT, int EPI>
__global__ __launch_bounds__(256) void gemm_rows_staged_kernel(const typename Mode<MODE>::ActT* __restrict__ A,
                                                               int64_t rows, const uint4* __restrict__ pack,
                                                               EpiArgs e) {
  typedef typename Mode<MODE>::ActT AT;
  static_assert(K <= 128 && NOUT % 64 == 0, "staged row GEMM: K <= 128, NOUT a multiple of 64");
  static_assert(EPI == EPI_GELU || EPI == EPI_DGELU || EPI == EPI_STORE_KV,
                "staged row GEMM: GELU, GELU' or K/V-type store epilogue");
  typedef typename std::conditional<EPI == EPI_STORE_KV, typename Mode<MODE>::KvT, AT>::type OT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int NC = K / KC;
  constexpr int NG = NOUT / 64;
  constexpr int RT = StagedRowTiles<EPI>::value; // 16-row tiles per wave
  constexpr int R = 64 * RT;                     // rows per workgroup
  constexpr size_t LO = (size_t)NOUT * K / 8;
  __shared__ __align__(16) float Ev[R][68];                               // out / outT values
  __shared__ __align__(16) float Eh[EPI == EPI_STORE_KV ? 1 : R][68];     // GELU: hpre_out; GELU': hpre_in
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, c = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  FragA<MODE> fa[RT][NC];                    // the wave's A fragments (rows 16 RT w ..), converted once
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t ra = std::min<int64_t>(r0 + wave * 16 * RT + 16 * rt + c, rows - 1);   // stores are guarded
    if (e.ln_x) {
      load_ln_frags<MODE, K>(e.ln_x, ra, e.ln_g, e.ln_b, g, fa[rt]);
    } else {
      const AT* arow = A + ra * K + g * LK;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        alignas(16) AT af[LK];
#pragma unroll
        for (int i = 0; i < LK; i += 16 / (int)sizeof(AT))
          *reinterpret_cast<uint4*>(&af[i]) = *reinterpret_cast<const uint4*>(arow + cc * KC + i);
        fa[rt][cc].load(af);
      }
    }
  }
  const bool full = r0 + R <= rows;
  OT* out = reinterpret_cast<OT*>(e.out);
  AT* outT = reinterpret_cast<AT*>(e.outT);
  for (int ng = 0; ng < NG; ++ng) {
    if constexpr (EPI == EPI_DGELU) {
      // stage the pre-activation tile (256-byte row segments)
#pragma unroll
      for (int k = 0; k < R / 16; ++k) {
        const int idx = tid + 256 * k, row = idx >> 4, c4 = (idx & 15) * 4;
        const int64_t r = std::min<int64_t>(r0 + row, rows - 1);
        *reinterpret_cast<float4*>(&Eh[row][c4]) =
            *reinterpret_cast<const float4*>(e.hpre_in + r * NOUT + ng * 64 + c4);
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int nt = ng * 4 + u;
      floatx4 acc[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt] = floatx4{0.f, 0.f, 0.f, 0.f};
      const uint4* bp = pack + (size_t)nt * NC * 64 + lane;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = fa[rt][cc].mma(bp + cc * 64, bp + cc * 64 + LO, acc[rt]);
      const int col = 16 * u + c;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = wave * 16 * RT + 16 * rt + 4 * g + i;
          if constexpr (EPI == EPI_GELU) {
            const float hv = acc[rt][i] + e.bias[ng * 64 + col];
            Eh[row][col] = hv;
            Ev[row][col] = gelu(hv);
          } else if constexpr (EPI == EPI_STORE_KV) {
            Ev[row][col] = acc[rt][i] + e.bias[ng * 64 + col];
          } else {
            Ev[row][col] = acc[rt][i] * gelu_grad(Eh[row][col]);
          }
        }
    }
    __syncthreads();
    const int n0 = ng * 64;
    // row-major outputs: thread -> (row, 4 columns); 16 threads cover a 64-column row segment
#pragma unroll
    for (int k = 0; k < R / 16; ++k) {
      const int idx = tid + 256 * k, row = idx >> 4, c4 = (idx & 15) * 4;
      const int64_t r = r0 + row;
      if (r < rows) {
        if (out) store4(out + r * NOUT + n0 + c4, Ev[row][c4], Ev[row][c4 + 1], Ev[row][c4 + 2], Ev[row][c4 + 3]);
        if constexpr (EPI == EPI_GELU) {
          if (e.hpre_out)
            *reinterpret_cast<float4*>(e.hpre_out + r * NOUT + n0 + c4) =
                *reinterpret_cast<const float4*>(&Eh[row][c4]);
        }
      }
    }
    // feature-major copy: thread -> (column, 4 rows); R/4 threads cover a column's R rows
    if constexpr (EPI != EPI_STORE_KV) {
      if (outT) {
#pragma unroll
        for (int k = 0; k < R / 16; ++k) {
          const int idx = tid + 256 * k, col = idx / (R / 4), q4 = (idx % (R / 4)) * 4;
          AT* dst = outT + (int64_t)(n0 + col) * e.ldT + r0 + q4;
          if (full) {
            store4(dst, Ev[q4][col], Ev[q4 + 1][col], Ev[q4 + 2][col], Ev[q4 + 3][col]);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (r0 + q4 + i < rows) dst[i] = from_f<AT>(Ev[q4 + i][col]);
          }
        }
      }
    }
    __syncthreads();
  }
}

// Fused feed-forward block of the teacher-forced forward pass:
//   out[r] = resid[r] + W2 GELU(W1 a[r] + b1) + b2,   W1 [4D x D], W2 [D x 4D],
// a[r] = LayerNorm(X rows; ln_g, ln_b) computed in the kernel.
// 128 rows per workgroup, one 16-row MFMA tile per wave (8 waves).  The hidden
// layer is walked 32 units at a time: the chunk's fragments of W1 (its rows)
// and W2 (its columns) are staged in LDS once for all eight waves, the next
// chunk's fetched into registers meanwhile, and each wave's hidden activations
// go through a wave-private LDS tile straight into the W2 product, so the
// 4D-wide hidden layer never reaches HBM.  (Each wave loading every weight for
// its own rows made the kernel bound by L2 reads of the weights.)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kFfnRows = 128;                // rows per fused-FFN workgroup

template <int MODE, int D>
__global__ __launch_bounds__(512, 4) void ffn_fused_kernel(const float* __restrict__ X, const float* __restrict__ ln_g,
                                                        const float* __restrict__ ln_b, int64_t rows,
                                                        const uint4* __restrict__ p1, const uint4* __restrict__ p2,
                                                        const float* __restrict__ b1, const float* __restrict__ b2,
                                                        const float* __restrict__ resid, float* __restrict__ out) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int NW = 8;                      // waves
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int NPL = Mode<MODE>::SPLIT ? 2 : 1;   // weight planes (hi, lo)
  constexpr int NC1 = D / KC;                // K chunks of the W1 product
  constexpr int HC = 32;                     // hidden units per chunk
  constexpr int NH = 4 * D / HC;
  constexpr int NT1 = HC / 16;               // W1 output tiles per chunk
  constexpr int NT2 = D / 16;                // W2 output tiles
  constexpr int NC2 = 4 * D / KC;            // K chunks of the W2 product
  constexpr int NC2H = HC / KC;              // ... per hidden chunk
  constexpr size_t LO = (size_t)4 * D * D / 8;   // hi-to-lo distance of a split pack (both matrices 4D^2)
  constexpr int S1 = NT1 * NC1 * 64;         // fragments of a W1 chunk, per plane
  constexpr int S2 = NT2 * NC2H * 64;        // fragments of a W2 chunk, per plane
  constexpr int SW = S1 + S2;
  constexpr int NPRE = (NPL * SW + 64 * NW - 1) / (64 * NW);
  static_assert(NPRE <= 4, "at most four staged fragments per thread");
  static_assert(64 * NW == 512, "staging strides assume 512 threads");
  constexpr int LDH = HC + 4;
  __shared__ __align__(16) uint4 Ws[NPL][SW];      // [W1 chunk | W2 chunk]
  __shared__ __align__(16) AT Hs[NW][16][LDH];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kFfnRows + wave * 16;
  auto src = [&](int hc, int idx) -> const uint4* {
    const int pl = idx / SW, j = idx % SW;
    const size_t lo = pl ? LO : 0;
    if (j < S1) return p1 + (size_t)hc * S1 + j + lo;
    const int k = j - S1, t2 = k / (NC2H * 64), rest = k % (NC2H * 64);
    return p2 + ((size_t)t2 * NC2 + (size_t)hc * NC2H) * 64 + rest + lo;
  };
  uint4 q0{}, q1{}, q2{}, q3{};
#define FVAN_FF_FETCH(hc)                                                            \
  do {                                                                               \
    if (NPRE > 0 && tid < NPL * SW) q0 = *src(hc, tid);                              \
    if (NPRE > 1 && tid + 512 < NPL * SW) q1 = *src(hc, tid + 512);                  \
    if (NPRE > 2 && tid + 1024 < NPL * SW) q2 = *src(hc, tid + 1024);                \
    if (NPRE > 3 && tid + 1536 < NPL * SW) q3 = *src(hc, tid + 1536);                \
  } while (0)
#define FVAN_FF_COMMIT()                                                             \
  do {                                                                               \
    uint4* w = &Ws[0][0];                                                            \
    if (NPRE > 0 && tid < NPL * SW) w[tid] = q0;                                     \
    if (NPRE > 1 && tid + 512 < NPL * SW) w[tid + 512] = q1;                         \
    if (NPRE > 2 && tid + 1024 < NPL * SW) w[tid + 1024] = q2;                       \
    if (NPRE > 3 && tid + 1536 < NPL * SW) w[tid + 1536] = q3;                       \
  } while (0)
  FVAN_FF_FETCH(0);
  FragA<MODE> fa[NC1];                       // the wave's A fragments, converted once (rows clamped)
  load_ln_frags<MODE, D>(X, std::min<int64_t>(rbase + c, rows - 1), ln_g, ln_b, g, fa);
  floatx4 acc2[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) acc2[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  FVAN_FF_COMMIT();
  __syncthreads();
  if (NH > 1) FVAN_FF_FETCH(1);
  AT (*H)[LDH] = Hs[wave];
  const uint4* W1s = &Ws[0][0];
  const uint4* W2s = &Ws[0][S1];
  constexpr int PLO = NPL > 1 ? SW : 0;      // hi-to-lo distance in the stage
  for (int hc = 0; hc < NH; ++hc) {
#pragma unroll
    for (int t = 0; t < NT1; ++t) {
      floatx4 a0 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int cc = 0; cc < NC1; ++cc) {
        const int f = (t * NC1 + cc) * 64 + lane;
        a0 = fa[cc].mma(W1s + f, W1s + f + PLO, a0);
      }
      const float bias = b1[hc * HC + t * 16 + c];
#pragma unroll
      for (int i = 0; i < 4; ++i) H[4 * g + i][t * 16 + c] = from_f<AT>(gelu(a0[i] + bias));
    }
    wave_lds_sync();
#pragma unroll
    for (int cc = 0; cc < NC2H; ++cc) {
      FragA<MODE> h0;
      h0.load(&H[c][cc * KC + g * LK]);
#pragma unroll
      for (int t = 0; t < NT2; ++t) {
        const int f = (t * NC2H + cc) * 64 + lane;
        acc2[t] = h0.mma(W2s + f, W2s + f + PLO, acc2[t]);
      }
    }
    __syncthreads();                         // every wave is done with this chunk's weights and tiles
    if (hc + 1 < NH) {
      FVAN_FF_COMMIT();
      __syncthreads();
      if (hc + 2 < NH) FVAN_FF_FETCH(hc + 2);
    }
  }
#undef FVAN_FF_FETCH
#undef FVAN_FF_COMMIT
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
    const int n = t * 16 + c;
    const float bias = b2[n];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rbase + 4 * g + i;
      if (r < rows) out[r * D + n] = resid[r * D + n] + acc2[t][i] + bias;
    }
  }
}

// LayerNorm backward of the 16 rows a wave holds as MFMA accumulators (lane
// (g, c): rows rbase+4g+i, columns 16t+c of dA, the gradient at the LayerNorm's
// output; y = LN(x) with gain ln_g, shift ln_b):
//   out[r] = resid[r] + LN'(dA[r])       (row-major, rows < rows)
//   At[k][r] = y[r][k]                   (feature-major, for a weight gradient)
//   Rt[k][r] = resid[r][k]               (feature-major, if Rt is set)
// and the wave's column sums of dA * xhat (the gain gradient) and of dA (the
// shift gradient) into red[0 .. D) and red[D .. 2D) (lanes with g = 0 write).
template <int D>
__device__ __forceinline__ void ln_bwd_rows(floatx4 (&acc)[D / 16], const float* __restrict__ X,
                                            const float* __restrict__ resid, const float* __restrict__ ln_g,
                                            const float* __restrict__ ln_b, int64_t rbase, int64_t rows, int g,
                                            int c, float* __restrict__ out, float* __restrict__ At,
                                            float* __restrict__ Rt, int64_t ldT, float* __restrict__ red) {
  constexpr int NT2 = D / 16;
  const bool full = rbase + 16 <= rows;
  float xh[NT2][4], dyv[NT2][4];
  bool live[4];
  float rstd[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = rbase + 4 * g + i;
    live[i] = r < rows;
    const int64_t rr = std::min<int64_t>(r, rows - 1);
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < NT2; ++t) {
      xh[t][i] = X[rr * D + 16 * t + c];
      dyv[t][i] = resid[rr * D + 16 * t + c];
      s += xh[t][i];
    }
    const float mean = row_sum16(s) * (1.0f / D);
    float q = 0.f;
#pragma unroll
    for (int t = 0; t < NT2; ++t) {
      xh[t][i] -= mean;
      q += xh[t][i] * xh[t][i];
    }
    rstd[i] = rsqrtf(row_sum16(q) * (1.0f / D) + kLnEps);
#pragma unroll
    for (int t = 0; t < NT2; ++t) xh[t][i] *= rstd[i];
  }
  float s1[4] = {0.f, 0.f, 0.f, 0.f}, s2[4] = {0.f, 0.f, 0.f, 0.f};
  float pg[NT2], pb[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
    const int k = 16 * t + c;
    const float gk = ln_g[k], bk = ln_b[k];
    pg[t] = 0.f;
    pb[t] = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float a = live[i] ? acc[t][i] : 0.f;
      pg[t] += a * xh[t][i];
      pb[t] += a;
      acc[t][i] = a * gk;                    // now dy = dA * gain
      s1[i] += acc[t][i];
      s2[i] += acc[t][i] * xh[t][i];
    }
    // feature-major LN output (and resid): four consecutive rows per lane
    float* ap = At + (int64_t)k * ldT + rbase + 4 * g;
    float* yp = Rt ? Rt + (int64_t)k * ldT + rbase + 4 * g : nullptr;
    if (full) {
      *reinterpret_cast<float4*>(ap) = make_float4(xh[t][0] * gk + bk, xh[t][1] * gk + bk, xh[t][2] * gk + bk,
                                                   xh[t][3] * gk + bk);
      if (yp) *reinterpret_cast<float4*>(yp) = make_float4(dyv[t][0], dyv[t][1], dyv[t][2], dyv[t][3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (live[i]) {
          ap[i] = xh[t][i] * gk + bk;
          if (yp) yp[i] = dyv[t][i];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s1[i] = row_sum16(s1[i]) * (1.0f / D);
    s2[i] = row_sum16(s2[i]) * (1.0f / D);
  }
#pragma unroll
  for (int t = 0; t < NT2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rbase + 4 * g + i;
      if (live[i]) out[r * D + 16 * t + c] = dyv[t][i] + rstd[i] * (acc[t][i] - s1[i] - xh[t][i] * s2[i]);
    }
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
    pg[t] = sum_xor32(sum_xor16(pg[t]));
    pb[t] = sum_xor32(sum_xor16(pb[t]));
    if (g == 0) {
      red[16 * t + c] = pg[t];
      red[D + 16 * t + c] = pb[t];
    }
  }
}

// Fused feed-forward backward of one layer, with the block's forward recomputed
// in place (x = the post-attention residual XM, dY = the gradient arriving at
// the block's output):
//   a = LN2(x), h = W1 a + b1, g = GELU(h)             (recompute)
//   dG = W2^T dY, dH = dG * GELU'(h), dA = W1^T dH      (back through W2, GELU, W1)
//   out = dY + LN2'(dA)                                 (LayerNorm backward and the residual)
// plus the feature-major operands of the weight gradients, Gt = g^T and
// dHt = dH^T [4D x ldT], At = a^T and dYt = dY^T [D x ldT], and per-workgroup
// partial sums of the LN2 gain and shift gradients (part[block][2D]).
// 128 rows per workgroup, one 16-row MFMA tile per wave (8 waves).  The hidden
// layer is walked 32 units at a time: the chunk's weight fragments (rows of W1
// and W2^T, columns of W1^T) are staged in LDS once for all eight waves, in two
// alternating buffers so that the next chunk is committed while the current one
// is read (one barrier per chunk), the chunk after it fetched into registers
// meanwhile.  g and dH reach HBM only as the two feature-major weight-gradient
// operands, stored straight from the accumulator layout (a lane holds four
// consecutive rows of one hidden unit); dH also goes through a wave-private LDS
// tile, where the dA product reads it in the A layout.  (One wave loading every weight for
// its own 16 rows made the kernel bound by L2 reads of the weights.)
// p1: W1 [4D x D] pack; p2t: W2^T [4D x D] pack; p1t: W1^T [D x 4D] pack.
constexpr int kFfnBwdRows = 128;

template <int MODE, int D>
__global__ __launch_bounds__(512) void ffn_bwd_fused_kernel(
    const float* __restrict__ X, const float* __restrict__ dY, const float* __restrict__ ln_g,
    const float* __restrict__ ln_b, int64_t rows, const uint4* __restrict__ p1, const uint4* __restrict__ p2t,
    const uint4* __restrict__ p1t, const float* __restrict__ b1, typename Mode<MODE>::ActT* __restrict__ Gt,
    typename Mode<MODE>::ActT* __restrict__ dHt, typename Mode<MODE>::ActT* __restrict__ At,
    typename Mode<MODE>::ActT* __restrict__ dYt, int64_t ldT, float* __restrict__ out, float* __restrict__ part) {
  typedef typename Mode<MODE>::ActT AT;
  static_assert(sizeof(AT) == 4, "FP32 activations");
  constexpr int NW = 8;                      // waves
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int NPL = Mode<MODE>::SPLIT ? 2 : 1;   // weight planes (hi, lo)
  constexpr int NC1 = D / KC;                // K chunks of the D-wide products
  constexpr int HC = 32;                     // hidden units per chunk
  constexpr int NH = 4 * D / HC;
  constexpr int NT1 = HC / 16;               // h / dG tiles per chunk
  constexpr int NT2 = D / 16;                // output tiles of dA
  constexpr int NC2 = 4 * D / KC;            // K chunks of the dA product
  constexpr int NC2H = HC / KC;              // ... per hidden chunk
  constexpr size_t LO = (size_t)4 * D * D / 8;
  constexpr int S1 = NT1 * NC1 * 64;         // fragments of a W1 (or W2^T) chunk, per plane
  constexpr int S3 = NT2 * NC2H * 64;        // fragments of a W1^T chunk, per plane
  constexpr int SW = 2 * S1 + S3;
  constexpr int NPRE = (NPL * SW + 64 * NW - 1) / (64 * NW);   // staged fragments per thread
  constexpr int LDH = HC + 4;
  __shared__ __align__(16) uint4 Ws[2][NPL][SW];   // two stages of [W1 chunk | W2^T chunk | W1^T chunk]
  __shared__ __align__(16) float Hd[NW][16][LDH];
  __shared__ float red[NW][2 * D];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kFfnBwdRows + wave * 16;
  const bool full = rbase + 16 <= rows;
  // staged fragment idx (plane pl, slot j) -> its place in the packs
  auto src = [&](int hc, int idx) -> const uint4* {
    const int pl = idx / SW, j = idx % SW;
    const size_t lo = pl ? LO : 0;
    if (j < S1) return p1 + (size_t)hc * S1 + j + lo;
    if (j < 2 * S1) return p2t + (size_t)hc * S1 + (j - S1) + lo;
    const int k = j - 2 * S1, t2 = k / (NC2H * 64), rest = k % (NC2H * 64);
    return p1t + ((size_t)t2 * NC2 + (size_t)hc * NC2H) * 64 + rest + lo;
  };
  // the next chunk's fragments, held in registers (p0..p5) between the fetch and the commit
  static_assert(NPRE <= 6, "at most six staged fragments per thread");
  uint4 p0{}, p1r{}, p2r{}, p3{}, p4{}, p5{};
#define FVAN_FB_FETCH(hc)                                                            \
  do {                                                                               \
    const int i0 = tid;                                                              \
    if (NPRE > 0 && i0 < NPL * SW) p0 = *src(hc, i0);                                \
    if (NPRE > 1 && i0 + 512 < NPL * SW) p1r = *src(hc, i0 + 512);                   \
    if (NPRE > 2 && i0 + 1024 < NPL * SW) p2r = *src(hc, i0 + 1024);                 \
    if (NPRE > 3 && i0 + 1536 < NPL * SW) p3 = *src(hc, i0 + 1536);                  \
    if (NPRE > 4 && i0 + 2048 < NPL * SW) p4 = *src(hc, i0 + 2048);                  \
    if (NPRE > 5 && i0 + 2560 < NPL * SW) p5 = *src(hc, i0 + 2560);                  \
  } while (0)
#define FVAN_FB_COMMIT(buf)                                                          \
  do {                                                                               \
    uint4* w = &Ws[buf][0][0];                                                       \
    if (NPRE > 0 && tid < NPL * SW) w[tid] = p0;                                     \
    if (NPRE > 1 && tid + 512 < NPL * SW) w[tid + 512] = p1r;                        \
    if (NPRE > 2 && tid + 1024 < NPL * SW) w[tid + 1024] = p2r;                      \
    if (NPRE > 3 && tid + 1536 < NPL * SW) w[tid + 1536] = p3;                       \
    if (NPRE > 4 && tid + 2048 < NPL * SW) w[tid + 2048] = p4;                       \
    if (NPRE > 5 && tid + 2560 < NPL * SW) w[tid + 2560] = p5;                       \
  } while (0)
  static_assert(64 * NW == 512, "staging strides assume 512 threads");
  FVAN_FB_FETCH(0);
  // A fragments of the wave's rows (clamped; every output below is guarded)
  const int64_t ra = std::min<int64_t>(rbase + c, rows - 1);
  FragA<MODE> fa[NC1], fy[NC1];
  load_ln_frags<MODE, D, true>(X, ra, ln_g, ln_b, g, fa);
#pragma unroll
  for (int cc = 0; cc < NC1; ++cc) {
    alignas(16) AT af[LK];
#pragma unroll
    for (int i = 0; i < LK; i += 4)
      *reinterpret_cast<float4*>(&af[i]) = load_nt4(dY + ra * D + cc * KC + g * LK + i);
    fy[cc].load(af);
  }
  FVAN_FB_COMMIT(0);
  __syncthreads();
  if (NH > 1) FVAN_FB_FETCH(1);
  floatx4 acc[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float (*HD)[LDH] = Hd[wave];
  constexpr int PLO = NPL > 1 ? SW : 0;      // hi-to-lo distance in the stage
  for (int hc = 0; hc < NH; ++hc) {
    const uint4* W1s = &Ws[hc & 1][0][0];
    const uint4* W2s = W1s + S1;
    const uint4* W3s = W1s + 2 * S1;
#pragma unroll
    for (int t = 0; t < NT1; ++t) {
      floatx4 ah = {0.f, 0.f, 0.f, 0.f}, ag = ah;
#pragma unroll
      for (int cc = 0; cc < NC1; ++cc) {
        const int f = (t * NC1 + cc) * 64 + lane;
        ah = fa[cc].mma(W1s + f, W1s + f + PLO, ah);
        ag = fy[cc].mma(W2s + f, W2s + f + PLO, ag);
      }
      const float bias = b1[hc * HC + t * 16 + c];
      float gv[4], dh[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float gpr;
        gelu_and_grad(ah[i] + bias, gv[i], gpr);
        dh[i] = ag[i] * gpr;
        HD[4 * g + i][16 * t + c] = dh[i];
      }
      // feature-major g and dH: hidden unit hc HC + 16 t + c, rows rbase + 4 g ..
      const int64_t n = (int64_t)hc * HC + 16 * t + c;
      AT* gq = Gt + n * ldT + rbase + 4 * g;
      AT* dq = dHt + n * ldT + rbase + 4 * g;
      if (full) {
        *reinterpret_cast<float4*>(gq) = make_float4(gv[0], gv[1], gv[2], gv[3]);
        *reinterpret_cast<float4*>(dq) = make_float4(dh[0], dh[1], dh[2], dh[3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (rbase + 4 * g + i < rows) {
            gq[i] = gv[i];
            dq[i] = dh[i];
          }
      }
    }
    wave_lds_sync();
    // dA += dH_chunk W1^T_chunk
#pragma unroll
    for (int cc = 0; cc < NC2H; ++cc) {
      FragA<MODE> hd;
      hd.load(&HD[c][cc * KC + g * LK]);
#pragma unroll
      for (int t = 0; t < NT2; ++t) {
        const int f = (t * NC2H + cc) * 64 + lane;
        acc[t] = hd.mma(W3s + f, W3s + f + PLO, acc[t]);
      }
    }
    // the other stage was last read in chunk hc - 1, which every wave finished
    // before the barrier that ended it
    if (hc + 1 < NH) FVAN_FB_COMMIT((hc + 1) & 1);
    __syncthreads();                         // chunk hc + 1 is staged; stage hc & 1 is free
    // issued after the barrier, whose fence would otherwise wait for these loads
    if (hc + 2 < NH) FVAN_FB_FETCH(hc + 2);
  }
  // LN2 backward on the wave's rows (the workgroup's partial sums below)
  ln_bwd_rows<D>(acc, X, dY, ln_g, ln_b, rbase, rows, g, c, out, At, dYt, ldT, red[wave]);
  __syncthreads();
  for (int k = tid; k < 2 * D; k += 64 * NW) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += red[w][k];
    part[(size_t)blockIdx.x * 2 * D + k] = sum;
  }
#undef FVAN_FB_FETCH
#undef FVAN_FB_COMMIT
}

// Input gradient of the LayerNorm-fed QKV projection, in one kernel:
//   dA = dQKV W_qkv                  (row GEMM, K = 3D, against the pack of W_qkv^T [D x 3D])
//   out = resid + LN1'(dA)           (LayerNorm backward; resid = the gradient at the residual)
//   At = LN1(x)^T                    (feature-major operand of the W_qkv gradient)
// plus per-workgroup partial sums of the LN1 gain and shift gradients.  128 rows
// per workgroup (8 waves x 16 rows); the weight fragments are staged in LDS for
// all waves, CG K-chunks at a time, in two alternating buffers (one barrier per
// group), the group after next fetched into registers meanwhile.
constexpr int kGlbRows = 128;

template <int MODE, int D, int K>
__global__ __launch_bounds__(512) void gemm_ln_bwd_kernel(const float* __restrict__ A, int64_t rows,
                                                          const uint4* __restrict__ pack, const float* __restrict__ X,
                                                          const float* __restrict__ ln_g,
                                                          const float* __restrict__ ln_b,
                                                          const float* __restrict__ resid, float* __restrict__ out,
                                                          float* __restrict__ At, int64_t ldT,
                                                          float* __restrict__ part) {
  typedef typename Mode<MODE>::ActT AT;
  static_assert(sizeof(AT) == 4, "FP32 activations");
  constexpr int NW = 8;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int NPL = Mode<MODE>::SPLIT ? 2 : 1;
  constexpr int NT = D / 16;
  constexpr int NC = K / KC;
  constexpr int CG = Mode<MODE>::SPLIT ? 3 : 6;   // K chunks per stage
  static_assert(NC % CG == 0, "whole stages");
  constexpr int NG = NC / CG;
  constexpr size_t LO = (size_t)D * K / 8;
  constexpr int SW = NT * CG * 64;           // fragments per plane and stage
  constexpr int NPRE = (NPL * SW + 64 * NW - 1) / (64 * NW);
  static_assert(NPRE <= 6, "at most six staged fragments per thread");
  __shared__ __align__(16) uint4 Ws[2][NPL][SW];
  __shared__ float red[NW][2 * D];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kGlbRows + wave * 16;
  const int64_t ra = std::min<int64_t>(rbase + c, rows - 1);
  // staged fragment idx (plane, tile t, chunk cc of the group, lane) -> its place in the pack
  auto src = [&](int grp, int idx) -> const uint4* {
    const int pl = idx / SW, rem = idx % SW, t = rem / (CG * 64), r2 = rem % (CG * 64);
    return pack + ((size_t)t * NC + (size_t)grp * CG) * 64 + r2 + (pl ? LO : 0);
  };
  uint4 q0{}, q1{}, q2{}, q3{}, q4{}, q5{};
#define FVAN_GL_FETCH(grp)                                                           \
  do {                                                                               \
    if (NPRE > 0 && tid < NPL * SW) q0 = *src(grp, tid);                             \
    if (NPRE > 1 && tid + 512 < NPL * SW) q1 = *src(grp, tid + 512);                 \
    if (NPRE > 2 && tid + 1024 < NPL * SW) q2 = *src(grp, tid + 1024);               \
    if (NPRE > 3 && tid + 1536 < NPL * SW) q3 = *src(grp, tid + 1536);               \
    if (NPRE > 4 && tid + 2048 < NPL * SW) q4 = *src(grp, tid + 2048);               \
    if (NPRE > 5 && tid + 2560 < NPL * SW) q5 = *src(grp, tid + 2560);               \
  } while (0)
#define FVAN_GL_COMMIT(buf)                                                          \
  do {                                                                               \
    uint4* w = &Ws[buf][0][0];                                                       \
    if (NPRE > 0 && tid < NPL * SW) w[tid] = q0;                                     \
    if (NPRE > 1 && tid + 512 < NPL * SW) w[tid + 512] = q1;                         \
    if (NPRE > 2 && tid + 1024 < NPL * SW) w[tid + 1024] = q2;                       \
    if (NPRE > 3 && tid + 1536 < NPL * SW) w[tid + 1536] = q3;                       \
    if (NPRE > 4 && tid + 2048 < NPL * SW) w[tid + 2048] = q4;                       \
    if (NPRE > 5 && tid + 2560 < NPL * SW) w[tid + 2560] = q5;                       \
  } while (0)
  static_assert(64 * NW == 512, "staging strides assume 512 threads");
  FVAN_GL_FETCH(0);
  FVAN_GL_COMMIT(0);
  __syncthreads();
  if (NG > 1) FVAN_GL_FETCH(1);
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  constexpr int PLO = NPL > 1 ? SW : 0;
  for (int grp = 0; grp < NG; ++grp) {
    const uint4* ws = &Ws[grp & 1][0][0];
#pragma unroll
    for (int cc = 0; cc < CG; ++cc) {
      FragA<MODE> fa;
      {
        alignas(16) AT af[LK];
        const float* ap = A + ra * K + (grp * CG + cc) * KC + g * LK;
#pragma unroll
        for (int i = 0; i < LK; i += 4) *reinterpret_cast<float4*>(&af[i]) = *reinterpret_cast<const float4*>(ap + i);
        fa.load(af);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int f = (t * CG + cc) * 64 + lane;
        acc[t] = fa.mma(ws + f, ws + f + PLO, acc[t]);
      }
    }
    // the other stage was last read in group grp - 1, finished before the barrier that ended it
    if (grp + 1 < NG) FVAN_GL_COMMIT((grp + 1) & 1);
    __syncthreads();                         // group grp + 1 is staged; stage grp & 1 is free
    // issued after the barrier, whose fence would otherwise wait for these loads
    if (grp + 2 < NG) FVAN_GL_FETCH(grp + 2);
  }
#undef FVAN_GL_FETCH
#undef FVAN_GL_COMMIT
  ln_bwd_rows<D>(acc, X, resid, ln_g, ln_b, rbase, rows, g, c, out, At, nullptr, ldT, red[wave]);
  __syncthreads();
  for (int k = tid; k < 2 * D; k += 64 * NW) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += red[w][k];
    part[(size_t)blockIdx.x * 2 * D + k] = sum;
  }
}

template <int MODE, int K, int NOUT, int EPI>
inline hipError_t gemm_rows(const typename Mode<MODE>::ActT* A, int64_t rows, const void* pack, const EpiArgs& e,
                            hipStream_t s) {
  // the rows come either from A or, for K <= 128, from LayerNorm(e.ln_x)
  if (e.ln_x ? (K > 128) : (A == nullptr)) return hipErrorInvalidValue;
  if constexpr ((EPI == EPI_GELU || EPI == EPI_DGELU || EPI == EPI_STORE_KV) && K <= 128 && NOUT % 64 == 0) {
    constexpr int R = 64 * StagedRowTiles<EPI>::value;
    hipLaunchKernelGGL((gemm_rows_staged_kernel<MODE, K, NOUT, EPI>), dim3((int)((rows + R - 1) / R)), dim3(256), 0,
                       s, A, rows, reinterpret_cast<const uint4*>(pack), e);
  } else {
    hipLaunchKernelGGL((gemm_rows_kernel<MODE, K, NOUT, EPI>), dim3((int)((rows + kGemmRows - 1) / kGemmRows)),
                       dim3(256), 0, s, A, rows, reinterpret_cast<const uint4*>(pack), e);
  }
  return hipGetLastError();
}

}  // namespace fvan
