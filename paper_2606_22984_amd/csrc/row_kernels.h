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
// hold it whole and the row statistics are two pair reductions.
template <int MODE, int K>
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
      const float4 v = *reinterpret_cast<const float4*>(X + row * K + cc * KC + g * LK + i);
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
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
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
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
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
//   out[r] = resid[r] + W2 GELU(W1 a[r] + b1) + b2,   W1 [4D x D], W2 [D x 4D].
// 128 rows per workgroup, one wave per 32 rows (two 16-row MFMA tiles, so every
// weight fragment a wave loads feeds both).  A wave's hidden activations go
// through a wave-private LDS tile, 64 hidden units at a time, straight into the
// W2 product, so the 4D-wide hidden layer never reaches HBM.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int kFfnRows = 128;                // rows per fused-FFN workgroup

// The input rows are LayerNorm(X rows; ln_g, ln_b), computed in the kernel.
template <int MODE, int D>
__global__ __launch_bounds__(256) void ffn_fused_kernel(const float* __restrict__ X, const float* __restrict__ ln_g,
                                                        const float* __restrict__ ln_b, int64_t rows,
                                                        const uint4* __restrict__ p1, const uint4* __restrict__ p2,
                                                        const float* __restrict__ b1, const float* __restrict__ b2,
                                                        const float* __restrict__ resid, float* __restrict__ out) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;                 // A elements per lane per chunk
  constexpr int NC1 = D / KC;                // K chunks of the W1 product
  constexpr int HC = 64;                     // hidden units per chunk
  constexpr int NH = 4 * D / HC;             // hidden chunks
  constexpr int NT1 = HC / 16;               // W1 output tiles per hidden chunk
  constexpr int NT2 = D / 16;                // W2 output tiles
  constexpr int NC2 = 4 * D / KC;            // K chunks of the W2 product
  constexpr int NC2H = HC / KC;              // ... per hidden chunk
  constexpr size_t LO = (size_t)4 * D * D / 8;   // hi-to-lo distance of a split pack (both matrices 4D^2)
  constexpr int LDH = HC + 16 / (int)sizeof(AT);
  __shared__ __align__(16) AT Hs[4][32][LDH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kFfnRows + wave * 32;
  if (rbase >= rows) return;                 // no block-wide barrier below
  FragA<MODE> fa[2][NC1];                    // both row tiles' A fragments, converted once
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
    load_ln_frags<MODE, D>(X, std::min<int64_t>(rbase + 16 * rt + c, rows - 1), ln_g, ln_b, g, fa[rt]);
  floatx4 acc2[2][NT2];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int t = 0; t < NT2; ++t) acc2[rt][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  AT (*H)[LDH] = Hs[wave];
  for (int hc = 0; hc < NH; ++hc) {
#pragma unroll
    for (int t = 0; t < NT1; ++t) {
      const int nt = hc * NT1 + t;
      floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0;
      const uint4* bp = p1 + (size_t)nt * NC1 * 64 + lane;
#pragma unroll
      for (int cc = 0; cc < NC1; ++cc) {
        a0 = fa[0][cc].mma(bp + cc * 64, bp + cc * 64 + LO, a0);
        a1 = fa[1][cc].mma(bp + cc * 64, bp + cc * 64 + LO, a1);
      }
      const float bias = b1[nt * 16 + c];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        H[4 * g + i][t * 16 + c] = from_f<AT>(gelu(a0[i] + bias));
        H[16 + 4 * g + i][t * 16 + c] = from_f<AT>(gelu(a1[i] + bias));
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int cc = 0; cc < NC2H; ++cc) {
      FragA<MODE> h0, h1;
      h0.load(&H[c][cc * KC + g * LK]);
      h1.load(&H[16 + c][cc * KC + g * LK]);
#pragma unroll
      for (int t = 0; t < NT2; ++t) {
        const uint4* bp = p2 + ((size_t)t * NC2 + hc * NC2H + cc) * 64 + lane;
        acc2[0][t] = h0.mma(bp, bp + LO, acc2[0][t]);
        acc2[1][t] = h1.mma(bp, bp + LO, acc2[1][t]);
      }
    }
    wave_lds_sync();                         // the next chunk overwrites H
  }
#pragma unroll
  for (int t = 0; t < NT2; ++t) {
    const int n = t * 16 + c;
    const float bias = b2[n];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rbase + 16 * rt + 4 * g + i;
        if (r < rows) out[r * D + n] = resid[r * D + n] + acc2[rt][t][i] + bias;
      }
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
