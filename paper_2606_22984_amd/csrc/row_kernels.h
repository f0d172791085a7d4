// Row-parallel kernels shared by the teacher-forced forward and the backward
// pass (which recomputes each layer's forward): LayerNorm, the row GEMM on
// packed weights with fused epilogues.
#pragma once

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

// ---------------------------------------------------------------- row GEMM
// C[r][n] = sum_k A[r][k] W[n][k] over a packed W [NOUT x K]; 64 rows per
// workgroup, one wave per 16 rows.  A is read from HBM once: for K <= 128 the
// wave's A fragments stay in registers across all output tiles; for larger K
// (NOUT <= 128) the loop runs K-outer with every output tile's accumulator live.
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
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * 64 + wave * 16;
  if (rbase >= rows) return;
  const int64_t ra = std::min<int64_t>(rbase + (lane & 15), rows - 1);   // clamp the A row; stores are guarded
  const AT* arow = A + ra * K + (lane >> 4) * LK;
  if constexpr (K <= 128) {
    alignas(16) AT af[NC][LK];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int i = 0; i < LK; i += 16 / (int)sizeof(AT))
        *reinterpret_cast<uint4*>(&af[c][i]) = *reinterpret_cast<const uint4*>(arow + c * KC + i);
    }
    for (int nt = 0; nt < NT; ++nt) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      const uint4* bp = pack + (size_t)nt * NC * 64 + lane;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc = Frag<MODE>::step(af[c], bp + c * 64, bp + c * 64 + LO, acc);
      const int n = nt * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rbase + 4 * (lane >> 4) + i;
        if (r < rows) Epi<MODE, EPI>::apply(e, r, n, NOUT, acc[i]);
      }
    }
  } else {
    static_assert(NT <= 8, "K-outer row GEMM keeps at most 8 output tiles live");
    floatx4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const uint4* bp = pack + lane;
    for (int c = 0; c < NC; ++c) {
      alignas(16) AT af[LK];
#pragma unroll
      for (int i = 0; i < LK; i += 16 / (int)sizeof(AT))
        *reinterpret_cast<uint4*>(&af[i]) = *reinterpret_cast<const uint4*>(arow + c * KC + i);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const uint4* b = bp + ((size_t)nt * NC + c) * 64;
        acc[nt] = Frag<MODE>::step(af, b, b + LO, acc[nt]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = rbase + 4 * (lane >> 4) + i;
        if (r < rows) Epi<MODE, EPI>::apply(e, r, n, NOUT, acc[nt][i]);
      }
    }
  }
}

template <int MODE, int K, int NOUT, int EPI>
inline hipError_t gemm_rows(const typename Mode<MODE>::ActT* A, int64_t rows, const void* pack, const EpiArgs& e,
                            hipStream_t s) {
  const int grid = (int)((rows + 63) / 64);
  hipLaunchKernelGGL((gemm_rows_kernel<MODE, K, NOUT, EPI>), dim3(grid), dim3(256), 0, s, A, rows,
                     reinterpret_cast<const uint4*>(pack), e);
  return hipGetLastError();
}

}  // namespace fvan
