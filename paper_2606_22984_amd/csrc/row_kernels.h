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
// workgroup, one wave per 16 rows, every 16-column tile of the output.
template <int MODE, int K, int NOUT, int EPI>
__global__ __launch_bounds__(256) void gemm_rows_kernel(const typename Mode<MODE>::ActT* __restrict__ A,
                                                        int64_t rows, const uint4* __restrict__ pack,
                                                        EpiArgs e) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int NC = K / KC;
  constexpr size_t LO = (size_t)NOUT * K / 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * 64 + wave * 16;
  if (rbase >= rows) return;
  const int64_t ra = std::min<int64_t>(rbase + (lane & 15), rows - 1);   // clamp the A row; stores are guarded
  const AT* arow = A + ra * K + (lane >> 4) * (KC / 4);
  for (int nt = 0; nt < NOUT / 16; ++nt) {
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const uint4* bp = pack + (size_t)nt * NC * 64 + lane;
#pragma unroll 4
    for (int c = 0; c < NC; ++c) acc = Frag<MODE>::step(arow + c * KC, bp + c * 64, bp + c * 64 + LO, acc);
    const int n = nt * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rbase + 4 * (lane >> 4) + i;
      if (r < rows) Epi<MODE, EPI>::apply(e, r, n, NOUT, acc[i]);
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
