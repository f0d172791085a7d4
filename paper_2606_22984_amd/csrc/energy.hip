// Spin energies E_b = - sum_{pairs} J_ij s_i s_j (Eq. 6 for SK, Eq. 8 for EA),
// each unordered pair counted once.
//
// ELL bonds: one workgroup per sample; the sample's int8 spin row is staged in
// LDS with coalesced 16-byte loads, each thread sums its sites' stored pairs
// (neighbour table and bonds are shared by all samples and stay in L2), then a
// fixed-order block reduction.  +/-J bonds accumulate in int32: exact.
// Dense (SK) bonds: one workgroup per 16 samples so every J row read from L2
// serves 16 samples; lanes stride over columns (coalesced) and waves over rows.
#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

constexpr int kEThreads = 256;

template <typename A>
__device__ __forceinline__ A block_sum(A v, A* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  A r = 0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
  }
  return r;
}

template <typename JT, typename A>
__global__ __launch_bounds__(kEThreads) void energy_ell_kernel(int n, int deg, const int32_t* __restrict__ nbr,
                                                              const JT* __restrict__ J,
                                                              const int8_t* __restrict__ spins, A* __restrict__ out) {
  extern __shared__ int8_t srow[];
  __shared__ A red[kEThreads / 64];
  const int b = blockIdx.x;
  const int8_t* row = spins + (size_t)b * n;
  // stage the row: 16-byte loads where aligned, bytes for the tail
  const int n16 = ((((uintptr_t)row) & 15) == 0) ? (n >> 4) : 0;
  for (int i = threadIdx.x; i < n16; i += kEThreads)
    reinterpret_cast<uint4*>(srow)[i] = reinterpret_cast<const uint4*>(row)[i];
  for (int i = n16 * 16 + threadIdx.x; i < n; i += kEThreads) srow[i] = row[i];
  __syncthreads();
  A acc = 0;
  for (int i = threadIdx.x; i < n; i += kEThreads) {
    const A si = (A)srow[i];
    A part = 0;
    for (int k = 0; k < deg; ++k) {
      const int j = nbr[(size_t)i * deg + k];
      if (j >= 0 && j < n) part += (A)J[(size_t)i * deg + k] * (A)srow[j];
    }
    acc += si * part;
  }
  const A tot = block_sum<A>(acc, red);
  if (threadIdx.x == 0) out[b] = -tot;
}

constexpr int kDenseS = 16;

__global__ __launch_bounds__(kEThreads) void energy_dense_kernel(int n, int batch, const float* __restrict__ J,
                                                                 const int8_t* __restrict__ spins,
                                                                 float* __restrict__ out) {
  extern __shared__ int8_t sm[];    // [kDenseS][n]
  __shared__ float red[kEThreads / 64];
  const int b0 = blockIdx.x * kDenseS;
  const int ns = min(kDenseS, batch - b0);
  for (int i = threadIdx.x; i < kDenseS * n; i += kEThreads) {
    const int s = i / n, j = i % n;
    sm[i] = s < ns ? spins[(size_t)(b0 + s) * n + j] : (int8_t)0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float acc[kDenseS];
#pragma unroll
  for (int s = 0; s < kDenseS; ++s) acc[s] = 0.f;
  for (int i = wave; i < n; i += kEThreads / 64) {
    const float* Ji = J + (size_t)i * n;
    for (int j = lane; j < n; j += 64) {
      const float w = Ji[j];
#pragma unroll
      for (int s = 0; s < kDenseS; ++s) acc[s] += w * (float)(sm[s * n + i] * sm[s * n + j]);
    }
  }
  for (int s = 0; s < kDenseS; ++s) {
    const float tot = block_sum<float>(acc[s], red);
    if (threadIdx.x == 0 && s < ns) out[b0 + s] = -0.5f * tot;
    __syncthreads();
  }
}

hipError_t launch_energy(const fvan_couplings& c, int32_t batch, const int8_t* spins, void* energy,
                         hipStream_t s) {
  const int n = c.n_spins;
  if (c.kind == FVAN_BONDS_PM1) {
    hipLaunchKernelGGL((energy_ell_kernel<int8_t, int>), dim3(batch), dim3(kEThreads), n, s, n, c.degree, c.nbr,
                       (const int8_t*)c.J, spins, (int*)energy);
  } else if (c.kind == FVAN_BONDS_F32) {
    hipLaunchKernelGGL((energy_ell_kernel<float, float>), dim3(batch), dim3(kEThreads), n, s, n, c.degree, c.nbr,
                       (const float*)c.J, spins, (float*)energy);
  } else {
    const int grid = (batch + kDenseS - 1) / kDenseS;
    hipLaunchKernelGGL(energy_dense_kernel, dim3(grid), dim3(kEThreads), kDenseS * n, s, n, batch,
                       (const float*)c.J, spins, (float*)energy);
  }
  return hipGetLastError();
}

}  // namespace fvan
