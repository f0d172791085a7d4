// Overlap distribution (Eq. overlap_distribution) of a batch of independent
// samples: counts[k] = number of pairs a < b whose configurations agree on k
// sites, i.e. whose overlap q = (1/N) s_a . s_b equals 2k/N - 1.
//
// The pair products are the dense contraction Q = S S^T of the +-1 spins, done
// on int8 MFMA (16x16x64, int32 accumulation: exact).  A workgroup (4 waves)
// takes 64 x 64 blocks (I <= J) of Q from a grid-stride list of the upper
// triangle; wave w owns rows 16w .. 16w+15 of block I against the four 16-row
// tiles of block J.  Each pair a < b adds one count to an LDS histogram, which
// the workgroup adds to the global counts once at the end (integer atomics:
// the result does not depend on their order).
#include <cmath>

#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

constexpr int kOvThreads = 256;
constexpr int kOvBlock = 64;
constexpr int kOvMaxSpins = 16000;
constexpr int kOvMaxGrid = 2048;

typedef int int4v __attribute__((ext_vector_type(4)));

// 16 spins of a row starting at k (zero past n); vec8: rows are 8-byte aligned
__device__ __forceinline__ int4v load16(const int8_t* row, int k, int n, bool vec8) {
  if (vec8 && k + 16 <= n) {
    const uint2 x = *reinterpret_cast<const uint2*>(row + k);
    const uint2 y = *reinterpret_cast<const uint2*>(row + k + 8);
    return int4v{(int)x.x, (int)x.y, (int)y.x, (int)y.y};
  }
  int w[4] = {0, 0, 0, 0};
  for (int j = 0; j < 16; ++j) {
    const int v = k + j < n ? (int)(uint8_t)row[k + j] : 0;
    w[j >> 2] |= v << (8 * (j & 3));
  }
  return int4v{w[0], w[1], w[2], w[3]};
}

__global__ __launch_bounds__(kOvThreads) void overlap_kernel(const int8_t* __restrict__ S, int B, int n,
                                                             unsigned long long* __restrict__ counts) {
  extern __shared__ unsigned int hist[];   // n + 1 bins
  for (int k = threadIdx.x; k <= n; k += kOvThreads) hist[k] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), r = lane & 15, g = lane >> 4;
  const int nblk = (B + kOvBlock - 1) / kOvBlock;
  const int npairs = nblk * (nblk + 1) / 2;
  const bool vec8 = (n & 7) == 0;
  for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
    // p-th block pair (I, J), I <= J, in row-major upper-triangle order
    int I = (int)floor(((2.0 * nblk + 1.0) - sqrt((2.0 * nblk + 1.0) * (2.0 * nblk + 1.0) - 8.0 * p)) * 0.5);
    while (I > 0 && I * (2 * nblk - I + 1) / 2 > p) --I;
    while ((I + 1) * (2 * nblk - I) / 2 <= p) ++I;
    const int J = I + (p - I * (2 * nblk - I + 1) / 2);
    const int a = I * kOvBlock + 16 * wave + r;
    const int8_t* arow = S + (int64_t)min(a, B - 1) * n;
    const int8_t* brow[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) brow[t] = S + (int64_t)min(J * kOvBlock + 16 * t + r, B - 1) * n;
    int4v acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = int4v{0, 0, 0, 0};
    // the next K step's fragments are loaded before the current step's products
    int4v fa = load16(arow, 16 * g, n, vec8), fb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) fb[t] = load16(brow[t], 16 * g, n, vec8);
    for (int k0 = 0; k0 < n; k0 += 64) {
      const int kn = k0 + 64 + 16 * g;
      int4v na = int4v{0, 0, 0, 0}, nbv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) nbv[t] = na;
      if (k0 + 64 < n) {
        na = load16(arow, kn, n, vec8);
#pragma unroll
        for (int t = 0; t < 4; ++t) nbv[t] = load16(brow[t], kn, n, vec8);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb[t], acc[t], 0, 0, 0);
      fa = na;
#pragma unroll
      for (int t = 0; t < 4; ++t) fb[t] = nbv[t];
    }
    // lane holds Q(row 16w + 4g + i of block I, row 16t + r of block J)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra = I * kOvBlock + 16 * wave + 4 * g + i, rb = J * kOvBlock + 16 * t + r;
        const int k = (acc[t][i] + n) >> 1;   // in [0, n] for +-1 spins; other values are not counted
        if (ra < rb && rb < B && k >= 0 && k <= n) atomicAdd(&hist[k], 1u);
      }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= n; k += kOvThreads)
    if (hist[k]) atomicAdd(&counts[k], (unsigned long long)hist[k]);
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

hipError_t launch_overlap(int32_t batch, int32_t n, const int8_t* spins, unsigned long long* counts, hipStream_t s) {
  if (batch < 1 || n < 1 || n > kOvMaxSpins) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 256) / 256), dim3(256), 0, s, counts, n + 1);
  const int nblk = (batch + kOvBlock - 1) / kOvBlock;
  const int npairs = nblk * (nblk + 1) / 2;
  hipLaunchKernelGGL(overlap_kernel, dim3(std::min(npairs, kOvMaxGrid)), dim3(kOvThreads),
                     (size_t)(n + 1) * sizeof(unsigned int), s, spins, batch, n, counts);
  return hipGetLastError();
}

}  // namespace fvan
