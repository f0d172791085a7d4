// Local Monte Carlo refinement of sampled configurations (Results, 3D EA;
// Methods, training strategy): checkerboard Metropolis sweeps at inverse
// temperature beta, in place.
//
// One workgroup per configuration.  The spins live in LDS for all sweeps; a
// sweep updates the sites of colour 0, then those of colour 1, every site's
// local field h_i = sum_j J_ij s_j taken from the configuration at the start
// of the half-sweep (the half-sweep reads one LDS copy of the configuration and
// writes the other).  A flip of s_i changes the
// energy by dE = 2 s_i h_i and is accepted iff u < exp(-beta dE), u from
// Philox4x32-10 with key (seed lo, seed hi), counter (i >> 2, b, sweep, tag),
// word i & 3, u = (word >> 8) 2^-24.  The neighbour table holds every
// neighbour of a site (both directions), -1 for an empty slot.
#include <cmath>

#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

constexpr int kLmcThreads = 256;
constexpr int kLmcMaxSpins = 16384;   // LDS copy of one configuration

__global__ __launch_bounds__(kLmcThreads) void lmc_kernel(const int32_t* __restrict__ nbr, const float* __restrict__ J,
                                                          const int8_t* __restrict__ colour, int n, int degree,
                                                          float beta, int sweeps, uint32_t k0, uint32_t k1,
                                                          uint32_t tag, int8_t* __restrict__ spins,
                                                          int32_t* __restrict__ accepted) {
  // two copies of the configuration: each half-sweep reads buf[p] and writes buf[p ^ 1]
  __shared__ int8_t buf[2][kLmcMaxSpins];
  __shared__ int red[kLmcThreads / 64];
  const int b = blockIdx.x;
  int8_t* row = spins + (int64_t)b * n;
  for (int i = threadIdx.x; i < n; i += kLmcThreads) buf[0][i] = row[i];
  __syncthreads();
  int p = 0, acc = 0;
  for (int k = 0; k < sweeps; ++k) {
    for (int c = 0; c < 2; ++c) {
      for (int i = threadIdx.x; i < n; i += kLmcThreads) {
        int8_t v = buf[p][i];
        if (colour[i] == c) {
          float h = 0.f;
          for (int d = 0; d < degree; ++d) {
            const int j = nbr[(int64_t)i * degree + d];
            if (j >= 0) h += J[(int64_t)i * degree + d] * (float)buf[p][j];
          }
          const float dE = 2.f * (float)v * h;
          const uint4 w = philox4x32_10(make_uint4((uint32_t)(i >> 2), (uint32_t)b, (uint32_t)k, tag), k0, k1);
          const uint32_t x = (i & 3) == 0 ? w.x : (i & 3) == 1 ? w.y : (i & 3) == 2 ? w.z : w.w;
          if (u24(x) < expf(-beta * dE)) {
            v = (int8_t)-v;
            ++acc;
          }
        }
        buf[p ^ 1][i] = v;
      }
      p ^= 1;
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += kLmcThreads) row[i] = buf[p][i];
  if (accepted) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w = 0; w < kLmcThreads / 64; ++w) t += red[w];
      accepted[b] = t;
    }
  }
}

hipError_t launch_lmc(int32_t n, int32_t degree, const int32_t* nbr, const float* J, const int8_t* colour,
                      int32_t batch, double beta, int32_t sweeps, uint64_t seed, uint32_t stream_tag, int8_t* spins,
                      int32_t* accepted, hipStream_t s) {
  if (n < 1 || n > kLmcMaxSpins || batch < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lmc_kernel, dim3(batch), dim3(kLmcThreads), 0, s, nbr, J, colour, n, degree, (float)beta, sweeps,
                     (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), stream_tag, spins, accepted);
  return hipGetLastError();
}

}  // namespace fvan
