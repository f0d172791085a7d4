// 2^D-spin patch tokens -> spins (Methods, model configurations and training
// settings): the energy of a sampled token sequence is that of the lattice
// configuration its tokens encode.  Bit m of token t is the spin at site
// sites[t][m] (bit value (sigma + 1) / 2).
#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

__global__ void tokens_to_spins_kernel(const uint8_t* __restrict__ tokens, const int32_t* __restrict__ sites,
                                       int T, int bits, int n, int64_t total, int8_t* __restrict__ spins) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / ((int64_t)T * bits);
    const int rem = (int)(i % ((int64_t)T * bits));
    const int t = rem / bits, m = rem % bits;
    const int site = sites[t * bits + m];
    if (site >= 0 && site < n)
      spins[b * n + site] = ((tokens[b * T + t] >> m) & 1) ? (int8_t)1 : (int8_t)-1;
  }
}

hipError_t launch_tokens_to_spins(int32_t T, int32_t bits, const int32_t* sites, int32_t n, int32_t batch,
                                  const uint8_t* tokens, int8_t* spins, hipStream_t s) {
  const int64_t total = (int64_t)batch * T * bits;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(tokens_to_spins_kernel, dim3(grid), dim3(256), 0, s, tokens, sites, T, bits, n, total, spins);
  return hipGetLastError();
}

}  // namespace fvan

using namespace fvan;

extern "C" int fvan_tokens_to_spins(int32_t n_tokens, int32_t bits, const int32_t* sites, int32_t n_spins,
                                    int32_t batch, const uint8_t* tokens, int8_t* spins, void* stream) {
  if (!sites || !tokens || !spins) return fail(FVAN_EINVAL, "NULL argument");
  if (n_tokens < 1 || bits < 1 || bits > 8 || batch < 1 || n_spins < 1 || (int64_t)n_tokens * bits != n_spins)
    return fail(FVAN_EINVAL, "need n_tokens >= 1, bits in [1, 8], batch >= 1 and n_tokens * bits == n_spins");
  FVAN_HIP(launch_tokens_to_spins(n_tokens, bits, sites, n_spins, batch, tokens, spins, (hipStream_t)stream));
  return FVAN_OK;
}
