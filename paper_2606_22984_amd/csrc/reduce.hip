// Batch reductions in FP64 on the device: the free-energy estimator (Eq. 5),
// its sample variance, the REINFORCE baseline and weights (Eq. 19), the mean
// energy and the gradient norm.  Each runs in ONE workgroup with a fixed
// per-thread stride and a fixed reduction tree, so results are bitwise
// reproducible run to run.
#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

constexpr int kRThreads = 1024;

__device__ double block_sum_d(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < kRThreads / 64; ++w) r += red[w];   // every thread, same order
  return r;
}

__device__ __forceinline__ double load_energy(const void* e, int is_int, int b) {
  return is_int ? (double)reinterpret_cast<const int*>(e)[b] : (double)reinterpret_cast<const float*>(e)[b];
}

__global__ __launch_bounds__(kRThreads) void free_energy_kernel(int batch, int n, double beta, int is_int,
                                                                const void* __restrict__ energy,
                                                                const float* __restrict__ logq,
                                                                double* __restrict__ stats) {
  __shared__ double red[kRThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < batch; b += kRThreads)
    s += (load_energy(energy, is_int, b) + (double)logq[b] / beta) / (double)n;
  const double mean = block_sum_d(s, red) / (double)batch;
  double v = 0.0;
  for (int b = threadIdx.x; b < batch; b += kRThreads) {
    const double f = (load_energy(energy, is_int, b) + (double)logq[b] / beta) / (double)n;
    v += (f - mean) * (f - mean);
  }
  const double var = block_sum_d(v, red);
  if (threadIdx.x == 0) {
    stats[0] = mean;
    stats[1] = batch > 1 ? var / (double)(batch - 1) : 0.0;
  }
}

// wlik: weight w of the likelihood term of Eq. (loss2): weights are
// ((L - Lbar) - w) / (beta batch), the 1/beta of the exact gradient scaling both
// of its terms (w = 0 gives the REINFORCE weights of Eq. 19).
__global__ __launch_bounds__(kRThreads) void reinforce_kernel(int batch, double beta, int is_int,
                                                              const void* __restrict__ energy,
                                                              const float* __restrict__ logq,
                                                              float* __restrict__ w, double* Lmean_out, double wlik) {
  __shared__ double red[kRThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < batch; b += kRThreads) s += beta * load_energy(energy, is_int, b) + (double)logq[b];
  const double Lbar = block_sum_d(s, red) / (double)batch;
  const double scale = 1.0 / (beta * (double)batch);
  for (int b = threadIdx.x; b < batch; b += kRThreads) {
    const double L = beta * load_energy(energy, is_int, b) + (double)logq[b];
    w[b] = (float)(((L - Lbar) - wlik) * scale);
  }
  if (threadIdx.x == 0 && Lmean_out) *Lmean_out = Lbar;
}

__global__ __launch_bounds__(kRThreads) void mean_energy_kernel(int batch, int n, int is_int,
                                                                const void* __restrict__ energy, double* out) {
  __shared__ double red[kRThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < batch; b += kRThreads) s += load_energy(energy, is_int, b);
  const double tot = block_sum_d(s, red);
  if (threadIdx.x == 0) *out = tot / ((double)batch * (double)n);
}

__global__ __launch_bounds__(kRThreads) void sumsq_kernel(const float* __restrict__ g, int64_t n, double* out) {
  __shared__ double red[kRThreads / 64];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRThreads) s += (double)g[i] * (double)g[i];
  const double tot = block_sum_d(s, red);
  if (threadIdx.x == 0) *out = sqrt(tot);
}

hipError_t launch_free_energy(int32_t batch, int32_t n, double beta, int is_int, const void* energy,
                              const float* logq, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(free_energy_kernel, dim3(1), dim3(kRThreads), 0, s, batch, n, beta, is_int, energy, logq, stats);
  return hipGetLastError();
}

hipError_t launch_reinforce(int32_t batch, double beta, int is_int, const void* energy, const float* logq,
                            float* weights, double* Lmean_out, hipStream_t s, double wlik) {
  hipLaunchKernelGGL(reinforce_kernel, dim3(1), dim3(kRThreads), 0, s, batch, beta, is_int, energy, logq, weights,
                     Lmean_out, wlik);
  return hipGetLastError();
}

hipError_t launch_mean_energy(int32_t batch, int32_t n, int is_int, const void* energy, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(mean_energy_kernel, dim3(1), dim3(kRThreads), 0, s, batch, n, is_int, energy, out);
  return hipGetLastError();
}

hipError_t launch_grad_norm(const float* g, int64_t n, double* out, double* /*scratch*/, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(kRThreads), 0, s, g, n, out);
  return hipGetLastError();
}

}  // namespace fvan
