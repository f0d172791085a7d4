// Parameter-side kernels: the packed weight copies the MFMA kernels read
// (FP32 or round-to-nearest-even BF16, in 16-byte lane-fragment order) and the
// Adam update of the flat FP32 parameters.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

// dst = pack of the [rows x K] matrix M, M[r][k] = src[r*K + k] (or src[k*rows + r]
// when transposed, i.e. M = W^T of a row-major W [K x rows]).  Split mode
// writes the bf16 hi parts at dst[0, rows*K) and the lo parts right after.
// valid: entries of M with row (or, transposed, k) index >= valid are zero
// (padding of the vocab-way head).
template <int MODE>
__global__ void pack_kernel(const float* __restrict__ src, int rows, int K, int transposed, int valid,
                            typename Mode<MODE>::WT* __restrict__ dst) {
  typedef typename Mode<MODE>::WT WT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int VEC = KC / 4;
  const int64_t total = (int64_t)rows * K;
  const int nchunk = K / KC;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(p % VEC);
    const int64_t pc = p / VEC;
    const int l = (int)(pc % 64);
    const int64_t rest = pc / 64;
    const int c = (int)(rest % nchunk);
    const int n = (int)(rest / nchunk);
    const int r = 16 * n + (l & 15);
    const int k = c * KC + (l >> 4) * VEC + e;
    const float v = transposed ? (k < valid ? src[(size_t)k * rows + r] : 0.f)
                               : (r < valid ? src[(size_t)r * K + k] : 0.f);
    const WT hi = from_f<WT>(v);
    dst[p] = hi;
    if (Mode<MODE>::SPLIT) dst[p + total] = from_f<WT>(v - to_f(hi));
  }
}

template <int MODE>
static hipError_t pack_all(const fvan_model_config& c, const float* theta, void* wpack, hipStream_t s) {
  typedef typename Mode<MODE>::WT WT;
  const ParamOffsets po = param_offsets(c);
  const PackOffsets pk = pack_offsets(c);
  const int D = c.d_model;
  for (int l = 0; l < c.n_layers; ++l) {
    const float* lp = theta + po.layer0 + (int64_t)l * po.layer_stride;
    char* w = reinterpret_cast<char*>(wpack) + (size_t)l * pk.layer_stride;
    struct Job { const float* src; int rows, K, tr; size_t off; } jobs[6] = {
        {lp + po.qkv_w, 3 * D, D, 0, pk.qkv},   {lp + po.ffn1_w, 4 * D, D, 0, pk.ffn1},
        {lp + po.ffn2_w, D, 4 * D, 0, pk.ffn2}, {lp + po.qkv_w, D, 3 * D, 1, pk.qkvT},
        {lp + po.ffn1_w, D, 4 * D, 1, pk.ffn1T}, {lp + po.ffn2_w, 4 * D, D, 1, pk.ffn2T}};
    for (auto& j : jobs) {
      const int64_t total = (int64_t)j.rows * j.K;
      const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
      hipLaunchKernelGGL((pack_kernel<MODE>), dim3(grid), dim3(256), 0, s, j.src, j.rows, j.K, j.tr,
                         j.tr ? j.K : j.rows, reinterpret_cast<WT*>(w + j.off));
    }
  }
  if (pk.vp) {   // the vocab-way head: W_h [vp x D] (rows >= vocab zero) and W_h^T [D x vp]
    char* w = reinterpret_cast<char*>(wpack);
    const int64_t total = (int64_t)pk.vp * D;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((pack_kernel<MODE>), dim3(grid), dim3(256), 0, s, theta + po.head_w, pk.vp, D, 0, c.vocab,
                       reinterpret_cast<WT*>(w + pk.head));
    hipLaunchKernelGGL((pack_kernel<MODE>), dim3(grid), dim3(256), 0, s, theta + po.head_w, D, pk.vp, 1, c.vocab,
                       reinterpret_cast<WT*>(w + pk.headT));
  }
  return hipGetLastError();
}

hipError_t launch_pack(const fvan_model_config& c, const float* theta, void* wpack, hipStream_t s) {
  switch (c.precision) {
    case FVAN_FP32: return pack_all<0>(c, theta, wpack, s);
    case FVAN_BF16_SPLIT: return pack_all<2>(c, theta, wpack, s);
    default: return hipErrorInvalidValue;
  }
}

// Adam (Kingma & Ba) with L2 weight decay folded into the gradient; the
// gradient is zeroed for the next accumulation.
__global__ void adam_kernel(float* __restrict__ theta, float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float wd,
                            float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i] + wd * theta[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    g[i] = 0.0f;
  }
}

hipError_t launch_adam(float* theta, float* grads, float* m, float* v, int64_t n, const fvan_adam& o, int64_t step,
                       hipStream_t s) {
  const double c1 = 1.0 - std::pow((double)o.beta1, (double)step);
  const double c2 = 1.0 - std::pow((double)o.beta2, (double)step);
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, s, theta, grads, m, v, n, o.lr, o.beta1, o.beta2, o.eps,
                     o.weight_decay, (float)c1, (float)c2);
  return hipGetLastError();
}

__global__ void zero_int_kernel(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_zero_int(int* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace fvan
