// Muon update (Methods, comparison of optimisers): momentum, Newton-Schulz
// orthogonalisation of the momentum matrix on FP32 MFMA, and the scaled step
// with decoupled weight decay; the parameters that are not layer weight
// matrices take Adam in the same call.
//
// One 8-wave workgroup owns one matrix for the whole update.  The matrix is
// iterated in place, viewed as the wide matrix Z (m x n, m = min(rows, cols)
// <= 128): a tall matrix is read through transposed strides.  Per iteration:
//   Gram     A = Z Z^T           upper-triangle 16x16 tiles, mirrored into LDS
//   poly     P = b A + c A A     LDS -> LDS (A A is symmetric: same mirroring)
//   update   Z <- a Z + P Z      each wave owns 16-column blocks of Z; it holds
//                                its block's K fragments in registers before
//                                it overwrites the block in global memory
// with (a, b, c) = (3.4445, -4.7750, 2.0315), the quintic coefficients
// published with the Muon optimiser.  Z lives in global memory (L2-resident:
// at most 128 x 512 floats per matrix here); the two Gram-sized operands live
// in LDS.  All products are FP32 MFMA 16x16x4 with FP32 accumulation.
#include <cmath>

#include "device_common.h"
#include "fvan_internal.h"

namespace fvan {

constexpr int kNsMaxGram = 128;          // largest min(rows, cols)
constexpr int kNsThreads = 512;          // 8 waves
constexpr int kNsWaves = kNsThreads / 64;
constexpr int kNsPitch = kNsMaxGram + 4; // LDS row pitch in floats
constexpr float kNsA = 3.4445f, kNsB = -4.7750f, kNsC = 2.0315f;

struct NsSmem {
  float gram[kNsMaxGram][kNsPitch];
  float poly[kNsMaxGram][kNsPitch];
  double part[kNsWaves];
};

// Z(i, j) = p[i * si + j * sj], 0 <= i < m <= n, 0 <= j < n.
struct ZView {
  float* p;
  int m, n;
  int64_t si, sj;
};

__device__ __forceinline__ ZView wide_view(float* p, int rows, int cols) {
  if (rows <= cols) return ZView{p, rows, cols, (int64_t)cols, 1};
  return ZView{p, cols, rows, 1, (int64_t)cols};
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// p-th pair (ti, tj), ti <= tj, of mt x mt tiles in row-major upper-triangle order.
__device__ __forceinline__ void upper_pair(int p, int mt, int& ti, int& tj) {
  ti = 0;
  while (p >= mt - ti) {
    p -= mt - ti;
    ++ti;
  }
  tj = ti + p;
}

// Sum of v over the workgroup in a fixed order (bitwise reproducible).
__device__ double block_sum(double v, NsSmem& sm) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sm.part[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kNsWaves; ++w) s += sm.part[w];
  __syncthreads();
  return s;
}

// steps Newton-Schulz iterations on Z in place (Z already normalised).
__device__ __forceinline__ void ns_iterate(const ZView z, int steps, NsSmem& sm) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  const int mt = (z.m + 15) >> 4;
  const int kg = 4 * mt;                 // K steps of 4 over the padded Gram dimension
  const int npairs = mt * (mt + 1) / 2;
  const int nb = (z.n + 15) >> 4;
  for (int it = 0; it < steps; ++it) {
    // ---- A = Z Z^T: lane supplies A-operand Z(16ti + r16, k) and B-operand Z(16tj + r16, k), k = k0 + g
    for (int p = wave; p < npairs; p += kNsWaves) {
      int ti, tj;
      upper_pair(p, mt, ti, tj);
      const int ia = 16 * ti + r16, ib = 16 * tj + r16;
      const float* za = z.p + (int64_t)min(ia, z.m - 1) * z.si;
      const float* zb = z.p + (int64_t)min(ib, z.m - 1) * z.si;
      const bool va = ia < z.m, vb = ib < z.m;
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      int k0 = 0;
      for (; k0 + 16 <= z.n; k0 += 16) {
        float a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t o = (int64_t)(k0 + 4 * u + g) * z.sj;
          a[u] = va ? za[o] : 0.f;
          b[u] = vb ? zb[o] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mfma4(a[u], b[u], acc);
      }
      for (; k0 < z.n; k0 += 4) {
        const int k = k0 + g;
        const int64_t o = (int64_t)min(k, z.n - 1) * z.sj;
        const float a = (va && k < z.n) ? za[o] : 0.f;
        const float b = (vb && k < z.n) ? zb[o] : 0.f;
        acc = mfma4(a, b, acc);
      }
      // lane holds A(16ti + 4g + i, 16tj + r16)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * ti + 4 * g + i, col = 16 * tj + r16;
        sm.gram[row][col] = acc[i];
        if (ti != tj) sm.gram[col][row] = acc[i];
      }
    }
    __syncthreads();
    // ---- P = b A + c A A (symmetric)
    for (int p = wave; p < npairs; p += kNsWaves) {
      int ti, tj;
      upper_pair(p, mt, ti, tj);
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int s = 0; s < kg; ++s) {
        const int k = 4 * s + g;
        acc = mfma4(sm.gram[16 * ti + r16][k], sm.gram[k][16 * tj + r16], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * ti + 4 * g + i, col = 16 * tj + r16;
        const float v = kNsB * sm.gram[row][col] + kNsC * acc[i];
        sm.poly[row][col] = v;
        if (ti != tj) sm.poly[col][row] = v;
      }
    }
    __syncthreads();
    // ---- Z <- a Z + P Z, one 16-column block per wave at a time
    for (int jb = wave; jb < nb; jb += kNsWaves) {
      const int j = 16 * jb + r16;
      const bool vj = j < z.n;
      float* zc = z.p + (int64_t)min(j, z.n - 1) * z.sj;
      float zf[kNsMaxGram / 4];          // Z(4s + g, j)
#pragma unroll
      for (int s = 0; s < kNsMaxGram / 4; ++s) {
        const int k = 4 * s + g;
        zf[s] = (s < kg && vj && k < z.m) ? zc[(int64_t)k * z.si] : 0.f;
      }
      for (int ti = 0; ti < mt; ++ti) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < kNsMaxGram / 4; ++s)
          if (s < kg) acc = mfma4(sm.poly[16 * ti + r16][4 * s + g], zf[s], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * ti + 4 * g + i;
          if (vj && row < z.m) {
            float* q = zc + (int64_t)row * z.si;
            *q = kNsA * *q + acc[i];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Standalone orthogonalisation: O = NewtonSchulz(M), O may alias M.
__global__ void __launch_bounds__(kNsThreads) newton_schulz_kernel(const float* M, float* O, int rows, int cols,
                                                                   int steps, float eps) {
  __shared__ NsSmem sm;
  const int64_t total = (int64_t)rows * cols;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += kNsThreads) {
    const float v = M[i];
    O[i] = v;
    ss += (double)v * v;
  }
  const float inv = (float)(1.0 / (sqrt(block_sum(ss, sm)) + (double)eps));
  for (int64_t i = threadIdx.x; i < total; i += kNsThreads) O[i] *= inv;
  __syncthreads();
  ns_iterate(wide_view(O, rows, cols), steps, sm);
}

// Offsets of the three weight matrices inside each layer's parameter block.
struct MuonLayout {
  int64_t layer0, stride;
  int64_t off[3];
  int rows[3], cols[3];
  int n_layers;
};

__device__ __forceinline__ bool in_muon_matrix(int64_t i, const MuonLayout& L) {
  if (i < L.layer0 || i >= L.layer0 + L.n_layers * L.stride) return false;
  const int64_t o = (i - L.layer0) % L.stride;
#pragma unroll
  for (int w = 0; w < 3; ++w)
    if (o >= L.off[w] && o < L.off[w] + (int64_t)L.rows[w] * L.cols[w]) return true;
  return false;
}

// Workgroup (layer, which): momentum, orthogonalisation in the gradient's
// storage, step, and the gradient cleared for the next accumulation.
__global__ void __launch_bounds__(kNsThreads) muon_kernel(float* __restrict__ theta, float* __restrict__ grads,
                                                          float* __restrict__ mom, MuonLayout L, float lr, float mu,
                                                          float wd, float rms_scale, float eps, int steps) {
  __shared__ NsSmem sm;
  const int layer = blockIdx.x / 3, w = blockIdx.x % 3;
  const int rows = L.rows[w], cols = L.cols[w];
  const int64_t base = L.layer0 + layer * L.stride + L.off[w];
  float* W = theta + base;
  float* Gm = grads + base;
  float* Mm = mom + base;
  const int64_t total = (int64_t)rows * cols;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < total; i += kNsThreads) {
    const float v = mu * Mm[i] + Gm[i];
    Mm[i] = v;
    Gm[i] = v;
    ss += (double)v * v;
  }
  const float inv = (float)(1.0 / (sqrt(block_sum(ss, sm)) + (double)eps));
  for (int64_t i = threadIdx.x; i < total; i += kNsThreads) Gm[i] *= inv;
  __syncthreads();
  ns_iterate(wide_view(Gm, rows, cols), steps, sm);
  const float scale = rms_scale * sqrtf((float)max(rows, cols));
  for (int64_t i = threadIdx.x; i < total; i += kNsThreads) {
    const float wv = W[i];
    W[i] = wv - lr * (scale * Gm[i] + wd * wv);
    Gm[i] = 0.0f;
  }
}

// Adam on the parameters outside the layer weight matrices; same update as
// the library's Adam step.
__global__ void adam_rest_kernel(float* __restrict__ theta, float* __restrict__ g, float* __restrict__ m,
                                 float* __restrict__ v, int64_t n, MuonLayout L, float lr, float b1, float b2,
                                 float eps, float wd, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (in_muon_matrix(i, L)) continue;
    const float gi = g[i] + wd * theta[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    g[i] = 0.0f;
  }
}

hipError_t launch_newton_schulz(const float* M, float* O, int rows, int cols, int steps, float eps, hipStream_t s) {
  if (rows < 1 || cols < 1 || (rows < cols ? rows : cols) > kNsMaxGram) return hipErrorInvalidValue;
  hipLaunchKernelGGL(newton_schulz_kernel, dim3(1), dim3(kNsThreads), 0, s, M, O, rows, cols, steps, eps);
  return hipGetLastError();
}

hipError_t launch_muon(const fvan_model_config& c, float* theta, float* grads, float* m, float* v, int64_t n,
                       const fvan_muon& o, int64_t step, hipStream_t s) {
  const ParamOffsets po = param_offsets(c);
  const int d = c.d_model;
  if (d > kNsMaxGram) return hipErrorInvalidValue;
  MuonLayout L{};
  L.layer0 = po.layer0;
  L.stride = po.layer_stride;
  L.n_layers = c.n_layers;
  L.off[0] = po.qkv_w;  L.rows[0] = 3 * d; L.cols[0] = d;
  L.off[1] = po.ffn1_w; L.rows[1] = 4 * d; L.cols[1] = d;
  L.off[2] = po.ffn2_w; L.rows[2] = d;     L.cols[2] = 4 * d;
  const double c1 = 1.0 - std::pow((double)o.adam.beta1, (double)step);
  const double c2 = 1.0 - std::pow((double)o.adam.beta2, (double)step);
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(adam_rest_kernel, dim3(grid), dim3(256), 0, s, theta, grads, m, v, n, L, o.adam.lr,
                     o.adam.beta1, o.adam.beta2, o.adam.eps, o.adam.weight_decay, (float)c1, (float)c2);
  if (c.n_layers > 0)
    hipLaunchKernelGGL(muon_kernel, dim3(3 * c.n_layers), dim3(kNsThreads), 0, s, theta, grads, m, L, o.lr,
                       o.momentum, o.weight_decay, o.rms_scale, o.ns_eps, o.ns_steps);
  return hipGetLastError();
}

}  // namespace fvan
