// Hand-written backward pass of ln q (Alg. 1) for the REINFORCE gradient
// (Eqs. 16-19): grads += sum_b w_b d ln q_b / d theta.
//
// Per chunk of samples the forward pass is run once to save every layer's
// input; then, layer by layer from the top, the layer's forward is recomputed
// (attention included: scores are rebuilt from Q, K and the saved
// log-sum-exp, never stored) and differentiated:
//   FFN:   dW2 = dy^T g, dg = dy W2, dh = dg * GELU'(h), dW1 = dh^T a2, da2 = dh W1, LN2'
//   attn:  dQ per query tile, dK/dV per key tile (both deterministic, no atomics)
//   QKV:   dWqkv = dqkv^T a1, da1 = dqkv Wqkv, LN1'
// Weight gradients are split-K MFMA GEMMs over the rows, with operands stored
// feature-major and a row of ones appended to the right operand so the bias
// gradient falls out as one more output column; partial sums are reduced in a
// fixed order and added to the caller's gradient vector.
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "fvan_model.h"

#include "passes.h"
#include "row_kernels.h"
#include "attn_mfma.h"
#include "attn_f16.h"
#include "attn_generic.h"

namespace fvan {

// Both operands as stored activations (not packed weights).
template <int MODE> struct FragAB;
template <> struct FragAB<0> {
  static __device__ __forceinline__ floatx4 step(const float* a, const float* b, floatx4 acc) {
    return Frag<0>::step(a, reinterpret_cast<const uint4*>(b), nullptr, acc);
  }
};
template <> struct FragAB<2> {
  static __device__ __forceinline__ floatx4 step(const float* a, const float* b, floatx4 acc) {
    float x[8], y[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) { x[i] = a[i]; y[i] = b[i]; }
    uint4 ah, al, bh, bl;
    split8(x, ah, al);
    split8(y, bh, bl);
    acc = mfma_bf16(al, bh, acc);
    acc = mfma_bf16(ah, bl, acc);
    return mfma_bf16(ah, bh, acc);
  }
};

// ---------------------------------------------------------------- head
// One workgroup per sample.  dz = w_b (onehot(s) - softmax(z)); dX = W_h^T dz;
// per-sample partial sums of dW_h (2 x D) and db_h (2) into part[b].
template <int D>
__global__ __launch_bounds__(256) void head_bwd_kernel(const float* __restrict__ X, const float* __restrict__ theta,
                                                       int64_t head_w, int64_t head_b, const int8_t* __restrict__ spins,
                                                       const float* __restrict__ w, int N, float* __restrict__ dX,
                                                       float* __restrict__ part) {
  __shared__ float red[16][2 * D + 2];
  const int b = blockIdx.x;
  const int grp = threadIdx.x >> 4, part_ = threadIdx.x & 15;
  const float* w0 = theta + head_w;
  const float* w1 = w0 + D;
  const float b0v = theta[head_b], b1v = theta[head_b + 1];
  const float wb = w[b];
  float gw0[D / 16], gw1[D / 16], gb0 = 0.f, gb1 = 0.f;
#pragma unroll
  for (int i = 0; i < D / 16; ++i) { gw0[i] = 0.f; gw1[i] = 0.f; }
  for (int t = grp; t < N; t += 16) {
    const int64_t r = (int64_t)b * N + t;
    const float* x = X + r * D;
    float xv[D / 16];
    float z0 = 0.f, z1 = 0.f;
#pragma unroll
    for (int i = 0; i < D / 16; ++i) {
      const int k = part_ + 16 * i;
      xv[i] = x[k];
      z0 += xv[i] * w0[k];
      z1 += xv[i] * w1[k];
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) { z0 += __shfl_xor(z0, o, 16); z1 += __shfl_xor(z1, o, 16); }
    const float d = (z1 + b1v) - (z0 + b0v);
    const float e = expf(-fabsf(d));
    const float p1 = d >= 0.f ? 1.0f / (1.0f + e) : e / (1.0f + e);   // softmax(z)[1]
    const int s = spins[r] > 0;
    const float dz1 = wb * ((float)s - p1);
    const float dz0 = -dz1;
#pragma unroll
    for (int i = 0; i < D / 16; ++i) {
      const int k = part_ + 16 * i;
      dX[r * D + k] = dz0 * w0[k] + dz1 * w1[k];
      gw0[i] += dz0 * xv[i];
      gw1[i] += dz1 * xv[i];
    }
    gb0 += dz0;
    gb1 += dz1;
  }
#pragma unroll
  for (int i = 0; i < D / 16; ++i) {
    red[grp][part_ + 16 * i] = gw0[i];
    red[grp][D + part_ + 16 * i] = gw1[i];
  }
  if (part_ == 0) { red[grp][2 * D] = gb0; red[grp][2 * D + 1] = gb1; }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * D + 2; k += 256) {
    float s = 0.f;
    for (int g = 0; g < 16; ++g) s += red[g][k];
    part[(size_t)b * (2 * D + 2) + k] = s;
  }
}

// out[k] += sum_{i < n} part[i * width + k] in a fixed order.  Two levels: each
// workgroup sums a fixed slice of partials for 64 columns into part2, then one
// pass adds the slices.
constexpr int kColSlices = 64;
__global__ __launch_bounds__(256) void colsum_slices_kernel(const float* __restrict__ part, int n, int width,
                                                            float* __restrict__ part2) {
  __shared__ float red[4][64];
  const int k = blockIdx.x * 64 + (threadIdx.x & 63);
  const int sub = threadIdx.x >> 6;
  const int slice = blockIdx.y;
  const int per = (n + kColSlices - 1) / kColSlices;
  const int i0 = slice * per, i1 = min(n, i0 + per);
  float s = 0.f;
  if (k < width)
    for (int i = i0 + sub; i < i1; i += 4) s += part[(size_t)i * width + k];
  red[sub][threadIdx.x & 63] = s;
  __syncthreads();
  if (sub == 0 && k < width)
    part2[(size_t)slice * width + k] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void colsum_final_kernel(const float* __restrict__ part2, int width, float* __restrict__ out) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < width; k += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int i = 0; i < kColSlices; ++i) s += part2[(size_t)i * width + k];
    out[k] += s;
  }
}

static void colsum_add(const float* part, int n, int width, float* part2, float* out, hipStream_t s) {
  hipLaunchKernelGGL(colsum_slices_kernel, dim3((width + 63) / 64, kColSlices), dim3(256), 0, s, part, n, width, part2);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((width + 255) / 256), dim3(256), 0, s, (const float*)part2, width, out);
}

// ---------------------------------------------------------------- transpose + cast
// dY (float, [rows x D]) -> Yrm (ActT, row-major; skipped when NULL) and YT (ActT, [D x ldT]).
// 16-byte loads and stores: each thread moves four consecutive features of a
// row in, and four consecutive rows of a feature out (ldT is a multiple of 64).
template <int D, typename AT>
__global__ __launch_bounds__(256) void transpose_cast_kernel(const float* __restrict__ Y, int64_t rows,
                                                             AT* __restrict__ Yrm, AT* __restrict__ YT, int64_t ldT) {
  __shared__ float tile[64][D + 1];
  constexpr int NV = 64 * D / 4 / 256;             // float4 per thread
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  float4 v[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int rr = i / (D / 4), k = 4 * (i % (D / 4));
    const int64_t r = r0 + rr;
    v[u] = r < rows ? *reinterpret_cast<const float4*>(Y + r * D + k) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int rr = i / (D / 4), k = 4 * (i % (D / 4));
    tile[rr][k] = v[u].x;
    tile[rr][k + 1] = v[u].y;
    tile[rr][k + 2] = v[u].z;
    tile[rr][k + 3] = v[u].w;
    const int64_t r = r0 + rr;
    if (Yrm && r < rows) {
      AT* d = Yrm + r * D + k;
      d[0] = from_f<AT>(v[u].x);
      d[1] = from_f<AT>(v[u].y);
      d[2] = from_f<AT>(v[u].z);
      d[3] = from_f<AT>(v[u].w);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int i = threadIdx.x + 256 * u;
    const int k = i / 16, rr = 4 * (i % 16);
    const int64_t r = r0 + rr;
    AT* d = YT + (int64_t)k * ldT + r;
    if (r + 3 < rows) {
      if constexpr (sizeof(AT) == 4) {
        *reinterpret_cast<float4*>(d) = make_float4(tile[rr][k], tile[rr + 1][k], tile[rr + 2][k], tile[rr + 3][k]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = from_f<AT>(tile[rr + e][k]);
      }
    } else {
      for (int e = 0; e < 4 && r + e < rows; ++e) d[e] = from_f<AT>(tile[rr + e][k]);
    }
  }
}

// ---------------------------------------------------------------- weight-gradient GEMM
// part[s][m][n] = sum_{k in slice s, k < K} A[m][k] B[n][k]; A [m_total x lda]
// and B [NB x ldb] feature-major, K = rows of the chunk.  One workgroup (8 waves)
// owns an M x NB block of the output (row block mbi, column block nbi) for its K slice, so
// the blocks of one K slice read its operand slices close in time on one XCD (L2 reuse); K chunks are staged in LDS (the next chunk is fetched into
// registers while the current one is multiplied) and every wave keeps a block of
// RT x CT accumulator tiles (rows split over WRG wave groups, columns over WCG).
template <int MT>
struct WaveGrid {
  static constexpr int WRG = (MT % 8 == 0) ? 8 : (MT % 4 == 0) ? 4 : (MT % 2 == 0) ? 2 : 1;
  static constexpr int WCG = 8 / WRG;
  static constexpr int RT = MT / WRG;
};

template <int MODE, int M, int NB>
__global__ __launch_bounds__(512) void wgrad_kernel(const typename Mode<MODE>::ActT* __restrict__ A, int64_t lda,
                                                    const typename Mode<MODE>::ActT* __restrict__ B, int64_t ldb,
                                                    int64_t K, int64_t kper, int m_total, int n_total,
                                                    int nsplit_m, int nsplit_n, float* __restrict__ part) {
  // in split mode an operand no other workgroup of this K slice re-reads (A when
  // the output's columns are not split, B when its rows are not) is streamed with
  // non-temporal loads, so that it does not evict what the co-running attention
  // backward re-reads from L2 (FP32 mode measured no gain)
  const bool nt_a = Mode<MODE>::SPLIT && nsplit_n == 1, nt_b = Mode<MODE>::SPLIT && nsplit_m == 1;
  typedef typename Mode<MODE>::ActT AT;
  // split mode stages each operand already split into BF16 hi and lo planes, so a
  // K chunk is converted once instead of once per wave that multiplies it
  constexpr bool SPLIT = Mode<MODE>::SPLIT;
  typedef typename std::conditional<SPLIT, __bf16, AT>::type ST;
  constexpr int NPL = SPLIT ? 2 : 1;                // LDS planes (hi, lo)
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int PADK = KC + 16 / (int)sizeof(ST);
  constexpr int MT = M / 16, NT = NB / 16;
  typedef WaveGrid<MT> G;
  constexpr int RT = G::RT, WCG = G::WCG;
  constexpr int CT = (NT + WCG - 1) / WCG;
  constexpr int VPL = 16 / (int)sizeof(AT);        // elements per 16-byte load
  __shared__ __attribute__((aligned(16))) ST As[NPL][M][PADK];
  __shared__ __attribute__((aligned(16))) ST Bs[NPL][NB][PADK];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave / WCG, wc = wave % WCG;
  // 1-D grid over (column block fastest, then row block, then K slice), dealt to
  // the XCDs in contiguous ranges: the workgroups of one K slice read the same
  // operand slice close in time on one XCD
  const int v = xcd_contiguous(blockIdx.x, gridDim.x);
  const int nbi = v % nsplit_n, mbi = (v / nsplit_n) % nsplit_m, s = v / (nsplit_n * nsplit_m);
  A += (int64_t)mbi * M * lda;                     // this workgroup's block of M output rows
  B += (int64_t)nbi * NB * ldb;                    // and of NB output columns
  const int64_t kb = (int64_t)s * kper;
  const int64_t ke = std::min<int64_t>(K, kb + kper);
  floatx4 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // K chunks are fetched into registers one chunk ahead of the MFMA loop
  constexpr int NPIECE = (M + NB) * (KC / VPL);    // 16-byte pieces per chunk
  constexpr int NLD = (NPIECE + 511) / 512;
  uint4 pre[NLD];
  auto fetch = [&](int64_t k) {
    const bool full = k + KC <= ke;
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int x = threadIdx.x + 512 * u;
      pre[u] = make_uint4(0u, 0u, 0u, 0u);
      if (x < NPIECE) {
        const int row = x / (KC / VPL), piece = x % (KC / VPL);
        const AT* src = row < M ? A + (int64_t)row * lda : B + (int64_t)(row - M) * ldb;
        const int64_t kk = k + piece * VPL;
        if (full) {
          if (row < M ? nt_a : nt_b) {
            const float4 f = load_nt4(reinterpret_cast<const float*>(src + kk));
            pre[u] = make_uint4(__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z), __float_as_uint(f.w));
          } else {
            pre[u] = *reinterpret_cast<const uint4*>(src + kk);
          }
        } else {
          alignas(16) AT tmp[VPL];
#pragma unroll
          for (int i = 0; i < VPL; ++i) tmp[i] = kk + i < ke ? src[kk + i] : from_f<AT>(0.f);
          pre[u] = *reinterpret_cast<const uint4*>(tmp);
        }
      }
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k = kb; k < ke; k += KC) {
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int x = threadIdx.x + 512 * u;
      if (x < NPIECE) {
        const int row = x / (KC / VPL), piece = x % (KC / VPL);
        ST* hi_dst = row < M ? &As[0][row][piece * VPL] : &Bs[0][row - M][piece * VPL];
        if constexpr (SPLIT) {
          ST* lo_dst = row < M ? &As[1][row][piece * VPL] : &Bs[1][row - M][piece * VPL];
          const SplitBf16x4 t = AOp<2>::make(__uint_as_float(pre[u].x), __uint_as_float(pre[u].y),
                                             __uint_as_float(pre[u].z), __uint_as_float(pre[u].w));
          *reinterpret_cast<bf16x4*>(hi_dst) = t.h;
          *reinterpret_cast<bf16x4*>(lo_dst) = t.l;
        } else {
          *reinterpret_cast<uint4*>(hi_dst) = pre[u];
        }
      }
    }
    __syncthreads();
    if (k + KC < ke) fetch(k + KC);
    if constexpr (SPLIT) {
      // lane fragments: 8 consecutive k of one row, hi and lo planes
      uint4 ah[RT], al[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int row = (wr * RT + i) * 16 + (lane & 15), k8 = (lane >> 4) * LK;
        ah[i] = *reinterpret_cast<const uint4*>(&As[0][row][k8]);
        al[i] = *reinterpret_cast<const uint4*>(&As[1][row][k8]);
      }
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        const int ct = wc * CT + j;
        if (ct < NT) {
          const int row = ct * 16 + (lane & 15), k8 = (lane >> 4) * LK;
          const uint4 bh = *reinterpret_cast<const uint4*>(&Bs[0][row][k8]);
          const uint4 bl = *reinterpret_cast<const uint4*>(&Bs[1][row][k8]);
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            acc[i][j] = mfma_bf16(al[i], bh, acc[i][j]);
            acc[i][j] = mfma_bf16(ah[i], bl, acc[i][j]);
            acc[i][j] = mfma_bf16(ah[i], bh, acc[i][j]);
          }
        }
      }
    } else {
    alignas(16) AT af[RT][LK];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const AT* ap = &As[0][(wr * RT + i) * 16 + (lane & 15)][(lane >> 4) * LK];
#pragma unroll
      for (int e = 0; e < LK; e += VPL) *reinterpret_cast<uint4*>(&af[i][e]) = *reinterpret_cast<const uint4*>(ap + e);
    }
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int ct = wc * CT + j;
      if (ct < NT) {
        alignas(16) AT bf[LK];
        const AT* bp = &Bs[0][ct * 16 + (lane & 15)][(lane >> 4) * LK];
#pragma unroll
        for (int e = 0; e < LK; e += VPL) *reinterpret_cast<uint4*>(&bf[e]) = *reinterpret_cast<const uint4*>(bp + e);
#pragma unroll
        for (int i = 0; i < RT; ++i) acc[i][j] = FragAB<MODE>::step(af[i], bf, acc[i][j]);
      }
    }
    }
    __syncthreads();
  }
  float* out = part + ((size_t)s * m_total + (size_t)mbi * M) * n_total + (size_t)nbi * NB;
#pragma unroll
  for (int i = 0; i < RT; ++i) {
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int ct = wc * CT + j;
      if (ct < NT) {
        const int n = ct * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(size_t)((wr * RT + i) * 16 + 4 * (lane >> 4) + q) * n_total + n] = acc[i][j][q];
      }
    }
  }
}

// grads: W[m][n] += sum_s part[s][m][n] for n < Nw; bias[m] += sum_s part[s][m][Nw]
// (rows m >= m_valid are padding and not written).
// A block owns 64 consecutive outputs; its four thread groups sum the slices
// s = grp, grp + 4, ... (eight loads in flight each) and the four partial sums
// are added in a fixed order: bitwise reproducible.
constexpr int kRedOut = 64, kRedGroups = 4;
__global__ __launch_bounds__(kRedOut * kRedGroups) void wgrad_reduce_kernel(const float* __restrict__ part, int S,
                                                                            int M, int NB, int Nw, int m_valid,
                                                                            float* __restrict__ gW,
                                                                            float* __restrict__ gb) {
  __shared__ float red[kRedGroups][kRedOut];
  const int total = M * (Nw + 1);
  const int o = threadIdx.x % kRedOut, grp = threadIdx.x / kRedOut;
  const int i = blockIdx.x * kRedOut + o;
  const int m = i / (Nw + 1), n = i % (Nw + 1);
  const size_t stride = (size_t)M * NB;
  const float* p = part + (size_t)min(m, M - 1) * NB + n;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (i < total) {
    int s = grp;
    for (; s + 7 * kRedGroups < S; s += 8 * kRedGroups) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += p[(size_t)(s + u * kRedGroups) * stride];
    }
    for (; s < S; s += kRedGroups) acc[0] += p[(size_t)s * stride];
  }
  red[grp][o] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (grp == 0 && i < total && m < m_valid) {
    const float v = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
    if (n < Nw) gW[(size_t)m * Nw + n] += v;
    else gb[m] += v;
  }
}

template <int MODE, int M, int Nw>
static hipError_t wgrad(fvan_model* m, const void* A, const void* B, int64_t K, float* gW, float* gb, hipStream_t s,
                        int m_valid = M, float* part = nullptr) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int NB = Nw + 16;
  auto& f = m->fw;
  if (!part) part = f.part;
  const int KC = Mode<MODE>::KC;
  int S = (int)std::max<int64_t>(1, std::min<int64_t>(512, K / (8 * KC)));
  while ((size_t)S * M * NB > f.part_floats) --S;
  int64_t kper = (K + S - 1) / S;
  kper = (kper + KC - 1) / KC * KC;
  S = (int)((K + kper - 1) / kper);
  // large outputs are split over several workgroups per K slice (keeps the
  // accumulators and the prefetch registers of a wave within 256 VGPRs): 512 rows
  // by rows, 512 + 16 columns into three column blocks, so that the split re-reads
  // the smaller operand
  constexpr int MS = M >= 512 ? M / 2 : M;
  constexpr int NBS = NB >= 512 && NB % 48 == 0 ? NB / 3 : NB;
  hipLaunchKernelGGL((wgrad_kernel<MODE, MS, NBS>), dim3(S * (M / MS) * (NB / NBS)), dim3(512), 0, s, (const AT*)A,
                     f.ldT, (const AT*)B, f.ldT, K, kper, M, NB, M / MS, NB / NBS, part);
  const int total = M * (Nw + 1);
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((total + kRedOut - 1) / kRedOut), dim3(kRedOut * kRedGroups), 0, s,
                     (const float*)part, S, M, NB, Nw, m_valid, gW, gb);
  return hipGetLastError();
}

// ---------------------------------------------------------------- LayerNorm backward
// out[r] = resid[r] + LN'(da[r]) for y = LN(x) with gain g; per 64-row tile
// partial sums of dg (= sum da * xhat) and db (= sum da) into part[tile][2D].
template <int D>
__global__ __launch_bounds__(256) void ln_bwd_kernel(const float* __restrict__ da, const float* __restrict__ X,
                                                     const float* __restrict__ g, const float* __restrict__ resid,
                                                     int64_t rows, float* __restrict__ out, float* __restrict__ part) {
  constexpr int PER = D / 16;
  __shared__ float red[16][2 * D];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int grp = threadIdx.x >> 4, p = threadIdx.x & 15;
  float pg[PER], pb[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) { pg[i] = 0.f; pb[i] = 0.f; }
  for (int rr = grp; rr < 64; rr += 16) {
    const int64_t r = r0 + rr;
    if (r >= rows) break;
    float x[PER], dy[PER];
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) { x[i] = X[r * D + p + 16 * i]; s += x[i]; }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
    const float mean = s * (1.0f / D);
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) { x[i] -= mean; q += x[i] * x[i]; }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) q += __shfl_xor(q, o, 16);
    const float rstd = rsqrtf(q * (1.0f / D) + kLnEps);
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = p + 16 * i;
      const float a = da[r * D + k];
      const float xh = x[i] * rstd;
      x[i] = xh;
      pg[i] += a * xh;
      pb[i] += a;
      dy[i] = a * g[k];
      s1 += dy[i];
      s2 += dy[i] * xh;
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) { s1 += __shfl_xor(s1, o, 16); s2 += __shfl_xor(s2, o, 16); }
    s1 *= 1.0f / D;
    s2 *= 1.0f / D;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int k = p + 16 * i;
      out[r * D + k] = resid[r * D + k] + rstd * (dy[i] - s1 - x[i] * s2);
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) { red[grp][p + 16 * i] = pg[i]; red[grp][D + p + 16 * i] = pb[i]; }
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * D; k += 256) {
    float s = 0.f;
    for (int gI = 0; gI < 16; ++gI) s += red[gI][k];
    part[(size_t)blockIdx.x * 2 * D + k] = s;
  }
}

// ---------------------------------------------------------------- embedding
// dP[t][k] += sum_b dX0[b*N + t][dt + k], in two fixed-order steps: workgroup
// column y sums the samples of its slice for every (t, k) into part[y][t][k],
// then pos_grad_final adds the slices in order.
constexpr int kPosSlices = 32;
__global__ void pos_grad_slices_kernel(const float* __restrict__ dX, int nsamp, int N, int D, int dt,
                                       float* __restrict__ part) {
  const int dp = D - dt;
  const int64_t total = (int64_t)N * dp;
  const int per = (nsamp + gridDim.y - 1) / gridDim.y;
  const int b0 = blockIdx.y * per, b1 = min(nsamp, b0 + per);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(i / dp), k = (int)(i % dp);
    float s = 0.f;
    for (int b = b0; b < b1; ++b) s += dX[((int64_t)b * N + t) * D + dt + k];
    part[(size_t)blockIdx.y * total + i] = s;
  }
}

__global__ void pos_grad_final_kernel(const float* __restrict__ part, int slices, int64_t total,
                                      float* __restrict__ gpos) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int y = 0; y < slices; ++y) s += part[(size_t)y * total + i];
    gpos[i] += s;
  }
}

// dT[tok][k] += sum over the rows fed token tok (vocab 2), in two fixed-order
// steps: workgroup (slice, k) sums its slice of rows into part[slice][tok * dt + k],
// then colsum_final_kernel adds the kColSlices partials.
__global__ __launch_bounds__(256) void tok_grad_slices_kernel(const float* __restrict__ dX,
                                                              const int8_t* __restrict__ spins, int64_t rows, int N,
                                                              int D, int dt, float* __restrict__ part) {
  __shared__ float red[2][4];
  const int k = blockIdx.y;
  const int64_t per = (rows + kColSlices - 1) / kColSlices;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = std::min<int64_t>(rows, r0 + per);
  float s0 = 0.f, s1 = 0.f;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const bool one = (r % N != 0) && spins[r - 1] > 0;   // token of row r is s_{t-1} (0 at t = 0)
    const float v = dX[r * D + k];
    s0 += one ? 0.f : v;
    s1 += one ? v : 0.f;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) { red[0][wave] = s0; red[1][wave] = s1; }
  __syncthreads();
  if (threadIdx.x < 2)
    part[(size_t)blockIdx.x * 2 * dt + threadIdx.x * dt + k] =
        red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

// ---------------------------------------------------------------- vocab-way head (patch tokens)
// 64 rows (positions) per workgroup, one 16-row MFMA tile per wave:
//   z = W_h h + b_h (MFMA against the padded head pack [vp x D]); p = softmax(z)
//   per row (the row's vp logits sit in 16 lanes x vp/16 tiles); dz = w_b
//   (onehot(tok) - p), the gradient of w_b ln p_t(tok_t) (a token >= vocab makes
//   its row's dz NaN); dz written feature-major into dZT [mrows][ldT] (rows >=
//   vocab zero) for the head's weight-gradient GEMM, and through a wave-private
//   LDS tile into dX = W_h^T dz (MFMA against the transposed pack [D x vp]).
constexpr int kHbRows = 64;
template <int MODE, int D, int VP>
__global__ __launch_bounds__(256) void head_vocab_bwd_kernel(const float* __restrict__ X, const uint4* __restrict__ ph,
                                                             const uint4* __restrict__ phT,
                                                             const float* __restrict__ hb, int V, int mrows,
                                                             const uint8_t* __restrict__ tokens,
                                                             const float* __restrict__ w, int N, int64_t rows,
                                                             float* __restrict__ dX, float* __restrict__ dZT,
                                                             int64_t ldT) {
  typedef typename Mode<MODE>::ActT AT;
  constexpr int KC = Mode<MODE>::KC;
  constexpr int LK = KC / 4;
  constexpr int NC = D / KC;                 // K chunks of z = h W_h^T
  constexpr int NZ = VP / 16;                // logit tiles
  constexpr int NC2 = VP / KC;               // K chunks of dX = dz W_h
  constexpr int NX = D / 16;                 // dX tiles
  constexpr size_t LO1 = (size_t)VP * D / 8, LO2 = LO1;
  constexpr int LDZ = VP + 4;
  __shared__ __align__(16) float Zs[4][16][LDZ];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), g = lane >> 4, c = lane & 15;
  const int64_t rbase = (int64_t)blockIdx.x * kHbRows + wave * 16;
  if (rbase >= rows) return;                 // no block-wide barrier below
  FragA<MODE> fa[NC];
  {
    const int64_t ra = std::min<int64_t>(rbase + c, rows - 1);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      alignas(16) AT af[LK];
#pragma unroll
      for (int i = 0; i < LK; i += 4)
        *reinterpret_cast<float4*>(&af[i]) = *reinterpret_cast<const float4*>(X + ra * D + cc * KC + g * LK + i);
      fa[cc].load(af);
    }
  }
  floatx4 z[NZ];
#pragma unroll
  for (int t = 0; t < NZ; ++t) {
    z[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const uint4* bp = ph + (size_t)t * NC * 64 + lane;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) z[t] = fa[cc].mma(bp + cc * 64, bp + cc * 64 + LO1, z[t]);
  }
  // softmax of each row: lane (g, c) holds logits of rows 4g+i at columns 16t+c
  float mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
  for (int t = 0; t < NZ; ++t) {
    const int col = 16 * t + c;
    const float bias = col < V ? hb[col] : 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z[t][i] = col < V ? z[t][i] + bias : -INFINITY;
      mx[i] = fmaxf(mx[i], z[t][i]);
    }
  }
  float sum[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i) mx[i] = row_max16(mx[i]);
#pragma unroll
  for (int t = 0; t < NZ; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      z[t][i] = 16 * t + c < V ? expf(z[t][i] - mx[i]) : 0.f;
      sum[i] += z[t][i];
    }
  int tok[4];
  float wb[4];
  bool live[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sum[i] = row_sum16(sum[i]);
    const int64_t r = rbase + 4 * g + i;
    live[i] = r < rows;
    const int64_t rr = live[i] ? r : rows - 1;
    tok[i] = tokens[rr];
    wb[i] = live[i] ? w[rr / N] : 0.f;
  }
  float (*Z)[LDZ] = Zs[wave];
#pragma unroll
  for (int t = 0; t < NZ; ++t) {
    const int col = 16 * t + c;
    float dz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dz[i] = col < V ? wb[i] * ((col == tok[i] ? 1.f : 0.f) - z[t][i] / sum[i]) : 0.f;
      if (live[i] && tok[i] >= V) dz[i] = __builtin_nanf("");
      Z[4 * g + i][col] = dz[i];
    }
    if (col < mrows) {
      float* dst = dZT + (int64_t)col * ldT + rbase + 4 * g;
      if (live[3]) {
        *reinterpret_cast<float4*>(dst) = make_float4(dz[0], dz[1], dz[2], dz[3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (live[i]) dst[i] = dz[i];
      }
    }
  }
  wave_lds_sync();
  floatx4 ax[NX];
#pragma unroll
  for (int t = 0; t < NX; ++t) ax[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int cc = 0; cc < NC2; ++cc) {
    FragA<MODE> dzf;
    dzf.load(&Z[c][cc * KC + g * LK]);
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const uint4* bp = phT + ((size_t)t * NC2 + cc) * 64 + lane;
      ax[t] = dzf.mma(bp, bp + LO2, ax[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NX; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (live[i]) dX[(rbase + 4 * g + i) * D + 16 * t + c] = ax[t][i];
}

// dT[tok][k] (k < dt) summed over the rows fed token tok (start token 0 at
// t = 0): one wave per slice of `per` rows, walked in order, accumulating into
// LDS [V][dt]; part[slice][V * dt] is then summed over the slices in a fixed
// order (colsum_add).  Tokens >= vocab are clamped (their dX is NaN already).
__global__ __launch_bounds__(64) void tok_grad_vocab_kernel(const float* __restrict__ dX,
                                                            const uint8_t* __restrict__ tokens, int64_t rows, int N,
                                                            int D, int dt, int V, int64_t per,
                                                            float* __restrict__ part) {
  extern __shared__ float acc[];                   // [V][dt]
  for (int i = threadIdx.x; i < V * dt; i += 64) acc[i] = 0.f;
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = std::min<int64_t>(rows, r0 + per);
  for (int64_t r = r0; r < r1; ++r) {
    const int tok = r % N == 0 ? 0 : min((int)tokens[r - 1], V - 1);
    for (int k = threadIdx.x; k < dt; k += 64) acc[tok * dt + k] += dX[r * D + k];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < V * dt; i += 64) part[(size_t)blockIdx.x * V * dt + i] = acc[i];
}

// ---------------------------------------------------------------- driver
// Attention backward of one layer for heads wider than 16 (attn_generic.h).
template <typename KT, typename AT, int DH>
static hipError_t attn_bwd_gen(fvan_model* m, const KT* QKV, const float* X, const float* XM, const float* LSE,
                               int nsamp, hipStream_t s) {
  const fvan_model_config& c = m->cfg;
  auto& f = m->fw;
  const int N = c.n_spins, D = c.d_model, H = c.n_heads;
  const int grid = (N + kGenRows - 1) / kGenRows * H * nsamp;
  hipLaunchKernelGGL((attn_bwd_dq_gen<KT, AT, DH>), dim3(grid), dim3(kGenThreads), 0, s, QKV, X, XM,
                     (const float*)f.dXM, LSE, f.DELTA, (AT*)f.dQKV, (AT*)f.T_e, f.ldT, N, D, H, c.window, m->kg.P);
  hipLaunchKernelGGL((attn_bwd_dkv_gen<KT, AT, DH>), dim3(grid), dim3(kGenThreads), 0, s, QKV, (const float*)f.dXM,
                     LSE, (const float*)f.DELTA, (AT*)f.dQKV, (AT*)f.T_e, f.ldT, N, D, H, c.window, m->kg.P);
  return hipGetLastError();
}

// seq: spins (int8, TOK false) or patch tokens (uint8, TOK true) [nsamp, N].
template <int MODE, int D, bool TOK>
static hipError_t backward_chunk_t(fvan_model* m, const void* seq, int nsamp, const float* w, hipStream_t s) {
  typedef typename Mode<MODE>::ActT AT;
  typedef typename Mode<MODE>::KvT KT;
  const fvan_model_config& c = m->cfg;
  auto& f = m->fw;
  const int N = c.n_spins, H = c.n_heads, L = c.n_layers;
  const int64_t rows = (int64_t)nsamp * N;
  const int rgrid = (int)((rows + 63) / 64);
  float* G = m->grads;
  const int8_t* spins = reinterpret_cast<const int8_t*>(seq);
  const uint8_t* tokens = reinterpret_cast<const uint8_t*>(seq);
  hipError_t err = TOK ? forward_chunk_tokens(m, tokens, nsamp, nullptr, s) : forward_chunk(m, spins, nsamp, nullptr, true, s);
  if (err != hipSuccess) return err;

  // head
  const float* XL = f.X + (size_t)L * f.rows * D;
  if constexpr (TOK) {
    const int mrows = c.vocab <= 16 ? 16 : 256;
    const char* wp = reinterpret_cast<const char*>(m->wpack);
    const uint4* ph = reinterpret_cast<const uint4*>(wp + m->pk.head);
    const uint4* phT = reinterpret_cast<const uint4*>(wp + m->pk.headT);
    const dim3 hgrid((unsigned)((rows + kHbRows - 1) / kHbRows));
    const float* hb = m->params + m->po.head_b;
    switch (m->pk.vp) {
#define HB_CASE(VPV)                                                                                             \
  case VPV:                                                                                                      \
    hipLaunchKernelGGL((head_vocab_bwd_kernel<MODE, D, VPV>), hgrid, dim3(256), 0, s, XL, ph, phT, hb, c.vocab, \
                       mrows, tokens, w, N, rows, f.dX, (float*)f.T_a, f.ldT);                                   \
    break;
      HB_CASE(32) HB_CASE(64) HB_CASE(96) HB_CASE(128) HB_CASE(160) HB_CASE(192) HB_CASE(224) HB_CASE(256)
#undef HB_CASE
      default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((transpose_cast_kernel<D, AT>), dim3(rgrid), dim3(256), 0, s, XL, rows, (AT*)nullptr,
                       (AT*)f.T_c, f.ldT);
    if (mrows == 16) {
      if ((err = wgrad<MODE, 16, D>(m, f.T_a, f.T_c, rows, G + m->po.head_w, G + m->po.head_b, s, c.vocab)))
        return err;
    } else {
      if constexpr (4 * D >= 256) {
        if ((err = wgrad<MODE, 256, D>(m, f.T_a, f.T_c, rows, G + m->po.head_w, G + m->po.head_b, s, c.vocab)))
          return err;
      } else {
        return hipErrorInvalidValue;
      }
    }
  } else {
    hipLaunchKernelGGL((head_bwd_kernel<D>), dim3(nsamp), dim3(256), 0, s, XL, m->params, m->po.head_w, m->po.head_b,
                       spins, w, N, f.dX, f.colpart);
    colsum_add(f.colpart, nsamp, 2 * D + 2, f.colpart2, G + m->po.head_w, s);
  }

  // The layer weight gradients go to the side stream as soon as their operands
  // are written, and run beside the attention backward and the next layer's FFN
  // backward; a buffer they read is written again only after its "read" event.
  // Every event waited on is recorded earlier in this chunk (the previous chunk
  // joined the side stream back before returning), so the fork and join also
  // hold under stream capture.
  hipStream_t ss = f.side;
  hipEvent_t ffn_ready = f.ev[0], ffn_read = f.ev[1], qkv_ready = f.ev[2], qkv_read = f.ev[3];
  for (int l = L - 1; l >= 0; --l) {
    const float* lp = m->params + m->po.layer0 + (int64_t)l * m->po.layer_stride;
    float* gl = G + m->po.layer0 + (int64_t)l * m->po.layer_stride;
    const char* wl = reinterpret_cast<const char*>(m->wpack) + (size_t)l * m->pk.layer_stride;
    const float* X = f.X + (size_t)l * f.rows * D;
    const float* XM = f.XM + (size_t)l * f.rows * D;
    const KT* QKV = reinterpret_cast<const KT*>(f.QKV) + (size_t)l * f.rows * 3 * D;
    const float* LSE = f.LSE + (size_t)l * f.rows * H;
    // ---- FFN: one fused kernel recomputes LN2, the pre-activation and GELU,
    // differentiates through W2, GELU' and W1 and the LayerNorm, and leaves the
    // feature-major operands of the two weight gradients
    if (l < L - 1 && (err = hipStreamWaitEvent(s, ffn_read, 0))) return err;   // recorded by layer l + 1
    hipLaunchKernelGGL((ffn_bwd_fused_kernel<MODE, D>), dim3((int)((rows + kFfnBwdRows - 1) / kFfnBwdRows)),
                       dim3(512), 0, s, XM, (const float*)f.dX, lp + m->po.ln2_g, lp + m->po.ln2_b, rows,
                       reinterpret_cast<const uint4*>(wl + m->pk.ffn1), reinterpret_cast<const uint4*>(wl + m->pk.ffn2T),
                       reinterpret_cast<const uint4*>(wl + m->pk.ffn1T), lp + m->po.ffn1_b, (AT*)f.T_b, (AT*)f.T_a,
                       (AT*)f.T_c, (AT*)f.T_d, f.ldT, f.dXM, f.colpart);
    if ((err = hipEventRecord(ffn_ready, s))) return err;
    if ((err = hipStreamWaitEvent(ss, ffn_ready, 0))) return err;
    if ((err = wgrad<MODE, D, 4 * D>(m, f.T_d, f.T_b, rows, gl + m->po.ffn2_w, gl + m->po.ffn2_b, ss, D, f.part2)))
      return err;
    if ((err = wgrad<MODE, 4 * D, D>(m, f.T_a, f.T_c, rows, gl + m->po.ffn1_w, gl + m->po.ffn1_b, ss, 4 * D,
                                     f.part2)))
      return err;
    if ((err = hipEventRecord(ffn_read, ss))) return err;
    colsum_add(f.colpart, (int)((rows + kFfnBwdRows - 1) / kFfnBwdRows), 2 * D, f.colpart2, gl + m->po.ln2_g, s);
    // ---- attention backward (dO = dXM: the heads' output is added to the residual directly);
    // probabilities are recomputed from Q, K and the saved log-sum-exp
    if (l < L - 1 && (err = hipStreamWaitEvent(s, qkv_read, 0))) return err;   // recorded by layer l + 1
    if (D / H == 16) {
      const dim3 qgrid((N + attn_rows(kDqThreads) - 1) / attn_rows(kDqThreads) * H * nsamp);
      const dim3 kgrid((N + attn_rows(kDkvThreads) - 1) / attn_rows(kDkvThreads) * H * nsamp);
      if constexpr (MODE == FVAN_BF16_SPLIT) {
        hipLaunchKernelGGL(attn_bwd_dq_f16, qgrid, dim3(kDqThreads), 0, s, (const _Float16*)QKV, X, XM,
                           (const float*)f.dXM, LSE, f.DELTA, (float*)f.dQKV, (float*)f.T_e, f.ldT, N, D, H, c.window,
                           m->kg.P);
        hipLaunchKernelGGL(attn_bwd_dkv_f16, kgrid, dim3(kDkvThreads), 0, s, (const _Float16*)QKV,
                           (const float*)f.dXM, LSE, (const float*)f.DELTA, (float*)f.dQKV, (float*)f.T_e, f.ldT, N,
                           D, H, c.window, m->kg.P);
      } else {
        hipLaunchKernelGGL((attn_bwd_dq_mfma<KT, AT, MODE>), qgrid, dim3(kDqThreads), 0, s, QKV, X, XM,
                           (const float*)f.dXM, LSE, f.DELTA, (AT*)f.dQKV, (AT*)f.T_e, f.ldT, N, D, H, c.window,
                           m->kg.P);
        hipLaunchKernelGGL((attn_bwd_dkv_mfma<KT, AT, MODE>), kgrid, dim3(kDkvThreads), 0, s, QKV,
                           (const float*)f.dXM, LSE, (const float*)f.DELTA, (AT*)f.dQKV, (AT*)f.T_e, f.ldT, N, D, H,
                           c.window, m->kg.P);
      }
    } else if (D / H == 32) {
      if ((err = attn_bwd_gen<KT, AT, 32>(m, QKV, X, XM, LSE, nsamp, s))) return err;
    } else {
      if constexpr (D >= 64)
        if ((err = attn_bwd_gen<KT, AT, 64>(m, QKV, X, XM, LSE, nsamp, s))) return err;
    }
    // ---- QKV backward: dA1 = dQKV W_qkv and the LN1 backward in one kernel, which
    // also leaves LN1(x) feature-major for the W_qkv gradient
    hipLaunchKernelGGL((gemm_ln_bwd_kernel<MODE, D, 3 * D>), dim3((int)((rows + kGlbRows - 1) / kGlbRows)), dim3(512),
                       0, s, (const float*)f.dQKV, rows, reinterpret_cast<const uint4*>(wl + m->pk.qkvT), X,
                       lp + m->po.ln1_g, lp + m->po.ln1_b, (const float*)f.dXM, f.dX, (float*)f.T_f, f.ldT, f.colpart);
    if ((err = hipEventRecord(qkv_ready, s))) return err;
    if ((err = hipStreamWaitEvent(ss, qkv_ready, 0))) return err;
    if ((err = wgrad<MODE, 3 * D, D>(m, f.T_e, f.T_f, rows, gl + m->po.qkv_w, gl + m->po.qkv_b, ss, 3 * D, f.part2)))
      return err;
    if ((err = hipEventRecord(qkv_read, ss))) return err;
    colsum_add(f.colpart, (int)((rows + kGlbRows - 1) / kGlbRows), 2 * D, f.colpart2, gl + m->po.ln1_g, s);
  }
  // join: every side-stream kernel precedes what follows on the caller's stream
  if ((err = hipStreamWaitEvent(s, qkv_read, 0))) return err;
  // embeddings
  const int64_t npos = (int64_t)N * (D - c.d_token);
  int slices = std::min(kPosSlices, nsamp);
  while (slices > 1 && (size_t)slices * npos > f.part_floats) --slices;
  hipLaunchKernelGGL(pos_grad_slices_kernel, dim3((unsigned)std::min<int64_t>((npos + 255) / 256, 4096), slices),
                     dim3(256), 0, s, (const float*)f.dX, nsamp, N, D, c.d_token, f.part);
  hipLaunchKernelGGL(pos_grad_final_kernel, dim3((unsigned)std::min<int64_t>((npos + 255) / 256, 4096)), dim3(256), 0,
                     s, (const float*)f.part, slices, npos, G + m->po.pos);
  if constexpr (TOK) {
    const int width = c.vocab * c.d_token;
    int S = (int)std::max<int64_t>(1, std::min<int64_t>(1024, rows / 64));
    while ((size_t)S * width > f.part_floats) --S;
    const int64_t per = (rows + S - 1) / S;
    S = (int)((rows + per - 1) / per);
    hipLaunchKernelGGL(tok_grad_vocab_kernel, dim3(S), dim3(64), (size_t)width * sizeof(float), s,
                       (const float*)f.dX, tokens, rows, N, D, c.d_token, c.vocab, per, f.part);
    colsum_add(f.part, S, width, f.colpart2, G + m->po.tok, s);
  } else {
    hipLaunchKernelGGL(tok_grad_slices_kernel, dim3(kColSlices, c.d_token), dim3(256), 0, s, (const float*)f.dX, spins,
                       rows, N, D, c.d_token, f.part);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((2 * c.d_token + 255) / 256), dim3(256), 0, s, (const float*)f.part,
                       2 * c.d_token, G + m->po.tok);
  }
  return hipGetLastError();
}

hipError_t backward_chunk(fvan_model* m, const int8_t* spins, int nsamp, const float* w, hipStream_t s) {
  const int D = m->cfg.d_model;
#define BWD_CASE(MODE, DD) \
  if (m->cfg.precision == MODE && D == DD) return backward_chunk_t<MODE, DD, false>(m, spins, nsamp, w, s);
  BWD_CASE(0, 32) BWD_CASE(0, 64) BWD_CASE(0, 128)
  BWD_CASE(2, 32) BWD_CASE(2, 64) BWD_CASE(2, 128)
#undef BWD_CASE
  return hipErrorInvalidValue;
}

hipError_t backward_chunk_tokens(fvan_model* m, const uint8_t* tokens, int nsamp, const float* w, hipStream_t s) {
  const int D = m->cfg.d_model;
#define BWD_CASE(MODE, DD) \
  if (m->cfg.precision == MODE && D == DD) return backward_chunk_t<MODE, DD, true>(m, tokens, nsamp, w, s);
  BWD_CASE(0, 32) BWD_CASE(0, 64) BWD_CASE(0, 128)
  BWD_CASE(2, 32) BWD_CASE(2, 64) BWD_CASE(2, 128)
#undef BWD_CASE
  return hipErrorInvalidValue;
}

}  // namespace fvan
