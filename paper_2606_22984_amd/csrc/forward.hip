// Teacher-forced pass of the network over every position at once (Alg. 1),
// and the row kernels the backward pass re-uses.  Rows r = b*N + t of a chunk
// of samples are processed in parallel:
//   embed      x0[r] = [tok_emb[tok]; pos_emb[t]]
//   ln         a = LN(x) (row-major GEMM operand and/or a feature-major copy)
//   gemm_rows  out = a W^T (packed weights, MFMA) with fused epilogues
//   attn_fwd   band+prefix masked attention, online softmax; writes o, x + o
//              and the per-(row, head) log-sum-exp the backward pass needs
//   head_fwd   log p_t(s_t) summed per sample in a fixed order
// and, for models over 2^D-spin patch tokens, the token embedding and the
// vocab-way head (embed_tokens, head_vocab).
#include <algorithm>

#include "device_common.h"
#include "fvan_model.h"
#include "passes.h"
#include "row_kernels.h"
#include "attn_mfma.h"
#include "attn_f16.h"
#include "attn_generic.h"

namespace fvan {

// ---------------------------------------------------------------- embedding
__global__ void embed_kernel(const float* __restrict__ theta, int64_t pos_off, int dt, int D, int N,
                             const int8_t* __restrict__ spins, int64_t rows, float* __restrict__ X) {
  const int64_t total = rows * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / D;
    const int k = (int)(i % D);
    const int t = (int)(r % N);
    float v;
    if (k < dt) {
      const int tok = t == 0 ? 0 : (spins[r - 1] + 1) >> 1;
      v = theta[tok * dt + k];
    } else {
      v = theta[pos_off + (int64_t)t * (D - dt) + (k - dt)];
    }
    X[i] = v;
  }
}

// ---------------------------------------------------------------- head
// One workgroup per sample; 16 lanes per position.  logq[b] = sum_t log p_t(s_t)
// in a fixed order.
template <int D>
__global__ __launch_bounds__(256) void head_fwd_kernel(const float* __restrict__ X, const float* __restrict__ theta,
                                                       int64_t head_w, int64_t head_b, const int8_t* __restrict__ spins,
                                                       int N, float* __restrict__ logq) {
  __shared__ float red[16];
  const int b = blockIdx.x;
  const int grp = threadIdx.x >> 4, part = threadIdx.x & 15;
  const float* w0 = theta + head_w;
  const float* w1 = w0 + D;
  const float b0v = theta[head_b], b1v = theta[head_b + 1];
  float acc = 0.f;
  for (int t = grp; t < N; t += 16) {
    const float* x = X + ((int64_t)b * N + t) * D;
    float z0 = 0.f, z1 = 0.f;
#pragma unroll
    for (int i = 0; i < D / 16; ++i) {
      const int k = part + 16 * i;
      z0 += x[k] * w0[k];
      z1 += x[k] * w1[k];
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) { z0 += __shfl_xor(z0, o, 16); z1 += __shfl_xor(z1, o, 16); }
    const float d = (z1 + b1v) - (z0 + b0v);
    const int s = spins[(int64_t)b * N + t] > 0;
    acc += s ? -softplus(-d) : -softplus(d);
  }
  if (part == 0) red[grp] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tot = 0.f;
    for (int i = 0; i < 16; ++i) tot += red[i];
    logq[b] = tot;
  }
}

// ---------------------------------------------------------------- patch tokens
// Embedding of a token sequence: position t is fed tok_{t-1} (start token 0 at
// t = 0).  A token >= vocab is clamped for the table read (its sample's ln q is
// NaN, set by the head below), so no read leaves the token table.
__global__ void embed_tokens_kernel(const float* __restrict__ theta, int64_t pos_off, int dt, int D, int N, int V,
                                    const uint8_t* __restrict__ tokens, int64_t rows, float* __restrict__ X) {
  const int64_t total = rows * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / D;
    const int k = (int)(i % D);
    const int t = (int)(r % N);
    float v;
    if (k < dt) {
      const int tok = t == 0 ? 0 : min((int)tokens[r - 1], V - 1);
      v = theta[tok * dt + k];
    } else {
      v = theta[pos_off + (int64_t)t * (D - dt) + (k - dt)];
    }
    X[i] = v;
  }
}

// Vocab-way head: one workgroup per sample, thread v computes the logit
// z_v = W_h[v] . h_t + b_v; ln p_t(tok_t) = z_tok - logsumexp(z) (FP32), summed
// over t in order.  Positions go kHeadPos at a time, so every weight a thread
// reads feeds kHeadPos products and the barriers are paid once per group.  A
// token >= vocab gives NaN for its sample.
constexpr int kHeadVocabThreads = 256, kHeadPos = 16;
template <int D>
__global__ __launch_bounds__(kHeadVocabThreads) void head_vocab_kernel(const float* __restrict__ X,
                                                                       const float* __restrict__ theta,
                                                                       int64_t head_w, int64_t head_b, int V,
                                                                       const uint8_t* __restrict__ tokens, int N,
                                                                       float* __restrict__ logq) {
  constexpr int NW = kHeadVocabThreads / 64;
  __shared__ __align__(16) float xs[kHeadPos][D];
  __shared__ float wmax[kHeadPos][NW], wsum[kHeadPos][NW];
  __shared__ float zsel[kHeadPos];
  const int b = blockIdx.x, v = threadIdx.x, lane = v & 63, wave = v >> 6;
  const bool live = v < V;
  const float* wrow = theta + head_w + (int64_t)(live ? v : 0) * D;
  const float bias = live ? theta[head_b + v] : 0.f;
  float acc = 0.f;                                   // used by thread 0
  for (int t0 = 0; t0 < N; t0 += kHeadPos) {
    const int np = min(kHeadPos, N - t0);
    const int64_t r0 = (int64_t)b * N + t0;
    for (int i = v; i < kHeadPos * D; i += kHeadVocabThreads) {
      const int p = i / D, k = i % D;
      xs[p][k] = p < np ? X[(r0 + p) * D + k] : 0.f;
    }
    if (v < kHeadPos) zsel[v] = __builtin_nanf("");
    __syncthreads();
    float z[kHeadPos];
#pragma unroll
    for (int p = 0; p < kHeadPos; ++p) z[p] = -INFINITY;
    if (live) {
      float a[kHeadPos];
#pragma unroll
      for (int p = 0; p < kHeadPos; ++p) a[p] = 0.f;
#pragma unroll 4
      for (int k = 0; k < D; ++k) {                  // the head's offset need not be 16-byte aligned
        const float w = wrow[k];
#pragma unroll
        for (int p = 0; p < kHeadPos; ++p) a[p] += w * xs[p][k];
      }
#pragma unroll
      for (int p = 0; p < kHeadPos; ++p) {
        z[p] = a[p] + bias;
        if (p < np && v == (int)tokens[r0 + p]) zsel[p] = z[p];
      }
    }
#pragma unroll
    for (int p = 0; p < kHeadPos; ++p) {
      float m = z[p];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
      if (lane == 0) wmax[p][wave] = m;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kHeadPos; ++p) {
      float mx = wmax[p][0];
#pragma unroll
      for (int w = 1; w < NW; ++w) mx = fmaxf(mx, wmax[p][w]);
      float e = live ? expf(z[p] - mx) : 0.f;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
      if (lane == 0) wsum[p][wave] = e;
      z[p] = mx;                                     // keep the maximum for the log-sum-exp
    }
    __syncthreads();
    if (v == 0) {
      for (int p = 0; p < np; ++p) {
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) tot += wsum[p][w];
        acc += zsel[p] - (z[p] + logf(tot));
      }
    }
    __syncthreads();                                 // xs, zsel and the partials are rewritten next
  }
  if (v == 0) logq[b] = acc;
}

// ---------------------------------------------------------------- drivers
template <int MODE, int D>
hipError_t forward_layer(fvan_model* m, int l, int64_t rows, int nsamp, hipStream_t s) {
  typedef typename Mode<MODE>::KvT KT;
  const fvan_model_config& c = m->cfg;
  auto& f = m->fw;
  const float* lp = m->params + m->po.layer0 + (int64_t)l * m->po.layer_stride;
  const char* wl = reinterpret_cast<const char*>(m->wpack) + (size_t)l * m->pk.layer_stride;
  const float* X = f.X + (size_t)l * f.rows * D;
  float* Xn = f.X + (size_t)(l + 1) * f.rows * D;
  float* XM = f.XM + (size_t)l * f.rows * D;
  KT* QKV = reinterpret_cast<KT*>(f.QKV) + (size_t)l * f.rows * 3 * D;
  float* LSE = f.LSE + (size_t)l * f.rows * c.n_heads;
  // LN1 is computed inside the QKV projection and LN2 inside the fused FFN
  EpiArgs e{};
  e.bias = lp + m->po.qkv_b;
  e.out = QKV;
  e.ln_x = X;
  e.ln_g = lp + m->po.ln1_g;
  e.ln_b = lp + m->po.ln1_b;
  hipError_t err = gemm_rows<MODE, D, 3 * D, EPI_STORE_KV>(nullptr, rows, wl + m->pk.qkv, e, s);
  if (err != hipSuccess) return err;
  const int H = c.n_heads, dh = D / H;
  const int ggrid = (c.n_spins + kGenRows - 1) / kGenRows * H * nsamp;
  if (dh == 16) {
    const dim3 agrid((c.n_spins + attn_rows(kFwdThreads) - 1) / attn_rows(kFwdThreads) * H * nsamp);
    if constexpr (MODE == FVAN_BF16_SPLIT)
      hipLaunchKernelGGL(attn_fwd_f16, agrid, dim3(kFwdThreads), 0, s, (const _Float16*)QKV, X, XM, LSE, c.n_spins, D,
                         H, c.window, m->kg.P);
    else
      hipLaunchKernelGGL((attn_fwd_mfma<KT, MODE>), agrid, dim3(kFwdThreads), 0, s, (const KT*)QKV, X, XM, LSE,
                         c.n_spins, D, H, c.window, m->kg.P);
  } else if (dh == 32) {
    hipLaunchKernelGGL((attn_fwd_gen<KT, 32>), dim3(ggrid), dim3(kGenThreads), 0, s, (const KT*)QKV, X, XM, LSE,
                       c.n_spins, D, H, c.window, m->kg.P);
  } else {
    if constexpr (D >= 64)
      hipLaunchKernelGGL((attn_fwd_gen<KT, 64>), dim3(ggrid), dim3(kGenThreads), 0, s, (const KT*)QKV, X, XM, LSE,
                         c.n_spins, D, H, c.window, m->kg.P);
  }
  hipLaunchKernelGGL((ffn_fused_kernel<MODE, D>), dim3((int)((rows + kFfnRows - 1) / kFfnRows)), dim3(512), 0, s,
                     (const float*)XM, lp + m->po.ln2_g, lp + m->po.ln2_b, rows,
                     reinterpret_cast<const uint4*>(wl + m->pk.ffn1), reinterpret_cast<const uint4*>(wl + m->pk.ffn2),
                     lp + m->po.ffn1_b, lp + m->po.ffn2_b, (const float*)XM, Xn);
  return hipGetLastError();
}

template <int MODE, int D>
static hipError_t forward_chunk_t(fvan_model* m, const int8_t* spins, int nsamp, float* logq, bool for_backward,
                                  hipStream_t s) {
  const fvan_model_config& c = m->cfg;
  const int64_t rows = (int64_t)nsamp * c.n_spins;
  const int grid = (int)std::min<int64_t>((rows * D + 255) / 256, 65536);
  hipLaunchKernelGGL(embed_kernel, dim3(grid), dim3(256), 0, s, m->params, m->po.pos, c.d_token, D, c.n_spins,
                     spins, rows, m->fw.X);
  for (int l = 0; l < c.n_layers; ++l) {
    hipError_t e = forward_layer<MODE, D>(m, l, rows, nsamp, s);
    if (e != hipSuccess) return e;
  }
  if (logq) {
    hipLaunchKernelGGL((head_fwd_kernel<D>), dim3(nsamp), dim3(256), 0, s,
                       (const float*)(m->fw.X + (size_t)c.n_layers * m->fw.rows * D), m->params, m->po.head_w,
                       m->po.head_b, spins, c.n_spins, logq);
  }
  return hipGetLastError();
}

template <int MODE, int D>
static hipError_t forward_chunk_tokens_t(fvan_model* m, const uint8_t* tokens, int nsamp, float* logq, hipStream_t s) {
  const fvan_model_config& c = m->cfg;
  const int64_t rows = (int64_t)nsamp * c.n_spins;
  const int grid = (int)std::min<int64_t>((rows * D + 255) / 256, 65536);
  hipLaunchKernelGGL(embed_tokens_kernel, dim3(grid), dim3(256), 0, s, m->params, m->po.pos, c.d_token, D, c.n_spins,
                     c.vocab, tokens, rows, m->fw.X);
  for (int l = 0; l < c.n_layers; ++l) {
    hipError_t e = forward_layer<MODE, D>(m, l, rows, nsamp, s);
    if (e != hipSuccess) return e;
  }
  if (logq)
    hipLaunchKernelGGL((head_vocab_kernel<D>), dim3(nsamp), dim3(kHeadVocabThreads), 0, s,
                       (const float*)(m->fw.X + (size_t)c.n_layers * m->fw.rows * D), m->params, m->po.head_w,
                       m->po.head_b, c.vocab, tokens, c.n_spins, logq);
  return hipGetLastError();
}

hipError_t forward_chunk_tokens(fvan_model* m, const uint8_t* tokens, int nsamp, float* logq, hipStream_t s) {
  const int D = m->cfg.d_model;
  if (m->cfg.vocab < 2 || m->cfg.vocab > kHeadVocabThreads) return hipErrorInvalidValue;
#define TOK_CASE(MODE, DD) if (m->cfg.precision == MODE && D == DD) return forward_chunk_tokens_t<MODE, DD>(m, tokens, nsamp, logq, s);
  TOK_CASE(0, 32) TOK_CASE(0, 64) TOK_CASE(0, 128)
  TOK_CASE(2, 32) TOK_CASE(2, 64) TOK_CASE(2, 128)
#undef TOK_CASE
  return hipErrorInvalidValue;
}

hipError_t forward_chunk(fvan_model* m, const int8_t* spins, int nsamp, float* logq, bool for_backward,
                         hipStream_t s) {
  const int D = m->cfg.d_model;
#define FWD_CASE(MODE, DD) if (m->cfg.precision == MODE && D == DD) return forward_chunk_t<MODE, DD>(m, spins, nsamp, logq, for_backward, s);
  FWD_CASE(0, 32) FWD_CASE(0, 64) FWD_CASE(0, 128)
  FWD_CASE(2, 32) FWD_CASE(2, 64) FWD_CASE(2, 128)
#undef FWD_CASE
  return hipErrorInvalidValue;
}

}  // namespace fvan
