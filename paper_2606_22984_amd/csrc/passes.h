// Epilogues of the row GEMM and the entry points of the teacher-forced
// forward / backward passes.
#pragma once

#include "device_common.h"
#include "fvan_model.h"

namespace fvan {

enum {
  EPI_STORE_KV = 0,   // out[r][n] (K/V element type) = acc + bias[n]
  EPI_GELU = 1,       // h = acc + bias[n]; hpre_out[r][n] = h (if set); out[r][n] = GELU(h); outT[n][r] = GELU(h) (if set)
  EPI_RESID = 2,      // out[r][n] (float) = resid[r][n] + acc + bias[n]
  EPI_DGELU = 3,      // d = acc * GELU'(hpre_in[r][n]); out[r][n] = d; outT[n][r] = d (if set)
  EPI_F32 = 4         // out[r][n] (float) = acc
};

struct EpiArgs {
  const float* bias = nullptr;
  const float* resid = nullptr;
  float* hpre_out = nullptr;
  const float* hpre_in = nullptr;
  void* out = nullptr;
  void* outT = nullptr;
  int64_t ldT = 0;
  // staged GEMM: when ln_x is set the A rows are LayerNorm(ln_x rows; ln_g, ln_b),
  // computed in the kernel, and the A argument is not read
  const float* ln_x = nullptr;
  const float* ln_g = nullptr;
  const float* ln_b = nullptr;
};

template <int MODE, int EPI> struct Epi;
template <int MODE> struct Epi<MODE, EPI_STORE_KV> {
  static __device__ __forceinline__ void apply(const EpiArgs& e, int64_t r, int n, int nout, float v) {
    typedef typename Mode<MODE>::KvT KT;
    reinterpret_cast<KT*>(e.out)[r * nout + n] = from_f<KT>(v + e.bias[n]);
  }
};
template <int MODE> struct Epi<MODE, EPI_GELU> {
  static __device__ __forceinline__ void apply(const EpiArgs& e, int64_t r, int n, int nout, float v) {
    typedef typename Mode<MODE>::ActT AT;
    const float h = v + e.bias[n];
    if (e.hpre_out) e.hpre_out[r * nout + n] = h;
    const float g = gelu(h);
    if (e.out) reinterpret_cast<AT*>(e.out)[r * nout + n] = from_f<AT>(g);
    if (e.outT) reinterpret_cast<AT*>(e.outT)[(int64_t)n * e.ldT + r] = from_f<AT>(g);
  }
};
template <int MODE> struct Epi<MODE, EPI_RESID> {
  static __device__ __forceinline__ void apply(const EpiArgs& e, int64_t r, int n, int nout, float v) {
    reinterpret_cast<float*>(e.out)[r * nout + n] = e.resid[r * nout + n] + v + e.bias[n];
  }
};
template <int MODE> struct Epi<MODE, EPI_DGELU> {
  static __device__ __forceinline__ void apply(const EpiArgs& e, int64_t r, int n, int nout, float v) {
    typedef typename Mode<MODE>::ActT AT;
    const float d = v * gelu_grad(e.hpre_in[r * nout + n]);
    reinterpret_cast<AT*>(e.out)[r * nout + n] = from_f<AT>(d);
    if (e.outT) reinterpret_cast<AT*>(e.outT)[(int64_t)n * e.ldT + r] = from_f<AT>(d);
  }
};
template <int MODE> struct Epi<MODE, EPI_F32> {
  static __device__ __forceinline__ void apply(const EpiArgs& e, int64_t r, int n, int nout, float v) {
    reinterpret_cast<float*>(e.out)[r * nout + n] = v;
  }
};

// Teacher-forced forward of one chunk of samples (rows = nsamp * N).  Saves, per
// layer, the input X, Q/K/V, the post-attention residual XM and the attention
// log-sum-exp (what the backward pass reads; attention probabilities are never
// stored).
// logq (may be NULL): per-sample ln q.
hipError_t forward_chunk(fvan_model* m, const int8_t* spins, int nsamp, float* logq, bool for_backward,
                         hipStream_t s);
// The same forward for a model over patch tokens (vocab >= 2): tokens [nsamp, N]
// in [0, vocab), a vocab-way head; logq: per-sample ln q (NULL: the head is not
// evaluated, as before a backward pass).
hipError_t forward_chunk_tokens(fvan_model* m, const uint8_t* tokens, int nsamp, float* logq, hipStream_t s);
// grads += sum_b w[b] d ln q_b / d theta for one chunk (recomputes the forward).
hipError_t backward_chunk(fvan_model* m, const int8_t* spins, int nsamp, const float* w, hipStream_t s);
// The same for a model over patch tokens (uint8 [nsamp, N]); needs vocab <= 16
// or d_model >= 64 (the head's dz is staged in a [4 d_model]-row buffer).
hipError_t backward_chunk_tokens(fvan_model* m, const uint8_t* tokens, int nsamp, const float* w, hipStream_t s);
// Enqueue a check of n floats / doubles: the model's non-finite flag is set if
// any is NaN or Inf.
hipError_t check_finite(fvan_model* m, const float* v, int64_t n, hipStream_t s);
hipError_t check_finite(fvan_model* m, const double* v, int64_t n, hipStream_t s);

}  // namespace fvan
