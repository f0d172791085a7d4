// Host-side internals of libfvan: the model object, parameter offsets and the
// launchers each kernel source file provides.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fvan.h"

namespace fvan {

// Offsets (in floats) of the tensors inside the flat FP32 parameter vector.
struct ParamOffsets {
  int64_t tok, pos, layer0, layer_stride, head_w, head_b, total;
  // offsets relative to a layer's base
  int64_t ln1_g, ln1_b, qkv_w, qkv_b, ln2_g, ln2_b, ffn1_w, ffn1_b, ffn2_w, ffn2_b;
};
ParamOffsets param_offsets(const fvan_model_config& c);

// Byte offsets of the packed weight copies of one layer inside the pack buffer.
// Forward packs: qkv [3D x D], ffn1 [4D x D], ffn2 [D x 4D];
// backward packs (transposes): qkvT [D x 3D], ffn1T [D x 4D], ffn2T [4D x D].
// A pack of a [rows x K] matrix stores, for tile n (16 rows) and K chunk c, the
// 64 lanes' 16-byte fragments contiguously: lane l holds row 16n + l%16,
// elements c*KC + (l/16)*KC/4 .. +KC/4.  Split packs store all hi fragments,
// then all lo fragments.
struct PackOffsets {
  size_t qkv, ffn1, ffn2, qkvT, ffn1T, ffn2T, layer_stride;
  // models over patch tokens (vocab > 2): the head W_h [vocab x d] padded to vp
  // rows (vp = vocab rounded up to 32, zero rows), and its transpose [d x vp]
  size_t head, headT;
  int vp;
  size_t total;
};
PackOffsets pack_offsets(const fvan_model_config& c);

// Bytes per K/V cache element and per packed weight (FP32, or a split pack's
// BF16 hi and lo).
inline int kv_elem_bytes(int precision) { return precision == FVAN_FP32 ? 4 : 2; }
inline int w_elem_bytes(int) { return 4; }

// KV cache geometry of the sampler: per (sample, layer) [2][S][D], slots
// [0, P) hold prefix positions, [P, P+R) a ring of the last R band positions.
struct KvGeom {
  int32_t P, R, S;
};
inline KvGeom kv_geom(const fvan_model_config& c) {
  KvGeom g;
  g.P = c.prefix < c.n_spins ? c.prefix : c.n_spins;
  int32_t band = c.window + 1;
  int32_t rest = c.n_spins - g.P;
  g.R = band < rest ? band : rest;
  g.S = g.P + g.R;
  return g;
}

// Samples per chunk of the teacher-forced forward / backward.
int64_t fwd_chunk_samples(const fvan_model_config& c);

struct fvan_model_impl;

// Work item table entry of the decode kernel (one per (unit, sample tile) range).
struct DecodeUnit {
  const float* theta;
  const void* wpack;
  void* kv;            // [B][n_layers][2][S][D]
  int8_t* spins;       // [B][N]
  float* logq;         // [B]
  int32_t N, W, P, R, S, B, n_layers, tile0, n_tiles;
  int32_t pos_off;     // offset of pos_emb in theta; tok_emb is at 0
  int64_t layer0, layer_stride, head_w, head_b;
  uint32_t seed_lo, seed_hi, stream_lo, stream_hi;
  // per-layer relative offsets
  int32_t o_ln1_g, o_ln1_b, o_qkv_b, o_ln2_g, o_ln2_b, o_ffn1_b, o_ffn2_b;
  int64_t p_qkv, p_ffn1, p_ffn2, p_layer_stride;   // pack byte offsets
  int32_t d_token;
  int32_t vocab;       // 2: spins; > 2: patch tokens (uint8 written to `spins`)
};

// Which decode kernel a model needs.
struct DecodeShape {
  int d_model, precision, d_head;
  bool tokens;         // vocab-way head and token draw
  int tile;            // samples per workgroup: 32, or 16 where decode_has_tile16
};
inline DecodeShape decode_shape(const fvan_model_config& c, int tile = 32) {
  return DecodeShape{c.d_model, c.precision, c.d_model / c.n_heads, c.vocab > 2, tile};
}
// Whether the decode kernel of this shape exists with 16-sample tiles.
bool decode_has_tile16(const DecodeShape& sh);

// Messages of the entry points a model's configuration does not provide.
constexpr const char* kBinaryOnly =
    "a model over patch tokens (vocab > 2) takes the token calls (fvan_sample_tokens, fvan_log_prob_tokens, "
    "fvan_log_prob_tokens_backward, fvan_train_step_tokens)";
constexpr const char* kNoSampler = "the model was created without FVAN_WS_SAMPLER (no KV cache)";
constexpr const char* kNoTeacher = "the model was created without FVAN_WS_TEACHER (no teacher-forced workspace)";
constexpr const char* kNoTrain = "a training step needs FVAN_WS_SAMPLER | FVAN_WS_TEACHER";

// ----- error slot -----
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
#define FVAN_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::fvan::fail(FVAN_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ----- launchers (return hipError_t of the launch) -----
hipError_t launch_decode(const DecodeShape& sh, const DecodeUnit* units_dev, int n_units, int total_tiles,
                         int* queue_counter, int grid, hipStream_t s);
int decode_tile_samples();

hipError_t launch_energy(const fvan_couplings& c, int32_t batch, const int8_t* spins, void* energy,
                         hipStream_t s);
hipError_t launch_free_energy(int32_t batch, int32_t n, double beta, int is_int, const void* energy,
                              const float* logq, double* stats, hipStream_t s);
hipError_t launch_reinforce(int32_t batch, double beta, int is_int, const void* energy, const float* logq,
                            float* weights, double* Lmean_out, hipStream_t s, double wlik = 0.0);
hipError_t launch_overlap(int32_t batch, int32_t n, const int8_t* spins, unsigned long long* counts, hipStream_t s);
hipError_t launch_lmc(int32_t n, int32_t degree, const int32_t* nbr, const float* J, const int8_t* colour,
                      int32_t batch, double beta, int32_t sweeps, uint64_t seed, uint32_t stream_tag, int8_t* spins,
                      int32_t* accepted, hipStream_t s);
hipError_t launch_pack(const fvan_model_config& c, const float* theta, void* wpack, hipStream_t s);
hipError_t launch_adam(float* theta, float* grads, float* m, float* v, int64_t n, const fvan_adam& o,
                       int64_t step, hipStream_t s);
// Host checks of optimiser hyper-parameters: NULL when valid, else the reason.
inline const char* check_adam(const fvan_adam& o) {
  const bool ok = o.lr >= 0.f && o.beta1 >= 0.f && o.beta1 < 1.f && o.beta2 >= 0.f && o.beta2 < 1.f && o.eps > 0.f &&
                  std::isfinite(o.lr) && std::isfinite(o.eps) && std::isfinite(o.weight_decay);
  return ok ? nullptr : "Adam hyper-parameters out of range";
}
inline const char* check_muon(const fvan_muon& o) {
  const bool ok = o.lr >= 0.f && std::isfinite(o.lr) && o.momentum >= 0.f && o.momentum < 1.f &&
                  o.weight_decay >= 0.f && std::isfinite(o.weight_decay) && o.rms_scale >= 0.f &&
                  std::isfinite(o.rms_scale) && o.ns_eps > 0.f && std::isfinite(o.ns_eps) && o.ns_steps >= 0 &&
                  o.ns_steps <= 16;
  if (!ok) return "Muon hyper-parameters out of range";
  return check_adam(o.adam);
}

hipError_t launch_newton_schulz(const float* M, float* O, int rows, int cols, int steps, float eps, hipStream_t s);
hipError_t launch_muon(const fvan_model_config& c, float* theta, float* grads, float* m, float* v, int64_t n,
                       const fvan_muon& o, int64_t step, hipStream_t s);
hipError_t launch_grad_norm(const float* g, int64_t n, double* out, double* scratch, hipStream_t s);
hipError_t launch_mean_energy(int32_t batch, int32_t n, int is_int, const void* energy, double* out,
                              hipStream_t s);
hipError_t launch_zero_int(int* p, int n, hipStream_t s);
hipError_t launch_tokens_to_spins(int32_t T, int32_t bits, const int32_t* sites, int32_t n, int32_t batch,
                                  const uint8_t* tokens, int8_t* spins, hipStream_t s);
// Bits per patch token of a vocabulary (log2 vocab), 0 when vocab is not a power of two above 2.
inline int token_bits(int vocab) {
  for (int b = 2; b <= 8; ++b)
    if (vocab == (1 << b)) return b;
  return 0;
}

}  // namespace fvan
