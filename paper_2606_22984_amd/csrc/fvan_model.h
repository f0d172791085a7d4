// The model object behind the opaque fvan_model handle.
#pragma once

#include "fvan_internal.h"


struct fvan_model {
  fvan_model_config cfg{};
  fvan::ParamOffsets po{};
  fvan::PackOffsets pk{};
  fvan::KvGeom kg{};
  int64_t n_params = 0;
  int device = 0;
  float* params = nullptr;   // caller-owned FP32 [n_params]
  float* grads = nullptr;    // caller-owned FP32 [n_params] (may be NULL)
  bool synced = false;

  // library-owned device workspaces
  void* wpack = nullptr;        // packed weight copies (precision-specific)
  int* nf_flag = nullptr;       // device: set to nonzero by a kernel that finds a non-finite result
  int* nf_host = nullptr;       // pinned host copy of nf_flag taken at the end of a training step
  hipEvent_t nf_event = nullptr;  // recorded after that copy
  bool nf_pending = false;      // a training step's copy is in flight
  void* kv = nullptr;           // sampler KV cache [max_batch][n_layers][2][S][D]
  size_t kv_bytes = 0;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  // train-step buffers
  int8_t* ts_spins = nullptr;   // [max_batch, N] (spins, or the tokens of a patch-token model)
  int8_t* ts_lattice = nullptr; // patch-token models: [max_batch, N * log2(vocab)] spins of the sampled tokens
  float* ts_logq = nullptr;     // [max_batch]
  void* ts_energy = nullptr;    // [max_batch] int32 or float
  float* ts_w = nullptr;        // [max_batch] REINFORCE weights
  double* ts_dbl = nullptr;     // small FP64 scratch
  // teacher-forced forward / backward workspace (one chunk of samples)
  struct Fwd {
    int64_t chunk = 0, rows = 0;   // samples per chunk, rows = chunk * N
    float* X = nullptr;            // [(n_layers+1)][rows][D] layer inputs
    float* XM = nullptr;           // [n_layers][rows][D] residual after attention
    float* LSE = nullptr;          // [n_layers][rows][H] log-sum-exp of the scores (base 2)
    float* DELTA = nullptr;        // [rows][H] dO . O per head (backward)
    void* T_c = nullptr;           // [(D+16)][ldT] feature-major LN outputs (+ ones row) for weight gradients
    void* T_d = nullptr;           // [D][ldT] feature-major gradient at a block's output (left operand of dW2)
    int64_t ldT = 0;               // row stride of the feature-major buffers (rows rounded up to 64)
    void* QKV = nullptr;           // [n_layers][rows][3D] (K/V element type)
    // backward
    float* dX = nullptr;           // [rows][D]
    float* dXM = nullptr;          // [rows][D]
    void* dQKV = nullptr;          // [rows][3D]
    void* T_a = nullptr;           // [4D][ldT] feature-major left operands of the weight gradients
    void* T_b = nullptr;           // [(4D+16)][ldT] feature-major GELU outputs (+ ones row)
    void* T_e = nullptr;           // [3D][ldT] feature-major dQKV (left operand of the W_qkv gradient)
    void* T_f = nullptr;           // [(D+16)][ldT] feature-major LN1 outputs (+ ones row) for the W_qkv gradient
    float* part = nullptr;         // split-K partial sums
    float* part2 = nullptr;        // split-K partial sums of the weight gradients on the side stream
    size_t part_floats = 0;
    // The layer weight gradients run on a stream of the model's own, forked from
    // and joined back to the caller's stream with events, beside the next kernels
    // of the backward: ev[0]/ev[1] = FFN operands ready / read, ev[2]/ev[3] =
    // W_qkv operands ready / read.
    hipStream_t side = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float* colpart = nullptr;      // per-tile partial column sums (LN gains, head, embeddings)
    float* colpart2 = nullptr;     // second-level column sums [64][2D+2]
    size_t colpart_floats = 0;
  } fw;
};

namespace fvan {
// Allocate and initialise every workspace cfg.workspaces asks for (synchronous).
int model_allocate(fvan_model* m);
inline bool has_sampler(const fvan_model* m) { return (m->cfg.workspaces & FVAN_WS_SAMPLER) != 0; }
inline bool has_teacher(const fvan_model* m) { return (m->cfg.workspaces & FVAN_WS_TEACHER) != 0; }
void model_free(fvan_model* m);
void model_free_fwd(fvan_model* m);
// tile: samples per decode workgroup (16 or 32; DecodeShape::tile of the launch).
DecodeUnit make_decode_unit(const fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, int8_t* spins,
                            float* log_q, void* kv, int tile0, int tile);
int device_cus(int dev);
int sample_tile(const fvan_model* m, DecodeShape sh, int32_t batch);
// Resolve (once per device; `dev` must be current) the device address of the
// static KV cache fvan_sample_noalloc uses.
int static_kv_setup(int dev);
hipError_t launch_decode_single(const DecodeShape& sh, const DecodeUnit& u, int tiles, hipStream_t s);
}  // namespace fvan
