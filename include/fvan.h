/*
 * fvan.h -- C ABI of the FlashVAN hot path for AMD Instinct MI355X (gfx950).
 *
 * The method ("Scalable Physics-Inspired Transformers for Spin Glasses"):
 * an autoregressive transformer q_theta(sigma) = prod_t q(sigma_t | sigma_<t)
 * (Eq. 1, Eq. 11) over Ising spins, with concatenated token/position
 * embeddings (Eq. 15), decoder blocks whose masked attention has no output
 * projection (Eqs. 2-3, Alg. 1), a sparse attention mask derived from the
 * interaction graph (Methods, ordered Markov boundary; SI Eq. S1), KV-cached
 * ancestral sampling (Alg. 2), the spin energy (Eq. 6, Eq. 8), the variational
 * free energy F_q (Eq. 5) and its REINFORCE gradient (Eqs. 16-19).
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE memory unless the argument name starts with host_.
 *    The caller owns every input/output buffer and the FP32 parameter and
 *    gradient vectors; the library owns its workspaces (KV cache, activations
 *    of the teacher-forced passes, packed weight copies, optimiser state),
 *    allocated and initialised by fvan_create_model from max_batch and freed
 *    by fvan_destroy_model.  No other call allocates device memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously on it; the backward (fvan_log_prob_backward, the token
 *    backward and the training steps) also runs the layer weight gradients on a
 *    stream the model owns, forked from `stream` and joined back to it with
 *    events within each chunk of samples, so every kernel of a call is ordered
 *    after the work already on `stream` and before the work enqueued on it
 *    afterwards (under stream capture: one fork and join per chunk).  Argument
 *    checks happen on the host, synchronously, before anything is enqueued.  A
 *    call that fails its checks enqueues nothing.  Only fvan_model_status and
 *    the training steps (which wait for the previous training step of their
 *    model, see fvan_train_step) synchronise with the device.
 *  - Every call returns an fvan_status.  On failure fvan_last_error() returns
 *    a thread-local message.  No C++ exception crosses the ABI.
 *  - Non-finite values: the model calls (sampling, log q, backward, training
 *    steps) check their results on the device (ln q, the gradient vector, the
 *    step statistics) and set a per-model flag on a NaN or Inf; the flag is
 *    reported as FVAN_ENONFINITE by the next synchronising call on that model.
 *  - One model is used by one stream at a time; calls on one model must not
 *    overlap (they share its workspaces).
 *  - Spins are int8 +1/-1, row-major [batch, n_spins] (sample-major).  Token
 *    s = (sigma + 1) / 2; head output index 1 is sigma = +1.
 *
 * Flat FP32 parameter layout (row-major tensors concatenated in this order):
 *   tok_emb [vocab, d_token]   row s = embedding of token s; row 0 is also the start token
 *   pos_emb [n_spins, d_pos]   d_pos = d_model - d_token
 *   per layer: ln1.g [d], ln1.b [d], qkv.w [3d, d], qkv.b [3d], ln2.g [d], ln2.b [d],
 *              ffn1.w [4d, d], ffn1.b [4d], ffn2.w [d, 4d], ffn2.b [d]
 *              (qkv rows: Q, then K, then V; head h owns rows h*d_h .. h*d_h+d_h-1 of each,
 *              d_h = d_model / n_heads)
 *   head.w [vocab, d], head.b [vocab]
 * Count: n_layers (11 d^2 + 12 d) + n_spins d_pos + vocab d_token + vocab (d + 1).
 *
 * Network (per position t, tok_0 = start, tok_t = s_{t-1}):
 *   h = [tok_emb[tok_t]; pos_emb[t]]
 *   per layer: h += concat_heads(softmax_j(q_t.k_j / sqrt(d_h)) v_j)  with q,k,v = qkv.w LN1(h) + qkv.b
 *              h += ffn2.w GELU(ffn1.w LN2(h) + ffn1.b) + ffn2.b
 *   z_t = head.w h + head.b ;  log p_t(s) = z_{t,s} - logsumexp(z_t)
 * LayerNorm: affine, population variance, eps 1e-5.  GELU: x Phi(x) (erf form).
 * Mask: key position j is visible from query t iff j <= t and
 *       (t - j <= window or j < prefix).
 */
#ifndef FVAN_H
#define FVAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FVAN_OK = 0,
  FVAN_EINVAL = -1,        /* bad argument: null pointer, size out of range, mismatch */
  FVAN_ENOMEM = -2,        /* workspace allocation failed at create time */
  FVAN_EDEVICE = -3,       /* a HIP runtime call failed (message names it) */
  FVAN_ENONFINITE = -4,    /* a kernel of this model produced a NaN or Inf (ln q, energy, gradient
                              or step statistics) since the last synchronising call */
  FVAN_EUNSUPPORTED = -5   /* valid request this library does not implement */
} fvan_status;

/* Arithmetic of a model's kernels.  Every mode accumulates in FP32, keeps the
 * residual stream, LayerNorm statistics, logits, log-softmax and log q in FP32,
 * and leaves the batch reductions (F_q, variance, baseline) to FP64.
 *   FVAN_FP32        FP32 MFMA GEMMs, FP32 K/V cache: the plain path.
 *   FVAN_BF16_SPLIT  BF16 MFMA GEMMs on split operands (x = hi + lo, both BF16;
 *                    three MFMAs per step: FP32-level GEMM accuracy), FP16 K/V
 *                    cache and attention operands (the paper runs attention in
 *                    FP16, SI Sec. II A): half the K/V bytes of FVAN_FP32.
 * Value 1 is not a mode: GEMM operands rounded to plain BF16 bias ln q by about
 * 1e-3 per site at the 3D EA L=10 workload, ten times the free-energy
 * tolerance (|dF_q / N| <= 1e-4) this library is held to. */
typedef enum { FVAN_FP32 = 0, FVAN_BF16_SPLIT = 2 } fvan_precision;

/* Workspaces fvan_create_model allocates (bit set). */
enum {
  FVAN_WS_SAMPLER = 1,     /* KV cache of fvan_sample (and of group launches) */
  FVAN_WS_TEACHER = 2      /* activations of the teacher-forced passes: fvan_log_prob, fvan_log_prob_tokens,
                              fvan_log_prob_backward and the training steps */
};

typedef enum {
  FVAN_BONDS_PM1 = 0,      /* ELL, int8 J in {-1, 0, +1}; energy int32, exact */
  FVAN_BONDS_F32 = 1,      /* ELL, float J; energy float */
  FVAN_BONDS_DENSE = 2     /* dense float J [n, n], symmetric, zero diagonal (SK); energy float */
} fvan_bond_kind;

typedef struct {
  int32_t n_spins;     /* N: sequence length (one site, or one patch token, per position) */
  int32_t d_model;     /* d = d_token + d_pos; 32, 64 or 128 */
  int32_t d_token;     /* token-embedding width (2 for single spins) */
  int32_t n_layers;
  int32_t n_heads;     /* d_h = d_model / n_heads must be 16, 32 or 64 (16: MFMA attention in the
                          teacher-forced passes; 32, 64: FP32 attention kernels) */
  int32_t vocab;       /* 2 (single spins); up to 256 for patch tokens (the token calls) */
  int32_t window;      /* W of the mask, 0 <= W; values >= n_spins-1 mean full causal */
  int32_t prefix;      /* P of the mask, 0 <= P <= n_spins */
  int32_t max_batch;   /* largest batch any call on this model will pass */
  int32_t precision;   /* fvan_precision */
  int32_t workspaces;  /* FVAN_WS_* bits; a call whose workspace was not requested returns EUNSUPPORTED.
                          The training steps need both. */
} fvan_model_config;

typedef struct {
  int32_t n_spins;
  int32_t kind;        /* fvan_bond_kind */
  int32_t degree;      /* ELL slots per site (ignored for FVAN_BONDS_DENSE) */
  const int32_t* nbr;  /* device int32 [n_spins, degree]: partner j of the pair (i, j) stored in
                          row i; each unordered pair appears in exactly one row; -1 = empty slot */
  const void* J;       /* device: int8 [n_spins, degree] | float [n_spins, degree] | float [n_spins, n_spins] */
} fvan_couplings;

typedef struct {
  float lr, beta1, beta2, eps, weight_decay;
} fvan_adam;

/* Neighbour graph for local Monte Carlo refinement: every neighbour of a site
 * (both directions of each pair, unlike fvan_couplings), -1 for an empty slot,
 * and a 2-colouring of the sites. */
typedef struct {
  int32_t degree;          /* slots per site, >= 1 */
  const int32_t* nbr;      /* device int32 [n_spins, degree] */
  const float* J;          /* device float [n_spins, degree]: bond of each slot (+-1.0 for +-J bonds) */
  const int8_t* colour;    /* device int8 [n_spins], 0 or 1; a proper colouring (no bond inside a colour)
                              makes every half-sweep exact sequential single-site Metropolis */
  int32_t sweeps;          /* checkerboard sweeps, >= 0 */
} fvan_lmc;

/* Muon (Methods, comparison of optimisers: momentum M, Newton-Schulz
 * orthogonalisation O of M, step W -= eta (s O + lambda W), with the weight
 * decay and RMS scale alignment the paper takes from the Muon-at-scale work it
 * cites).  Applies to the per-layer matrices W_qkv, W1, W2; every other
 * parameter takes the Adam step given in `adam`. */
typedef struct {
  float lr;            /* eta >= 0 */
  float momentum;      /* mu in [0, 1): M = mu M + G */
  float weight_decay;  /* lambda >= 0, decoupled: adds lambda W to the step direction */
  float rms_scale;     /* >= 0; s = rms_scale * sqrt(max(rows, cols)); 0.2 aligns the update RMS with Adam's */
  float ns_eps;        /* > 0, added to ||M||_F before the first iteration */
  int32_t ns_steps;    /* Newton-Schulz iterations, 0..16 (5 in the published method) */
  fvan_adam adam;      /* embeddings, head, biases, LayerNorm gains and shifts */
} fvan_muon;

typedef struct fvan_model fvan_model;
typedef struct fvan_group fvan_group;

/* Number of FP32 parameters of a configuration (host only; the count formula
 * above, which reproduces the counts the paper prints in SI Secs. III-IV). */
int fvan_num_params(const fvan_model_config* cfg, int64_t* n_params);

/* Attention mask from the interaction graph (host only).  Sites are ordered by
 * index (raster scan).  Computes the ordered Markov boundary of every site
 * (Methods: past sites adjacent to i or joined to i through future sites) and
 * returns the (window, prefix) pair minimising window + prefix among those
 * that keep every boundary site visible, where site j reaches the query that
 * predicts site i iff position j+1 is visible from position i and the window
 * is counted in sites (SI Eq. S1: A_ij = 0 for i - j > W, W >= d_max).
 * host_i/host_j: the n_edges pairs, each unordered pair once.  EINVAL on an
 * index outside [0, n_spins). */
int fvan_derive_mask(int32_t n_spins, int64_t n_edges, const int32_t* host_i, const int32_t* host_j,
                     int32_t* window, int32_t* prefix);

/* Create a model on the current HIP device, allocate the workspaces
 * cfg->workspaces asks for, sized for cfg->max_batch samples, and initialise
 * them (synchronously: this call waits for its own device work).  The
 * teacher-forced workspace holds one chunk of about 2^21 positions
 * (min(max_batch, 2^21 / n_spins) samples); longer batches run chunk by chunk.
 * EINVAL on a bad shape, EUNSUPPORTED on a shape the kernels do not cover,
 * ENOMEM when the workspaces do not fit. */
int fvan_create_model(const fvan_model_config* cfg, fvan_model** out);
int fvan_destroy_model(fvan_model* model);

/* Attach the caller's FP32 parameter vector [n_params] and gradient vector
 * [n_params] (grads may be NULL if no backward is run).  The library reads
 * params, writes params only in the optimiser steps (fvan_adam_step, fvan_muon_step
 * and the train steps), and
 * accumulates into grads.  Call fvan_sync_params after the caller changes params. */
int fvan_bind_params(fvan_model* model, float* params, float* grads);

/* Rebuild the packed weight copies (FP32 or BF16 by the model's precision,
 * round-to-nearest-even) from the bound FP32 parameters. */
int fvan_sync_params(fvan_model* model, void* stream);

/* Ancestral sampling with a KV cache (Alg. 2): for t = 0..N-1 every layer
 * computes only q_t, k_t, v_t, appends k_t, v_t to its cache and attends over
 * the visible cached keys including position t; the head gives
 * p = p_t(sigma_t = +1) and sigma_t = +1 iff u(b, t) < p, with
 *   u(b, t) = (word[t & 3] >> 8) * 2^-24 of Philox4x32-10,
 *   key = (seed mod 2^32, seed >> 32), counter = (t >> 2, b, stream_id mod 2^32, stream_id >> 32).
 * Outputs spins [batch, N] and log_q [batch] = sum_t log p_t(sigma_t) (FP32).
 * EINVAL if batch is not in [1, max_batch]. */
int fvan_sample(fvan_model* model, int32_t batch, uint64_t seed, uint64_t stream_id,
                int8_t* spins, float* log_q, void* stream);

/* Teacher-forced ln q(sigma) (Alg. 1), FP32 [batch]. */
int fvan_log_prob(fvan_model* model, int32_t batch, const int8_t* spins, float* log_q, void* stream);

/* Teacher-forced ln q of token sequences for a model over 2^D-spin patches
 * (Methods, model configurations and training settings: each 2^D block of the
 * lattice is one token, vocabulary 2^(2^D), sequence (L/2)^D).  tokens: device
 * uint8 [batch, n_spins] (row-major, caller-owned), values in [0, vocab); the
 * token fed at position t is tokens[t-1] (token 0 at t = 0) and the head has
 * vocab outputs: ln q = sum_t (z_t[tok_t] - logsumexp(z_t)), FP32 [batch].  The
 * spin-to-token map is the caller's: patches in raster order of their
 * coordinates, the site at offset o in {0,1}^D giving bit sum_k o_k 2^(D-1-k),
 * bit value (sigma + 1) / 2.  Any vocab in [2, 256]; with vocab 2 and
 * tokens (sigma + 1) / 2 it equals fvan_log_prob up to FP32 rounding.  A token
 * >= vocab makes its sample's ln q NaN (no read leaves the parameter vector).
 * EINVAL for NULL pointers, unsynced parameters or batch outside [1, max_batch].
 * A model with vocab > 2 takes the token calls (this one, fvan_sample_tokens,
 * fvan_log_prob_tokens_backward, fvan_train_step_tokens) and the optimiser
 * steps; the spin calls (fvan_sample, fvan_log_prob, fvan_log_prob_backward,
 * the spin training steps, groups) return EUNSUPPORTED for it. */
int fvan_log_prob_tokens(fvan_model* model, int32_t batch, const uint8_t* tokens, float* log_q, void* stream);

/* Ancestral sampling of token sequences (Alg. 2 over 2^D-spin patch tokens,
 * Methods, model configurations and training settings): at position t the
 * head gives z_t (vocab outputs, FP32) and p_t = softmax(z_t); with one uniform
 * u(b, t) per position, drawn exactly as in fvan_sample, the token is the
 * largest k >= 1 with u < sum_{j >= k} p_t(j), else 0 (the vocabulary walked
 * from the top; for vocab 2 this is fvan_sample's rule with token (sigma+1)/2),
 * and it is fed to the token embedding of position t + 1.  Outputs tokens
 * uint8 [batch, n_spins] and log_q [batch] = sum_t ln p_t(tok_t) (FP32).  Any
 * vocab in [2, 256].  EINVAL if batch is not in [1, max_batch]. */
int fvan_sample_tokens(fvan_model* model, int32_t batch, uint64_t seed, uint64_t stream_id, uint8_t* tokens,
                       float* log_q, void* stream);

/* grads += sum_b grad_log_q[b] * d ln q(tok_b) / d theta for token sequences
 * (the backward of fvan_log_prob_tokens; the forward is recomputed).
 * EUNSUPPORTED when vocab > 16 with d_model < 64, or vocab * d_token > 16384. */
int fvan_log_prob_tokens_backward(fvan_model* model, int32_t batch, const uint8_t* tokens,
                                  const float* grad_log_q, void* stream);

/* Spins of token sequences (the inverse of the patch map): for every sample b,
 * token t and bit m < bits, spins[b][sites[t * bits + m]] = bit m of
 * tokens[b][t] ? +1 : -1.  sites: device int32 [n_tokens, bits], a permutation
 * of [0, n_spins) (entries outside that range are skipped); spins: device int8
 * [batch, n_spins].  EINVAL unless n_tokens * bits == n_spins, bits in [1, 8]. */
int fvan_tokens_to_spins(int32_t n_tokens, int32_t bits, const int32_t* sites, int32_t n_spins, int32_t batch,
                         const uint8_t* tokens, int8_t* spins, void* stream);

/* One training step of a model over 2^D-spin patch tokens (vocab = 2^bits,
 * bits = 2^D; the sequence is the model's n_spins tokens): sample tokens
 * (seed, stream_id = step) -> spins through `sites` (as fvan_tokens_to_spins)
 * -> energies -> F_q statistics per lattice site (n = n_spins * bits) ->
 * REINFORCE weights -> token backward -> gradient norm -> Muon update.  stats
 * as fvan_train_step.  couplings->n_spins must be n_spins * bits. */
int fvan_train_step_tokens(fvan_model* model, const fvan_couplings* couplings, const int32_t* sites, double beta,
                           int32_t batch, uint64_t seed, uint64_t step, const fvan_muon* opt, double* stats,
                           void* stream);

/* grads += sum_b grad_log_q[b] * d ln q(sigma_b) / d theta.  Recomputes the
 * forward pass (attention included) in chunks of samples; nothing from an
 * earlier call is reused. */
int fvan_log_prob_backward(fvan_model* model, int32_t batch, const int8_t* spins,
                           const float* grad_log_q, void* stream);

/* E_b = - sum over stored pairs of J_ij sigma_i sigma_j (Eq. 6 / Eq. 8; each
 * unordered pair once).  energy: int32 [batch] for FVAN_BONDS_PM1 (exact),
 * float [batch] otherwise. */
int fvan_energy(const fvan_couplings* couplings, int32_t batch, const int8_t* spins, void* energy,
                void* stream);

/* Free-energy estimator (Eq. 5) in FP64 on the device:
 *   f_b = (E_b + log_q_b / beta) / n_spins,
 *   stats[0] = mean_b f_b  (= F_q / N estimate),  stats[1] = sum_b (f_b - mean)^2 / (batch - 1).
 * energy is int32 when energy_is_int, else float.  stats: device double [2].
 * Fixed-order reduction: bitwise reproducible. */
int fvan_free_energy(int32_t batch, int32_t n_spins, double beta, int32_t energy_is_int,
                     const void* energy, const float* log_q, double* stats, void* stream);

/* REINFORCE weights (Eq. 19 with the exact 1/beta scale):
 *   L_b = beta E_b + log_q_b,  Lbar = mean_b L_b (FP64),
 *   weights[b] = (L_b - Lbar) / (beta * batch)  (float)
 * so that sum_b weights[b] grad ln q_b estimates grad F_q. */
int fvan_reinforce_weights(int32_t batch, double beta, int32_t energy_is_int, const void* energy,
                           const float* log_q, float* weights, void* stream);

/* One Adam step on the bound parameters with the bound gradients, then zero
 * the gradients and refresh the packed weights.  step counts from 1. */
int fvan_adam_step(fvan_model* model, const fvan_adam* opt, int64_t step, void* stream);

/* One training step of the paper's procedure (Results: optimisation;
 * Methods: training strategy):
 *   sample batch (seed, stream_id = step) -> energies -> F_q stats ->
 *   REINFORCE weights from the sampled log q -> backward -> Adam.
 * stats: device double [4] = { F_q/N, Var[f], <E>/N, ||grad||_2 }.
 * The model's grads must be bound; they are zeroed by the update.  The model
 * needs both workspaces (FVAN_WS_SAMPLER | FVAN_WS_TEACHER).
 * A training step first waits for the previous training step of the same
 * model to finish and returns FVAN_ENONFINITE, enqueuing nothing, if that
 * step's statistics were not finite (the flag is then cleared); otherwise it
 * enqueues its own work asynchronously, ending with a device copy of its
 * finiteness check for the next call to read. */
int fvan_train_step(fvan_model* model, const fvan_couplings* couplings, double beta, int32_t batch,
                    uint64_t seed, uint64_t step, const fvan_adam* opt, double* stats, void* stream);

/* Newton-Schulz orthogonalisation used by Muon (Methods, comparison of
 * optimisers; quintic iteration published with the Muon optimiser the paper
 * cites, coefficients (a, b, c) = (3.4445, -4.7750, 2.0315)):
 *   X_0 = M / (||M||_F + eps);  a wide X (rows <= cols) is iterated as
 *   X <- a X + (b A + c A^2) X with A = X X^T, a tall one as its transpose;
 *   O = X after `steps` iterations.
 * M, O: FP32 row-major [rows, cols]; O may be M (in place).  FP32 MFMA
 * products with FP32 accumulation, one workgroup.  EINVAL if rows or cols < 1,
 * min(rows, cols) > 128, rows * cols >= 2^31, steps outside 0..16, or eps not
 * finite and > 0. */
int fvan_newton_schulz(int32_t rows, int32_t cols, int32_t steps, float eps, const float* M, float* O,
                       void* stream);

/* One Muon step on the bound parameters with the bound gradients (fvan_muon),
 * then zero the gradients and refresh the packed weights.  step counts from 1
 * (Adam bias correction of the non-matrix parameters).  Optimiser state: the
 * momentum of the matrices shares the storage of Adam's first moment, so
 * switching between fvan_adam_step and fvan_muon_step carries it over as is. */
int fvan_muon_step(fvan_model* model, const fvan_muon* opt, int64_t step, void* stream);

/* Local Monte Carlo refinement (Results, 3D EA; Methods, training strategy;
 * SI Sec. I C): lmc->sweeps checkerboard Metropolis sweeps at inverse
 * temperature beta on each configuration of spins [batch, n_spins], in place.
 * A sweep updates the sites of colour 0, then those of colour 1; within a
 * half-sweep every local field h_i = sum_j J_ij s_j comes from the
 * configuration at its start.  Flipping s_i changes E (Eq. 8) by
 * dE = 2 s_i h_i; the flip is accepted iff u < exp(-beta dE) (FP32), with
 *   u(b, k, i) = (word[i & 3] >> 8) * 2^-24 of Philox4x32-10,
 *   key = (seed mod 2^32, seed >> 32), counter = (i >> 2, b, k, stream_tag).
 * accepted: device int32 [batch] accepted flips per configuration, or NULL.
 * EINVAL on NULL graph arrays, n_spins outside [1, 16384], degree < 1,
 * sweeps < 0, batch < 1, or beta not finite and >= 0. */
int fvan_lmc_refine(int32_t n_spins, const fvan_lmc* lmc, int32_t batch, double beta, uint64_t seed,
                    uint32_t stream_tag, int8_t* spins, int32_t* accepted, void* stream);

/* Weights of the self-distillation gradient, Eq. (loss2), on M = batch
 * (refined) configurations with their energies and teacher-forced log q:
 *   L_m = beta E_m + log_q_m,  Lbar = mean_m L_m (FP64),
 *   weights[m] = ((L_m - Lbar) - w) / (beta M),
 * i.e. Eq. (loss2)'s (1/M) sum_m ((L - Lbar) - w) grad ln q_m with the 1/beta
 * of the exact F_q gradient (Eq. 18) as its proportionality constant, applied
 * to both terms; w = 0 gives fvan_reinforce_weights. */
int fvan_distill_weights(int32_t batch, double beta, double w, int32_t energy_is_int, const void* energy,
                         const float* log_q, float* weights, void* stream);

/* fvan_train_step with the Muon update (the paper's default optimiser) in
 * place of Adam; same stats. */
int fvan_train_step_muon(fvan_model* model, const fvan_couplings* couplings, double beta, int32_t batch,
                         uint64_t seed, uint64_t step, const fvan_muon* opt, double* stats, void* stream);

/* Overlap distribution (Eq. overlap_distribution): every pair a < b of the
 * batch is a pair of independent replicas;
 *   counts[k] = #{a < b : sum_i s_a,i s_b,i = 2k - n_spins},  k = 0..n_spins,
 * i.e. the pairs with overlap q = 2k / n_spins - 1.  spins: device int8 +-1
 * [batch, n_spins] (pairs whose product falls outside [-n_spins, n_spins],
 * possible only for entries other than +-1, are not counted); counts: device
 * uint64 [n_spins + 1], overwritten.  Exact (integer MFMA products).  EINVAL on
 * NULL, batch outside [1, 2^20] or n_spins outside [1, 16000]. */
int fvan_overlap_histogram(int32_t batch, int32_t n_spins, const int8_t* spins, uint64_t* counts, void* stream);

/* Annealing schedule (Methods, variational annealing; host only):
 *   T = T0                                                 step <= n_warmup,
 *   T = T0 - (T0 / n_anneal) min(floor((step - n_warmup) / n_eq), n_anneal)  otherwise,
 * reaching 0 at step = n_warmup + n_eq * n_anneal (no finite beta there).
 * EINVAL on T0 not finite and > 0, n_warmup < 0, n_eq < 1 or n_anneal < 1. */
int fvan_anneal_temperature(int64_t step, double T0, int64_t n_warmup, int64_t n_eq, int32_t n_anneal,
                            double* host_T);

/* One training step of the paper's 3D EA procedure (Results, 3D EA; Methods,
 * training strategy): sample (seed, stream_id = step); energies and the F_q
 * statistics of the raw samples (stats as fvan_train_step); refine the samples
 * in place with fvan_lmc_refine (key seed, stream_tag = 2^31 | (step mod 2^31));
 * energies and teacher-forced log q of the refined samples; weights of
 * Eq. (loss2) with likelihood weight w; backward; gradient norm; Muon update.
 * The refined samples stay in the model's sample buffer. */
int fvan_train_step_distill(fvan_model* model, const fvan_couplings* couplings, const fvan_lmc* lmc, double beta,
                            double w, int32_t batch, uint64_t seed, uint64_t step, const fvan_muon* opt,
                            double* stats, void* stream);

/* ---------------------------------------------------------------------------
 * Batched launches: many (instance, temperature, size) units sampled in ONE
 * persistent kernel launch.  All models of a group must share d_model,
 * n_layers, n_heads and precision; n_spins, the mask, the parameters and the
 * couplings may differ per unit.
 * ------------------------------------------------------------------------- */
typedef struct {
  fvan_model* model;                /* parameters bound and synced */
  const fvan_couplings* couplings;  /* copied at group creation */
  double beta;
  int32_t batch;                    /* samples of this unit, <= model max_batch */
  uint64_t seed, stream_id;
  int8_t* spins;                    /* device [batch, N] */
  float* log_q;                     /* device [batch] */
  void* energy;                     /* device [batch], int32 or float as fvan_energy */
  double* stats;                    /* device [2] as fvan_free_energy */
} fvan_group_unit;

/* Build the device unit table and choose the launch shape (many instances,
 * sizes and temperatures in one persistent launch).  tile_samples: samples
 * per work item and decode workgroup, 16 or 32, or 0 to let the autotuner
 * choose it.  The autotuner searches the tile and the persistent grid size
 * (1, 2 and 4 workgroups per compute unit, and the grid whose samples in
 * flight keep their K/V caches within the 256 MB MALL), timing each candidate
 * on the same prefix of the work queue, and keeps the fastest per sample.  The
 * choice is persisted per launch shape (model shape, precision, compute units,
 * the units' sizes, masks and batches) in the JSON file named by
 * $FVAN_TUNE_FILE (default $HOME/.cache/fvan_tuning.json); a later group of the
 * same shape, in any process, takes the stored choice without timing.
 * Creation synchronises the device.  EINVAL when the models disagree in shape;
 * EUNSUPPORTED for a tile of 16 the model's decode kernel does not have. */
int fvan_group_create(const fvan_group_unit* units, int32_t n_units, int32_t tile_samples,
                      fvan_group** out);
/* The launch shape a group runs with: tile (samples per workgroup), grid
 * (persistent workgroups), from_store = 1 when it came from the persisted
 * store (no timing), and ms = the timed prefix of that shape.  Any output
 * pointer may be NULL (host pointers). */
int fvan_group_launch_shape(const fvan_group* group, int32_t* host_tile, int32_t* host_grid,
                            int32_t* host_from_store, double* host_ms);
int fvan_group_destroy(fvan_group* group);
/* Sampling of every unit in one persistent launch (work queue over
 * (unit, sample tile)), followed by the energies and free-energy statistics. */
int fvan_group_run(fvan_group* group, void* stream);
/* Capture fvan_group_run into a HIP graph on `stream` (once) and replay it. */
int fvan_group_run_graph(fvan_group* group, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fvan_sample
 * with its KV cache in a static device array of the library, of
 * FVAN_NOALLOC_KV_BYTES (64 MiB) per GPU, instead of the model's sampler
 * workspace.  fvan_create_model sets the array up on its device (the runtime
 * backs it with device memory then), and the GPU holds it until the process
 * ends.  The model
 * needs no FVAN_WS_SAMPLER.  Same kernel and same outputs (bitwise) as
 * fvan_sample; this call allocates nothing and enqueues only on `stream`.
 * A sample's cache takes n_layers * 2 * S * d_model * e bytes, S = P + min(W + 1,
 * N - P) slots (P = min(prefix, N), W = window) and e = 4 (FVAN_FP32) or 2
 * (FVAN_BF16_SPLIT).  EINVAL (nothing enqueued) when batch times that exceeds
 * FVAN_NOALLOC_KV_BYTES, when the current HIP device is not the model's, or as
 * fvan_sample.  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (nothing in it needs clearing: a sample's keys are
 * written before they are read): calls that overlap in time on one GPU (other
 * streams, threads or models) race on it and must be serialised by the caller. */
#define FVAN_NOALLOC_KV_BYTES ((size_t)64 << 20)
int fvan_sample_noalloc(fvan_model* model, int32_t batch, uint64_t seed, uint64_t stream_id,
                        int8_t* spins, float* log_q, void* stream);

/* Synchronise `stream`, then report and clear the model's non-finite flag:
 * FVAN_ENONFINITE if any kernel of this model found a NaN or Inf in its
 * results since the flag was last reported, else FVAN_OK. */
int fvan_model_status(fvan_model* model, void* stream);

/* Thread-local message describing the last failure on this thread. */
const char* fvan_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FVAN_H */
