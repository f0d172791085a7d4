// Host implementation of the C ABI declared in include/fvan.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "fvan_internal.h"
#include "fvan_model.h"
#include "passes.h"

namespace fvan {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

ParamOffsets param_offsets(const fvan_model_config& c) {
  ParamOffsets o;
  const int64_t d = c.d_model;
  o.tok = 0;
  o.pos = (int64_t)c.vocab * c.d_token;
  o.layer0 = o.pos + (int64_t)c.n_spins * (d - c.d_token);
  o.ln1_g = 0;
  o.ln1_b = d;
  o.qkv_w = 2 * d;
  o.qkv_b = o.qkv_w + 3 * d * d;
  o.ln2_g = o.qkv_b + 3 * d;
  o.ln2_b = o.ln2_g + d;
  o.ffn1_w = o.ln2_b + d;
  o.ffn1_b = o.ffn1_w + 4 * d * d;
  o.ffn2_w = o.ffn1_b + 4 * d;
  o.ffn2_b = o.ffn2_w + 4 * d * d;
  o.layer_stride = o.ffn2_b + d;   // = 11 d^2 + 12 d
  o.head_w = o.layer0 + (int64_t)c.n_layers * o.layer_stride;
  o.head_b = o.head_w + (int64_t)c.vocab * d;
  o.total = o.head_b + c.vocab;
  return o;
}

PackOffsets pack_offsets(const fvan_model_config& c) {
  PackOffsets p;
  const size_t d = c.d_model, e = w_elem_bytes(c.precision);
  p.qkv = 0;
  p.ffn1 = p.qkv + 3 * d * d * e;
  p.ffn2 = p.ffn1 + 4 * d * d * e;
  p.qkvT = p.ffn2 + 4 * d * d * e;
  p.ffn1T = p.qkvT + 3 * d * d * e;
  p.ffn2T = p.ffn1T + 4 * d * d * e;
  p.layer_stride = p.ffn2T + 4 * d * d * e;
  p.head = p.headT = p.total = p.layer_stride * c.n_layers;
  p.vp = 0;
  if (c.vocab > 2) {
    p.vp = (c.vocab + 31) / 32 * 32;
    p.headT = p.head + (size_t)p.vp * d * e;
    p.total = p.headT + d * (size_t)p.vp * e;
  }
  return p;
}

static int check_config(const fvan_model_config* c) {
  if (!c) return fail(FVAN_EINVAL, "config is NULL");
  if (c->n_spins < 1) return fail(FVAN_EINVAL, "n_spins must be >= 1");
  if (c->d_model != 32 && c->d_model != 64 && c->d_model != 128)
    return fail(FVAN_EUNSUPPORTED, "d_model must be 32, 64 or 128");
  if (c->n_heads < 1 || c->d_model % c->n_heads != 0 ||
      (c->d_model / c->n_heads != 16 && c->d_model / c->n_heads != 32 && c->d_model / c->n_heads != 64))
    return fail(FVAN_EUNSUPPORTED, "d_model / n_heads must be 16, 32 or 64");
  if (c->d_token < 1 || c->d_token >= c->d_model) return fail(FVAN_EINVAL, "d_token out of range");
  if (c->vocab < 2 || c->vocab > 256) return fail(FVAN_EUNSUPPORTED, "vocab must be in [2, 256]");
  if (c->n_layers < 0 || c->n_layers > 64) return fail(FVAN_EINVAL, "n_layers out of range");
  if (c->window < 0 || c->prefix < 0 || c->prefix > c->n_spins) return fail(FVAN_EINVAL, "mask out of range");
  if (c->max_batch < 1) return fail(FVAN_EINVAL, "max_batch must be >= 1");
  if (c->precision != FVAN_FP32 && c->precision != FVAN_BF16_SPLIT)
    return fail(FVAN_EINVAL, "unknown precision (FVAN_FP32 = 0 or FVAN_BF16_SPLIT = 2)");
  if (c->workspaces & ~(FVAN_WS_SAMPLER | FVAN_WS_TEACHER)) return fail(FVAN_EINVAL, "unknown workspace bits");
  return FVAN_OK;
}

int64_t fwd_chunk_samples(const fvan_model_config& c) {
  // about 2^21 rows (positions) per chunk of the teacher-forced passes
  int64_t s = std::max<int64_t>(1, (int64_t(1) << 21) / c.n_spins);
  s = std::min<int64_t>(s, c.max_batch);
  return std::min<int64_t>(s, 65535);   // keeps the 1-D attention grids (tiles x heads x samples) in int range
}

static fvan_model_config clamp_mask(fvan_model_config c) {
  if (c.window > c.n_spins - 1) c.window = c.n_spins - 1;
  return c;
}

}  // namespace fvan

using namespace fvan;

extern "C" {

const char* fvan_last_error(void) { return g_err.c_str(); }

int fvan_num_params(const fvan_model_config* cfg, int64_t* n_params) {
  if (!cfg || !n_params) return fail(FVAN_EINVAL, "NULL argument");
  if (cfg->d_model < 1 || cfg->d_token < 0 || cfg->d_token > cfg->d_model || cfg->n_layers < 0 || cfg->vocab < 1 ||
      cfg->n_spins < 1)
    return fail(FVAN_EINVAL, "config out of range");
  *n_params = param_offsets(*cfg).total;
  return FVAN_OK;
}

int fvan_derive_mask(int32_t n, int64_t n_edges, const int32_t* host_i, const int32_t* host_j, int32_t* window,
                     int32_t* prefix) {
  if (n < 1 || n_edges < 0 || !window || !prefix || (n_edges > 0 && (!host_i || !host_j)))
    return fail(FVAN_EINVAL, "bad arguments");
  std::vector<std::vector<int32_t>> adj(n);
  for (int64_t e = 0; e < n_edges; ++e) {
    const int32_t a = host_i[e], b = host_j[e];
    if (a < 0 || a >= n || b < 0 || b >= n) return fail(FVAN_EINVAL, "edge index outside [0, n_spins)");
    if (a == b) continue;
    adj[a].push_back(b);
    adj[b].push_back(a);
  }
  // far[j]: largest i - j over sites i whose ordered Markov boundary contains j.
  std::vector<int32_t> far(n + 1, 0), mark(n, -1);
  std::vector<int32_t> stack;
  for (int32_t i = 0; i < n; ++i) {
    // region reachable from i through future sites; past neighbours of it form the boundary
    stack.clear();
    stack.push_back(i);
    mark[i] = i;
    while (!stack.empty()) {
      const int32_t v = stack.back();
      stack.pop_back();
      for (int32_t w : adj[v]) {
        if (w < i) {
          far[w] = std::max(far[w], i - w);
        } else if (w > i && mark[w] != i) {
          mark[w] = i;
          stack.push_back(w);
        }
      }
    }
  }
  // suffix maxima: W(P) = max_{j >= P-1} far[j]
  std::vector<int32_t> suf(n + 2, 0);
  for (int32_t j = n; j >= 0; --j) suf[j] = std::max(far[j], suf[j + 1]);
  int64_t best = -1;
  int32_t bw = 0, bp = 0;
  for (int32_t P = 0; P <= n; ++P) {
    const int32_t W = suf[std::max(P - 1, 0)];
    const int64_t cost = (int64_t)P + W;
    if (best < 0 || cost < best) {
      best = cost;
      bw = W;
      bp = P;
    }
  }
  *window = bw;
  *prefix = bp;
  return FVAN_OK;
}

int fvan_create_model(const fvan_model_config* cfg, fvan_model** out) {
  if (!out) return fail(FVAN_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_config(cfg);
  if (rc) return rc;
  fvan_model* m = new (std::nothrow) fvan_model();
  if (!m) return fail(FVAN_ENOMEM, "host allocation failed");
  m->cfg = clamp_mask(*cfg);
  rc = model_allocate(m);
  // the static KV cache of fvan_sample_noalloc is resolved here, at set-up on
  // the model's device, so that the sampling call itself never makes the
  // runtime materialise it
  if (!rc) rc = static_kv_setup(m->device);
  if (rc) {
    model_free(m);
    delete m;
    return rc;
  }
  *out = m;
  return FVAN_OK;
}

int fvan_destroy_model(fvan_model* m) {
  if (!m) return fail(FVAN_EINVAL, "model is NULL");
  model_free(m);
  delete m;
  return FVAN_OK;
}

int fvan_bind_params(fvan_model* m, float* params, float* grads) {
  if (!m || !params) return fail(FVAN_EINVAL, "model or params is NULL");
  m->params = params;
  m->grads = grads;
  return FVAN_OK;
}

int fvan_sync_params(fvan_model* m, void* stream) {
  if (!m || !m->params) return fail(FVAN_EINVAL, "model has no bound parameters");
  FVAN_HIP(launch_pack(m->cfg, m->params, m->wpack, (hipStream_t)stream));
  m->synced = true;
  return FVAN_OK;
}

int fvan_sample(fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, int8_t* spins, float* log_q,
                void* stream) {
  if (!m || !spins || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (m->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  if (!has_sampler(m)) return fail(FVAN_EUNSUPPORTED, kNoSampler);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  DecodeShape sh = decode_shape(m->cfg);
  sh.tile = sample_tile(m, sh, batch);
  DecodeUnit u = make_decode_unit(m, batch, seed, stream_id, spins, log_q, m->kv, 0, sh.tile);
  FVAN_HIP(launch_decode_single(sh, u, u.n_tiles, (hipStream_t)stream));
  FVAN_HIP(check_finite(m, log_q, batch, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_sample_tokens(fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, uint8_t* tokens,
                       float* log_q, void* stream) {
  if (!m || !tokens || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (!has_sampler(m)) return fail(FVAN_EUNSUPPORTED, kNoSampler);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  DecodeShape sh = decode_shape(m->cfg);
  sh.tokens = true;
  sh.tile = sample_tile(m, sh, batch);
  DecodeUnit u = make_decode_unit(m, batch, seed, stream_id, reinterpret_cast<int8_t*>(tokens), log_q, m->kv, 0,
                                  sh.tile);
  FVAN_HIP(launch_decode_single(sh, u, u.n_tiles, (hipStream_t)stream));
  FVAN_HIP(check_finite(m, log_q, batch, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_energy(const fvan_couplings* c, int32_t batch, const int8_t* spins, void* energy, void* stream) {
  if (!c || !spins || !energy || !c->J) return fail(FVAN_EINVAL, "NULL argument");
  if (batch < 1 || c->n_spins < 1) return fail(FVAN_EINVAL, "batch and n_spins must be >= 1");
  if (c->kind != FVAN_BONDS_PM1 && c->kind != FVAN_BONDS_F32 && c->kind != FVAN_BONDS_DENSE)
    return fail(FVAN_EINVAL, "unknown bond kind");
  if (c->kind != FVAN_BONDS_DENSE && (!c->nbr || c->degree < 0)) return fail(FVAN_EINVAL, "ELL table missing");
  if (c->kind == FVAN_BONDS_DENSE && c->n_spins > 4096) return fail(FVAN_EUNSUPPORTED, "dense bonds need n <= 4096");
  if (c->kind != FVAN_BONDS_DENSE && c->n_spins > 32768) return fail(FVAN_EUNSUPPORTED, "ELL bonds need n <= 32768");
  FVAN_HIP(launch_energy(*c, batch, spins, energy, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_free_energy(int32_t batch, int32_t n, double beta, int32_t is_int, const void* energy, const float* log_q,
                     double* stats, void* stream) {
  if (!energy || !log_q || !stats) return fail(FVAN_EINVAL, "NULL argument");
  if (batch < 1 || n < 1 || !(beta > 0.0) || !std::isfinite(beta)) return fail(FVAN_EINVAL, "batch, n or beta out of range");
  FVAN_HIP(launch_free_energy(batch, n, beta, is_int != 0, energy, log_q, stats, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_reinforce_weights(int32_t batch, double beta, int32_t is_int, const void* energy, const float* log_q,
                           float* weights, void* stream) {
  if (!energy || !log_q || !weights) return fail(FVAN_EINVAL, "NULL argument");
  if (batch < 1 || !(beta > 0.0) || !std::isfinite(beta)) return fail(FVAN_EINVAL, "batch or beta out of range");
  FVAN_HIP(launch_reinforce(batch, beta, is_int != 0, energy, log_q, weights, nullptr, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_adam_step(fvan_model* m, const fvan_adam* opt, int64_t step, void* stream) {
  if (!m || !opt) return fail(FVAN_EINVAL, "NULL argument");
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (!m->params || !m->grads) return fail(FVAN_EINVAL, "parameters and gradients must be bound");
  if (step < 1) return fail(FVAN_EINVAL, "step counts from 1");
  if (const char* why = check_adam(*opt)) return fail(FVAN_EINVAL, why);
  hipStream_t s = (hipStream_t)stream;
  FVAN_HIP(launch_adam(m->params, m->grads, m->adam_m, m->adam_v, m->n_params, *opt, step, s));
  FVAN_HIP(launch_pack(m->cfg, m->params, m->wpack, s));
  return FVAN_OK;
}

int fvan_lmc_refine(int32_t n, const fvan_lmc* g, int32_t batch, double beta, uint64_t seed, uint32_t tag,
                    int8_t* spins, int32_t* accepted, void* stream) {
  if (!g || !spins) return fail(FVAN_EINVAL, "NULL argument");
  if (!g->nbr || !g->J || !g->colour) return fail(FVAN_EINVAL, "NULL neighbour graph array");
  if (n < 1 || n > 16384) return fail(FVAN_EINVAL, "n_spins must be in [1, 16384] for refinement");
  if (g->degree < 1 || g->sweeps < 0 || batch < 1) return fail(FVAN_EINVAL, "degree, sweeps or batch out of range");
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(FVAN_EINVAL, "beta must be finite and >= 0");
  if (g->sweeps == 0) return FVAN_OK;
  FVAN_HIP(launch_lmc(n, g->degree, g->nbr, g->J, g->colour, batch, beta, g->sweeps, seed, tag, spins, accepted,
                      (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_distill_weights(int32_t batch, double beta, double w, int32_t is_int, const void* energy,
                         const float* log_q, float* weights, void* stream) {
  if (!energy || !log_q || !weights) return fail(FVAN_EINVAL, "NULL argument");
  if (batch < 1 || !(beta > 0.0) || !std::isfinite(beta) || !std::isfinite(w))
    return fail(FVAN_EINVAL, "batch, beta or w out of range");
  FVAN_HIP(launch_reinforce(batch, beta, is_int != 0, energy, log_q, weights, nullptr, (hipStream_t)stream, w));
  return FVAN_OK;
}

int fvan_overlap_histogram(int32_t batch, int32_t n, const int8_t* spins, uint64_t* counts, void* stream) {
  if (!spins || !counts) return fail(FVAN_EINVAL, "NULL argument");
  if (batch < 1 || batch > (1 << 20) || n < 1 || n > 16000)
    return fail(FVAN_EINVAL, "overlap histogram needs batch in [1, 2^20] and n_spins in [1, 16000]");
  FVAN_HIP(launch_overlap(batch, n, spins, reinterpret_cast<unsigned long long*>(counts), (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_anneal_temperature(int64_t step, double T0, int64_t n_warmup, int64_t n_eq, int32_t n_anneal,
                            double* host_T) {
  if (!host_T) return fail(FVAN_EINVAL, "NULL argument");
  if (!(T0 > 0.0) || !std::isfinite(T0) || n_warmup < 0 || n_eq < 1 || n_anneal < 1)
    return fail(FVAN_EINVAL, "annealing schedule parameters out of range");
  if (step <= n_warmup) {
    *host_T = T0;
  } else {
    const int64_t k = std::min<int64_t>((step - n_warmup) / n_eq, n_anneal);
    *host_T = T0 - (T0 / n_anneal) * (double)k;
  }
  return FVAN_OK;
}

int fvan_newton_schulz(int32_t rows, int32_t cols, int32_t steps, float eps, const float* M, float* O,
                       void* stream) {
  if (!M || !O) return fail(FVAN_EINVAL, "NULL argument");
  if (rows < 1 || cols < 1 || std::min(rows, cols) > 128 || (int64_t)rows * cols >= ((int64_t)1 << 31))
    return fail(FVAN_EINVAL, "Newton-Schulz needs 1 <= min(rows, cols) <= 128 and rows * cols < 2^31");
  if (steps < 0 || steps > 16) return fail(FVAN_EINVAL, "Newton-Schulz steps must be in 0..16");
  if (!(eps > 0.f) || !std::isfinite(eps)) return fail(FVAN_EINVAL, "eps must be finite and > 0");
  FVAN_HIP(launch_newton_schulz(M, O, rows, cols, steps, eps, (hipStream_t)stream));
  return FVAN_OK;
}

int fvan_muon_step(fvan_model* m, const fvan_muon* opt, int64_t step, void* stream) {
  if (!m || !opt) return fail(FVAN_EINVAL, "NULL argument");
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (!m->params || !m->grads) return fail(FVAN_EINVAL, "parameters and gradients must be bound");
  if (step < 1) return fail(FVAN_EINVAL, "step counts from 1");
  if (const char* why = check_muon(*opt)) return fail(FVAN_EINVAL, why);
  hipStream_t s = (hipStream_t)stream;
  FVAN_HIP(launch_muon(m->cfg, m->params, m->grads, m->adam_m, m->adam_v, m->n_params, *opt, step, s));
  FVAN_HIP(launch_pack(m->cfg, m->params, m->wpack, s));
  return FVAN_OK;
}

}  // extern "C"
