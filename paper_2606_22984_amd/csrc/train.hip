// Teacher-forced log q, its backward, and the training step (host side).
#include <algorithm>

#include "device_common.h"
#include "fvan_model.h"
#include "passes.h"

namespace fvan {

// Training steps: wait for the previous step of this model and report its
// finiteness check (see fvan_train_step); FVAN_OK when it was finite.
static int previous_step_status(fvan_model* m) {
  if (!m->nf_pending) return FVAN_OK;
  if (hipEventSynchronize(m->nf_event) != hipSuccess) return fail(FVAN_EDEVICE, "hipEventSynchronize failed");
  m->nf_pending = false;
  if (*m->nf_host) {
    *m->nf_host = 0;
    if (hipMemset(m->nf_flag, 0, 4) != hipSuccess) return fail(FVAN_EDEVICE, "hipMemset of the flag failed");
    return fail(FVAN_ENONFINITE, "the previous training step of this model produced a non-finite value");
  }
  return FVAN_OK;
}

// End of a training step: check the statistics and hand the flag to the host.
static int finish_step(fvan_model* m, const double* stats, hipStream_t s) {
  FVAN_HIP(check_finite(m, stats, 4, s));
  FVAN_HIP(hipMemcpyAsync(m->nf_host, m->nf_flag, 4, hipMemcpyDeviceToHost, s));
  FVAN_HIP(hipEventRecord(m->nf_event, s));
  m->nf_pending = true;
  return FVAN_OK;
}

}  // namespace fvan

using namespace fvan;

extern "C" {

int fvan_log_prob(fvan_model* m, int32_t batch, const int8_t* spins, float* log_q, void* stream) {
  if (!m || !spins || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (m->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(forward_chunk(m, spins + b0 * N, nb, log_q + b0, false, s));
  }
  FVAN_HIP(check_finite(m, log_q, batch, s));
  return FVAN_OK;
}

int fvan_log_prob_tokens(fvan_model* m, int32_t batch, const uint8_t* tokens, float* log_q, void* stream) {
  if (!m || !tokens || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(forward_chunk_tokens(m, tokens + b0 * N, nb, log_q + b0, s));
  }
  return FVAN_OK;
}

int fvan_log_prob_backward(fvan_model* m, int32_t batch, const int8_t* spins, const float* grad_log_q,
                           void* stream) {
  if (!m || !spins || !grad_log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (m->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (!m->grads) return fail(FVAN_EINVAL, "no gradient buffer bound");
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(backward_chunk(m, spins + b0 * N, nb, grad_log_q + b0, s));
  }
  FVAN_HIP(check_finite(m, m->grads, m->n_params, s));
  return FVAN_OK;
}

int fvan_log_prob_tokens_backward(fvan_model* m, int32_t batch, const uint8_t* tokens, const float* grad_log_q,
                                  void* stream) {
  if (!m || !tokens || !grad_log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (!m->grads) return fail(FVAN_EINVAL, "no gradient buffer bound");
  if (!has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTeacher);
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  if (m->cfg.vocab > 16 && m->cfg.d_model < 64)
    return fail(FVAN_EUNSUPPORTED, "the token backward needs vocab <= 16 or d_model >= 64");
  if (m->cfg.vocab * m->cfg.d_token > 16384) return fail(FVAN_EUNSUPPORTED, "vocab * d_token must be <= 16384");
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(backward_chunk_tokens(m, tokens + b0 * N, nb, grad_log_q + b0, s));
  }
  FVAN_HIP(check_finite(m, m->grads, m->n_params, s));
  return FVAN_OK;
}

// Everything of a training step before the update: sample, energies, F_q
// statistics, REINFORCE weights, backward and the gradient norm.
static int train_step_gradient(fvan_model* m, const fvan_couplings* c, double beta, int32_t batch, uint64_t seed,
                               uint64_t step, double* stats, void* stream) {
  if (!m || !c || !stats) return fail(FVAN_EINVAL, "NULL argument");
  if (c->n_spins != m->cfg.n_spins) return fail(FVAN_EINVAL, "couplings and model disagree on n_spins");
  if (!(beta > 0.0)) return fail(FVAN_EINVAL, "beta must be > 0");
  if (step < 1) return fail(FVAN_EINVAL, "step counts from 1");
  if (!m->params || !m->grads) return fail(FVAN_EINVAL, "parameters and gradients must be bound");
  if (!has_sampler(m) || !has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTrain);
  hipStream_t s = (hipStream_t)stream;
  int rc = previous_step_status(m);
  if (rc) return rc;
  rc = fvan_sample(m, batch, seed, step, m->ts_spins, m->ts_logq, stream);
  if (rc) return rc;
  if ((rc = fvan_energy(c, batch, m->ts_spins, m->ts_energy, stream))) return rc;
  const int is_int = c->kind == FVAN_BONDS_PM1;
  if ((rc = fvan_free_energy(batch, m->cfg.n_spins, beta, is_int, m->ts_energy, m->ts_logq, stats, stream)))
    return rc;
  FVAN_HIP(launch_mean_energy(batch, m->cfg.n_spins, is_int, m->ts_energy, stats + 2, s));
  FVAN_HIP(launch_reinforce(batch, beta, is_int, m->ts_energy, m->ts_logq, m->ts_w, nullptr, s));
  if ((rc = fvan_log_prob_backward(m, batch, m->ts_spins, m->ts_w, stream))) return rc;
  FVAN_HIP(launch_grad_norm(m->grads, m->n_params, stats + 3, nullptr, s));
  return FVAN_OK;
}

int fvan_train_step(fvan_model* m, const fvan_couplings* c, double beta, int32_t batch, uint64_t seed,
                    uint64_t step, const fvan_adam* opt, double* stats, void* stream) {
  if (!opt) return fail(FVAN_EINVAL, "NULL argument");
  if (const char* why = check_adam(*opt)) return fail(FVAN_EINVAL, why);
  int rc = train_step_gradient(m, c, beta, batch, seed, step, stats, stream);
  if (rc) return rc;
  if ((rc = fvan_adam_step(m, opt, (int64_t)step, stream))) return rc;
  return finish_step(m, stats, (hipStream_t)stream);
}

int fvan_train_step_distill(fvan_model* m, const fvan_couplings* c, const fvan_lmc* g, double beta, double w,
                            int32_t batch, uint64_t seed, uint64_t step, const fvan_muon* opt, double* stats,
                            void* stream) {
  if (!m || !c || !g || !opt || !stats) return fail(FVAN_EINVAL, "NULL argument");
  if (const char* why = check_muon(*opt)) return fail(FVAN_EINVAL, why);
  if (c->n_spins != m->cfg.n_spins) return fail(FVAN_EINVAL, "couplings and model disagree on n_spins");
  if (!(beta > 0.0) || !std::isfinite(beta) || !std::isfinite(w)) return fail(FVAN_EINVAL, "beta or w out of range");
  if (step < 1) return fail(FVAN_EINVAL, "step counts from 1");
  if (!m->params || !m->grads) return fail(FVAN_EINVAL, "parameters and gradients must be bound");
  if (!g->nbr || !g->J || !g->colour || g->degree < 1 || g->sweeps < 0 || m->cfg.n_spins > 16384)
    return fail(FVAN_EINVAL, "refinement graph or sweeps out of range");
  if (!has_sampler(m) || !has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTrain);
  hipStream_t s = (hipStream_t)stream;
  int rc = previous_step_status(m);
  if (rc) return rc;
  rc = fvan_sample(m, batch, seed, step, m->ts_spins, m->ts_logq, stream);
  if (rc) return rc;
  const int is_int = c->kind == FVAN_BONDS_PM1;
  if ((rc = fvan_energy(c, batch, m->ts_spins, m->ts_energy, stream))) return rc;
  if ((rc = fvan_free_energy(batch, m->cfg.n_spins, beta, is_int, m->ts_energy, m->ts_logq, stats, stream)))
    return rc;
  FVAN_HIP(launch_mean_energy(batch, m->cfg.n_spins, is_int, m->ts_energy, stats + 2, s));
  const uint32_t tag = 0x80000000u | (uint32_t)(step & 0x7FFFFFFFu);
  if ((rc = fvan_lmc_refine(m->cfg.n_spins, g, batch, beta, seed, tag, m->ts_spins, nullptr, stream))) return rc;
  if ((rc = fvan_energy(c, batch, m->ts_spins, m->ts_energy, stream))) return rc;
  if ((rc = fvan_log_prob(m, batch, m->ts_spins, m->ts_logq, stream))) return rc;
  FVAN_HIP(launch_reinforce(batch, beta, is_int, m->ts_energy, m->ts_logq, m->ts_w, nullptr, s, w));
  if ((rc = fvan_log_prob_backward(m, batch, m->ts_spins, m->ts_w, stream))) return rc;
  FVAN_HIP(launch_grad_norm(m->grads, m->n_params, stats + 3, nullptr, s));
  if ((rc = fvan_muon_step(m, opt, (int64_t)step, stream))) return rc;
  return finish_step(m, stats, s);
}

int fvan_model_status(fvan_model* m, void* stream) {
  if (!m) return fail(FVAN_EINVAL, "model is NULL");
  FVAN_HIP(hipStreamSynchronize((hipStream_t)stream));
  m->nf_pending = false;                       // a training step's copy, if any, has landed
  *m->nf_host = 0;
  int v = 0;
  FVAN_HIP(hipMemcpy(&v, m->nf_flag, 4, hipMemcpyDeviceToHost));
  if (v) {
    FVAN_HIP(hipMemset(m->nf_flag, 0, 4));
    return fail(FVAN_ENONFINITE, "a kernel of this model produced a non-finite value");
  }
  return FVAN_OK;
}

int fvan_train_step_tokens(fvan_model* m, const fvan_couplings* c, const int32_t* sites, double beta, int32_t batch,
                           uint64_t seed, uint64_t step, const fvan_muon* opt, double* stats, void* stream) {
  if (!m || !c || !sites || !opt || !stats) return fail(FVAN_EINVAL, "NULL argument");
  if (const char* why = check_muon(*opt)) return fail(FVAN_EINVAL, why);
  const int bits = token_bits(m->cfg.vocab);
  if (!bits) return fail(FVAN_EUNSUPPORTED, "a patch-token training step needs vocab = 2^bits, bits in [2, 8]");
  const int32_t n = m->cfg.n_spins * bits;
  if (c->n_spins != n) return fail(FVAN_EINVAL, "couplings must cover n_spins * log2(vocab) lattice sites");
  if (!(beta > 0.0) || !std::isfinite(beta)) return fail(FVAN_EINVAL, "beta must be finite and > 0");
  if (step < 1) return fail(FVAN_EINVAL, "step counts from 1");
  if (!m->params || !m->grads) return fail(FVAN_EINVAL, "parameters and gradients must be bound");
  if (!has_sampler(m) || !has_teacher(m)) return fail(FVAN_EUNSUPPORTED, kNoTrain);
  hipStream_t s = (hipStream_t)stream;
  int rc = previous_step_status(m);
  if (rc) return rc;
  uint8_t* tok = reinterpret_cast<uint8_t*>(m->ts_spins);
  if ((rc = fvan_sample_tokens(m, batch, seed, step, tok, m->ts_logq, stream))) return rc;
  FVAN_HIP(launch_tokens_to_spins(m->cfg.n_spins, bits, sites, n, batch, tok, m->ts_lattice, s));
  if ((rc = fvan_energy(c, batch, m->ts_lattice, m->ts_energy, stream))) return rc;
  const int is_int = c->kind == FVAN_BONDS_PM1;
  if ((rc = fvan_free_energy(batch, n, beta, is_int, m->ts_energy, m->ts_logq, stats, stream))) return rc;
  FVAN_HIP(launch_mean_energy(batch, n, is_int, m->ts_energy, stats + 2, s));
  FVAN_HIP(launch_reinforce(batch, beta, is_int, m->ts_energy, m->ts_logq, m->ts_w, nullptr, s));
  if ((rc = fvan_log_prob_tokens_backward(m, batch, tok, m->ts_w, stream))) return rc;
  FVAN_HIP(launch_grad_norm(m->grads, m->n_params, stats + 3, nullptr, s));
  if ((rc = fvan_muon_step(m, opt, (int64_t)step, stream))) return rc;
  return finish_step(m, stats, s);
}

int fvan_train_step_muon(fvan_model* m, const fvan_couplings* c, double beta, int32_t batch, uint64_t seed,
                         uint64_t step, const fvan_muon* opt, double* stats, void* stream) {
  if (!opt) return fail(FVAN_EINVAL, "NULL argument");
  if (const char* why = check_muon(*opt)) return fail(FVAN_EINVAL, why);
  int rc = train_step_gradient(m, c, beta, batch, seed, step, stats, stream);
  if (rc) return rc;
  if ((rc = fvan_muon_step(m, opt, (int64_t)step, stream))) return rc;
  return finish_step(m, stats, (hipStream_t)stream);
}

}  // extern "C"
