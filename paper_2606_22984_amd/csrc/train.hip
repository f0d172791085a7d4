// Teacher-forced log q, its backward, and the training step (host side).
#include <algorithm>

#include "device_common.h"
#include "fvan_model.h"
#include "passes.h"

namespace fvan {

template <typename T>
__global__ void set_rows_kernel(T* p, int64_t ld, int row0, int nrows, int64_t cols, float value) {
  const int64_t total = (int64_t)nrows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    p[(int64_t)(row0 + i / cols) * ld + i % cols] = from_f<T>(value);
}

template <typename T>
static hipError_t set_rows(void* p, int64_t ld, int row0, int nrows, int64_t cols, float v) {
  const int64_t total = (int64_t)nrows * cols;
  hipLaunchKernelGGL((set_rows_kernel<T>), dim3((int)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0,
                     nullptr, (T*)p, ld, row0, nrows, cols, v);
  return hipGetLastError();
}

static int walloc(void** p, size_t bytes, const char* what) {
  if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(FVAN_ENOMEM, std::string("hipMalloc failed for the forward/backward workspace (") + what + ", " +
                                 std::to_string(bytes) + " bytes)");
  }
  return FVAN_OK;
}

int ensure_fwd_workspace(fvan_model* m) {
  auto& f = m->fw;
  if (f.X) return FVAN_OK;
  const fvan_model_config& c = m->cfg;
  const int64_t D = c.d_model, H = c.n_heads, L = c.n_layers, N = c.n_spins;
  f.chunk = fwd_chunk_samples(c);
  f.rows = f.chunk * N;
  f.ldT = (f.rows + 63) / 64 * 64;
  const size_t R = (size_t)f.rows, ldT = (size_t)f.ldT;
  const size_t at = c.precision == FVAN_BF16 ? 2 : 4;
  const size_t kt = kv_elem_bytes(c.precision);
  f.part_floats = (size_t)512 * 4 * D * (D + 16);
  f.colpart_floats = std::max<size_t>((size_t)f.chunk * (2 * D + 2), ((R + 63) / 64) * 2 * D);
  struct A { void** p; size_t bytes; const char* what; } allocs[] = {
      {(void**)&f.X, (size_t)(L + 1) * R * D * 4, "X"},   {(void**)&f.XM, (size_t)L * R * D * 4, "XM"},
      {(void**)&f.LSE, (size_t)L * R * H * 4, "LSE"},
      {(void**)&f.DELTA, R * H * 4, "DELTA"},             {(void**)&f.TMP, R * D * 4, "TMP"},
      {&f.DY, R * D * at, "DY"},
      {&f.QKV, (size_t)L * R * 3 * D * kt, "QKV"},       {(void**)&f.HPRE, R * 4 * D * 4, "HPRE"},
      {(void**)&f.dX, R * D * 4, "dX"},                   {(void**)&f.dXM, R * D * 4, "dXM"},
      {&f.dQKV, R * 3 * D * at, "dQKV"},                  {&f.dH, R * 4 * D * at, "dH"},
      {&f.T_a, 4 * D * ldT * at, "T_a"},
      {&f.T_b, (4 * D + 16) * ldT * at, "T_b"},           {&f.T_c, (D + 16) * ldT * at, "T_c"},
      {(void**)&f.part, f.part_floats * 4, "partials"},   {(void**)&f.colpart, f.colpart_floats * 4, "column partials"},
      {(void**)&f.colpart2, (size_t)64 * (2 * D + 2) * 4, "column slices"},
  };
  for (auto& a : allocs) {
    int rc = walloc(a.p, a.bytes, a.what);
    if (rc) {
      model_free_fwd(m);
      return rc;
    }
  }
  // ones row (bias gradients) and zero rows of the padded right operands
  hipError_t e;
  if (at == 2) {
    e = set_rows<__bf16>(f.T_b, f.ldT, 4 * D, 1, f.ldT, 1.f);
    if (e == hipSuccess) e = set_rows<__bf16>(f.T_b, f.ldT, 4 * D + 1, 15, f.ldT, 0.f);
    if (e == hipSuccess) e = set_rows<__bf16>(f.T_c, f.ldT, D, 1, f.ldT, 1.f);
    if (e == hipSuccess) e = set_rows<__bf16>(f.T_c, f.ldT, D + 1, 15, f.ldT, 0.f);
  } else {
    e = set_rows<float>(f.T_b, f.ldT, 4 * D, 1, f.ldT, 1.f);
    if (e == hipSuccess) e = set_rows<float>(f.T_b, f.ldT, 4 * D + 1, 15, f.ldT, 0.f);
    if (e == hipSuccess) e = set_rows<float>(f.T_c, f.ldT, D, 1, f.ldT, 1.f);
    if (e == hipSuccess) e = set_rows<float>(f.T_c, f.ldT, D + 1, 15, f.ldT, 0.f);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    model_free_fwd(m);
    return fail(FVAN_EDEVICE, std::string("workspace initialisation: ") + hipGetErrorString(e));
  }
  return FVAN_OK;
}

}  // namespace fvan

using namespace fvan;

extern "C" {

int fvan_log_prob(fvan_model* m, int32_t batch, const int8_t* spins, float* log_q, void* stream) {
  if (!m || !spins || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (m->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  int rc = ensure_fwd_workspace(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(forward_chunk(m, spins + b0 * N, nb, log_q + b0, false, s));
  }
  return FVAN_OK;
}

int fvan_log_prob_tokens(fvan_model* m, int32_t batch, const uint8_t* tokens, float* log_q, void* stream) {
  if (!m || !tokens || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  int rc = ensure_fwd_workspace(m);
  if (rc) return rc;
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
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  int rc = ensure_fwd_workspace(m);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = m->cfg.n_spins;
  for (int64_t b0 = 0; b0 < batch; b0 += m->fw.chunk) {
    const int nb = (int)std::min<int64_t>(m->fw.chunk, batch - b0);
    FVAN_HIP(backward_chunk(m, spins + b0 * N, nb, grad_log_q + b0, s));
  }
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
  hipStream_t s = (hipStream_t)stream;
  int rc = fvan_sample(m, batch, seed, step, m->ts_spins, m->ts_logq, stream);
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
  return fvan_adam_step(m, opt, (int64_t)step, stream);
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
  hipStream_t s = (hipStream_t)stream;
  int rc = fvan_sample(m, batch, seed, step, m->ts_spins, m->ts_logq, stream);
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
  return fvan_muon_step(m, opt, (int64_t)step, stream);
}

int fvan_train_step_muon(fvan_model* m, const fvan_couplings* c, double beta, int32_t batch, uint64_t seed,
                         uint64_t step, const fvan_muon* opt, double* stats, void* stream) {
  if (!opt) return fail(FVAN_EINVAL, "NULL argument");
  if (const char* why = check_muon(*opt)) return fail(FVAN_EINVAL, why);
  int rc = train_step_gradient(m, c, beta, batch, seed, step, stats, stream);
  if (rc) return rc;
  return fvan_muon_step(m, opt, (int64_t)step, stream);
}

}  // extern "C"
