// Model workspaces and the per-call decode descriptor.
#include <algorithm>

#include "fvan_model.h"

namespace fvan {

template <typename T>
static int dalloc(T** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return FVAN_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(FVAN_ENOMEM, std::string("hipMalloc failed for ") + what + " (" + std::to_string(bytes) + " bytes)");
  }
  return FVAN_OK;
}

int model_allocate(fvan_model* m) {
  const fvan_model_config& c = m->cfg;
  m->po = param_offsets(c);
  m->pk = pack_offsets(c);
  m->kg = kv_geom(c);
  m->n_params = m->po.total;
  if (hipGetDevice(&m->device) != hipSuccess) return fail(FVAN_EDEVICE, "hipGetDevice failed");
  const size_t B = (size_t)c.max_batch;
  const size_t eb = kv_elem_bytes(c.precision);
  m->kv_bytes = B * c.n_layers * 2 * (size_t)m->kg.S * c.d_model * eb;
  int rc;
  if ((rc = dalloc(&m->wpack, std::max<size_t>(m->pk.total, 16), "packed weights"))) return rc;
  if ((rc = dalloc(&m->kv, std::max<size_t>(m->kv_bytes, 16), "KV cache"))) return rc;
  if ((rc = dalloc(&m->adam_m, m->n_params * 4, "Adam m"))) return rc;
  if ((rc = dalloc(&m->adam_v, m->n_params * 4, "Adam v"))) return rc;
  if ((rc = dalloc(&m->ts_spins, B * c.n_spins, "train-step spins"))) return rc;
  if ((rc = dalloc(&m->ts_logq, B * 4, "train-step log q"))) return rc;
  if ((rc = dalloc(&m->ts_energy, B * 4, "train-step energies"))) return rc;
  if ((rc = dalloc(&m->ts_w, B * 4, "train-step weights"))) return rc;
  if ((rc = dalloc(&m->ts_dbl, 64 * 8, "FP64 scratch"))) return rc;
  if (hipMemset(m->adam_m, 0, m->n_params * 4) != hipSuccess || hipMemset(m->adam_v, 0, m->n_params * 4) != hipSuccess)
    return fail(FVAN_EDEVICE, "hipMemset of optimiser state failed");
  return FVAN_OK;
}

static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void model_free(fvan_model* m) {
  dfree(m->wpack); dfree(m->kv); dfree(m->adam_m); dfree(m->adam_v);
  dfree(m->ts_spins); dfree(m->ts_logq); dfree(m->ts_energy); dfree(m->ts_w); dfree(m->ts_dbl);
  model_free_fwd(m);
}

void model_free_fwd(fvan_model* m) {
  auto& f = m->fw;
  dfree(f.X); dfree(f.XM); dfree(f.LSE); dfree(f.DELTA); dfree(f.TMP); dfree(f.DY);
  dfree(f.QKV); dfree(f.HPRE); dfree(f.logp); dfree(f.dX); dfree(f.dXM); dfree(f.dQKV); dfree(f.dH);
  dfree(f.T_a); dfree(f.T_b); dfree(f.T_c); dfree(f.part); dfree(f.colpart); dfree(f.colpart2);
  m->fw = fvan_model::Fwd();
}

DecodeUnit make_decode_unit(const fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, int8_t* spins,
                            float* log_q, void* kv, int tile0) {
  const fvan_model_config& c = m->cfg;
  DecodeUnit u{};
  u.theta = m->params;
  u.wpack = m->wpack;
  u.kv = kv;
  u.spins = spins;
  u.logq = log_q;
  u.N = c.n_spins;
  u.W = c.window;
  u.P = m->kg.P;
  u.R = m->kg.R;
  u.S = m->kg.S;
  u.B = batch;
  u.n_layers = c.n_layers;
  u.tile0 = tile0;
  u.n_tiles = (batch + decode_tile_samples() - 1) / decode_tile_samples();
  u.pos_off = (int32_t)m->po.pos;
  u.layer0 = m->po.layer0;
  u.layer_stride = m->po.layer_stride;
  u.head_w = m->po.head_w;
  u.head_b = m->po.head_b;
  u.seed_lo = (uint32_t)(seed & 0xffffffffu);
  u.seed_hi = (uint32_t)(seed >> 32);
  u.stream_lo = (uint32_t)(stream_id & 0xffffffffu);
  u.stream_hi = (uint32_t)(stream_id >> 32);
  u.o_ln1_g = (int32_t)m->po.ln1_g;
  u.o_ln1_b = (int32_t)m->po.ln1_b;
  u.o_qkv_b = (int32_t)m->po.qkv_b;
  u.o_ln2_g = (int32_t)m->po.ln2_g;
  u.o_ln2_b = (int32_t)m->po.ln2_b;
  u.o_ffn1_b = (int32_t)m->po.ffn1_b;
  u.o_ffn2_b = (int32_t)m->po.ffn2_b;
  u.p_qkv = (int64_t)m->pk.qkv;
  u.p_ffn1 = (int64_t)m->pk.ffn1;
  u.p_ffn2 = (int64_t)m->pk.ffn2;
  u.p_layer_stride = (int64_t)m->pk.layer_stride;
  u.d_token = c.d_token;
  return u;
}

}  // namespace fvan
