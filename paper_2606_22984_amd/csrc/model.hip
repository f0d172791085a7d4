// Model workspaces (allocated and initialised at create time) and the
// per-call decode descriptor.
#include <algorithm>
#include <map>
#include <mutex>

#include "device_common.h"
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

// rows [row0, row0 + nrows) of a [* x ld] float matrix set to value
__global__ void set_rows_kernel(float* p, int64_t ld, int row0, int nrows, int64_t cols, float value) {
  const int64_t total = (int64_t)nrows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    p[(int64_t)(row0 + i / cols) * ld + i % cols] = value;
}

static hipError_t set_rows(void* p, int64_t ld, int row0, int nrows, int64_t cols, float v, hipStream_t s) {
  const int64_t total = (int64_t)nrows * cols;
  hipLaunchKernelGGL(set_rows_kernel, dim3((int)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0, s,
                     (float*)p, ld, row0, nrows, cols, v);
  return hipGetLastError();
}

// The teacher-forced forward/backward workspace: one chunk of samples
// (fwd_chunk_samples), every layer's input and post-attention residual, Q/K/V
// and the attention log-sum-exp, plus the backward's transients.
static int allocate_fwd(fvan_model* m, hipStream_t s) {
  auto& f = m->fw;
  const fvan_model_config& c = m->cfg;
  const int64_t D = c.d_model, H = c.n_heads, L = c.n_layers, N = c.n_spins;
  f.chunk = fwd_chunk_samples(c);
  f.rows = f.chunk * N;
  f.ldT = (f.rows + 63) / 64 * 64;
  const size_t R = (size_t)f.rows, ldT = (size_t)f.ldT;
  const size_t kt = kv_elem_bytes(c.precision);
  f.part_floats = (size_t)512 * 4 * D * (D + 16);
  f.colpart_floats = std::max<size_t>((size_t)f.chunk * (2 * D + 2), ((R + 63) / 64) * 2 * D);
  struct A { void** p; size_t bytes; const char* what; } allocs[] = {
      {(void**)&f.X, (size_t)(L + 1) * R * D * 4, "X"},   {(void**)&f.XM, (size_t)L * R * D * 4, "XM"},
      {(void**)&f.LSE, (size_t)L * R * H * 4, "LSE"},
      {(void**)&f.DELTA, R * H * 4, "DELTA"},
      {&f.QKV, (size_t)L * R * 3 * D * kt, "QKV"},
      {(void**)&f.dX, R * D * 4, "dX"},                   {(void**)&f.dXM, R * D * 4, "dXM"},
      {&f.dQKV, R * 3 * D * 4, "dQKV"},
      {&f.T_a, 4 * D * ldT * 4, "T_a"},
      {&f.T_b, (4 * D + 16) * ldT * 4, "T_b"},            {&f.T_c, (D + 16) * ldT * 4, "T_c"},
      {&f.T_d, D * ldT * 4, "T_d"},
      {&f.T_e, 3 * D * ldT * 4, "T_e"},                   {&f.T_f, (D + 16) * ldT * 4, "T_f"},
      {(void**)&f.part, f.part_floats * 4, "partials"},   {(void**)&f.part2, f.part_floats * 4, "side partials"},   {(void**)&f.colpart, f.colpart_floats * 4, "column partials"},
      {(void**)&f.colpart2, (size_t)64 * std::max<size_t>(2 * D + 2, (size_t)c.vocab * c.d_token) * 4,
       "column slices"},
  };
  for (auto& a : allocs) {
    int rc = dalloc(a.p, std::max<size_t>(a.bytes, 16), a.what);
    if (rc) return rc;
  }
  // the ones row (bias gradients) and the zero rows of the padded right operands
  hipError_t e = set_rows(f.T_b, f.ldT, 4 * D, 1, f.ldT, 1.f, s);
  if (e == hipSuccess) e = set_rows(f.T_b, f.ldT, 4 * D + 1, 15, f.ldT, 0.f, s);
  if (e == hipSuccess) e = set_rows(f.T_c, f.ldT, D, 1, f.ldT, 1.f, s);
  if (e == hipSuccess) e = set_rows(f.T_c, f.ldT, D + 1, 15, f.ldT, 0.f, s);
  if (e == hipSuccess) e = set_rows(f.T_f, f.ldT, D, 1, f.ldT, 1.f, s);
  if (e == hipSuccess) e = set_rows(f.T_f, f.ldT, D + 1, 15, f.ldT, 0.f, s);
  if (e != hipSuccess) return fail(FVAN_EDEVICE, std::string("workspace initialisation: ") + hipGetErrorString(e));
  // the side stream of the layer weight gradients (default priority) and its events
  if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) {
    f.side = nullptr;
    return fail(FVAN_EDEVICE, "hipStreamCreate failed for the weight-gradient stream");
  }
  for (auto& ev : f.ev) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
      return fail(FVAN_EDEVICE, "hipEventCreate failed for the weight-gradient stream");
    }
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
  int rc;
  if ((rc = dalloc(&m->wpack, std::max<size_t>(m->pk.total, 16), "packed weights"))) return rc;
  if ((rc = dalloc(&m->nf_flag, 4, "non-finite flag"))) return rc;
  if (hipHostMalloc(reinterpret_cast<void**>(&m->nf_host), 4, hipHostMallocDefault) != hipSuccess) {
    m->nf_host = nullptr;
    (void)hipGetLastError();
    return fail(FVAN_ENOMEM, "hipHostMalloc failed for the non-finite flag");
  }
  *m->nf_host = 0;
  if (hipEventCreateWithFlags(&m->nf_event, hipEventDisableTiming) != hipSuccess) {
    m->nf_event = nullptr;
    return fail(FVAN_EDEVICE, "hipEventCreate failed");
  }
  if (has_sampler(m)) {
    m->kv_bytes = B * c.n_layers * 2 * (size_t)m->kg.S * c.d_model * eb;
    if ((rc = dalloc(&m->kv, std::max<size_t>(m->kv_bytes, 16), "KV cache"))) return rc;
  }
  if (has_teacher(m)) {
    if ((rc = dalloc(&m->adam_m, m->n_params * 4, "Adam m"))) return rc;
    if ((rc = dalloc(&m->adam_v, m->n_params * 4, "Adam v"))) return rc;
  }
  if (has_sampler(m) && has_teacher(m)) {
    if ((rc = dalloc(&m->ts_spins, B * c.n_spins, "train-step spins"))) return rc;
    if ((rc = dalloc(&m->ts_logq, B * 4, "train-step log q"))) return rc;
    if ((rc = dalloc(&m->ts_energy, B * 4, "train-step energies"))) return rc;
    if ((rc = dalloc(&m->ts_w, B * 4, "train-step weights"))) return rc;
    if ((rc = dalloc(&m->ts_dbl, 64 * 8, "FP64 scratch"))) return rc;
    if (token_bits(c.vocab) &&
        (rc = dalloc(&m->ts_lattice, B * c.n_spins * token_bits(c.vocab), "train-step lattice spins")))
      return rc;
  }
  // initialisation on the null stream, waited for here: create is the one call
  // that may block
  hipStream_t s = nullptr;
  if (hipMemsetAsync(m->nf_flag, 0, 4, s) != hipSuccess) return fail(FVAN_EDEVICE, "hipMemset of the flag failed");
  if (has_teacher(m)) {
    if (hipMemsetAsync(m->adam_m, 0, m->n_params * 4, s) != hipSuccess ||
        hipMemsetAsync(m->adam_v, 0, m->n_params * 4, s) != hipSuccess)
      return fail(FVAN_EDEVICE, "hipMemset of optimiser state failed");
    if ((rc = allocate_fwd(m, s))) return rc;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(FVAN_EDEVICE, "workspace initialisation failed");
  return FVAN_OK;
}

static void dfree(void* p) {
  if (p) (void)hipFree(p);
}

void model_free(fvan_model* m) {
  dfree(m->wpack); dfree(m->kv); dfree(m->adam_m); dfree(m->adam_v);
  dfree(m->ts_spins); dfree(m->ts_lattice); dfree(m->ts_logq); dfree(m->ts_energy); dfree(m->ts_w); dfree(m->ts_dbl);
  dfree(m->nf_flag);
  if (m->nf_host) (void)hipHostFree(m->nf_host);
  if (m->nf_event) (void)hipEventDestroy(m->nf_event);
  m->nf_host = nullptr;
  m->nf_event = nullptr;
  model_free_fwd(m);
}

void model_free_fwd(fvan_model* m) {
  auto& f = m->fw;
  dfree(f.X); dfree(f.XM); dfree(f.LSE); dfree(f.DELTA);
  dfree(f.QKV); dfree(f.dX); dfree(f.dXM); dfree(f.dQKV);
  dfree(f.T_e); dfree(f.T_f); dfree(f.part2);
  for (auto& ev : f.ev) {
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
  }
  if (f.side) (void)hipStreamDestroy(f.side);
  f.side = nullptr;
  dfree(f.T_a); dfree(f.T_b); dfree(f.T_c); dfree(f.T_d); dfree(f.part); dfree(f.colpart); dfree(f.colpart2);
  m->fw = fvan_model::Fwd();
}

// ---------------------------------------------------------------- non-finite checks
template <typename T>
__global__ void nonfinite_kernel(const T* __restrict__ v, int64_t n, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(v[i]);
  if (bad) atomicOr(flag, 1);
}

template <typename T>
static hipError_t check_finite_t(fvan_model* m, const T* v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(nonfinite_kernel<T>, dim3(grid), dim3(256), 0, s, v, n, m->nf_flag);
  return hipGetLastError();
}
hipError_t check_finite(fvan_model* m, const float* v, int64_t n, hipStream_t s) { return check_finite_t(m, v, n, s); }
hipError_t check_finite(fvan_model* m, const double* v, int64_t n, hipStream_t s) { return check_finite_t(m, v, n, s); }

int device_cus(int dev) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    n = 256;
  }
  cache[dev] = n;
  return n;
}

// Samples per decode workgroup for a sampling call of `batch` samples: 16 when
// 32-sample tiles would leave compute units idle and the kernel exists with
// 16-sample tiles (the per-sample arithmetic is the same for both), else 32.
int sample_tile(const fvan_model* m, DecodeShape sh, int32_t batch) {
  sh.tile = 16;
  if (!decode_has_tile16(sh)) return 32;
  return (batch + 31) / 32 < device_cus(m->device) ? 16 : 32;
}

DecodeUnit make_decode_unit(const fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, int8_t* spins,
                            float* log_q, void* kv, int tile0, int tile) {
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
  u.n_tiles = (batch + tile - 1) / tile;
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
  u.vocab = c.vocab;
  return u;
}

}  // namespace fvan
