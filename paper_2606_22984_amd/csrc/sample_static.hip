// Sampling for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation):
// fvan_sample_noalloc runs the same KV-cached decode kernel as fvan_sample, with
// its KV cache in a fixed device array of this library instead of the model's
// sampler workspace.  The array is file-scope, so each GPU the library runs on
// holds one copy of it, at its own address, until the process ends.
#include <mutex>

#include "device_common.h"
#include "fvan_model.h"
#include "passes.h"

namespace fvan {

constexpr size_t kStaticKvBytes = FVAN_NOALLOC_KV_BYTES;   // 64 MiB per GPU

// The KV cache of fvan_sample_noalloc.  Host code never uses this name as an
// address: it is a host-side stand-in for the device symbol.  The per-device
// address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kStaticKvBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current: looked up
// once per device and kept.  fvan_create_model calls it for the model's device
// (static_kv_setup), so the lookup, and the runtime's first-use allocation of
// the array behind it, happen at set-up and never inside fvan_sample_noalloc.
static int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FVAN_EUNSUPPORTED, "device index beyond the supported 64");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(FVAN_EDEVICE, std::string("hipGetSymbolAddress of the static KV cache: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FVAN_OK;
}

int static_kv_setup(int dev) {
  void* p = nullptr;
  return scratch_address(dev, &p);
}

}  // namespace fvan

using namespace fvan;

extern "C" int fvan_sample_noalloc(fvan_model* m, int32_t batch, uint64_t seed, uint64_t stream_id, int8_t* spins,
                                   float* log_q, void* stream) {
  if (!m || !spins || !log_q) return fail(FVAN_EINVAL, "NULL argument");
  if (m->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  if (!m->params || !m->synced) return fail(FVAN_EINVAL, "parameters not bound/synced");
  if (batch < 1 || batch > m->cfg.max_batch) return fail(FVAN_EINVAL, "batch outside [1, max_batch]");
  const size_t per_sample =
      (size_t)m->cfg.n_layers * 2 * (size_t)m->kg.S * m->cfg.d_model * kv_elem_bytes(m->cfg.precision);
  if (per_sample * (size_t)batch > kStaticKvBytes)
    return fail(FVAN_EINVAL, "fvan_sample_noalloc: the KV cache of " + std::to_string(batch) + " samples needs " +
                                 std::to_string(per_sample * (size_t)batch) + " bytes, beyond the static " +
                                 std::to_string(kStaticKvBytes) + "-byte cache (at most " +
                                 std::to_string(per_sample ? kStaticKvBytes / per_sample : 0) +
                                 " samples of this model)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FVAN_EDEVICE, "hipGetDevice failed");
  if (dev != m->device) return fail(FVAN_EINVAL, "the current device is not the model's device");
  void* kv = nullptr;
  if (int rc = scratch_address(dev, &kv)) return rc;
  DecodeShape sh = decode_shape(m->cfg);
  sh.tile = sample_tile(m, sh, batch);
  DecodeUnit u = make_decode_unit(m, batch, seed, stream_id, spins, log_q, kv, 0, sh.tile);
  FVAN_HIP(launch_decode_single(sh, u, u.n_tiles, (hipStream_t)stream));
  FVAN_HIP(check_finite(m, log_q, batch, (hipStream_t)stream));
  return FVAN_OK;
}
