// Batched launches over many (instance, temperature, size) units.
//
// Sampling of every unit runs in ONE persistent decode launch: the device
// table holds one descriptor per unit (its parameters, packed weights, K/V
// cache, mask, outputs and Philox stream), work items are (unit, 16-sample
// tile) ranges ordered longest-sequence first, and workgroups pull items from
// an atomic counter until the queue is empty (every workgroup reaches the
// exit test, so the grid always drains).  Energies and free-energy statistics
// of all units follow as one launch each.  The whole sequence can be captured
// once into a HIP graph and replayed; the queue counter is reset by a kernel,
// not a memset node, so replays stay correct.
//
// The launch shape is chosen by an autotuner: samples per workgroup (16 or 32)
// and the persistent grid size, including a grid sized so that the K/V caches
// of the samples in flight fit the 256 MB MALL (the last-level cache in front of
// HBM) rather than streaming from HBM.  Each candidate is timed on the same
// prefix of the work queue (the longest units); the fastest is kept and
// persisted per shape (tune_cache.h), so later groups of that shape, in this
// or another process, reuse it without timing.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "device_common.h"
#include "fvan_model.h"
#include "tune_cache.h"

namespace fvan {

struct GroupEnergyUnit {
  int32_t n, kind, degree, batch;
  const int32_t* nbr;
  const void* J;
  const int8_t* spins;
  void* energy;
};

struct GroupStatUnit {
  int32_t n, batch, is_int;
  double beta;
  const void* energy;
  const float* logq;
  double* stats;
};

// One workgroup per (unit, sample); ELL bonds only (dense SK units use the
// per-unit path).  Same arithmetic and summation order as the single-model
// kernel (energy_ell_kernel), so the energies are bitwise equal to fvan_energy's.
__global__ __launch_bounds__(256) void group_energy_kernel(const GroupEnergyUnit* __restrict__ units,
                                                           const int64_t* __restrict__ first, int n_units) {
  __shared__ int8_t srow[4096];
  const int64_t item = blockIdx.x;
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid; else hi = mid - 1;
  }
  const GroupEnergyUnit u = units[lo];
  const int b = (int)(item - first[lo]);
  const int8_t* row = u.spins + (size_t)b * u.n;
  for (int i = threadIdx.x; i < u.n; i += 256) srow[i] = row[i];
  __syncthreads();
  const bool pm1 = u.kind == FVAN_BONDS_PM1;
  int iacc = 0;
  float facc = 0.f;
  for (int i = threadIdx.x; i < u.n; i += 256) {
    int ip = 0;
    float fp = 0.f;
    for (int k = 0; k < u.degree; ++k) {
      const int j = u.nbr[(size_t)i * u.degree + k];
      if (j >= 0 && j < u.n) {
        if (pm1) ip += (int)reinterpret_cast<const int8_t*>(u.J)[(size_t)i * u.degree + k] * srow[j];
        else fp += reinterpret_cast<const float*>(u.J)[(size_t)i * u.degree + k] * (float)srow[j];
      }
    }
    iacc += srow[i] * ip;
    facc += (float)srow[i] * fp;
  }
  // the single-model kernel's reduction: lanes, then the waves in order, in the
  // accumulation type (int32 for +-J bonds, float otherwise)
  __shared__ int ired[4];
  __shared__ float fred[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    iacc += __shfl_xor(iacc, off);
    facc += __shfl_xor(facc, off);
  }
  if ((threadIdx.x & 63) == 0) {
    ired[threadIdx.x >> 6] = iacc;
    fred[threadIdx.x >> 6] = facc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int it = 0;
    float ft = 0.f;
    for (int w = 0; w < 4; ++w) {
      it += ired[w];
      ft += fred[w];
    }
    if (pm1) reinterpret_cast<int*>(u.energy)[b] = -it;
    else reinterpret_cast<float*>(u.energy)[b] = -ft;
  }
}

// One workgroup per unit: F_q/N and Var[f] in FP64, fixed order.
__global__ __launch_bounds__(256) void group_stats_kernel(const GroupStatUnit* __restrict__ units) {
  __shared__ double red[4];
  const GroupStatUnit u = units[blockIdx.x];
  auto f = [&](int b) {
    const double e = u.is_int ? (double)reinterpret_cast<const int*>(u.energy)[b]
                              : (double)reinterpret_cast<const float*>(u.energy)[b];
    return (e + (double)u.logq[b] / u.beta) / (double)u.n;
  };
  auto bsum = [&](double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
  };
  double s = 0.0;
  for (int b = threadIdx.x; b < u.batch; b += 256) s += f(b);
  const double mean = bsum(s) / (double)u.batch;
  double v = 0.0;
  for (int b = threadIdx.x; b < u.batch; b += 256) {
    const double d = f(b) - mean;
    v += d * d;
  }
  const double var = bsum(v);
  if (threadIdx.x == 0) {
    u.stats[0] = mean;
    u.stats[1] = u.batch > 1 ? var / (double)(u.batch - 1) : 0.0;
  }
}

}  // namespace fvan

struct fvan_group {
  int d_model = 0, precision = 0, n_layers = 0;
  fvan::DecodeShape shape{};
  int n_units = 0, total_tiles = 0, grid = 0, device = 0;
  std::vector<fvan::DecodeUnit> host_table;   // tile0 / n_tiles for shape.tile
  std::string tune_key;
  bool tuned_from_cache = false;
  double tuned_ms = 0.0;                      // timed prefix of the chosen shape
  size_t kv_sample_max = 0;                   // largest per-sample K/V cache of the units
  std::vector<fvan_group_unit> units;
  std::vector<fvan_couplings> coup;
  fvan::DecodeUnit* d_table = nullptr;
  fvan::GroupEnergyUnit* d_energy = nullptr;
  fvan::GroupStatUnit* d_stats = nullptr;
  int64_t* d_first = nullptr;
  int64_t total_samples = 0;
  int* d_queue = nullptr;
  bool ell_energy = true;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace fvan {

constexpr size_t kMallBytes = size_t(256) << 20;   // MI355X Infinity Cache (MALL)

static hipError_t group_sample_n(fvan_group* g, int grid, int n_tiles, hipStream_t s) {
  hipError_t e = launch_zero_int(g->d_queue, 1, s);
  if (e != hipSuccess) return e;
  return launch_decode(g->shape, g->d_table, g->n_units, n_tiles, g->d_queue, grid, s);
}

static hipError_t group_sample(fvan_group* g, int grid, hipStream_t s) {
  return group_sample_n(g, grid, g->total_tiles, s);
}

// Re-tile the unit table for `tile` samples per workgroup and upload it (synchronous).
static hipError_t group_set_tile(fvan_group* g, int tile) {
  int t0 = 0;
  for (auto& d : g->host_table) {
    d.tile0 = t0;
    d.n_tiles = (d.B + tile - 1) / tile;
    t0 += d.n_tiles;
  }
  g->shape.tile = tile;
  g->total_tiles = t0;
  return hipMemcpy(g->d_table, g->host_table.data(), g->host_table.size() * sizeof(DecodeUnit),
                   hipMemcpyHostToDevice);
}

static int group_run_impl(fvan_group* g, hipStream_t s) {
  FVAN_HIP(group_sample(g, g->grid, s));
  if (g->ell_energy) {
    hipLaunchKernelGGL(group_energy_kernel, dim3((unsigned)g->total_samples), dim3(256), 0, s,
                       (const GroupEnergyUnit*)g->d_energy, (const int64_t*)g->d_first, g->n_units);
    FVAN_HIP(hipGetLastError());
  } else {
    for (int i = 0; i < g->n_units; ++i)
      FVAN_HIP(launch_energy(g->coup[i], g->units[i].batch, g->units[i].spins, g->units[i].energy, s));
  }
  hipLaunchKernelGGL(group_stats_kernel, dim3(g->n_units), dim3(256), 0, s, (const GroupStatUnit*)g->d_stats);
  FVAN_HIP(hipGetLastError());
  return FVAN_OK;
}

// Key of a group's launch shape: model shape, precision, compute units and a
// hash of the units' (N, W, P, batch) in table order.
static std::string group_tune_key(const fvan_group* g, int cus) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const auto& d : g->host_table) {
    mix(d.N); mix(d.W); mix(d.P); mix(d.B);
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "group_d%d_l%d_h%d_p%d_cu%d_u%d_%016llx", g->d_model, g->n_layers,
                g->shape.d_head, g->precision, cus, g->n_units, (unsigned long long)h);
  return buf;
}

// Choose (tile, grid): a persisted entry for this shape if there is one, else
// time every candidate on the same prefix of the work queue and persist the
// fastest.  fixed_tile (16 or 32) restricts the search to that tile.
static int autotune(fvan_group* g, int fixed_tile) {
  const int cus = device_cus(g->device);
  g->tune_key = group_tune_key(g, cus);
  std::vector<int> tiles;
  if (fixed_tile) {
    tiles.push_back(fixed_tile);
  } else {
    DecodeShape sh16 = g->shape;
    sh16.tile = 16;
    if (decode_has_tile16(sh16)) tiles.push_back(16);
    tiles.push_back(32);
  }
  const std::string path = tune_file_path();
  {
    std::lock_guard<std::mutex> lock(tune_mutex());
    const auto stored = tune_read(path);
    auto it = stored.find(g->tune_key);
    if (it != stored.end() && it->second.grid > 0 &&
        std::find(tiles.begin(), tiles.end(), it->second.tile) != tiles.end()) {
      FVAN_HIP(group_set_tile(g, it->second.tile));
      g->grid = std::min(it->second.grid, g->total_tiles);
      g->tuned_ms = it->second.ms;
      g->tuned_from_cache = true;
      return FVAN_OK;
    }
  }
  hipStream_t s;
  FVAN_HIP(hipStreamCreate(&s));
  hipEvent_t a, b;
  FVAN_HIP(hipEventCreate(&a));
  FVAN_HIP(hipEventCreate(&b));
  // the prefix every candidate runs: the first ~12 tiles of 32 samples per compute unit
  const int64_t prefix_samples = std::min<int64_t>(g->total_samples, (int64_t)cus * 32 * 12);
  float best = 1e30f;
  int best_tile = tiles.back(), best_grid = 0;
  for (int tile : tiles) {
    FVAN_HIP(group_set_tile(g, tile));
    const int n_pre = (int)std::min<int64_t>(g->total_tiles, (prefix_samples + tile - 1) / tile);
    std::vector<int> cand;
    for (int k : {1, 2, 4}) cand.push_back(std::min(n_pre, k * cus));
    const int64_t mall = (int64_t)(kMallBytes / std::max<size_t>(1, (size_t)tile * g->kv_sample_max));
    if (mall >= cus / 4 && mall < n_pre) cand.push_back((int)mall);
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    FVAN_HIP(group_sample_n(g, cand.front(), n_pre, s));   // loads this tile's kernel
    for (int grid : cand) {
      FVAN_HIP(hipEventRecord(a, s));
      FVAN_HIP(group_sample_n(g, grid, n_pre, s));
      FVAN_HIP(hipEventRecord(b, s));
      FVAN_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      FVAN_HIP(hipEventElapsedTime(&ms, a, b));
      // per sample, so tiles of 16 and 32 compare on the same prefix
      const float per = ms / (float)std::min<int64_t>(g->total_samples, (int64_t)n_pre * tile);
      if (std::getenv("FVAN_TUNE_LOG"))
        std::fprintf(stderr, "[fvan tune] %s tile %d grid %d: %.3f ms for %d work items (%.3f us per sample)\n",
                     g->tune_key.c_str(), tile, grid, ms, n_pre, 1e3 * per);
      if (per < best) {
        best = per;
        best_tile = tile;
        best_grid = grid;
      }
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  FVAN_HIP(group_set_tile(g, best_tile));
  g->grid = std::min(best_grid, g->total_tiles);
  g->tuned_ms = (double)best * (double)prefix_samples;
  g->tuned_from_cache = false;
  {
    std::lock_guard<std::mutex> lock(tune_mutex());
    auto stored = tune_read(path);
    stored[g->tune_key] = TuneEntry{best_tile, best_grid, g->tuned_ms};
    (void)tune_write(path, stored);          // best effort: an unwritable store only costs re-tuning
  }
  return FVAN_OK;
}

static void group_free(fvan_group* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->d_table) (void)hipFree(g->d_table);
  if (g->d_energy) (void)hipFree(g->d_energy);
  if (g->d_stats) (void)hipFree(g->d_stats);
  if (g->d_first) (void)hipFree(g->d_first);
  if (g->d_queue) (void)hipFree(g->d_queue);
}

}  // namespace fvan

using namespace fvan;

extern "C" {

int fvan_group_create(const fvan_group_unit* units, int32_t n_units, int32_t tile_samples, fvan_group** out) {
  if (!units || !out || n_units < 1) return fail(FVAN_EINVAL, "units and out must be non-NULL, n_units >= 1");
  *out = nullptr;
  if (tile_samples != 0 && tile_samples != 16 && tile_samples != 32)
    return fail(FVAN_EUNSUPPORTED, "tile_samples must be 0 (autotuned), 16 or 32");
  const fvan_model* m0 = units[0].model;
  if (!m0) return fail(FVAN_EINVAL, "unit 0 has no model");
  for (int i = 0; i < n_units; ++i)
    if (units[i].model && units[i].model->cfg.vocab != 2) return fail(FVAN_EUNSUPPORTED, kBinaryOnly);
  for (int i = 0; i < n_units; ++i)
    for (int j = 0; j < i; ++j)
      if (units[i].model == units[j].model)
        return fail(FVAN_EINVAL, "units " + std::to_string(j) + " and " + std::to_string(i) +
                                     " share a model; each unit needs its own (its K/V cache is per model)");
  fvan_group* g = new (std::nothrow) fvan_group();
  if (!g) return fail(FVAN_ENOMEM, "host allocation failed");
  g->d_model = m0->cfg.d_model;
  g->precision = m0->cfg.precision;
  g->n_layers = m0->cfg.n_layers;
  g->shape = decode_shape(m0->cfg);
  g->n_units = n_units;
  g->device = m0->device;
  g->units.assign(units, units + n_units);
  // longest sequences first: the persistent grid then ends on short work items
  std::vector<int> order(n_units);
  for (int i = 0; i < n_units; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return units[a].model && units[b].model && units[a].model->cfg.n_spins > units[b].model->cfg.n_spins;
  });
  std::vector<DecodeUnit> table;
  std::vector<GroupEnergyUnit> en(n_units);
  std::vector<GroupStatUnit> st(n_units);
  std::vector<int64_t> first(n_units);
  int tiles = 0;
  int64_t samples = 0;
  for (int k = 0; k < n_units; ++k) {
    const int i = order[k];
    const fvan_group_unit& u = units[i];
    const fvan_model* m = u.model;
    if (!m || !m->params || !m->synced || !u.couplings || !u.spins || !u.log_q || !u.energy || !u.stats) {
      delete g;
      return fail(FVAN_EINVAL, "unit " + std::to_string(i) + ": model not bound/synced or NULL buffer");
    }
    if (!has_sampler(m)) {
      delete g;
      return fail(FVAN_EUNSUPPORTED, "unit " + std::to_string(i) + ": " + kNoSampler);
    }
    if (m->cfg.d_model != g->d_model || m->cfg.precision != g->precision || m->cfg.n_heads != m0->cfg.n_heads) {
      delete g;
      return fail(FVAN_EINVAL, "unit " + std::to_string(i) + ": models of a group must share d_model, heads, precision");
    }
    if (u.batch < 1 || u.batch > m->cfg.max_batch || !(u.beta > 0.0) || u.couplings->n_spins != m->cfg.n_spins) {
      delete g;
      return fail(FVAN_EINVAL, "unit " + std::to_string(i) + ": batch, beta or couplings out of range");
    }
    DecodeUnit d = make_decode_unit(m, u.batch, u.seed, u.stream_id, u.spins, u.log_q, m->kv, tiles, 32);
    tiles += d.n_tiles;
    table.push_back(d);
    g->kv_sample_max = std::max(g->kv_sample_max, m->kv_bytes / (size_t)m->cfg.max_batch);
    g->coup.push_back(*u.couplings);
    if (u.couplings->kind == FVAN_BONDS_DENSE || u.couplings->n_spins > 4096) g->ell_energy = false;
    en[k] = GroupEnergyUnit{m->cfg.n_spins, u.couplings->kind, u.couplings->degree, u.batch, u.couplings->nbr,
                            u.couplings->J, u.spins, u.energy};
    st[k] = GroupStatUnit{m->cfg.n_spins, u.batch, u.couplings->kind == FVAN_BONDS_PM1 ? 1 : 0, u.beta, u.energy,
                          u.log_q, u.stats};
    first[k] = samples;
    samples += u.batch;
  }
  // keep g->units / g->coup in table order for the per-unit fallback path
  std::vector<fvan_group_unit> ord_units(n_units);
  for (int k = 0; k < n_units; ++k) ord_units[k] = units[order[k]];
  g->units = ord_units;
  g->total_tiles = tiles;
  g->total_samples = samples;
  hipError_t e = hipMalloc(&g->d_table, table.size() * sizeof(DecodeUnit));
  if (e == hipSuccess) e = hipMalloc(&g->d_energy, n_units * sizeof(GroupEnergyUnit));
  if (e == hipSuccess) e = hipMalloc(&g->d_stats, n_units * sizeof(GroupStatUnit));
  if (e == hipSuccess) e = hipMalloc(&g->d_first, n_units * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&g->d_queue, sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(g->d_table, table.data(), table.size() * sizeof(DecodeUnit), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_energy, en.data(), n_units * sizeof(GroupEnergyUnit), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_stats, st.data(), n_units * sizeof(GroupStatUnit), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_first, first.data(), n_units * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    group_free(g);
    delete g;
    return fail(FVAN_ENOMEM, std::string("group tables: ") + hipGetErrorString(e));
  }
  g->host_table = table;
  if (tile_samples == 16) {
    DecodeShape sh16 = g->shape;
    sh16.tile = 16;
    if (!decode_has_tile16(sh16)) {
      group_free(g);
      delete g;
      return fail(FVAN_EUNSUPPORTED, "no 16-sample decode tile for this model shape");
    }
  }
  int rc = autotune(g, tile_samples);
  if (rc) {
    group_free(g);
    delete g;
    return rc;
  }
  *out = g;
  return FVAN_OK;
}

int fvan_group_launch_shape(const fvan_group* g, int32_t* tile, int32_t* grid, int32_t* from_store, double* ms) {
  if (!g) return fail(FVAN_EINVAL, "group is NULL");
  if (tile) *tile = g->shape.tile;
  if (grid) *grid = g->grid;
  if (from_store) *from_store = g->tuned_from_cache ? 1 : 0;
  if (ms) *ms = g->tuned_ms;
  return FVAN_OK;
}

int fvan_group_destroy(fvan_group* g) {
  if (!g) return fail(FVAN_EINVAL, "group is NULL");
  group_free(g);
  delete g;
  return FVAN_OK;
}

int fvan_group_run(fvan_group* g, void* stream) {
  if (!g) return fail(FVAN_EINVAL, "group is NULL");
  return group_run_impl(g, (hipStream_t)stream);
}

int fvan_group_run_graph(fvan_group* g, void* stream) {
  if (!g) return fail(FVAN_EINVAL, "group is NULL");
  if (!g->exec) {
    if (!g->cap_stream) FVAN_HIP(hipStreamCreate(&g->cap_stream));
    FVAN_HIP(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = group_run_impl(g, g->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    FVAN_HIP(e);
    g->graph = graph;
    FVAN_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  }
  FVAN_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return FVAN_OK;
}

}  // extern "C"
