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
// The persistent grid size is chosen by a small autotuner that times the
// sampling launch for a few grid sizes and keeps the fastest; results are
// cached per (d_model, n_layers, precision, work items) for the process.
#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "device_common.h"
#include "fvan_model.h"

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

static std::map<std::tuple<int, int, int, int>, int>& tuned_grids() {
  static std::map<std::tuple<int, int, int, int>, int> m;
  return m;
}

static hipError_t group_sample(fvan_group* g, int grid, hipStream_t s) {
  hipError_t e = launch_zero_int(g->d_queue, 1, s);
  if (e != hipSuccess) return e;
  return launch_decode(g->shape, g->d_table, g->n_units, g->total_tiles, g->d_queue, grid, s);
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

// Time the sampling launch at a few persistent grid sizes; keep the fastest.
static int autotune_grid(fvan_group* g) {
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const auto key = std::make_tuple(g->d_model, g->n_layers, g->precision, g->total_tiles);
  auto it = tuned_grids().find(key);
  if (it != tuned_grids().end()) {
    g->grid = it->second;
    return FVAN_OK;
  }
  std::vector<int> cand;
  for (int k : {1, 2, 3, 4}) cand.push_back(std::min(g->total_tiles, k * cus));
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  hipStream_t s;
  FVAN_HIP(hipStreamCreate(&s));
  hipEvent_t a, b;
  FVAN_HIP(hipEventCreate(&a));
  FVAN_HIP(hipEventCreate(&b));
  float best = 1e30f;
  int best_grid = cand.back();
  for (int grid : cand) {
    FVAN_HIP(group_sample(g, grid, s));     // warm
    FVAN_HIP(hipEventRecord(a, s));
    FVAN_HIP(group_sample(g, grid, s));
    FVAN_HIP(hipEventRecord(b, s));
    FVAN_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    FVAN_HIP(hipEventElapsedTime(&ms, a, b));
    if (ms < best) {
      best = ms;
      best_grid = grid;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  g->grid = best_grid;
  tuned_grids()[key] = best_grid;
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
  if (tile_samples != 0 && tile_samples != decode_tile_samples())
    return fail(FVAN_EUNSUPPORTED, "tile_samples must be 0 or " + std::to_string(decode_tile_samples()));
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
    DecodeUnit d = make_decode_unit(m, u.batch, u.seed, u.stream_id, u.spins, u.log_q, m->kv, tiles);
    tiles += d.n_tiles;
    table.push_back(d);
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
  int rc = autotune_grid(g);
  if (rc) {
    group_free(g);
    delete g;
    return rc;
  }
  *out = g;
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
