// Batched evaluation of a population whose genomes differ widely in size.
//
// Padding every genome to the largest one wastes memory and time (the
// space-time trade-off of the tensorized encoding, TensorNEAT Section 3.3);
// one launch per genome size wastes the chip on small launches. A plan sorts
// the genomes once into length buckets by the on-chip rows their forward pass
// needs (tn_transformed.prog_rows / n_rows):
//   prog_rows <= 50, 100, 128, 160, 200   register engine, a register file of
//                                         that many rows per tile (50: four
//                                         tiles of 64 observations per
//                                         wavefront, 100: two), for B >= 256;
//                                         fewer tiles per wavefront (and the
//                                         one-tile sizes 32, 64, 96) for B
//                                         spanning fewer tiles
//   larger: n_rows <= 256, <= the LDS capacity   level-parallel LDS engine
// and orders each bucket longest first. Two ways to run it:
//   tn_plan_forward_buckets  one plain launch per bucket, in order;
//   tn_plan_forward          one persistent kernel per bucket (workgroups or
//                            wavefronts take genomes / tiles from a counter,
//                            longest first), all captured once into a hipGraph
//                            whose buckets are independent branches, replayed
//                            with a single launch.
// Both call the same per-tile arithmetic, so their outputs are bitwise equal
// to each other and to tn_forward. tn_plan_tune times the tile candidates of
// every bucket and keeps the fastest, with an optional text cache file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fwd_launch.hpp"
#include "tn_internal.hpp"

namespace {

struct Bucket {
  int engine = TN_ENGINE_REG;
  int rows_class = 32;  // REG: register-file rows (bound of prog_rows); LDS: bound of n_rows
  int count = 0;
  int max_rows = 0;     // LDS: largest n_rows in the bucket (the tile's rows)
  int64_t edges = 0;    // enabled edges over the bucket
  int K = 1, waves = 4; // tile
  int grid = 0;         // workgroups of the persistent kernel
  int32_t* list = nullptr;  // device: genome indices, longest first
};

__global__ void zero_counters(int32_t* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

constexpr int kCountersPerBucket = 8;  // the register engine's XCD shares

}  // namespace

struct tn_plan {
  tn_population pop;
  tn_transformed tr;
  int B = 0;
  int device = 0;
  std::vector<Bucket> buckets;
  int32_t* d_lists = nullptr;
  int32_t* d_counters = nullptr;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;
  hipGraphExec_t exec = nullptr;
  const float* g_obs = nullptr;
  int64_t g_stride = -1;
  float* g_out = nullptr;
};

namespace {

using tn::record_hip;

// Resident workgroups of the bucket's persistent kernel, capped by its work.
int persistent_grid(const tn_plan& pl, const Bucket& b) {
  if (b.engine == TN_ENGINE_REG) {
    const int kt = tn::rf_tiles_of(b.rows_class);  // tiles per wavefront
    const int64_t items = (int64_t)b.count * (((pl.B + tn::kWave - 1) / tn::kWave + kt - 1) / kt);
    const int64_t need = (items + b.waves - 1) / b.waves;
    return (int)std::min<int64_t>(tn::reg_queue_grid(b.rows_class, b.waves, pl.pop.n_in), need);
  }
  return std::min(tn::lds_queue_grid(pl.pop, b.K, b.waves, b.max_rows), b.count);
}

// One bucket: the plain grid launch, or (counter != nullptr) the persistent
// kernel with b.grid workgroups.
int launch_bucket(const tn_plan& pl, const Bucket& b, const float* obs, int64_t stride, float* out,
                  int32_t* counter, hipStream_t s) {
  tn::FwdWork w;
  w.genomes = b.list;
  w.n_genomes = b.count;
  if (counter) {
    if (b.grid <= 0) return TN_EHIP;
    w.queue = counter;
    w.grid = b.grid;
  }
  if (b.engine == TN_ENGINE_REG) {
    tn::RegTile t;
    t.waves = b.waves;
    t.rf = b.rows_class;
    return tn::launch_forward_reg(pl.pop, pl.tr, obs, stride, pl.B, out, t, w, s);
  }
  tn::LdsTile t;
  t.K = b.K;
  t.waves = b.waves;
  t.rows = b.max_rows;
  return tn::launch_forward(pl.pop, pl.tr, obs, stride, pl.B, out, t, w, s);
}

void drop_graph(tn_plan& pl) {
  if (pl.exec) (void)hipGraphExecDestroy(pl.exec);
  pl.exec = nullptr;
  pl.g_obs = nullptr;
  pl.g_out = nullptr;
  pl.g_stride = -1;
}

// Captures: zero the counters (a kernel, not a memset node), then every
// bucket's persistent kernel on a branch of its own, joined at the end.
int build_graph(tn_plan& pl, const float* obs, int64_t stride, float* out) {
  drop_graph(pl);
  const int nb = (int)pl.buckets.size();
  for (Bucket& b : pl.buckets) {  // device queries stay outside the capture
    b.grid = persistent_grid(pl, b);
    if (b.grid <= 0) return TN_EHIP;
  }
  int rc = record_hip(hipStreamBeginCapture(pl.cap, hipStreamCaptureModeThreadLocal));
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, pl.cap, pl.d_counters,
                     nb * kCountersPerBucket);
  rc = tn::check_launch();
  if (rc == TN_OK) rc = record_hip(hipEventRecord(pl.ev[0], pl.cap));
  for (int i = 0; i < nb && rc == TN_OK; ++i) {
    rc = record_hip(hipStreamWaitEvent(pl.side[i], pl.ev[0], 0));
    if (rc == TN_OK)
      rc = launch_bucket(pl, pl.buckets[i], obs, stride, out,
                         pl.d_counters + i * kCountersPerBucket, pl.side[i]);
    if (rc == TN_OK) rc = record_hip(hipEventRecord(pl.ev[i + 1], pl.side[i]));
    if (rc == TN_OK) rc = record_hip(hipStreamWaitEvent(pl.cap, pl.ev[i + 1], 0));
  }
  hipGraph_t graph = nullptr;
  const int rc_end = record_hip(hipStreamEndCapture(pl.cap, &graph));
  if (rc == TN_OK) rc = rc_end;
  if (rc == TN_OK) rc = record_hip(hipGraphInstantiate(&pl.exec, graph, nullptr, nullptr, 0));
  if (graph) (void)hipGraphDestroy(graph);
  if (rc != TN_OK) {
    pl.exec = nullptr;
    return rc;
  }
  pl.g_obs = obs;
  pl.g_stride = stride;
  pl.g_out = out;
  return TN_OK;
}

std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

int ilog2(int64_t x) {
  int r = 0;
  while (x > 1) {
    x >>= 1;
    ++r;
  }
  return r;
}

// Cache key of a bucket: device, engine class, io shape, batch, and the
// bucket's size and mean edge count on a log2 scale.
std::string cache_key(const tn_plan& pl, const Bucket& b) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s e%d r%d i%d o%d B%d n%d c%d", arch_name(pl.device).c_str(),
                b.engine, b.rows_class, pl.pop.n_in, pl.pop.n_out, pl.B, ilog2(b.count),
                ilog2(b.count ? b.edges / b.count : 0));
  return buf;
}

// Cache file: one line per bucket class, "<key> = <K> <waves>".
std::map<std::string, std::pair<int, int>> read_cache(const char* path) {
  std::map<std::string, std::pair<int, int>> m;
  if (!path || !*path) return m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char* eq = std::strstr(line, " = ");
    if (!eq) continue;
    int K = 0, W = 0;
    if (std::sscanf(eq + 3, "%d %d", &K, &W) != 2) continue;
    if ((K != 1 && K != 2 && K != 4) || W < 1 || W > tn::lds_max_waves(K)) continue;
    m[std::string(line, eq)] = {K, W};
  }
  std::fclose(f);
  return m;
}

int write_cache(const char* path, const std::map<std::string, std::pair<int, int>>& m) {
  if (!path || !*path) return TN_OK;
  FILE* f = std::fopen(path, "w");
  if (!f) return TN_EINVAL;
  for (const auto& kv : m) std::fprintf(f, "%s = %d %d\n", kv.first.c_str(), kv.second.first,
                                        kv.second.second);
  return std::fclose(f) == 0 ? TN_OK : TN_EINVAL;
}

void apply_cache(tn_plan& pl, const char* path) {
  const auto m = read_cache(path);
  for (Bucket& b : pl.buckets) {
    const auto it = m.find(cache_key(pl, b));
    if (it == m.end()) continue;
    if (b.engine == TN_ENGINE_REG && (it->second.first != 1 || it->second.second > 8)) continue;
    if (b.engine == TN_ENGINE_LDS && tn::lds_tile_bytes(pl.pop, it->second.first, b.max_rows) == 0)
      continue;
    b.K = it->second.first;
    b.waves = it->second.second;
  }
}

void destroy(tn_plan* pl) {
  if (!pl) return;
  drop_graph(*pl);
  for (hipStream_t s : pl->side) (void)hipStreamDestroy(s);
  if (pl->cap) (void)hipStreamDestroy(pl->cap);
  for (hipEvent_t e : pl->ev) (void)hipEventDestroy(e);
  if (pl->d_lists) (void)hipFree(pl->d_lists);
  if (pl->d_counters) (void)hipFree(pl->d_counters);
  delete pl;
}

template <class T>
int to_host(std::vector<T>& v, const T* d, int64_t n, hipStream_t s) {
  v.resize((size_t)std::max<int64_t>(n, 1));
  if (n == 0) return TN_OK;
  int rc = record_hip(hipMemcpyAsync(v.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  return rc;
}

int check_plan_call(const tn_plan* pl, const float* obs, int64_t stride, const float* out) {
  if (!pl) return TN_EINVAL;
  int rc = tn::check_obs(&pl->pop, obs, stride, pl->B);
  if (rc != TN_OK) return rc;
  if (pl->B > 0 && pl->pop.P > 0 && !out) return TN_EINVAL;
  return TN_OK;
}

}  // namespace

extern "C" {

int tn_plan_create(const tn_population* pop, const tn_transformed* tr, int32_t B,
                   const char* tune_cache, tn_plan** plan, hipStream_t stream) {
  if (!plan) return TN_EINVAL;
  *plan = nullptr;
  int rc = tn::check_population(pop);
  if (rc != TN_OK) return rc;
  rc = tn::check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (B < 0) return TN_EINVAL;
  tn_plan* pl = new (std::nothrow) tn_plan;
  if (!pl) return TN_ENOMEM;
  pl->pop = *pop;
  pl->tr = *tr;
  pl->B = B;
  rc = record_hip(hipGetDevice(&pl->device));
  const int P = pop->P;
  const bool ragged = pop->node_off != nullptr;
  // per-genome sizes, read back once
  std::vector<int32_t> status, prog_rows, n_rows, n_valid, row_ptr;
  std::vector<int64_t> node_off;
  const int64_t rowptr_elems = (ragged ? pop->total_nodes : (int64_t)P * pop->N_max) + P;
  if (rc == TN_OK) rc = to_host(status, tr->status, P, stream);
  if (rc == TN_OK) rc = to_host(prog_rows, tr->prog_rows, P, stream);
  if (rc == TN_OK) rc = to_host(n_rows, tr->n_rows, P, stream);
  if (rc == TN_OK) rc = to_host(n_valid, tr->n_valid, P, stream);
  if (rc == TN_OK) rc = to_host(row_ptr, tr->row_ptr, P ? rowptr_elems : 0, stream);
  if (rc == TN_OK && ragged) rc = to_host(node_off, pop->node_off, P + 1, stream);
  if (rc == TN_OK) rc = record_hip(hipStreamSynchronize(stream));
  if (rc != TN_OK) {
    destroy(pl);
    return rc;
  }
  // buckets
  const int cap = tn::lds_rows_cap(*pop);
  std::vector<Bucket> classes;
  int reg_cls[6];
  const int n_reg = tn::reg_classes(B, reg_cls);
  for (int i = 0; i < n_reg; ++i) {
    Bucket b;
    b.engine = TN_ENGINE_REG;
    b.rows_class = reg_cls[i];
    classes.push_back(b);
  }
  std::vector<int> bounds;
  for (int r : {256, cap})
    if (std::min(r, cap) > tn::kRegRowsMax) bounds.push_back(std::min(r, cap));
  bounds.erase(std::unique(bounds.begin(), bounds.end()), bounds.end());
  for (int r : bounds) {
    Bucket b;
    b.engine = TN_ENGINE_LDS;
    b.rows_class = r;
    classes.push_back(b);
  }
  std::vector<std::vector<std::pair<int64_t, int>>> members(classes.size());
  for (int g = 0; g < P; ++g) {
    const int64_t rb = ragged ? (int64_t)node_off[g] + g : (int64_t)g * (pop->N_max + 1);
    const int64_t edges = status[g] ? 0 : row_ptr[rb + n_valid[g]];
    const int64_t cost = edges + n_valid[g];
    int c = -1;
    if (status[g]) {
      c = 0;
    } else {
      for (int k = 0; k < n_reg && c < 0; ++k)
        if (prog_rows[g] <= classes[k].rows_class) c = k;
      for (size_t k = n_reg; k < classes.size() && c < 0; ++k)
        if (n_rows[g] <= classes[k].rows_class) c = (int)k;
    }
    if (c < 0) {  // more value rows than the LDS engine holds
      destroy(pl);
      return TN_EUNSUPPORTED;
    }
    members[c].push_back({cost, g});
    classes[c].edges += edges;
    if (classes[c].engine == TN_ENGINE_LDS) classes[c].max_rows = std::max(classes[c].max_rows, n_rows[g]);
  }
  std::vector<int32_t> lists;
  std::vector<size_t> offs;
  for (size_t k = 0; k < classes.size(); ++k) {
    if (members[k].empty()) continue;
    // longest first; ties by genome index, so the plan is deterministic
    std::sort(members[k].begin(), members[k].end(),
              [](const std::pair<int64_t, int>& a, const std::pair<int64_t, int>& b) {
                return a.first != b.first ? a.first > b.first : a.second < b.second;
              });
    Bucket b = classes[k];
    b.count = (int)members[k].size();
    if (b.engine == TN_ENGINE_REG) b.K = 1;
    offs.push_back(lists.size());
    for (const auto& m : members[k]) lists.push_back(m.second);
    pl->buckets.push_back(b);
  }
  const int nb = (int)pl->buckets.size();
  if (nb > 0) {
    rc = record_hip(hipMalloc(&pl->d_lists, sizeof(int32_t) * lists.size()));
    if (rc == TN_OK)
      rc = record_hip(hipMalloc(&pl->d_counters, sizeof(int32_t) * nb * kCountersPerBucket));
    if (rc == TN_OK)
      rc = record_hip(hipMemcpy(pl->d_lists, lists.data(), sizeof(int32_t) * lists.size(),
                                hipMemcpyHostToDevice));
    for (int i = 0; i < nb; ++i) pl->buckets[i].list = pl->d_lists + offs[i];
  }
  if (rc == TN_OK) rc = record_hip(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking));
  for (int i = 0; i < nb && rc == TN_OK; ++i) {
    hipStream_t s = nullptr;
    rc = record_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    if (rc == TN_OK) pl->side.push_back(s);
  }
  for (int i = 0; i <= nb && rc == TN_OK; ++i) {
    hipEvent_t e = nullptr;
    rc = record_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (rc == TN_OK) pl->ev.push_back(e);
  }
  if (rc != TN_OK) {
    destroy(pl);
    return rc == TN_EHIP && tn_last_error()[0] ? rc : TN_ENOMEM;
  }
  apply_cache(*pl, tune_cache);
  *plan = pl;
  return TN_OK;
}

void tn_plan_destroy(tn_plan* plan) { destroy(plan); }

int tn_plan_num_buckets(const tn_plan* plan) { return plan ? (int)plan->buckets.size() : 0; }

int tn_plan_bucket(const tn_plan* plan, int32_t i, tn_bucket_info* info) {
  if (!plan || !info || i < 0 || i >= (int)plan->buckets.size()) return TN_EINVAL;
  const Bucket& b = plan->buckets[i];
  info->engine = b.engine;
  info->rows_class = b.rows_class;
  info->count = b.count;
  info->edges = b.edges;
  info->tile.engine = b.engine;
  info->tile.obs_per_lane = b.K;
  info->tile.waves_per_genome = b.waves;
  info->tile.rows = b.engine == TN_ENGINE_REG ? b.rows_class : b.max_rows;
  return TN_OK;
}

int tn_plan_set_tile(tn_plan* plan, int32_t i, int32_t obs_per_lane, int32_t waves) {
  if (!plan || i < 0 || i >= (int)plan->buckets.size() || waves < 1) return TN_EINVAL;
  Bucket& b = plan->buckets[i];
  if (waves > (b.engine == TN_ENGINE_REG ? 8 : tn::lds_max_waves(obs_per_lane))) return TN_EINVAL;
  if (b.engine == TN_ENGINE_REG ? obs_per_lane != 1
                                : (obs_per_lane != 1 && obs_per_lane != 2 && obs_per_lane != 4))
    return TN_EINVAL;
  if (b.engine == TN_ENGINE_LDS && tn::lds_tile_bytes(plan->pop, obs_per_lane, b.max_rows) == 0)
    return TN_EUNSUPPORTED;
  b.K = obs_per_lane;
  b.waves = waves;
  drop_graph(*plan);
  return TN_OK;
}

int tn_plan_forward_buckets(tn_plan* plan, const float* obs, int64_t obs_genome_stride, float* out,
                            hipStream_t stream) {
  int rc = check_plan_call(plan, obs, obs_genome_stride, out);
  if (rc != TN_OK || plan->B == 0) return rc;
  for (const Bucket& b : plan->buckets) {
    rc = launch_bucket(*plan, b, obs, obs_genome_stride, out, nullptr, stream);
    if (rc != TN_OK) return rc;
  }
  return TN_OK;
}

int tn_plan_forward(tn_plan* plan, const float* obs, int64_t obs_genome_stride, float* out,
                    hipStream_t stream) {
  int rc = check_plan_call(plan, obs, obs_genome_stride, out);
  if (rc != TN_OK || plan->B == 0 || plan->buckets.empty()) return rc;
  if (!plan->exec || plan->g_obs != obs || plan->g_out != out ||
      plan->g_stride != obs_genome_stride) {
    rc = build_graph(*plan, obs, obs_genome_stride, out);
    if (rc != TN_OK) return rc;
  }
  return record_hip(hipGraphLaunch(plan->exec, stream));
}

int tn_plan_forward_bucket(tn_plan* plan, int32_t i, int32_t persistent, const float* obs,
                           int64_t obs_genome_stride, float* out, hipStream_t stream) {
  int rc = check_plan_call(plan, obs, obs_genome_stride, out);
  if (rc != TN_OK) return rc;
  if (i < 0 || i >= (int)plan->buckets.size()) return TN_EINVAL;
  if (plan->B == 0) return TN_OK;
  Bucket& b = plan->buckets[i];
  if (!persistent) return launch_bucket(*plan, b, obs, obs_genome_stride, out, nullptr, stream);
  b.grid = persistent_grid(*plan, b);
  if (b.grid <= 0) return TN_EHIP;
  int32_t* counters = plan->d_counters + i * kCountersPerBucket;
  hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, stream, counters, kCountersPerBucket);
  rc = tn::check_launch();
  if (rc != TN_OK) return rc;
  return launch_bucket(*plan, b, obs, obs_genome_stride, out, counters, stream);
}

int tn_plan_tune(tn_plan* plan, const float* obs, int64_t obs_genome_stride, float* out,
                 const char* tune_cache, hipStream_t stream) {
  int rc = check_plan_call(plan, obs, obs_genome_stride, out);
  if (rc != TN_OK || plan->B == 0) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rc = record_hip(hipEventCreate(&e0));
  if (rc == TN_OK) rc = record_hip(hipEventCreate(&e1));
  auto cache = read_cache(tune_cache);
  for (size_t i = 0; i < plan->buckets.size() && rc == TN_OK; ++i) {
    Bucket& b = plan->buckets[i];
    std::vector<std::pair<int, int>> cand;
    for (int W : {1, 2, 4, 8, 16}) {
      if (b.engine == TN_ENGINE_REG) {
        if (W <= 8) cand.push_back({1, W});
      } else {
        for (int K : {1, 2, 4})
          if (W <= tn::lds_max_waves(K) && tn::lds_tile_bytes(plan->pop, K, b.max_rows) > 0)
            cand.push_back({K, W});
      }
    }
    float best = INFINITY;
    std::pair<int, int> pick{b.K, b.waves};
    for (const auto& c : cand) {
      b.K = c.first;
      b.waves = c.second;
      // the persistent form, as the graph runs it (grid sized for this tile)
      b.grid = persistent_grid(*plan, b);
      if (b.grid <= 0) {
        rc = TN_EHIP;
        break;
      }
      int32_t* counters = plan->d_counters + i * kCountersPerBucket;
      float ms = INFINITY;
      for (int rep = 0; rep < 6 && rc == TN_OK; ++rep) {  // the first run warms up
        hipLaunchKernelGGL(zero_counters, dim3(1), dim3(64), 0, stream, counters,
                           kCountersPerBucket);
        rc = tn::check_launch();
        if (rc == TN_OK) rc = record_hip(hipEventRecord(e0, stream));
        if (rc == TN_OK) rc = launch_bucket(*plan, b, obs, obs_genome_stride, out, counters, stream);
        if (rc == TN_OK) rc = record_hip(hipEventRecord(e1, stream));
        if (rc == TN_OK) rc = record_hip(hipEventSynchronize(e1));
        float t = 0.0f;
        if (rc == TN_OK) rc = record_hip(hipEventElapsedTime(&t, e0, e1));
        if (rc == TN_OK && rep > 0) ms = std::min(ms, t);
      }
      if (rc != TN_OK) break;
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    b.K = pick.first;
    b.waves = pick.second;
    b.grid = persistent_grid(*plan, b);
    cache[cache_key(*plan, b)] = pick;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  drop_graph(*plan);
  if (rc != TN_OK) return rc;
  return write_cache(tune_cache, cache);
}

}  // extern "C"
