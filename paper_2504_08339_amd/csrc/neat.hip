// One NEAT generation on the device (Algorithm 1's loop body: divide the
// population into species by distance, decide each species' number of
// children from the fitness, make them by crossover and mutation) and the
// initial population (Algorithm 1's first step); hyperparameters of Appendix
// A. The paper names these steps, not their rules; the rules implemented are
// stated at tn_neat_generation in the public header.
//
// Launches of one generation, all on the caller's stream:
//   prep (x2)   sorted gene lists of the population and of the species
//               representatives (the node-inclusive distance's genes);
//   speciate    one workgroup: every genome against the representatives
//               (threads over genomes), then the unassigned genomes in index
//               order (founders' distances on threads over slots), then the
//               species fitness, stagnation and offspring counts (one thread,
//               in slot order, float32 as specified);
//   rank        thread per genome: its rank in its species, scattered into
//               the member order;
//   parents     thread per child: elites, then two survivor picks;
//   reproduce   the crossover / mutation kernels;
//   table       workgroup per slot: next representatives and slot state.
// Every float decision (distance below the threshold, nearest species,
// counts) uses float32 operations in a fixed order with no contraction.
#include <algorithm>
#include <cmath>

#include "genes.hpp"
#include "tn_internal.hpp"

#pragma clang fp contract(off)

namespace tn {

size_t reproduce_workspace_bytes(int n);
int launch_reproduce(const tn_population& p, int n, const int32_t* parents, const float* U,
                     const float* Z, const tn_mutation_params& prm, int32_t next_key,
                     const tn_population_arrays& out, int32_t* next_key_out, void* workspace,
                     hipStream_t stream);

namespace {

constexpr int kBlock = 256;
constexpr int kMaxSpecies = TN_NEAT_MAX_SPECIES;

struct NeatWs {
  WsN pop;             // gene lists of the population
  WsN reps;            // gene lists of the representatives
  int32_t* sp;         // [P] species slot of each genome
  int32_t* order;      // [P] genomes by slot, then rank
  int32_t* parents;    // [P][2]
  int32_t* member_off; // [S + 1]
  int32_t* child_off;  // [S + 1]
  int32_t* counts;     // [S]
  int32_t* nmem;       // [S]
  int32_t* surv;       // [S]
  float* best;         // [S] updated best species fitness
  int32_t* last;       // [S] updated generation of the last improvement
  void* repro;         // workspace of the reproduction kernels
};

struct Table {
  int32_t* alive;
  float* best;
  int32_t* last;
  int32_t* size;
  tn_population_arrays reps;
};

size_t ws_bytes(int P, int S, int N, int C) {
  return ws_nodes_bytes(P, N, C) + ws_nodes_bytes(S, N, C) + 4 * gene_align(4 * (size_t)P) +
         8 * gene_align(4 * (size_t)(S + 1)) + gene_align(reproduce_workspace_bytes(P));
}

NeatWs carve(void* base, int P, int S, int N, int C) {
  unsigned char* p = (unsigned char*)base;
  size_t o = 0;
  NeatWs w;
  w.pop = carve_nodes(p + o, P, N, C);
  o += ws_nodes_bytes(P, N, C);
  w.reps = carve_nodes(p + o, S, N, C);
  o += ws_nodes_bytes(S, N, C);
  auto ints = [&](size_t n) {
    int32_t* q = (int32_t*)(p + o);
    o += gene_align(4 * n);
    return q;
  };
  w.sp = ints(P);
  w.order = ints(P);
  w.parents = ints(2 * (size_t)P);
  w.member_off = ints(S + 1);
  w.child_off = ints(S + 1);
  w.counts = ints(S + 1);
  w.nmem = ints(S + 1);
  w.surv = ints(S + 1);
  w.best = (float*)ints(S + 1);
  w.last = ints(S + 1);
  w.repro = p + o;
  return w;
}

__device__ __forceinline__ float draw(float mean, float std_, float z) {
  const float t = std_ * z;
  return mean + t;
}

__global__ __launch_bounds__(kBlock) void init_kernel(int n_in, int n_out, int N, int C,
                                                      const float* Z, int64_t nZ,
                                                      tn_mutation_params m,
                                                      tn_population_arrays out) {
  const int g = blockIdx.x;
  const float* z = Z + (int64_t)g * nZ;
  const int nio = n_in + n_out;
  const int64_t nb = (int64_t)g * N, cb = (int64_t)g * C;
  for (int r = threadIdx.x; r < N; r += kBlock) {
    const bool v = r < nio;
    out.node_key[nb + r] = v ? r : -1;
    out.node_bias[nb + r] = v ? draw(m.bias_init_mean, m.bias_init_std, z[4 + 2 * r]) : 0.0f;
    out.node_resp[nb + r] = v ? draw(m.resp_init_mean, m.resp_init_std, z[4 + 2 * r + 1]) : 0.0f;
    out.node_act[nb + r] = v ? (uint8_t)m.act_default : 0;
    out.node_agg[nb + r] = v ? (uint8_t)m.agg_default : 0;
  }
  for (int r = threadIdx.x; r < C; r += kBlock) {
    const bool v = r < n_in * n_out;
    out.conn_in[cb + r] = v ? r / n_out : -1;
    out.conn_out[cb + r] = v ? n_in + r % n_out : -1;
    out.conn_w[cb + r] =
        v ? draw(m.weight_init_mean, m.weight_init_std, z[4 + 2 * (int64_t)N + r]) : 0.0f;
    out.conn_en[cb + r] = v ? 1 : 0;
  }
}

__global__ __launch_bounds__(kBlock) void clear_table_kernel(Table t, int N, int C) {
  const int s = blockIdx.x;
  if (threadIdx.x == 0) {
    t.alive[s] = 0;
    t.best[s] = -INFINITY;
    t.last[s] = 0;
    t.size[s] = 0;
  }
  const int64_t nb = (int64_t)s * N, cb = (int64_t)s * C;
  for (int r = threadIdx.x; r < N; r += kBlock) {
    t.reps.node_key[nb + r] = -1;
    t.reps.node_bias[nb + r] = t.reps.node_resp[nb + r] = 0.0f;
    t.reps.node_act[nb + r] = t.reps.node_agg[nb + r] = 0;
  }
  for (int r = threadIdx.x; r < C; r += kBlock) {
    t.reps.conn_in[cb + r] = t.reps.conn_out[cb + r] = -1;
    t.reps.conn_w[cb + r] = 0.0f;
    t.reps.conn_en[cb + r] = 0;
  }
}

// (c_d * D + c_h * H) / max(n1, n2) of one gene kind by a merge of the two
// sorted lists: H summed in ascending key order, each term
// ((|da0| + |da1|) + [c0 differ]) + [c1 differ].
__device__ float kind_term(const GeneList& A, int PA, int a, int na, const GeneList& B, int PB,
                           int b, int nb, float c_d, float c_h) {
  const int n = max(na, nb);
  if (n == 0) return 0.0f;
  int i = 0, j = 0, hom = 0;
  float H = 0.0f;
  while (i < na && j < nb) {
    const int64_t oa = (int64_t)i * PA + a, ob = (int64_t)j * PB + b;
    const long long ka = A.keyT[oa], kb = B.keyT[ob];
    if (ka < kb) {
      ++i;
    } else if (kb < ka) {
      ++j;
    } else {
      float t = fabsf(A.a0T[oa] - B.a0T[ob]) + fabsf(A.a1T[oa] - B.a1T[ob]);
      const uint32_t ca = A.codeT[oa], cb = B.codeT[ob];
      t = t + ((ca & 0xffu) != (cb & 0xffu) ? 1.0f : 0.0f);
      t = t + ((ca >> 8) != (cb >> 8) ? 1.0f : 0.0f);
      H = H + t;
      ++hom;
      ++i;
      ++j;
    }
  }
  const float x = c_d * (float)(na + nb - 2 * hom);
  const float y = c_h * H;
  const float num = x + y;
  return num / (float)n;
}

// Node-inclusive distance of genome a of A and genome b of B (NaN when either
// has no gene set).
__device__ float pair_distance(const WsN& A, int PA, int a, const WsN& B, int PB, int b,
                               float c_d, float c_h) {
  const int an = A.cnt_n[a], bn = B.cnt_n[b];
  if (an < 0 || bn < 0) return __builtin_nanf("");
  const float tn = kind_term(A.nodes, PA, a, an, B.nodes, PB, b, bn, c_d, c_h);
  const float tc = kind_term(A.conns, PA, a, A.cnt_c[a], B.conns, PB, b, B.cnt_c[b], c_d, c_h);
  float total = 0.0f;
  total = total + tn;
  total = total + tc;
  return total;
}

struct SpecArgs {
  int P, S, gen;
  float thr, c_d, c_h;
  int species_elitism, max_stagnation;
  float rate;
};

__global__ __launch_bounds__(kBlock) void speciate_kernel(NeatWs ws, Table t, const float* fit,
                                                          SpecArgs a) {
  __shared__ int alive[kMaxSpecies];
  __shared__ int founder[kMaxSpecies];
  __shared__ float dsh[kMaxSpecies];
  __shared__ int nfree;
  __shared__ int smin_valid;
  __shared__ float smax[kMaxSpecies], smin[kMaxSpecies], ssum[kMaxSpecies];
  const int tid = threadIdx.x;
  const int P = a.P, S = a.S;
  if (tid < S) {
    alive[tid] = t.alive[tid] != 0;
    founder[tid] = -1;
  }
  __syncthreads();
  if (tid == 0) {
    int f = 0;
    for (int s = 0; s < S; ++s) f += !alive[s];
    nfree = f;
  }
  // a) every genome against the alive representatives
  for (int g = tid; g < P; g += kBlock) {
    int best = -1;
    float bd = 0.0f;
    for (int s = 0; s < S; ++s) {
      if (!alive[s]) continue;
      const float d = pair_distance(ws.pop, P, g, ws.reps, S, s, a.c_d, a.c_h);
      if (d < a.thr && (best < 0 || d < bd)) {
        best = s;
        bd = d;
      }
    }
    ws.sp[g] = best;
  }
  __syncthreads();
  // b) the others in index order: join a species founded earlier in this step
  // (below the threshold) or found one; with no free slot, the nearest one
  for (int g = 0; g < P; ++g) {
    if (ws.sp[g] >= 0) continue;  // the same value on every thread
    if (nfree > 0) {
      if (tid < S) {
        const int f = founder[tid];
        dsh[tid] = f >= 0 ? pair_distance(ws.pop, P, g, ws.pop, P, f, a.c_d, a.c_h) : 0.0f;
      }
      __syncthreads();
      if (tid == 0) {
        int best = -1;
        float bd = 0.0f;
        for (int s = 0; s < S; ++s) {
          if (founder[s] < 0) continue;
          const float d = dsh[s];
          if (d < a.thr && (best < 0 || d < bd)) {
            best = s;
            bd = d;
          }
        }
        if (best < 0) {
          for (int s = 0; s < S; ++s)
            if (!alive[s]) {
              best = s;
              break;
            }
          alive[best] = 1;
          founder[best] = g;
          nfree = nfree - 1;
        }
        ws.sp[g] = best;
      }
    } else {
      if (tid < S && alive[tid]) {
        const int f = founder[tid];
        float d = f >= 0 ? pair_distance(ws.pop, P, g, ws.pop, P, f, a.c_d, a.c_h)
                         : pair_distance(ws.pop, P, g, ws.reps, S, tid, a.c_d, a.c_h);
        dsh[tid] = d != d ? INFINITY : d;
      }
      __syncthreads();
      if (tid == 0) {
        int best = -1;
        float bd = 0.0f;
        for (int s = 0; s < S; ++s) {
          if (!alive[s]) continue;
          if (best < 0 || dsh[s] < bd) {
            best = s;
            bd = dsh[s];
          }
        }
        ws.sp[g] = best;
      }
    }
    __syncthreads();
  }
  // species statistics, per slot: members, largest and smallest fitness, sum
  // in ascending genome order
  if (tid < S) {
    int n = 0;
    float mx = -INFINITY, mn = INFINITY, sum = 0.0f;
    for (int g = 0; g < P; ++g) {
      if (ws.sp[g] != tid) continue;
      const float f = fit[g];
      ++n;
      mx = f > mx ? f : mx;
      mn = f < mn ? f : mn;
      sum = sum + f;
    }
    ws.nmem[tid] = n;
    smax[tid] = mx;
    smin[tid] = mn;
    ssum[tid] = sum;
  }
  __syncthreads();
  if (tid != 0) return;
  // stagnation and offspring counts, one thread in slot order
  float best[kMaxSpecies];
  int last[kMaxSpecies], surv[kMaxSpecies], cnt[kMaxSpecies], prot[kMaxSpecies];
  for (int s = 0; s < S; ++s) {
    const bool founded = founder[s] >= 0;
    best[s] = founded ? -INFINITY : t.best[s];
    last[s] = founded ? a.gen : t.last[s];
    prot[s] = 0;
    surv[s] = 0;
    cnt[s] = 0;
    if (ws.nmem[s] > 0 && smax[s] > best[s]) {
      best[s] = smax[s];
      last[s] = a.gen;
    }
  }
  for (int k = 0; k < a.species_elitism; ++k) {  // the largest species fitness first
    int pick = -1;
    for (int s = 0; s < S; ++s)
      if (ws.nmem[s] > 0 && !prot[s] && (pick < 0 || smax[s] > smax[pick])) pick = s;
    if (pick < 0) break;
    prot[pick] = 1;
  }
  int nsurv = 0;
  float lo = INFINITY, hi = -INFINITY;
  for (int s = 0; s < S; ++s) {
    surv[s] = ws.nmem[s] > 0 && (prot[s] || a.gen - last[s] < a.max_stagnation);
    if (!surv[s]) continue;
    ++nsurv;
    lo = smin[s] < lo ? smin[s] : lo;
    hi = smax[s] > hi ? smax[s] : hi;
  }
  smin_valid = 1;
  if (nsurv > 0) {
    const float d = hi - lo;
    const float rng = d > 1.0f ? d : 1.0f;
    float af[kMaxSpecies], share[kMaxSpecies];
    float af_sum = 0.0f;
    for (int s = 0; s < S; ++s) {
      if (!surv[s]) continue;
      const float mean = ssum[s] / (float)ws.nmem[s];
      af[s] = (mean - lo) / rng;
      af_sum = af_sum + af[s];
    }
    const float fP = (float)P, ns = (float)nsurv;
    float sp_sum = 0.0f;
    for (int s = 0; s < S; ++s) {
      if (!surv[s]) continue;
      const float target = af_sum > 0.0f ? (fP * af[s]) / af_sum : fP / ns;
      const float prev = (float)t.size[s] * (founder[s] >= 0 ? 0.0f : 1.0f);
      const float spawn = prev + (target - prev) * a.rate;
      share[s] = spawn;
      sp_sum = sp_sum + spawn;
    }
    int total = 0;
    bool ok = true;
    for (int s = 0; s < S; ++s) {
      if (!surv[s]) continue;
      share[s] = sp_sum > 0.0f ? (share[s] * fP) / sp_sum : fP / ns;
      ok = ok && __builtin_isfinite(share[s]) && share[s] >= 0.0f && share[s] < 1073741824.0f;
      cnt[s] = ok ? (int)floorf(share[s]) : 0;
      total += cnt[s];
    }
    int left = P - total;
    if (!ok || left < 0 || left > nsurv) {  // non-finite fitness: equal split
      for (int s = 0; s < S; ++s) cnt[s] = 0;
      int k = 0;
      for (int s = 0; s < S; ++s)
        if (surv[s]) cnt[s] = P / nsurv + (k++ < P % nsurv ? 1 : 0);
      left = 0;
    }
    int given[kMaxSpecies];
    for (int s = 0; s < S; ++s) given[s] = 0;
    for (; left > 0; --left) {  // largest remainder first, ties lowest slot
      int pick = -1;
      float pr = 0.0f;
      for (int s = 0; s < S; ++s) {
        if (!surv[s] || given[s]) continue;
        const float r = share[s] - (float)cnt[s];
        if (pick < 0 || r > pr) {
          pick = s;
          pr = r;
        }
      }
      given[pick] = 1;
      ++cnt[pick];
    }
  }
  int mo = 0, co = 0;
  for (int s = 0; s < S; ++s) {
    ws.member_off[s] = mo;
    ws.child_off[s] = co;
    mo += ws.nmem[s];
    co += cnt[s];
    ws.counts[s] = cnt[s];
    ws.surv[s] = surv[s];
    ws.best[s] = best[s];
    ws.last[s] = last[s];
  }
  ws.member_off[S] = mo;
  ws.child_off[S] = co;
}

__global__ __launch_bounds__(kBlock) void rank_kernel(NeatWs ws, const float* fit, int P) {
  const int g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= P) return;
  const int s = ws.sp[g];
  const float f = fit[g];
  int rank = 0;
  for (int h = 0; h < P; ++h) {
    if (ws.sp[h] != s) continue;
    const float fh = fit[h];
    rank += (fh > f || (fh == f && h < g)) ? 1 : 0;
  }
  ws.order[ws.member_off[s] + rank] = g;
}

__device__ __forceinline__ int pick(float u, int n) {
  const int k = (int)floorf(u * (float)n);
  return min(k, n - 1);
}

__global__ __launch_bounds__(kBlock) void parents_kernel(NeatWs ws, const float* fit,
                                                         const float* sel, int P, int S,
                                                         int genome_elitism, float survival) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= P) return;
  int s = 0;
  while (s < S && !(ws.child_off[s] <= c && c < ws.child_off[s] + ws.counts[s])) ++s;
  int pa = -1, pb = -1;
  if (s < S) {
    const int i = c - ws.child_off[s];
    const int n = ws.nmem[s];
    const int* ms = ws.order + ws.member_off[s];
    const int e = min(min(genome_elitism, ws.counts[s]), n);
    if (i < e) {
      pa = ms[i];
    } else {
      const int k = max(1, (int)ceilf(survival * (float)n));
      pa = ms[pick(sel[2 * (int64_t)c], k)];
      pb = ms[pick(sel[2 * (int64_t)c + 1], k)];
      if (fit[pb] > fit[pa] || (fit[pb] == fit[pa] && pb < pa)) {
        const int x = pa;
        pa = pb;
        pb = x;
      }
    }
  }
  ws.parents[2 * (int64_t)c] = pa;
  ws.parents[2 * (int64_t)c + 1] = pb;
}

__global__ __launch_bounds__(kBlock) void table_kernel(NeatWs ws, Table t, PopView pop) {
  const int s = blockIdx.x;
  const bool keep = ws.surv[s] && ws.counts[s] > 0;
  if (threadIdx.x == 0) {
    t.alive[s] = keep ? 1 : 0;
    t.best[s] = keep ? ws.best[s] : -INFINITY;
    t.last[s] = keep ? ws.last[s] : 0;
    t.size[s] = keep ? ws.counts[s] : 0;
  }
  if (!keep) return;
  const int g = ws.order[ws.member_off[s]];
  const int N = pop.N_max, C = pop.C_max;
  const int64_t sb = (int64_t)s * N, gb = (int64_t)g * N;
  for (int r = threadIdx.x; r < N; r += kBlock) {
    t.reps.node_key[sb + r] = pop.node_key[gb + r];
    t.reps.node_bias[sb + r] = pop.node_bias[gb + r];
    t.reps.node_resp[sb + r] = pop.node_resp[gb + r];
    t.reps.node_act[sb + r] = pop.node_act[gb + r];
    t.reps.node_agg[sb + r] = pop.node_agg[gb + r];
  }
  const int64_t sc = (int64_t)s * C, gc = (int64_t)g * C;
  for (int r = threadIdx.x; r < C; r += kBlock) {
    t.reps.conn_in[sc + r] = pop.conn_in[gc + r];
    t.reps.conn_out[sc + r] = pop.conn_out[gc + r];
    t.reps.conn_w[sc + r] = pop.conn_w[gc + r];
    t.reps.conn_en[sc + r] = pop.conn_en[gc + r];
  }
}

__global__ void copy_ints_kernel(const int32_t* src, int32_t* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

Table table_of(const tn_species_table& t) {
  Table x;
  x.alive = t.alive;
  x.best = t.best;
  x.last = t.last_improved;
  x.size = t.size;
  x.reps = t.reps;
  return x;
}

}  // namespace

size_t neat_workspace_bytes(int P, int S, int N, int C) { return ws_bytes(P, S, N, C); }

int launch_neat_init(int P, int n_in, int n_out, int N, int C, const float* Z,
                     const tn_mutation_params& m, const tn_population_arrays& out,
                     const tn_species_table* table, hipStream_t stream) {
  if (P > 0) {
    int nU = 0, nZ = 0;
    tn_reproduce_draws(N, C, &nU, &nZ);
    hipLaunchKernelGGL(init_kernel, dim3(P), dim3(kBlock), 0, stream, n_in, n_out, N, C, Z,
                       (int64_t)nZ, m, out);
    int rc = check_launch();
    if (rc != TN_OK) return rc;
  }
  if (table) {
    hipLaunchKernelGGL(clear_table_kernel, dim3(table->max_species), dim3(kBlock), 0, stream,
                       table_of(*table), N, C);
    return check_launch();
  }
  return TN_OK;
}

int launch_neat_generation(const tn_population& p, const float* fit, int gen,
                           const tn_neat_params& prm, const tn_species_table& table,
                           const float* sel, const float* U, const float* Z, int32_t next_key,
                           const tn_population_arrays& children, int32_t* species_of,
                           int32_t* parents, int32_t* next_key_out, void* workspace,
                           hipStream_t stream) {
  const int P = p.P, S = table.max_species, N = p.N_max, C = p.C_max;
  const size_t prep_lds = prep_nodes_lds(N, C);
  int rc = allow_lds((const void*)prep_nodes_kernel, prep_lds);
  if (rc != TN_OK) return rc;
  NeatWs ws = carve(workspace, P, S, N, C);
  const Table t = table_of(table);
  // gene lists of the population and of the representatives
  const PopView pv = make_view(p);
  tn_population rp = p;
  rp.P = S;
  rp.node_key = table.reps.node_key;
  rp.node_bias = table.reps.node_bias;
  rp.node_resp = table.reps.node_resp;
  rp.node_act = table.reps.node_act;
  rp.node_agg = table.reps.node_agg;
  rp.conn_in = table.reps.conn_in;
  rp.conn_out = table.reps.conn_out;
  rp.conn_w = table.reps.conn_w;
  rp.conn_en = table.reps.conn_en;
  const int Sp = gene_pow2(std::max(N, C));
  hipLaunchKernelGGL(prep_nodes_kernel, dim3(P), dim3(kWave), prep_lds, stream, pv, ws.pop, Sp);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(prep_nodes_kernel, dim3(S), dim3(kWave), prep_lds, stream, make_view(rp),
                     ws.reps, Sp);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  SpecArgs a;
  a.P = P;
  a.S = S;
  a.gen = gen;
  a.thr = prm.compatibility_threshold;
  a.c_d = prm.compatibility_disjoint;
  a.c_h = prm.compatibility_homologous;
  a.species_elitism = prm.species_elitism;
  a.max_stagnation = prm.max_stagnation;
  a.rate = prm.spawn_number_change_rate;
  hipLaunchKernelGGL(speciate_kernel, dim3(1), dim3(kBlock), 0, stream, ws, t, fit, a);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  const int blocks = (P + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(rank_kernel, dim3(blocks), dim3(kBlock), 0, stream, ws, fit, P);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(parents_kernel, dim3(blocks), dim3(kBlock), 0, stream, ws, fit, sel, P, S,
                     prm.genome_elitism, prm.survival_threshold);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  rc = launch_reproduce(p, P, ws.parents, U, Z, prm.mutation, next_key, children, next_key_out,
                        ws.repro, stream);
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(table_kernel, dim3(S), dim3(kBlock), 0, stream, ws, t, pv);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  if (species_of) {
    hipLaunchKernelGGL(copy_ints_kernel, dim3(std::min(blocks, 1024)), dim3(kBlock), 0, stream,
                       ws.sp, species_of, (int64_t)P);
    rc = check_launch();
    if (rc != TN_OK) return rc;
  }
  if (parents) {
    hipLaunchKernelGGL(copy_ints_kernel, dim3(std::min(2 * blocks, 1024)), dim3(kBlock), 0,
                       stream, ws.parents, parents, 2 * (int64_t)P);
    rc = check_launch();
  }
  return rc;
}

}  // namespace tn
