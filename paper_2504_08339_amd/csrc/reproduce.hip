// Tensorized reproduction (TensorNEAT Section 3.2; hyperparameters of
// Appendices A and C): crossover aligned by historical marking, then mutation
// as the paper's row operations on the padded tensors (add a node or a
// connection in the first empty row, empty a row, change attributes in place).
// Random draws are inputs, so the children are a pure function of the parents
// and the draws.
//
// Four launches, all on the caller's stream:
//   cross    one workgroup per child: the fitter parent's rows copied, the
//            other parent's node keys / markings hashed in LDS (first row of
//            each), homologous genes take the other parent's attributes on a
//            coin below 1/2; then the add-node decision and the connection it
//            splits (marking recorded for the innovation table).
//   first    one thread per child: is its split marking the first occurrence
//            among the children (block-tiled pass over the children before it).
//   keys     one thread per child: new key = next_key + the number of distinct
//            split markings below its own (the rank in lexicographic order).
//   mutate   one workgroup per child: the split, delete node, add connection
//            (cycle check by a breadth-first sweep over a key set in LDS),
//            delete connection, attribute rules.
#include <algorithm>

#include "tn_internal.hpp"

// Every float product and sum below is rounded on its own: no fused
// multiply-add (HIP's __fmul_rn / __fadd_rn are plain operators that the
// compiler may contract).
#pragma clang fp contract(off)

namespace tn {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kStruct = 16;  // structural draws at the head of each child's uniforms
constexpr int kZHead = 4;    // normals at the head of each child's normals

struct Rows {
  int32_t* key;
  float* bias;
  float* resp;
  uint8_t* act;
  uint8_t* agg;
  int32_t* cin;
  int32_t* cout;
  float* w;
  uint8_t* en;
};

struct Ws {
  int32_t* split_row;   // [n] connection row the add-node mutation splits, -1: none
  long long* mark;      // [n] its marking (in << 32 | out), -1: none
  int32_t* first;       // [n] 1 if the child's marking appears in no earlier child
  int32_t* split_key;   // [n] key of the new node
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

size_t ws_bytes(int n) {
  return 3 * align_up(sizeof(int32_t) * (size_t)n) + align_up(sizeof(long long) * (size_t)n);
}

Ws carve(void* base, int n) {
  unsigned char* p = (unsigned char*)base;
  size_t o = 0;
  Ws w;
  w.split_row = (int32_t*)(p + o);
  o += align_up(sizeof(int32_t) * (size_t)n);
  w.mark = (long long*)(p + o);
  o += align_up(sizeof(long long) * (size_t)n);
  w.first = (int32_t*)(p + o);
  o += align_up(sizeof(int32_t) * (size_t)n);
  w.split_key = (int32_t*)(p + o);
  return w;
}

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

__device__ __forceinline__ uint32_t hash32(uint32_t k) {
  // lowbias32 (Chris Wellons' integer hash constants)
  k ^= k >> 16;
  k *= 0x7feb352du;
  k ^= k >> 15;
  k *= 0x846ca68bu;
  k ^= k >> 16;
  return k;
}

__device__ __forceinline__ uint32_t hash64(long long k) {
  return hash32((uint32_t)k ^ hash32((uint32_t)((unsigned long long)k >> 32)));
}

__device__ __forceinline__ bool conn_valid(const Rows& c, int r) {
  return c.cin[r] >= 0 && c.cout[r] >= 0;
}

// Index floor(u * n) of n candidates, the product rounded to float32, at most n - 1.
__device__ __forceinline__ int pick(float u, int n) {
  const int k = (int)floorf(u * (float)n);
  return min(k, n - 1);
}

// mean + std * z, the product rounded before the sum (contraction is off).
__device__ __forceinline__ float draw(float mean, float std_, float z) {
  const float t = std_ * z;
  return mean + t;
}

// Float attribute rule: v + power * z below `rate`, mean + std * z below
// rate + replace, else v; each product and sum rounded on its own.
__device__ __forceinline__ float mutate_float(float v, float u, float z, float mean, float std_,
                                              float power, float rate, float replace) {
  if (u < rate) {
    const float t = power * z;
    return v + t;
  }
  if (u < rate + replace) return draw(mean, std_, z);
  return v;
}

// Number of rows r in [0, R) with pred(r), on every thread of the workgroup.
template <typename Pred>
__device__ int block_count(int R, Pred pred, int* sh) {
  int c = 0;
  for (int r = threadIdx.x; r < R; r += kBlock) c += pred(r) ? 1 : 0;
  c = wave_sum_int(c);
  if (lane_id() == 0) sh[wave_id()] = c;
  __syncthreads();
  int total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) total += sh[w];
  __syncthreads();
  return total;
}

// Row of the k-th (from 0, ascending rows) r in [0, R) with pred(r), or -1, on
// every thread of the workgroup.
template <typename Pred>
__device__ int block_select(int R, int k, Pred pred, int* sh) {
  int before = 0;
  if (threadIdx.x == 0) sh[kWaves] = -1;
  for (int base = 0; base < R; base += kBlock) {
    const int r = base + (int)threadIdx.x;
    const bool p = r < R && pred(r);
    const uint64_t m = __ballot(p);
    if (lane_id() == 0) sh[wave_id()] = __popcll(m);
    __syncthreads();
    int off = before, chunk = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      if (w < wave_id()) off += sh[w];
      chunk += sh[w];
    }
    if (p && off + mbcnt(m) == k) sh[kWaves] = r;
    before += chunk;
    __syncthreads();
    if (before > k) break;
  }
  const int res = sh[kWaves];
  __syncthreads();
  return res;
}

__device__ __forceinline__ Rows child_rows(const tn_population_arrays& o, int c, int N, int C) {
  Rows r;
  const int64_t nb = (int64_t)c * N, cb = (int64_t)c * C;
  r.key = o.node_key + nb;
  r.bias = o.node_bias + nb;
  r.resp = o.node_resp + nb;
  r.act = o.node_act + nb;
  r.agg = o.node_agg + nb;
  r.cin = o.conn_in + cb;
  r.cout = o.conn_out + cb;
  r.w = o.conn_w + cb;
  r.en = o.conn_en + cb;
  return r;
}

struct Parent {
  const int32_t* key;
  const float* bias;
  const float* resp;
  const uint8_t* act;
  const uint8_t* agg;
  const int32_t* cin;
  const int32_t* cout;
  const float* w;
  const uint8_t* en;
};

__device__ __forceinline__ Parent parent_rows(const PopView& pop, int g) {
  Parent p;
  const int64_t nb = (int64_t)g * pop.N_max, cb = (int64_t)g * pop.C_max;
  p.key = pop.node_key + nb;
  p.bias = pop.node_bias + nb;
  p.resp = pop.node_resp + nb;
  p.act = pop.node_act + nb;
  p.agg = pop.node_agg + nb;
  p.cin = pop.conn_in + cb;
  p.cout = pop.conn_out + cb;
  p.w = pop.conn_w + cb;
  p.en = pop.conn_en + cb;
  return p;
}

__device__ __forceinline__ int32_t cas(int32_t* p, int32_t cmp, int32_t v) {
  return atomicCAS(p, cmp, v);
}

__device__ __forceinline__ long long cas(long long* p, long long cmp, long long v) {
  return (long long)atomicCAS((unsigned long long*)p, (unsigned long long)cmp,
                              (unsigned long long)v);
}

// LDS hash: key -> smallest row holding it (keys >= 0; empty slot key -1).
template <typename K>
__device__ __forceinline__ void hash_insert_min(K* hk, int32_t* hr, int H, K key, uint32_t h,
                                                int32_t row) {
  h &= (uint32_t)(H - 1);
  while (true) {
    const K prev = cas(&hk[h], (K)-1, key);
    if (prev == (K)-1 || prev == key) {
      atomicMin(&hr[h], row);
      return;
    }
    h = (h + 1) & (uint32_t)(H - 1);
  }
}

template <typename K>
__device__ __forceinline__ int32_t hash_find(const K* hk, const int32_t* hr, int H, K key,
                                             uint32_t h) {
  h &= (uint32_t)(H - 1);
  while (true) {
    const K k = hk[h];
    if (k == key) return hr[h];
    if (k == (K)-1) return -1;
    h = (h + 1) & (uint32_t)(H - 1);
  }
}

__device__ __forceinline__ long long marking(int32_t a, int32_t b) {
  return ((long long)a << 32) | (long long)(uint32_t)b;
}

__global__ __launch_bounds__(kBlock) void cross_kernel(PopView pop, int n, const int32_t* parents,
                                                       const float* U, int64_t nU,
                                                       float node_add, tn_population_arrays out,
                                                       Ws ws, int HN, int HC, int32_t next_key,
                                                       int32_t* next_key_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh[kWaves + 1];
  const int c = blockIdx.x;
  const int N = pop.N_max, C = pop.C_max;
  if (c == 0 && threadIdx.x == 0) *next_key_out = next_key;
  const int p1 = parents[2 * (int64_t)c], p2 = parents[2 * (int64_t)c + 1];
  Rows ch = child_rows(out, c, N, C);
  if (p1 < 0 || p1 >= pop.P) {  // no such parent: an all-empty child
    for (int r = threadIdx.x; r < N; r += kBlock) {
      ch.key[r] = -1;
      ch.bias[r] = ch.resp[r] = 0.0f;
      ch.act[r] = ch.agg[r] = 0;
    }
    for (int r = threadIdx.x; r < C; r += kBlock) {
      ch.cin[r] = ch.cout[r] = -1;
      ch.w[r] = 0.0f;
      ch.en[r] = 0;
    }
    if (threadIdx.x == 0) {
      ws.split_row[c] = -1;
      ws.mark[c] = -1;
    }
    return;
  }
  const Parent a = parent_rows(pop, p1);
  const bool cross = p2 >= 0 && p2 < pop.P;
  const float* u = U + (int64_t)c * nU;
  if (!cross) {  // an elite: the parent unchanged
    for (int r = threadIdx.x; r < N; r += kBlock) {
      ch.key[r] = a.key[r];
      ch.bias[r] = a.bias[r];
      ch.resp[r] = a.resp[r];
      ch.act[r] = a.act[r];
      ch.agg[r] = a.agg[r];
    }
    for (int r = threadIdx.x; r < C; r += kBlock) {
      ch.cin[r] = a.cin[r];
      ch.cout[r] = a.cout[r];
      ch.w[r] = a.w[r];
      ch.en[r] = a.en[r];
    }
    if (threadIdx.x == 0) {
      ws.split_row[c] = -1;
      ws.mark[c] = -1;
    }
    return;
  }
  const Parent b = parent_rows(pop, p2);
  // node rows: hash of the other parent's keys (first row of each)
  int32_t* nk = (int32_t*)smem;   // [HN]
  int32_t* nr = nk + HN;          // [HN]
  for (int h = threadIdx.x; h < HN; h += kBlock) {
    nk[h] = -1;
    nr[h] = 0x7fffffff;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N; r += kBlock) {
    const int32_t k = b.key[r];
    if (k >= 0) hash_insert_min(nk, nr, HN, k, hash32((uint32_t)k), r);
  }
  __syncthreads();
  for (int r = threadIdx.x; r < N; r += kBlock) {
    const int32_t k = a.key[r];
    int q = -1;
    if (k >= 0 && u[kStruct + r] < 0.5f) q = hash_find(nk, nr, HN, k, hash32((uint32_t)k));
    const Parent& s = q >= 0 ? b : a;
    const int sr = q >= 0 ? q : r;
    ch.key[r] = k;
    ch.bias[r] = s.bias[sr];
    ch.resp[r] = s.resp[sr];
    ch.act[r] = s.act[sr];
    ch.agg[r] = s.agg[sr];
  }
  __syncthreads();
  // connection rows: hash of the other parent's markings (first row of each)
  long long* ck = (long long*)smem;          // [HC]
  int32_t* cr = (int32_t*)(ck + HC);         // [HC]
  for (int h = threadIdx.x; h < HC; h += kBlock) {
    ck[h] = -1;
    cr[h] = 0x7fffffff;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < C; r += kBlock) {
    const int32_t x = b.cin[r], y = b.cout[r];
    if (x >= 0 && y >= 0) {
      const long long m = marking(x, y);
      hash_insert_min(ck, cr, HC, m, hash64(m), r);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < C; r += kBlock) {
    const int32_t x = a.cin[r], y = a.cout[r];
    int q = -1;
    if (x >= 0 && y >= 0 && u[kStruct + N + r] < 0.5f) {
      const long long m = marking(x, y);
      q = hash_find(ck, cr, HC, m, hash64(m));
    }
    ch.cin[r] = x;
    ch.cout[r] = y;
    ch.w[r] = q >= 0 ? b.w[q] : a.w[r];
    ch.en[r] = q >= 0 ? b.en[q] : a.en[r];
  }
  __syncthreads();
  // add-node decision on the crossed-over child: an enabled connection to
  // split, a free node row and two free connection rows
  int split = -1;
  if (u[0] < node_add) {
    const int cand = block_count(C, [&](int r) { return conn_valid(ch, r) && ch.en[r] != 0; }, sh);
    const int free_node = block_count(N, [&](int r) { return ch.key[r] < 0; }, sh);
    const int free_conn = block_count(C, [&](int r) { return !conn_valid(ch, r); }, sh);
    if (cand > 0 && free_node > 0 && free_conn >= 2)
      split = block_select(C, pick(u[1], cand),
                           [&](int r) { return conn_valid(ch, r) && ch.en[r] != 0; }, sh);
  }
  if (threadIdx.x == 0) {
    ws.split_row[c] = split;
    ws.mark[c] = split >= 0 ? marking(ch.cin[split], ch.cout[split]) : -1;
  }
}

// first[c] = child c splits a marking that no child before it splits.
__global__ __launch_bounds__(kBlock) void first_kernel(int n, Ws ws, int32_t* next_key_out) {
  __shared__ long long tile[kBlock];
  __shared__ int sh[kWaves];
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const long long m = c < n ? ws.mark[c] : -1;
  bool first = m >= 0;
  const int end = min(n, (int)(blockIdx.x + 1) * kBlock);
  for (int base = 0; base < end; base += kBlock) {
    const int t = base + (int)threadIdx.x;
    tile[threadIdx.x] = t < n ? ws.mark[t] : -1;
    __syncthreads();
    const int lim = min(kBlock, max(0, c - base));  // children base .. c-1 of this tile
    for (int i = 0; i < lim; ++i) first &= tile[i] != m;
    __syncthreads();
  }
  if (c < n) ws.first[c] = first ? 1 : 0;
  // distinct markings of this block, added to the next free key
  const int cnt = wave_sum_int(first ? 1 : 0);
  if (lane_id() == 0) sh[wave_id()] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < kWaves; ++w) total += sh[w];
    if (total) atomicAdd(next_key_out, total);
  }
}

// split_key[c] = next_key + #{distinct split markings below child c's}.
__global__ __launch_bounds__(kBlock) void keys_kernel(int n, Ws ws, int32_t next_key) {
  __shared__ long long tile[kBlock];
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const long long m = c < n ? ws.mark[c] : -1;
  int rank = 0;
  for (int base = 0; base < n; base += kBlock) {
    const int t = base + (int)threadIdx.x;
    tile[threadIdx.x] = (t < n && ws.first[t]) ? ws.mark[t] : -1;
    __syncthreads();
    const int lim = min(kBlock, n - base);
    for (int i = 0; i < lim; ++i) {
      const long long x = tile[i];
      rank += (x >= 0 && x < m) ? 1 : 0;
    }
    __syncthreads();
  }
  if (c < n) ws.split_key[c] = m >= 0 ? next_key + rank : -1;
}

// Key set in LDS for the reachability sweep (keys >= 0; empty slot -1).
// Returns true if `key` was not there before.
__device__ __forceinline__ bool set_insert(int32_t* s, int H, int32_t key) {
  uint32_t h = hash32((uint32_t)key) & (uint32_t)(H - 1);
  while (true) {
    const int32_t prev = atomicCAS(&s[h], -1, key);
    if (prev == -1) return true;
    if (prev == key) return false;
    h = (h + 1) & (uint32_t)(H - 1);
  }
}

__device__ __forceinline__ bool set_has(const int32_t* s, int H, int32_t key) {
  uint32_t h = hash32((uint32_t)key) & (uint32_t)(H - 1);
  while (true) {
    const int32_t k = s[h];
    if (k == key) return true;
    if (k == -1) return false;
    h = (h + 1) & (uint32_t)(H - 1);
  }
}

__global__ __launch_bounds__(kBlock) void mutate_kernel(PopView pop, int n, const int32_t* parents,
                                                        const float* U, int64_t nU,
                                                        const float* Z, int64_t nZ,
                                                        tn_mutation_params prm,
                                                        tn_population_arrays out, Ws ws, int HR) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh[kWaves + 1];
  __shared__ int flag;
  const int c = blockIdx.x;
  const int N = pop.N_max, C = pop.C_max;
  const int n_in = pop.n_in, n_out = pop.n_out;
  const int p1 = parents[2 * (int64_t)c], p2 = parents[2 * (int64_t)c + 1];
  if (p1 < 0 || p1 >= pop.P || p2 < 0 || p2 >= pop.P) return;  // empty child or elite
  Rows ch = child_rows(out, c, N, C);
  const float* u = U + (int64_t)c * nU;
  const float* z = Z + (int64_t)c * nZ;
  // 1. add node: split the chosen connection a -> b into a -> new (weight 1)
  // and new -> b (the old weight), the old one disabled
  const int split = ws.split_row[c];
  if (split >= 0) {
    const int32_t a = ch.cin[split], b = ch.cout[split];
    const float w_old = ch.w[split];
    const int32_t key = ws.split_key[c];
    const int rn = block_select(N, 0, [&](int r) { return ch.key[r] < 0; }, sh);
    const int r1 = block_select(C, 0, [&](int r) { return !conn_valid(ch, r); }, sh);
    const int r2 = block_select(C, 1, [&](int r) { return !conn_valid(ch, r); }, sh);
    // (the crossover kernel chose the split only with these rows free)
    if (threadIdx.x == 0 && rn >= 0 && r1 >= 0 && r2 >= 0) {
      ch.en[split] = 0;
      ch.key[rn] = key;
      ch.bias[rn] = draw(prm.bias_init_mean, prm.bias_init_std, z[0]);
      ch.resp[rn] = draw(prm.resp_init_mean, prm.resp_init_std, z[1]);
      ch.act[rn] = (uint8_t)prm.act_default;
      ch.agg[rn] = (uint8_t)prm.agg_default;
      ch.cin[r1] = a;
      ch.cout[r1] = key;
      ch.w[r1] = 1.0f;
      ch.en[r1] = 1;
      ch.cin[r2] = key;
      ch.cout[r2] = b;
      ch.w[r2] = w_old;
      ch.en[r2] = 1;
    }
    __syncthreads();
  }
  // 2. delete node: a hidden node row and every connection naming its key
  if (u[2] < prm.node_delete) {
    auto hidden = [&](int r) { return ch.key[r] >= n_in + n_out; };
    const int cand = block_count(N, hidden, sh);
    if (cand > 0) {
      const int r = block_select(N, pick(u[3], cand), hidden, sh);
      const int32_t k = ch.key[r];
      __syncthreads();
      if (threadIdx.x == 0) {
        ch.key[r] = -1;
        ch.bias[r] = ch.resp[r] = 0.0f;
        ch.act[r] = ch.agg[r] = 0;
      }
      for (int q = threadIdx.x; q < C; q += kBlock) {
        if (conn_valid(ch, q) && (ch.cin[q] == k || ch.cout[q] == k)) {
          ch.cin[q] = ch.cout[q] = -1;
          ch.w[q] = 0.0f;
          ch.en[q] = 0;
        }
      }
      __syncthreads();
    }
  }
  // 3. add connection src -> dst in the first free row
  if (u[4] < prm.conn_add) {
    auto is_src = [&](int r) {
      const int32_t k = ch.key[r];
      return k >= 0 && !(k >= n_in && k < n_in + n_out);
    };
    auto is_dst = [&](int r) { return ch.key[r] >= n_in; };
    auto is_free = [&](int r) { return !conn_valid(ch, r); };
    const int ns = block_count(N, is_src, sh);
    const int nd = block_count(N, is_dst, sh);
    const int nf = block_count(C, is_free, sh);
    if (ns > 0 && nd > 0 && nf > 0) {
      const int32_t s = ch.key[block_select(N, pick(u[5], ns), is_src, sh)];
      const int32_t d = ch.key[block_select(N, pick(u[6], nd), is_dst, sh)];
      const int present = block_count(
          C, [&](int r) { return conn_valid(ch, r) && ch.cin[r] == s && ch.cout[r] == d; }, sh);
      bool ok = s != d && present == 0;
      if (ok && !prm.allow_cycles) {
        // would close a cycle: d reaches s over valid connections
        int32_t* set = (int32_t*)smem;  // [HR]
        for (int h = threadIdx.x; h < HR; h += kBlock) set[h] = -1;
        __syncthreads();
        if (threadIdx.x == 0) set_insert(set, HR, d);
        __syncthreads();
        bool reached = false;
        for (int it = 0; it <= C + 1 && !reached; ++it) {
          if (threadIdx.x == 0) flag = 0;
          __syncthreads();
          for (int r = threadIdx.x; r < C; r += kBlock) {
            if (!conn_valid(ch, r)) continue;
            if (set_has(set, HR, ch.cin[r]) && set_insert(set, HR, ch.cout[r])) flag = 1;
          }
          __syncthreads();
          reached = set_has(set, HR, s);
          const int changed = flag;
          __syncthreads();
          if (!changed) break;
        }
        ok = !reached;
      }
      if (ok) {
        const int r = block_select(C, 0, is_free, sh);
        if (threadIdx.x == 0) {
          ch.cin[r] = s;
          ch.cout[r] = d;
          ch.en[r] = 1;
          ch.w[r] = draw(prm.weight_init_mean, prm.weight_init_std, z[2]);
        }
      }
      __syncthreads();
    }
  }
  // 4. delete connection
  if (u[7] < prm.conn_delete) {
    auto valid = [&](int r) { return conn_valid(ch, r); };
    const int cand = block_count(C, valid, sh);
    if (cand > 0) {
      const int r = block_select(C, pick(u[8], cand), valid, sh);
      if (threadIdx.x == 0) {
        ch.cin[r] = ch.cout[r] = -1;
        ch.w[r] = 0.0f;
        ch.en[r] = 0;
      }
      __syncthreads();
    }
  }
  // 5. attributes of every valid non-input node row and valid connection row
  const int64_t un = kStruct + N + C, uc = kStruct + 7 * (int64_t)N + C;
  for (int r = threadIdx.x; r < N; r += kBlock) {
    if (ch.key[r] < n_in) continue;  // empty or input
    const float* d = u + un + 6 * (int64_t)r;
    ch.bias[r] = mutate_float(ch.bias[r], d[0], z[kZHead + 2 * r], prm.bias_init_mean,
                              prm.bias_init_std, prm.bias_mutate_power, prm.bias_mutate_rate,
                              prm.bias_replace_rate);
    ch.resp[r] = mutate_float(ch.resp[r], d[1], z[kZHead + 2 * r + 1], prm.resp_init_mean,
                              prm.resp_init_std, prm.resp_mutate_power, prm.resp_mutate_rate,
                              prm.resp_replace_rate);
    if (d[2] < prm.act_replace_rate) ch.act[r] = prm.act_options[pick(d[3], prm.n_act_options)];
    if (d[4] < prm.agg_replace_rate) ch.agg[r] = prm.agg_options[pick(d[5], prm.n_agg_options)];
  }
  for (int r = threadIdx.x; r < C; r += kBlock) {
    if (!conn_valid(ch, r)) continue;
    ch.w[r] = mutate_float(ch.w[r], u[uc + r], z[kZHead + 2 * (int64_t)N + r],
                           prm.weight_init_mean, prm.weight_init_std, prm.weight_mutate_power,
                           prm.weight_mutate_rate, prm.weight_replace_rate);
  }
}

__global__ void store_kernel(int32_t* p, int32_t v) { *p = v; }

}  // namespace

size_t reproduce_workspace_bytes(int n) { return ws_bytes(n); }

int launch_reproduce(const tn_population& p, int n, const int32_t* parents, const float* U,
                     const float* Z, const tn_mutation_params& prm, int32_t next_key,
                     const tn_population_arrays& out, int32_t* next_key_out, void* workspace,
                     hipStream_t stream) {
  const int HN = next_pow2(2 * p.N_max), HC = next_pow2(2 * p.C_max);
  const size_t cross_lds = std::max(sizeof(int32_t) * 2 * (size_t)HN,
                                    (sizeof(long long) + sizeof(int32_t)) * (size_t)HC);
  const int HR = next_pow2(2 * (p.C_max + 1));
  const size_t mutate_lds = sizeof(int32_t) * (size_t)HR;
  int rc = allow_lds((const void*)cross_kernel, cross_lds);
  if (rc == TN_OK) rc = allow_lds((const void*)mutate_kernel, mutate_lds);
  if (rc != TN_OK) return rc;
  if (n == 0) {
    hipLaunchKernelGGL(store_kernel, dim3(1), dim3(1), 0, stream, next_key_out, next_key);
    return check_launch();
  }
  int nU = 0, nZ = 0;
  tn_reproduce_draws(p.N_max, p.C_max, &nU, &nZ);
  Ws ws = carve(workspace, n);
  const PopView v = make_view(p);
  hipLaunchKernelGGL(cross_kernel, dim3(n), dim3(kBlock), cross_lds, stream, v, n, parents, U,
                     (int64_t)nU, prm.node_add, out, ws, HN, HC, next_key, next_key_out);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  const int blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(first_kernel, dim3(blocks), dim3(kBlock), 0, stream, n, ws, next_key_out);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(keys_kernel, dim3(blocks), dim3(kBlock), 0, stream, n, ws, next_key);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(mutate_kernel, dim3(n), dim3(kBlock), mutate_lds, stream, v, n, parents, U,
                     (int64_t)nU, Z, (int64_t)nZ, prm, out, ws, HR);
  return check_launch();
}

}  // namespace tn
