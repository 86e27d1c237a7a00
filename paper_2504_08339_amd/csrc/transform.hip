// Transformation stage of tensorized inference (TensorNEAT Section 3.3):
// per genome, the topological order N_order and the expanded connections
// C_exp, the latter kept as a compressed in-edge list per topological position.
//
// One workgroup of 1..8 wavefronts per genome (more for populations of larger
// genomes: every loop over node rows, connection rows, positions and edges is
// split over the workgroup's threads); everything for the genome lives in LDS:
//   1. node keys -> rows through an open-addressing hash (duplicate keys flagged)
//   2. connection markings (in-key, out-key) through a 64-bit hash (duplicates
//      flagged), enabled rows resolved to (source row, destination row)
//   3. level-synchronous Kahn sort: each round marks the node rows whose
//      remaining in-degree is 0, places them in ascending row order (a prefix
//      sum over the workgroup), then decrements their successors through an
//      out-edge list
//   4. in-edge lists grouped by destination position: rows are dropped into
//      buckets with LDS atomics, then each edge computes its rank among the
//      bucket's rows, which makes the result independent of atomic order.
//   5. value-row assignment for the forward pass: input k takes row k; then,
//      level by level, every non-input position takes the lowest free row (or a
//      new one), and after the level the rows of positions whose last consumer
//      is in that level are freed (outputs keep theirs). A row freed in level L
//      is only reused from level L+1 on, so the positions of one level can be
//      evaluated concurrently.
#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "tn_internal.hpp"

namespace tn {

namespace {

constexpr int32_t kEmptyKey = -1;
constexpr unsigned long long kEmptyMark = ~0ull;

__device__ __forceinline__ uint32_t hash32(uint32_t k) {
  // lowbias32 (Chris Wellons' integer hash constants)
  k ^= k >> 16;
  k *= 0x7feb352du;
  k ^= k >> 15;
  k *= 0x846ca68bu;
  k ^= k >> 16;
  return k;
}

__device__ __forceinline__ uint32_t hash64(unsigned long long k) {
  return hash32((uint32_t)k ^ hash32((uint32_t)(k >> 32)));
}

struct Layout {
  // genomes this launch takes: node rows <= n_cap and connection rows <= c_cap,
  // and not both within (n_prev, c_prev) (an earlier launch's); the launch
  // with the population's capacities also takes the oversize genomes
  int n_cap, c_cap, n_prev, c_prev;
  bool last;
  int HN, HC;              // hash table sizes (powers of two)
  int off_hkey, off_hslot, off_nkey, off_deg, off_rem, off_outdeg, off_pos,
      off_order, off_level, off_ptr, off_cursor, off_outlist, off_esrc, off_edst,
      off_tmp, off_chash, off_csr_row, off_lstart;
  size_t bytes;
};

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

Layout make_layout(int N, int C) {
  Layout L;
  L.n_cap = N;
  L.c_cap = C;
  L.n_prev = L.c_prev = -1;
  L.last = true;
  L.HN = next_pow2(2 * N);
  L.HC = next_pow2(C + C / 4 + 1);  // marking hash at most 80 % full
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (bytes + 15) & ~size_t(15);
    return (int)at;
  };
  // 8-byte aligned first; reused for the free-event list of step 9b
  L.off_chash = take(std::max(sizeof(unsigned long long) * L.HC, sizeof(int16_t) * (2 * N + C)));
  L.off_hkey = take(sizeof(int32_t) * L.HN);
  L.off_hslot = take(sizeof(int16_t) * L.HN);
  L.off_nkey = take(sizeof(int32_t) * N);
  L.off_deg = take(sizeof(int32_t) * N);
  L.off_rem = take(sizeof(int32_t) * N);
  L.off_outdeg = take(sizeof(int32_t) * N);
  L.off_pos = take(sizeof(int16_t) * N);
  L.off_order = take(sizeof(int16_t) * N);
  L.off_level = take(sizeof(int16_t) * N);
  L.off_ptr = take(sizeof(int32_t) * (N + 1));
  L.off_cursor = take(sizeof(int32_t) * N);
  L.off_outlist = take(sizeof(int16_t) * C);
  L.off_esrc = take(sizeof(int16_t) * C);
  L.off_edst = take(sizeof(int16_t) * C);
  L.off_tmp = take(sizeof(int16_t) * C);
  L.off_csr_row = take(sizeof(int16_t) * C);
  L.off_lstart = take(sizeof(int16_t) * (N + 1));
  L.bytes = o;
  return L;
}

__device__ int lookup_node(const int32_t* hkey, const int16_t* hslot, int HN, int32_t k) {
  if (k < 0) return -1;
  uint32_t h = hash32((uint32_t)k) & (uint32_t)(HN - 1);
  while (true) {
    int32_t kk = hkey[h];
    if (kk == k) return hslot[h];
    if (kk == kEmptyKey) return -1;
    h = (h + 1) & (uint32_t)(HN - 1);
  }
}

// Writes the "no valid transformation" form of genome g.
__device__ void write_flagged(const PopView& pop, const TrView& tr, int g, int st,
                              int64_t nb, int64_t nrows, int64_t cb, int64_t crows) {
  const int lane = threadIdx.x, T = blockDim.x;
  const int64_t rb = pop.rowptr_base(g);
  for (int64_t p = lane; p < nrows; p += T) {
    tr.order[nb + p] = -1;
    tr.level[nb + p] = -1;
    tr.pos_bias[nb + p] = 0.0f;
    tr.pos_resp[nb + p] = 0.0f;
    tr.pos_fn[nb + p] = 0;
    tr.pos_row[nb + p] = -1;
    tr.prog_node[nb + p] = make_int4(0, 0, 0, 0);
    for (int j = 0; j < 4; ++j) reinterpret_cast<int4*>(tr.prog_rec)[(nb + p) * 4 + j] = make_int4(0, 0, 0, 0);
  }
  for (int64_t p = lane; p <= nrows; p += T) tr.row_ptr[rb + p] = 0;
  for (int64_t e = lane; e < crows; e += T) {
    tr.edge_src[cb + e] = -1;
    tr.edge_row[cb + e] = -1;
    tr.edge_w[cb + e] = 0.0f;
    tr.prog_edge[cb + e] = make_int2(0, 0);
  }
  const int nio = pop.n_in + pop.n_out;
  for (int k = lane; k < nio; k += T) tr.io_pos[(int64_t)g * nio + k] = -1;
  if (lane == 0) {
    tr.status[g] = st;
    tr.n_valid[g] = 0;
    tr.n_rows[g] = 0;
    tr.prog_rows[g] = 0;
  }
}

constexpr int kTfMaxWaves = 8;
// Ragged populations of at least this many genomes are transformed by size class.
constexpr int kTfClassMinGenomes = 2048;

// Workgroup barrier that orders LDS accesses only: the kernel never reads back
// what it stores to global memory, so its stores stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup-wide steps of the transform for workgroups of up to kW
// wavefronts, over the threads in index order; with kW == 1 everything stays
// inside the wavefront (no workgroup barrier). The multi-wavefront forms wait
// at barriers: every thread of the workgroup calls them.
template <int kW>
struct Group {
  int* sh;  // kW ints of LDS

  __device__ __forceinline__ void sync() const {
    if constexpr (kW == 1)
      wave_sync();
    else
      lds_barrier();
  }

  // Sum of x over the earlier threads; *total: over the workgroup.
  __device__ __forceinline__ int excl_sum(int x, int* total) const {
    const int inc = wave_inclusive_scan(x);
    if constexpr (kW == 1) {
      *total = __shfl(inc, kWave - 1, kWave);
      return inc - x;
    } else {
      const int lane = lane_id(), wave = (int)(threadIdx.x / kWave), W = (int)(blockDim.x / kWave);
      if (lane == kWave - 1) sh[wave] = inc;
      lds_barrier();
      int before = 0, tot = 0;
      for (int w = 0; w < W; ++w) {
        const int t = sh[w];
        before += w < wave ? t : 0;
        tot += t;
      }
      lds_barrier();
      *total = tot;
      return before + inc - x;
    }
  }

  // Number of earlier threads with f set; *total: over the workgroup.
  __device__ __forceinline__ int excl_count(bool f, int* total) const {
    const uint64_t m = __ballot(f);
    if constexpr (kW == 1) {
      *total = __popcll(m);
      return mbcnt(m);
    } else {
      const int lane = lane_id(), wave = (int)(threadIdx.x / kWave), W = (int)(blockDim.x / kWave);
      if (lane == 0) sh[wave] = __popcll(m);
      lds_barrier();
      int before = 0, tot = 0;
      for (int w = 0; w < W; ++w) {
        const int t = sh[w];
        before += w < wave ? t : 0;
        tot += t;
      }
      lds_barrier();
      *total = tot;
      return before + mbcnt(m);
    }
  }

  // max(carry, x of this and every earlier thread); *prev: the same at the
  // previous thread (carry at thread 0), *all: at the last thread.
  __device__ __forceinline__ int incl_max(int x, int carry, int* prev, int* all) const {
    const int lane = lane_id();
    int before = carry, tot;
    const int inc = wave_inclusive_max(x);
    if constexpr (kW == 1) {
      tot = max(carry, __shfl(inc, kWave - 1, kWave));
    } else {
      const int wave = (int)(threadIdx.x / kWave), W = (int)(blockDim.x / kWave);
      if (lane == kWave - 1) sh[wave] = inc;
      lds_barrier();
      tot = carry;
      for (int w = 0; w < W; ++w) {
        const int t = sh[w];
        if (w < wave) before = max(before, t);
        tot = max(tot, t);
      }
      lds_barrier();
    }
    const int v = max(before, inc);
    int pv = __shfl_up(v, 1, kWave);
    if (lane == 0) pv = before;
    *prev = pv;
    *all = tot;
    return v;
  }
};

template <int kW>
__global__ __launch_bounds__(kWave * kW) void transform_kernel(PopView pop, TrView tr, Layout L) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int flags;
  __shared__ int scan_sh[kW];
  const Group<kW> G{scan_sh};

  const int g = blockIdx.x;
  const int tid = threadIdx.x, T = blockDim.x;
  const int N = pop.N_max, C = pop.C_max;

  const int64_t nb = pop.node_base(g);
  const int64_t cb = pop.conn_base(g);
  const int64_t nrows64 = pop.node_rows(g);
  const int64_t crows64 = pop.conn_rows(g);
  const bool bad = nrows64 > N || crows64 > C || nrows64 < 0 || crows64 < 0;
  if (bad ? !L.last
          : (nrows64 <= L.n_prev && crows64 <= L.c_prev) ||
                (!L.last && (nrows64 > L.n_cap || crows64 > L.c_cap)))
    return;  // another launch's genome
  if (bad) {
    write_flagged(pop, tr, g, TN_OVERSIZE, nb, nrows64 > 0 ? nrows64 : 0, cb,
                  crows64 > 0 ? crows64 : 0);
    return;
  }
  const int nrows = (int)nrows64, crows = (int)crows64;

  unsigned long long* chash = (unsigned long long*)(smem + L.off_chash);
  int32_t* hkey = (int32_t*)(smem + L.off_hkey);
  int16_t* hslot = (int16_t*)(smem + L.off_hslot);
  int32_t* nkey = (int32_t*)(smem + L.off_nkey);
  int32_t* deg = (int32_t*)(smem + L.off_deg);
  int32_t* rem = (int32_t*)(smem + L.off_rem);
  int32_t* outdeg = (int32_t*)(smem + L.off_outdeg);
  int16_t* pos_of = (int16_t*)(smem + L.off_pos);
  int16_t* order_l = (int16_t*)(smem + L.off_order);
  int16_t* level_l = (int16_t*)(smem + L.off_level);
  int32_t* ptr = (int32_t*)(smem + L.off_ptr);
  int32_t* cursor = (int32_t*)(smem + L.off_cursor);
  int16_t* outlist = (int16_t*)(smem + L.off_outlist);
  int16_t* esrc = (int16_t*)(smem + L.off_esrc);
  int16_t* edst = (int16_t*)(smem + L.off_edst);
  int16_t* tmp = (int16_t*)(smem + L.off_tmp);
  int16_t* csr_row = (int16_t*)(smem + L.off_csr_row);  // connection row of CSR entry e
  int16_t* csr_src = outlist;                              // source position of entry e
  int16_t* lstart = (int16_t*)(smem + L.off_lstart);    // first position of each level

  for (int i = tid; i < L.HN; i += T) hkey[i] = kEmptyKey;
  for (int i = tid; i < L.HC; i += T) chash[i] = kEmptyMark;
  for (int i = tid; i < nrows; i += T) {
    deg[i] = 0;
    outdeg[i] = 0;
    cursor[i] = 0;
    pos_of[i] = -1;
  }
  if (tid == 0) flags = 0;
  G.sync();

  // 1. node rows -> hash
  int my_valid = 0;
  for (int r = tid; r < nrows; r += T) {
    const int32_t k = pop.node_key[nb + r];
    nkey[r] = k;
    if (k < 0) continue;
    ++my_valid;
    if (pop.node_act[nb + r] > TN_ACT_ABS || pop.node_agg[nb + r] > TN_AGG_MAXABS)
      atomicOr(&flags, TN_BAD_ATTR);
    uint32_t h = hash32((uint32_t)k) & (uint32_t)(L.HN - 1);
    while (true) {
      const int32_t old = atomicCAS(&hkey[h], kEmptyKey, k);
      if (old == kEmptyKey) {
        hslot[h] = (int16_t)r;
        break;
      }
      if (old == k) {
        atomicOr(&flags, TN_DUP_NODE);
        break;
      }
      h = (h + 1) & (uint32_t)(L.HN - 1);
    }
  }
  int n_valid;
  (void)G.excl_sum(my_valid, &n_valid);
  G.sync();

  // 2. inputs / outputs present
  const int nio = pop.n_in + pop.n_out;
  for (int k = tid; k < nio; k += T)
    if (lookup_node(hkey, hslot, L.HN, k) < 0) atomicOr(&flags, TN_MISSING_IO);

  // 3. connection rows
  for (int r = tid; r < crows; r += T) {
    const int32_t a = pop.conn_in[cb + r];
    const int32_t b = pop.conn_out[cb + r];
    int16_t s = -1, d = -1;
    if (a >= 0 && b >= 0) {
      const unsigned long long mark = ((unsigned long long)(uint32_t)a << 32) | (uint32_t)b;
      uint32_t h = hash64(mark) & (uint32_t)(L.HC - 1);
      while (true) {
        const unsigned long long old = atomicCAS(&chash[h], kEmptyMark, mark);
        if (old == kEmptyMark) break;
        if (old == mark) {
          atomicOr(&flags, TN_DUP_CONN);
          break;
        }
        h = (h + 1) & (uint32_t)(L.HC - 1);
      }
      if (pop.conn_en[cb + r]) {
        const int sa = lookup_node(hkey, hslot, L.HN, a);
        const int sb = lookup_node(hkey, hslot, L.HN, b);
        if (sa < 0 || sb < 0) atomicOr(&flags, TN_DANGLING);
        if (b < pop.n_in) atomicOr(&flags, TN_INPUT_DST);
        if (sa >= 0 && sb >= 0) {
          s = (int16_t)sa;
          d = (int16_t)sb;
          atomicAdd(&deg[sb], 1);
          atomicAdd(&outdeg[sa], 1);
        }
      }
    }
    esrc[r] = s;
    edst[r] = d;
  }
  G.sync();
  const int st = flags;
  if (st) {
    write_flagged(pop, tr, g, st, nb, nrows, cb, crows);
    return;
  }

  // 4. out-edge lists by source row
  {
    int carry = 0;
    for (int base = 0; base < nrows; base += T) {
      const int i = base + tid;
      const int x = i < nrows ? outdeg[i] : 0;
      int tot;
      const int ex = G.excl_sum(x, &tot);
      if (i < nrows) {
        ptr[i] = carry + ex;
        rem[i] = deg[i];
      }
      carry += tot;
    }
    if (tid == 0) ptr[nrows] = carry;
  }
  G.sync();
  for (int r = tid; r < crows; r += T) {
    const int s = esrc[r];
    if (s >= 0) outlist[ptr[s] + atomicAdd(&cursor[s], 1)] = edst[r];
  }
  G.sync();

  // 5. level-synchronous Kahn rounds; a round's rows are placed in ascending
  // row order
  __shared__ uint32_t free_bits[TN_MAX_NODES / 32];  // here: rows ready for the next round
  int emitted = 0;
  bool scan = true;
  if constexpr (kW > 1) scan = nrows <= T;
  if (scan) {
    // each round tests every row (one pass of the workgroup when the rows fit)
    for (int lvl = 0;; ++lvl) {
      const int start = emitted;
      for (int base = 0; base < nrows; base += T) {
        const int i = base + tid;
        const bool ready = i < nrows && nkey[i] >= 0 && pos_of[i] < 0 && rem[i] == 0;
        int cnt;
        const int ex = G.excl_count(ready, &cnt);
        if (ready) {
          const int p = emitted + ex;
          pos_of[i] = (int16_t)p;
          order_l[p] = (int16_t)i;
          level_l[p] = (int16_t)lvl;
        }
        emitted += cnt;
      }
      if (emitted == start) break;
      G.sync();
      for (int p = start + tid; p < emitted; p += T) {
        const int s = order_l[p];
        const int j1 = ptr[s + 1];
        int j = ptr[s];
        for (; j + 4 <= j1; j += 4) {  // four removals in flight
          const int d0 = outlist[j], d1 = outlist[j + 1], d2 = outlist[j + 2],
                    d3 = outlist[j + 3];
          atomicSub(&rem[d0], 1);
          atomicSub(&rem[d1], 1);
          atomicSub(&rem[d2], 1);
          atomicSub(&rem[d3], 1);
        }
        for (; j < j1; ++j) atomicSub(&rem[outlist[j]], 1);
      }
      G.sync();
    }
  } else {
    // more rows than threads (a padded population): the rounds on the first
    // wavefront, the rows ready for the next round the bits of a bitmap, set
    // when a row's last in-edge is removed; a round places them in ascending
    // row order (lane w expands word w at its prefix offset), without testing
    // every row
    uint32_t* ready = free_bits;
    for (int w = tid; w < TN_MAX_NODES / 32; w += T) ready[w] = 0u;
    G.sync();
    for (int i = tid; i < nrows; i += T)
      if (nkey[i] >= 0 && rem[i] == 0) atomicOr(&ready[i >> 5], 1u << (i & 31));
    G.sync();
    if (tid < kWave) {
      const int lane = tid;
      int done = 0;
      for (int lvl = 0;; ++lvl) {
        const uint32_t bits = lane < TN_MAX_NODES / 32 ? ready[lane] : 0u;
        const int c = __popc(bits);
        const int incl = wave_inclusive_scan(c);
        const int cnt = __shfl(incl, kWave - 1, kWave);
        if (cnt == 0) break;
        int o = done + incl - c;
        for (uint32_t x = bits; x != 0u; x &= x - 1, ++o) {
          const int i = lane * 32 + (__ffs(x) - 1);
          pos_of[i] = (int16_t)o;
          order_l[o] = (int16_t)i;
          level_l[o] = (int16_t)lvl;
        }
        if (lane < TN_MAX_NODES / 32) ready[lane] = 0u;
        const int start = done;
        done += cnt;
        wave_sync();
        for (int p = start + lane; p < done; p += kWave) {
          const int s = order_l[p];
          const int j1 = ptr[s + 1];
          int j = ptr[s];
          for (; j + 4 <= j1; j += 4) {  // four removals in flight
            const int d0 = outlist[j], d1 = outlist[j + 1], d2 = outlist[j + 2],
                      d3 = outlist[j + 3];
            const int r0 = atomicSub(&rem[d0], 1), r1 = atomicSub(&rem[d1], 1),
                      r2 = atomicSub(&rem[d2], 1), r3 = atomicSub(&rem[d3], 1);
            if (r0 == 1) atomicOr(&ready[d0 >> 5], 1u << (d0 & 31));
            if (r1 == 1) atomicOr(&ready[d1 >> 5], 1u << (d1 & 31));
            if (r2 == 1) atomicOr(&ready[d2 >> 5], 1u << (d2 & 31));
            if (r3 == 1) atomicOr(&ready[d3 >> 5], 1u << (d3 & 31));
          }
          for (; j < j1; ++j) {
            const int d = outlist[j];
            if (atomicSub(&rem[d], 1) == 1) atomicOr(&ready[d >> 5], 1u << (d & 31));
          }
        }
        wave_sync();
      }
      if (lane == 0) flags = done;  // the status word has been read; it carries the count
    }
    G.sync();
    emitted = flags;
  }
  if (emitted < n_valid) {
    write_flagged(pop, tr, g, TN_CYCLE, nb, nrows, cb, crows);
    return;
  }

  // 6. in-edge row pointers over topological positions
  G.sync();
  {
    int carry = 0;
    for (int base = 0; base < n_valid; base += T) {
      const int p = base + tid;
      const int x = p < n_valid ? deg[order_l[p]] : 0;
      int tot;
      const int ex = G.excl_sum(x, &tot);
      if (p < n_valid) ptr[p] = carry + ex;
      carry += tot;
    }
    if (tid == 0) ptr[n_valid] = carry;
    for (int i = tid; i < nrows; i += T) cursor[i] = 0;
  }
  G.sync();
  const int n_edges = ptr[n_valid];
  for (int r = tid; r < crows; r += T) {
    const int d = edst[r];
    if (d >= 0) tmp[ptr[pos_of[d]] + atomicAdd(&cursor[d], 1)] = (int16_t)r;
  }
  G.sync();

  // 7. stable order inside each bucket, written out
  for (int idx = tid; idx < n_edges; idx += T) {
    const int r = tmp[idx];
    const int pd = pos_of[edst[r]];
    const int lo = ptr[pd], hi = ptr[pd + 1];
    int rank = 0;
    for (int j = lo; j < hi; ++j) rank += tmp[j] < r;
    const int64_t o = cb + lo + rank;
    tr.edge_row[o] = r;
    tr.edge_src[o] = pos_of[esrc[r]];
    tr.edge_w[o] = pop.conn_w[cb + r];
    csr_row[lo + rank] = (int16_t)r;
    csr_src[lo + rank] = pos_of[esrc[r]];
  }
  for (int e = n_edges + tid; e < crows; e += T) {
    tr.edge_row[cb + e] = -1;
    tr.edge_src[cb + e] = -1;
    tr.edge_w[cb + e] = 0.0f;
  }
  const int64_t rb = pop.rowptr_base(g);
  for (int p = tid; p <= nrows; p += T) tr.row_ptr[rb + p] = ptr[p < n_valid ? p : n_valid];

  // 8. node attributes by position; level starts (the start of level L is the
  // one position of level L whose predecessor has a lower level)
  for (int p = tid; p < nrows; p += T) {
    if (p < n_valid) {
      const int s = order_l[p];
      tr.order[nb + p] = s;
      tr.level[nb + p] = level_l[p];
      tr.pos_bias[nb + p] = pop.node_bias[nb + s];
      tr.pos_resp[nb + p] = pop.node_resp[nb + s];
      const int k = nkey[s];
      uint32_t fn = (uint32_t)pop.node_act[nb + s] | ((uint32_t)pop.node_agg[nb + s] << 8);
      if (k < pop.n_in) fn = kFnInput | ((uint32_t)k << 16) | fn;
      tr.pos_fn[nb + p] = (int32_t)fn;
      if (p == 0 || level_l[p - 1] != level_l[p]) lstart[level_l[p]] = (int16_t)p;
    } else {
      tr.order[nb + p] = -1;
      tr.level[nb + p] = -1;
      tr.pos_bias[nb + p] = 0.0f;
      tr.pos_resp[nb + p] = 0.0f;
      tr.pos_fn[nb + p] = 0;
    }
  }
  const int n_levels = n_valid > 0 ? level_l[n_valid - 1] + 1 : 0;
  if (tid == 0) lstart[n_levels] = (int16_t)n_valid;
  for (int k = tid; k < nio; k += T)
    tr.io_pos[(int64_t)g * nio + k] = pos_of[lookup_node(hkey, hslot, L.HN, k)];

  // 9. value rows with reuse (see the header). last[s]: position of the last
  // consumer of s (-1: none; outputs never free their row).
  __shared__ int next_row;
  int32_t* last = deg;        // both are free now
  int32_t* row = rem;
  int32_t* fl_end = outdeg;   // per level: end of the list of rows it frees
  int32_t* fl_list = cursor;  // positions whose row is freed, by level
  for (int p = tid; p < n_valid; p += T) last[p] = -1;
  for (int l = tid; l < n_levels; l += T) fl_end[l] = 0;
  for (int w = tid; w < TN_MAX_NODES / 32; w += T) free_bits[w] = 0u;
  G.sync();
  for (int p = tid; p < n_valid; p += T)
    for (int j = ptr[p]; j < ptr[p + 1]; ++j) atomicMax(&last[csr_src[j]], p);
  G.sync();
  // The level after which the row of position p is freed: that of its last
  // consumer, or its own for a non-input position nothing reads; never for an
  // output, nor for an input nobody reads (free from the start).
  auto free_level = [&](int p, int k) {
    if (k >= pop.n_in && k < nio) return -1;
    if (last[p] >= 0) return (int)level_l[last[p]];
    return k >= pop.n_in ? (int)level_l[p] : -1;
  };
  // input k takes row k; an input nobody reads is free at once
  for (int p = tid; p < n_valid; p += T) {
    const int k = nkey[order_l[p]];
    if (k < pop.n_in) {
      row[p] = k;
      if (last[p] < 0) atomicOr(&free_bits[k >> 5], 1u << (k & 31));
    }
    const int fl = free_level(p, k);
    if (fl >= 0) atomicAdd(&fl_end[fl], 1);
  }
  if (tid == 0) next_row = pop.n_in;
  G.sync();
  {
    int carry = 0;  // counts -> start offsets
    for (int base = 0; base < n_levels; base += T) {
      const int l = base + tid;
      const int c = l < n_levels ? fl_end[l] : 0;
      int tot;
      const int ex = G.excl_sum(c, &tot);
      if (l < n_levels) fl_end[l] = carry + ex;
      carry += tot;
    }
  }
  G.sync();
  for (int p = tid; p < n_valid; p += T) {  // start offsets -> ends
    const int fl = free_level(p, nkey[order_l[p]]);
    if (fl >= 0) fl_list[atomicAdd(&fl_end[fl], 1)] = p;
  }
  G.sync();
  // level by level, on the first wavefront (its own syncs only)
  if (tid < kWave) {
    const int lane = tid;
    for (int l = 0; l < n_levels; ++l) {
      const int lb = lstart[l], le = lstart[l + 1];
      // allocate the level's non-input positions, in order: the i-th takes
      // the i-th lowest free row, or a new one once the free rows are used up
      for (int base = lb; base < le; base += kWave) {
        const int p = base + lane;
        const bool node = p < le && nkey[order_l[p]] >= pop.n_in;
        const uint64_t m = __ballot(node);
        const int k = __popcll(m);
        if (k == 0) continue;
        const int i = mbcnt(m);
        int nfree = 0;
        for (int w = 0; w < TN_MAX_NODES / 32; ++w) nfree += __popc(free_bits[w]);
        const int nr = next_row;
        if (node) {
          int r;
          if (i < nfree) {
            int skip = i, w = 0;
            while (__popc(free_bits[w]) <= skip) skip -= __popc(free_bits[w++]);
            uint32_t x = free_bits[w];
            for (int t = 0; t < skip; ++t) x &= x - 1;
            r = w * 32 + (__ffs(x) - 1);
          } else {
            r = nr + (i - nfree);
          }
          row[p] = r;
        }
        wave_sync();
        if (node && i < nfree) atomicAnd(&free_bits[row[p] >> 5], ~(1u << (row[p] & 31)));
        if (lane == 0 && k > nfree) next_row = nr + (k - nfree);
        wave_sync();
      }
      // free the rows whose last consumer sits in this level, and those of
      // this level's positions that nothing reads
      for (int j = (l ? fl_end[l - 1] : 0) + lane; j < fl_end[l]; j += kWave) {
        const int q = fl_list[j];
        atomicOr(&free_bits[row[q] >> 5], 1u << (row[q] & 31));
      }
      wave_sync();
    }
  }
  G.sync();
  for (int p = tid; p < nrows; p += T) tr.pos_row[nb + p] = p < n_valid ? row[p] : -1;
  G.sync();

  // 9b. value rows of the packed program, which is evaluated one position
  // after the other: a value's row is free as soon as its last consumer has
  // read it (that consumer may take it for its own result). Any reuse policy
  // then needs the fewest rows, the largest number of values live at once.
  // The one used serves allocations from freed rows in the order they were
  // freed (first in, first out), so the u-th allocation served from freed rows
  // takes the u-th freed row, and allocation needs only prefix sums and one
  // prefix maximum: with F(p) the rows freed up to position p and A(p) the
  // non-input positions up to p, the rows created up to p are
  // max(0, max_{q <= p} A(q) - F(q)).
  // Free events, in order: the unused inputs (at position 0); then at each
  // position p the dead value at p-1 (a hidden node nobody reads), followed by
  // the sources whose last consumer is p, in in-edge order. Outputs keep their
  // rows.
  int32_t* fcum = outdeg;                        // F(p)
  int32_t* seq = cursor;                         // row, or -(s+1): the row of position s
  int16_t* ev = (int16_t*)(smem + L.off_chash);  // position whose row the u-th event frees
  int n_unused = 0;
  for (int base = 0; base < n_valid; base += T) {
    const int p = base + tid;
    const bool un = p < n_valid && nkey[order_l[p]] < pop.n_in && last[p] < 0;
    int cnt;
    const int ex = G.excl_count(un, &cnt);
    if (un) ev[n_unused + ex] = (int16_t)p;
    n_unused += cnt;
  }
  {
    int carry = n_unused;
    for (int base = 0; base < n_valid; base += T) {
      const int p = base + tid;
      int c = 0;
      if (p < n_valid) {
        if (p > 0) c += nkey[order_l[p - 1]] >= nio && last[p - 1] < 0;
        for (int j = ptr[p]; j < ptr[p + 1]; ++j) {
          const int s = csr_src[j];
          const int ks = nkey[order_l[s]];
          c += last[s] == p && !(ks >= pop.n_in && ks < nio);
        }
      }
      int tot;
      const int ex = G.excl_sum(c, &tot);
      if (p < n_valid) fcum[p] = carry + ex + c;
      carry += tot;
    }
  }
  G.sync();
  for (int p = 1 + tid; p < n_valid; p += T) {
    int i = fcum[p - 1];
    if (nkey[order_l[p - 1]] >= nio && last[p - 1] < 0) ev[i++] = (int16_t)(p - 1);
    for (int j = ptr[p]; j < ptr[p + 1]; ++j) {
      const int s = csr_src[j];
      const int ks = nkey[order_l[s]];
      if (last[s] == p && !(ks >= pop.n_in && ks < nio)) ev[i++] = (int16_t)s;
    }
  }
  G.sync();
  int n_new = 0;  // rows created so far (beyond the n_in input rows)
  {
    int a_carry = 0;
    for (int base = 0; base < n_valid; base += T) {
      const int p = base + tid;
      const int k = p < n_valid ? nkey[order_l[p]] : 0;
      const bool node = p < n_valid && k >= pop.n_in;
      int a_tot;
      const int a = a_carry + G.excl_count(node, &a_tot) + (node ? 1 : 0);
      const int d = node ? a - fcum[p] : INT_MIN;
      int prev, all;
      const int nn = G.incl_max(d, n_new, &prev, &all);
      if (p < n_valid) {
        if (!node)
          seq[p] = k;
        else if (nn > prev)
          seq[p] = pop.n_in + nn - 1;
        else
          seq[p] = -(ev[a - nn - 1] + 1);
      }
      a_carry += a_tot;
      n_new = all;
    }
  }
  G.sync();
  // resolve "same row as position s" links by pointer jumping (s < p always;
  // a link read while another thread replaces it is either value, both on the
  // same chain, so the rounds end with every position holding its chain's row)
  for (;;) {
    bool more = false;
    for (int p = tid; p < n_valid; p += T) {
      const int v = seq[p];
      if (v < 0) {
        const int t = seq[-v - 1];
        seq[p] = t;
        more |= t < 0;
      }
    }
    G.sync();
    int n_more;
    (void)G.excl_count(more, &n_more);
    if (n_more == 0) break;
  }

  // 10. packed program of the forward pass
  for (int p = tid; p < nrows; p += T) {
    int4 q = make_int4(0, 0, 0, 0);
    if (p < n_valid) {
      const int s = order_l[p];
      const int k = nkey[s];
      int32_t fn = (int32_t)((uint32_t)pop.node_act[nb + s] | ((uint32_t)pop.node_agg[nb + s] << 8));
      fn = k < pop.n_in ? (int32_t)(kFnInput | ((uint32_t)k << 16)) : (fn | (seq[p] << 16));
      q = make_int4(ptr[p + 1], fn, __float_as_int(pop.node_bias[nb + s]),
                    __float_as_int(pop.node_resp[nb + s]));
    }
    tr.prog_node[nb + p] = q;
  }
  for (int e = tid; e < crows; e += T) {
    int2 q = make_int2(0, 0);
    if (e < n_edges) q = make_int2(seq[csr_src[e]], __float_as_int(pop.conn_w[cb + csr_row[e]]));
    tr.prog_edge[cb + e] = q;
  }
  // 11. the same program as one 16-word record per non-input position (in
  // order; inputs are staged separately): word 0 = act | agg << 3 | row << 6 |
  // in-edge count << 17, word 1 bias, word 2 response, word 3 the in-edge
  // list index of the node's 7th in-edge (for nodes with more than 6), words
  // 4..15 its first 6 in-edges as (source row, weight); unused slots hold
  // (prog_rows, +0), a row past every live value: the engines read only the
  // record's in-edge count of slots, so these entries are never dereferenced.
  {
    const int zrow = pop.n_in + n_new;
    int in_before = 0;
    for (int base = 0; base < n_valid; base += T) {
      const int p = base + tid;
      const bool inp = p < n_valid && nkey[order_l[p]] < pop.n_in;
      int cnt;
      const int ex = G.excl_count(inp, &cnt);
      if (p < n_valid && !inp) {
        const int s = order_l[p];
        const int r = p - (in_before + ex);
        const int e0 = ptr[p], ne = ptr[p + 1] - e0;
        int32_t w[16];
        w[0] = (int32_t)((uint32_t)pop.node_act[nb + s] | ((uint32_t)pop.node_agg[nb + s] << 3) |
                         ((uint32_t)seq[p] << 6) | ((uint32_t)ne << 17));
        w[1] = __float_as_int(pop.node_bias[nb + s]);
        w[2] = __float_as_int(pop.node_resp[nb + s]);
        w[3] = e0 + 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const bool real = i < ne;
          w[4 + 2 * i] = real ? seq[csr_src[e0 + i]] : zrow;
          w[5 + 2 * i] = real ? __float_as_int(pop.conn_w[cb + csr_row[e0 + i]]) : 0;
        }
        int4* rec = reinterpret_cast<int4*>(tr.prog_rec) + (nb + r) * 4;
        rec[0] = make_int4(w[0], w[1], w[2], w[3]);
        rec[1] = make_int4(w[4], w[5], w[6], w[7]);
        rec[2] = make_int4(w[8], w[9], w[10], w[11]);
        rec[3] = make_int4(w[12], w[13], w[14], w[15]);
      }
      in_before += cnt;
    }
    const int n_nodes = n_valid - in_before;
    for (int i = n_nodes * 4 + tid; i < nrows * 4; i += T)
      reinterpret_cast<int4*>(tr.prog_rec)[nb * 4 + i] = make_int4(0, 0, 0, 0);
  }
  if (tid == 0) {
    tr.status[g] = 0;
    tr.n_valid[g] = n_valid;
    tr.n_rows[g] = next_row;
    tr.prog_rows[g] = pop.n_in + n_new;
  }
}

}  // namespace

size_t transform_lds_bytes(int N_max, int C_max) { return make_layout(N_max, C_max).bytes; }

namespace {

// The size classes of one call run side by side: the caller's stream takes
// the largest class, side streams the others, forked from the caller's stream
// and joined back to it with events, so the last, partly filled round of one
// class's workgroups overlaps the others' work (the classes write disjoint
// genomes). Side streams (default priority, non-blocking) and events are made
// once per device; the mutex keeps the fork / launch / join sequence of one
// call from interleaving with another's on the same events.
constexpr int kTfMaxClasses = 5;
constexpr int kMaxDevices = 64;
struct ClassStreams {
  hipStream_t side[kTfMaxClasses - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kTfMaxClasses - 1] = {};
};
std::mutex g_class_mu;
ClassStreams g_class[kMaxDevices];
bool g_class_ready[kMaxDevices] = {};

// The current device's side streams and events (caller holds g_class_mu).
int class_streams(ClassStreams** out) {
  int dev = 0;
  int rc = record_hip(hipGetDevice(&dev));
  if (rc != TN_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return TN_EUNSUPPORTED;
  ClassStreams& cs = g_class[dev];
  if (!g_class_ready[dev]) {
    if (!cs.fork) rc = record_hip(hipEventCreateWithFlags(&cs.fork, hipEventDisableTiming));
    for (int i = 0; i < kTfMaxClasses - 1 && rc == TN_OK; ++i) {
      if (!cs.side[i]) rc = record_hip(hipStreamCreateWithFlags(&cs.side[i], hipStreamNonBlocking));
      if (rc == TN_OK && !cs.join[i])
        rc = record_hip(hipEventCreateWithFlags(&cs.join[i], hipEventDisableTiming));
    }
    if (rc != TN_OK) return rc;  // what was made is kept and completed next time
    g_class_ready[dev] = true;
  }
  *out = &cs;
  return TN_OK;
}

// Wavefronts per workgroup of a class: one per 256 rows of the larger
// capacity, at most kTfMaxWaves (eight were measured fastest on genomes of up
// to 535 nodes / 1894 connections: 4 and 16 slower).
int class_waves(const Layout& L) {
  int waves = 1;
  while (waves < kTfMaxWaves && waves * 256 < std::max(L.n_cap, L.c_cap)) waves *= 2;
  return waves;
}

int class_lds(const Layout& L) {
  return allow_lds(class_waves(L) == 1 ? (const void*)transform_kernel<1>
                                       : (const void*)transform_kernel<kTfMaxWaves>,
                   L.bytes);
}

int launch_class(const tn_population& p, const tn_transformed& t, const Layout& L,
                 hipStream_t stream) {
  const int waves = class_waves(L);
  const int rc = class_lds(L);
  if (rc != TN_OK) return rc;
  if (waves == 1)
    hipLaunchKernelGGL(transform_kernel<1>, dim3(p.P), dim3(kWave), L.bytes, stream,
                       make_view(p), make_view(t), L);
  else
    hipLaunchKernelGGL(transform_kernel<kTfMaxWaves>, dim3(p.P), dim3(kWave * waves), L.bytes,
                       stream, make_view(p), make_view(t), L);
  return check_launch();
}

}  // namespace

int launch_transform(const tn_population& p, const tn_transformed& t, hipStream_t stream) {
  // Size classes of a large ragged population: one launch per class, each with
  // the LDS of its largest genome, so the many small genomes are not held to
  // the few large ones' LDS (two workgroups per CU at 535 nodes / 1894
  // connections). A padded population, or a small one, is one launch.
  std::vector<Layout> cls;
  if (p.node_off && p.P >= kTfClassMinGenomes) {
    int n_prev = -1, c_prev = -1;
    for (int n : {96, 192, 320, 400}) {
      const int c = std::min(p.C_max, 4 * n);
      if (n >= p.N_max) break;
      Layout L = make_layout(n, c);
      L.last = false;
      L.n_prev = n_prev;
      L.c_prev = c_prev;
      cls.push_back(L);
      n_prev = n;
      c_prev = c;
    }
    Layout L = make_layout(p.N_max, p.C_max);
    L.n_prev = n_prev;
    L.c_prev = c_prev;
    cls.push_back(L);
  } else {
    cls.push_back(make_layout(p.N_max, p.C_max));
  }
  if (p.P == 0) return class_lds(cls[0]);  // nothing to launch; the LDS check still applies
  const int nc = (int)cls.size();
  if (nc > kTfMaxClasses) return TN_EUNSUPPORTED;
  // Under stream capture the classes go one after another on the caller's
  // stream: side streams that joined a capture stay in it until it ends, and
  // they are shared with every other call on the device.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  int rc = record_hip(hipStreamIsCapturing(stream, &cap));
  if (rc != TN_OK) return rc;
  if (nc == 1 || cap != hipStreamCaptureStatusNone) {
    for (int i = nc - 1; i >= 0 && rc == TN_OK; --i) rc = launch_class(p, t, cls[i], stream);
    return rc;
  }

  std::lock_guard<std::mutex> lock(g_class_mu);
  ClassStreams* cs = nullptr;
  rc = class_streams(&cs);
  if (rc == TN_OK) rc = record_hip(hipEventRecord(cs->fork, stream));
  if (rc != TN_OK) return rc;
  // largest class first, on the caller's stream
  rc = launch_class(p, t, cls[nc - 1], stream);
  int forked = 0;
  for (int i = 0; i < nc - 1 && rc == TN_OK; ++i) {
    rc = record_hip(hipStreamWaitEvent(cs->side[i], cs->fork, 0));
    if (rc != TN_OK) break;
    ++forked;
    rc = launch_class(p, t, cls[i], cs->side[i]);
  }
  // join every side stream that was forked, also after a failed launch
  for (int i = 0; i < forked; ++i) {
    int r = record_hip(hipEventRecord(cs->join[i], cs->side[i]));
    if (r == TN_OK) r = record_hip(hipStreamWaitEvent(stream, cs->join[i], 0));
    if (rc == TN_OK) rc = r;
  }
  return rc;
}

}  // namespace tn
