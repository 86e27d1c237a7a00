// Per-genome sorted gene lists for the node-inclusive compatibility distance
// (node genes by key, connection genes by marking, with the attributes the
// distance compares), shared by the distance matrix and the speciation of
// one NEAT generation. Included by one translation unit each: everything here
// has internal linkage.
#pragma once

#include "tn_internal.hpp"

namespace tn {
namespace {

constexpr long long kGenePad = 0x7fffffffffffffffll;

__device__ __forceinline__ uint32_t gene_mix32(uint32_t k) {
  // lowbias32 (Chris Wellons' integer hash constants)
  k ^= k >> 16;
  k *= 0x7feb352du;
  k ^= k >> 15;
  k *= 0x846ca68bu;
  k ^= k >> 16;
  return k;
}

__device__ __forceinline__ uint32_t gene_hash(long long k) {
  return gene_mix32((uint32_t)k ^ gene_mix32((uint32_t)((unsigned long long)k >> 32)));
}

inline size_t gene_align(size_t x) { return (x + 255) & ~size_t(255); }

inline int gene_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct GeneList {
  long long* keyT;   // [cap][P]
  int32_t* hT;       // [cap][P] hash_mark of the key
  float* a0T;        // [cap][P]
  float* a1T;        // [cap][P]
  uint32_t* codeT;   // [cap][P] c0 | c1 << 8
};

struct WsN {
  int32_t* cnt_n;    // [P] node genes, -1 for a genome without a gene set
  int32_t* cnt_c;    // [P] connection genes, -1 likewise
  GeneList nodes;    // cap N_max
  GeneList conns;    // cap C_max
};

inline size_t gene_list_bytes(int P, int cap) {
  const size_t n = (size_t)P * cap;
  return gene_align(sizeof(long long) * n) + 4 * gene_align(4 * n);
}

inline GeneList carve_list(unsigned char* p, size_t& o, int P, int cap) {
  const size_t n = (size_t)P * cap;
  GeneList l;
  l.keyT = (long long*)(p + o);
  o += gene_align(sizeof(long long) * n);
  l.hT = (int32_t*)(p + o);
  o += gene_align(4 * n);
  l.a0T = (float*)(p + o);
  o += gene_align(4 * n);
  l.a1T = (float*)(p + o);
  o += gene_align(4 * n);
  l.codeT = (uint32_t*)(p + o);
  o += gene_align(4 * n);
  return l;
}

inline size_t ws_nodes_bytes(int P, int N, int C) {
  return 2 * gene_align(sizeof(int32_t) * P) + gene_list_bytes(P, N) + gene_list_bytes(P, C);
}

inline WsN carve_nodes(void* base, int P, int N, int C) {
  unsigned char* p = (unsigned char*)base;
  size_t o = 0;
  WsN w;
  w.cnt_n = (int32_t*)(p + o);
  o += gene_align(sizeof(int32_t) * P);
  w.cnt_c = (int32_t*)(p + o);
  o += gene_align(sizeof(int32_t) * P);
  w.nodes = carve_list(p, o, P, N);
  w.conns = carve_list(p, o, P, C);
  return w;
}

// Bitonic sort of S (a power of two) (key, row) pairs in LDS by key; one
// wavefront.
__device__ void wave_bitonic(long long* key, int32_t* row, int S) {
  const int lane = lane_id();
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < S; i += kWave) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const long long ki = key[i], kj = key[ixj];
          if ((ki > kj) == ((i & k) == 0)) {
            key[i] = kj;
            key[ixj] = ki;
            const int32_t t = row[i];
            row[i] = row[ixj];
            row[ixj] = t;
          }
        }
      }
      wave_sync();
    }
  }
}

__global__ __launch_bounds__(kWave) void prep_nodes_kernel(PopView pop, WsN ws, int S) {
  extern __shared__ __align__(16) unsigned char smem[];
  long long* key = (long long*)smem;               // [S]
  int32_t* row = (int32_t*)(smem + sizeof(long long) * S);  // [S]
  const int g = blockIdx.x;
  const int lane = lane_id();
  const int P = pop.P;
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g);
  const int64_t nrows = pop.node_rows(g), crows = pop.conn_rows(g);
  if (nrows > pop.N_max || nrows < 0 || crows > pop.C_max || crows < 0) {
    if (lane == 0) {
      ws.cnt_n[g] = -1;
      ws.cnt_c[g] = -1;
    }
    return;
  }
  // node genes: every valid key is sorted (a repeated input key also leaves
  // the genome without a gene set); the inputs, keys 0 .. n_in-1, come first
  // and are skipped when storing
  int n = 0;
  for (int base = 0; base < (int)nrows; base += kWave) {
    const int r = base + lane;
    const int32_t k = r < nrows ? pop.node_key[nb + r] : -1;
    const uint64_t m = __ballot(k >= 0);
    if (k >= 0) {
      key[n + mbcnt(m)] = (long long)k;
      row[n + mbcnt(m)] = r;
    }
    n += __popcll(m);
  }
  for (int i = n + lane; i < S; i += kWave) {
    key[i] = kGenePad;
    row[i] = -1;
  }
  wave_sync();
  wave_bitonic(key, row, S);
  bool dup = false;
  for (int i = lane + 1; i < n; i += kWave) dup |= key[i] == key[i - 1];
  int n_inputs = 0;
  for (int i = lane; i < n; i += kWave) n_inputs += key[i] < (long long)pop.n_in;
  const bool dup_n = __ballot(dup) != 0;
  n_inputs = wave_sum_int(n_inputs);
  const int nn = n - n_inputs;
  for (int k = lane; k < nn; k += kWave) {
    const long long kk = key[n_inputs + k];
    const int r = row[n_inputs + k];
    const int64_t o = (int64_t)k * P + g;
    ws.nodes.keyT[o] = kk;
    ws.nodes.hT[o] = (int32_t)gene_hash(kk);
    ws.nodes.a0T[o] = pop.node_bias[nb + r];
    ws.nodes.a1T[o] = pop.node_resp[nb + r];
    ws.nodes.codeT[o] = (uint32_t)pop.node_act[nb + r] | ((uint32_t)pop.node_agg[nb + r] << 8);
  }
  wave_sync();
  // connection genes
  n = 0;
  for (int base = 0; base < (int)crows; base += kWave) {
    const int r = base + lane;
    int32_t a = -1, b = -1;
    if (r < crows) {
      a = pop.conn_in[cb + r];
      b = pop.conn_out[cb + r];
    }
    const bool valid = a >= 0 && b >= 0;
    const uint64_t m = __ballot(valid);
    if (valid) {
      key[n + mbcnt(m)] = ((long long)a << 32) | (long long)(uint32_t)b;
      row[n + mbcnt(m)] = r;
    }
    n += __popcll(m);
  }
  for (int i = n + lane; i < S; i += kWave) {
    key[i] = kGenePad;
    row[i] = -1;
  }
  wave_sync();
  wave_bitonic(key, row, S);
  dup = false;
  for (int i = lane + 1; i < n; i += kWave) dup |= key[i] == key[i - 1];
  const bool dup_c = __ballot(dup) != 0;
  for (int k = lane; k < n; k += kWave) {
    const long long kk = key[k];
    const int r = row[k];
    const int64_t o = (int64_t)k * P + g;
    ws.conns.keyT[o] = kk;
    ws.conns.hT[o] = (int32_t)gene_hash(kk);
    ws.conns.a0T[o] = pop.conn_w[cb + r];
    ws.conns.a1T[o] = 0.0f;
    ws.conns.codeT[o] = (uint32_t)(pop.conn_en[cb + r] != 0);
  }
  if (lane == 0) {
    const bool bad = dup_n || dup_c;
    ws.cnt_n[g] = bad ? -1 : nn;
    ws.cnt_c[g] = bad ? -1 : n;
  }
}

// LDS bytes of prep_nodes_kernel for capacities N, C.
inline size_t prep_nodes_lds(int N, int C) {
  return (sizeof(long long) + sizeof(int32_t)) * (size_t)gene_pow2(N > C ? N : C);
}

}  // namespace
}  // namespace tn
