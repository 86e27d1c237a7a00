// Compatibility distance matrix (NEAT speciation; TensorNEAT Section 2.1,
// Algorithm 1, coefficients of Appendix A), over connection genes identified
// by their marking (in-key, out-key) in lexicographic order.
//
// Two launches:
//   prep  one wavefront per genome: gather the valid connection rows into LDS,
//         bitonic-sort them by marking, flag repeated markings, and store the
//         sorted list position-major (keysT[k][g]) so that 64 genomes' k-th
//         genes are 64 consecutive words.
//   pairs block = up to kMaxRows "row" genomes x 256 "column" genomes (see
//         pair_kernel): row genes in LDS hashes, each column gene read once
//         and probed against every row; only the pairs on or above the
//         diagonal are evaluated, each written to both halves.
#include <algorithm>
#include <mutex>

#include "genes.hpp"
#include "tn_internal.hpp"

namespace tn {

namespace {

constexpr long long kPadKey = 0x7fffffffffffffffll;

__device__ __forceinline__ uint32_t mix32(uint32_t k) {
  // lowbias32 (Chris Wellons' integer hash constants)
  k ^= k >> 16;
  k *= 0x7feb352du;
  k ^= k >> 15;
  k *= 0x846ca68bu;
  k ^= k >> 16;
  return k;
}

__device__ __forceinline__ uint32_t hash_mark(long long k) {
  return mix32((uint32_t)k ^ mix32((uint32_t)((unsigned long long)k >> 32)));
}

struct Ws {
  int32_t* cnt;      // [P] gene count, -1 when a marking repeats
  long long* maxk;   // [P] largest marking, -1 when there are none
  long long* keysT;  // [C_max][P]
  float* wT;         // [C_max][P]
  int32_t* hT;       // [C_max][P] hash of each marking (hash_mark), computed once
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Ws carve(void* base, int P, int C) {
  unsigned char* p = (unsigned char*)base;
  Ws w;
  size_t o = 0;
  w.cnt = (int32_t*)(p + o);
  o += align_up(sizeof(int32_t) * P);
  w.maxk = (long long*)(p + o);
  o += align_up(sizeof(long long) * P);
  w.keysT = (long long*)(p + o);
  o += align_up(sizeof(long long) * (size_t)P * C);
  w.wT = (float*)(p + o);
  o += align_up(sizeof(float) * (size_t)P * C);
  w.hT = (int32_t*)(p + o);
  return w;
}

size_t ws_bytes(int P, int C) {
  return align_up(sizeof(int32_t) * P) + align_up(sizeof(long long) * P) +
         align_up(sizeof(long long) * (size_t)P * C) + align_up(sizeof(float) * (size_t)P * C) +
         align_up(sizeof(int32_t) * (size_t)P * C);
}

int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

__global__ __launch_bounds__(kWave) void prep_kernel(PopView pop, Ws ws, int S) {
  extern __shared__ __align__(16) unsigned char smem[];
  long long* key = (long long*)smem;          // [S]
  float* w = (float*)(smem + sizeof(long long) * S);  // [S]
  __shared__ int dup;
  const int g = blockIdx.x;
  const int lane = lane_id();
  const int P = pop.P;
  const int64_t cb = pop.conn_base(g);
  const int64_t crows = pop.conn_rows(g);
  if (crows > pop.C_max || crows < 0) {
    if (lane == 0) {
      ws.cnt[g] = -1;
      ws.maxk[g] = -1;
    }
    return;
  }
  if (lane == 0) dup = 0;
  int n = 0;
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
      const int at = n + mbcnt(m);
      key[at] = ((long long)a << 32) | (long long)(uint32_t)b;
      w[at] = pop.conn_w[cb + r];
    }
    n += __popcll(m);
  }
  for (int i = n + lane; i < S; i += kWave) {
    key[i] = kPadKey;
    w[i] = 0.0f;
  }
  __syncthreads();
  // bitonic sort of S entries (S is a power of two)
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < S; i += kWave) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const long long ki = key[i], kj = key[ixj];
          const bool up = (i & k) == 0;
          if ((ki > kj) == up) {
            key[i] = kj;
            key[ixj] = ki;
            const float t = w[i];
            w[i] = w[ixj];
            w[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = lane + 1; i < n; i += kWave)
    if (key[i] == key[i - 1]) dup = 1;
  __syncthreads();
  for (int k = lane; k < n; k += kWave) {
    ws.keysT[(int64_t)k * P + g] = key[k];
    ws.wT[(int64_t)k * P + g] = w[k];
    ws.hT[(int64_t)k * P + g] = (int32_t)hash_mark(key[k]);
  }
  if (lane == 0) {
    ws.cnt[g] = dup ? -1 : n;
    ws.maxk[g] = n > 0 ? key[n - 1] : -1;
  }
}

constexpr int kPairBlock = 256;
constexpr int kMaxRows = 2;  // row genomes per block (measured best of 1, 2, 4, 8)

// Block = up to kMaxRows "row" genomes i0 .. i0+R-1 x 256 "column" genomes.
// Each row genome's genes go into an LDS hash (marking -> weight) plus its
// sorted list. Each lane walks its column genome's sorted list once
// (coalesced across the wavefront), hashes every marking once and probes all
// R tables: matches (|dw| summed in ascending marking order per row), column
// genes beyond each row's largest marking; then per row a binary search for
// the row's genes beyond the column's largest marking. The column genes are
// read from memory once per R rows.
__global__ __launch_bounds__(kPairBlock) void pair_kernel(Ws ws, int P, int HC, int C, int R,
                                                           float c1, float c2, float c3,
                                                           float* dist, int32_t* E_out,
                                                           int32_t* D_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  // per row r: hash keys [HC], hash weights [HC], sorted list [C]
  long long* hk_all = (long long*)smem;                                   // [R][HC]
  long long* si_all = hk_all + (size_t)R * HC;                             // [R][C]
  float* hw_all = (float*)(si_all + (size_t)R * C);                        // [R][HC]
  const int i0 = blockIdx.y * R;
  const int j = blockIdx.x * kPairBlock + threadIdx.x;
  const int nr = min(R, P - i0);
  // the distance is symmetric bit for bit (the matched markings are visited
  // in ascending order from either side): only pairs j >= i are evaluated,
  // each written to both halves of the matrix
  if ((int)(blockIdx.x * kPairBlock + kPairBlock - 1) < i0) return;  // all below the diagonal
  for (int h = threadIdx.x; h < nr * HC; h += kPairBlock) hk_all[h] = -1;
  __syncthreads();
  for (int r = 0; r < nr; ++r) {
    const int i = i0 + r;
    const int ni = ws.cnt[i];
    long long* hk = hk_all + (size_t)r * HC;
    float* hw = hw_all + (size_t)r * HC;
    long long* si = si_all + (size_t)r * C;
    for (int k = threadIdx.x; k < ni; k += kPairBlock) {
      const long long key = ws.keysT[(int64_t)k * P + i];
      si[k] = key;
      uint32_t h = (uint32_t)ws.hT[(int64_t)k * P + i] & (uint32_t)(HC - 1);
      while (atomicCAS((unsigned long long*)&hk[h], ~0ull, (unsigned long long)key) != ~0ull)
        h = (h + 1) & (uint32_t)(HC - 1);
      hw[h] = ws.wT[(int64_t)k * P + i];
    }
  }
  __syncthreads();
  if (j >= P) return;
  const int nj = ws.cnt[j];
  int ni[kMaxRows];
  long long maxi[kMaxRows];
  int M[kMaxRows], ex[kMaxRows];
  float S[kMaxRows];
#pragma unroll
  for (int r = 0; r < kMaxRows; ++r) {
    ni[r] = r < nr ? ws.cnt[i0 + r] : 0;
    maxi[r] = r < nr ? ws.maxk[i0 + r] : -1;
    M[r] = 0;
    ex[r] = 0;
    S[r] = 0.0f;
  }
  for (int k = 0; k < max(nj, 0); ++k) {
    const long long key = ws.keysT[(int64_t)k * P + j];
    const float w = ws.wT[(int64_t)k * P + j];
    const uint32_t h0 = (uint32_t)ws.hT[(int64_t)k * P + j] & (uint32_t)(HC - 1);
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
      if (r >= nr || ni[r] < 0 || j < i0 + r) continue;
      ex[r] += key > maxi[r];
      const long long* hk = hk_all + (size_t)r * HC;
      uint32_t h = h0;
      while (true) {
        const long long kk = hk[h];
        if (kk == key) {
          ++M[r];
          S[r] += fabsf(hw_all[(size_t)r * HC + h] - w);
          break;
        }
        if (kk == -1) break;
        h = (h + 1) & (uint32_t)(HC - 1);
      }
    }
  }
  const long long maxj = ws.maxk[j];
#pragma unroll
  for (int r = 0; r < kMaxRows; ++r) {
    if (r >= nr || j < i0 + r) continue;
    const int64_t o = (int64_t)(i0 + r) * P + j;
    const int64_t ot = (int64_t)j * P + (i0 + r);  // the mirrored entry (o itself on the diagonal)
    if (ni[r] < 0 || nj < 0) {
      dist[o] = __builtin_nanf("");
      dist[ot] = __builtin_nanf("");
      if (E_out) {
        E_out[o] = -1;
        D_out[o] = -1;
        E_out[ot] = -1;
        D_out[ot] = -1;
      }
      continue;
    }
    // row genes beyond the column's largest marking: ni - upper_bound(si, maxj)
    const long long* si = si_all + (size_t)r * C;
    int lo = 0, hi = ni[r];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (si[mid] <= maxj) lo = mid + 1;
      else hi = mid;
    }
    const int E = ex[r] + (ni[r] - lo);
    const int D = ni[r] + nj - 2 * M[r] - E;
    const int N = max(ni[r], nj);
    float d = 0.0f;
    if (N > 0) {
      const float fN = (float)N;
      d = c1 * (float)E / fN + c2 * (float)D / fN + c3 * (M[r] > 0 ? S[r] / (float)M[r] : 0.0f);
    }
    dist[o] = d;
    dist[ot] = d;
    if (E_out) {
      E_out[o] = E;
      D_out[o] = D;
      E_out[ot] = E;
      D_out[ot] = D;
    }
  }
}


// ------------------------------------------------ node-inclusive distance
//
// delta = sum over the two gene kinds X (node genes, connection genes) of
//   (c_d * D_X + c_h * H_X) / max(|X1|, |X2|)          (0 when both are empty)
// node genes: valid non-input node rows by key; connection genes: valid
// connection rows (enabled or not) by marking. D_X counts the genes only one
// genome holds; H_X sums, over the shared ones in ascending identity order,
// |a0 - a0'| + |a1 - a1'| + [c0 != c0'] + [c1 != c1'] with (a0, a1, c0, c1) =
// (bias, response, act, agg) for a node and (weight, 0, enabled, 0) for a
// connection (the zero terms add exactly nothing).
//
// Same two-launch shape as the connection-gene distance: a prep wavefront per
// genome sorts both gene lists (keys + the row they came from, bitonic in
// LDS), checks repeated keys / markings, and stores them position-major with
// their attributes; the pair kernel hashes R row genomes' genes in LDS and
// walks each column genome's sorted lists once.

struct Gene {
  float a0, a1;
  uint32_t code;
};

__device__ __forceinline__ float attr_distance(Gene p, float a0, float a1, uint32_t code) {
  float t = fabsf(p.a0 - a0) + fabsf(p.a1 - a1);
  t += (p.code & 0xffu) != (code & 0xffu) ? 1.0f : 0.0f;
  t += (p.code >> 8) != (code >> 8) ? 1.0f : 0.0f;
  return t;
}

// Inserts row genome i's genes of one kind into an LDS hash of HC slots.
__device__ __forceinline__ void fill_hash(const GeneList& l, int P, int i, int n, int HC,
                                          long long* hk, Gene* hv) {
  for (int k = threadIdx.x; k < n; k += kPairBlock) {
    const int64_t o = (int64_t)k * P + i;
    const long long key = l.keyT[o];
    uint32_t h = (uint32_t)l.hT[o] & (uint32_t)(HC - 1);
    while (atomicCAS((unsigned long long*)&hk[h], ~0ull, (unsigned long long)key) != ~0ull)
      h = (h + 1) & (uint32_t)(HC - 1);
    hv[h] = Gene{l.a0T[o], l.a1T[o], l.codeT[o]};
  }
}

// Walks column genome j's sorted genes of one kind against the row hashes:
// homologous counts and attribute sums per row, in ascending key order.
__device__ __forceinline__ void walk_genes(const GeneList& l, int P, int j, int nj, int nr,
                                           int i0, const int* ni, int HC,
                                           const long long* hk_all, const Gene* hv_all,
                                           int* hom, float* H) {
  for (int k = 0; k < nj; ++k) {
    const int64_t o = (int64_t)k * P + j;
    const long long key = l.keyT[o];
    const float a0 = l.a0T[o], a1 = l.a1T[o];
    const uint32_t code = l.codeT[o];
    const uint32_t h0 = (uint32_t)l.hT[o] & (uint32_t)(HC - 1);
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
      if (r >= nr || ni[r] < 0 || j < i0 + r) continue;
      const long long* hk = hk_all + (size_t)r * HC;
      uint32_t h = h0;
      while (true) {
        const long long kk = hk[h];
        if (kk == key) {
          ++hom[r];
          H[r] += attr_distance(hv_all[(size_t)r * HC + h], a0, a1, code);
          break;
        }
        if (kk == -1) break;
        h = (h + 1) & (uint32_t)(HC - 1);
      }
    }
  }
}

__device__ __forceinline__ float kind_term(int n1, int n2, int hom, float H, float c_d,
                                           float c_h) {
  const int n = max(n1, n2);
  if (n == 0) return 0.0f;
  return (c_d * (float)(n1 + n2 - 2 * hom) + c_h * H) / (float)n;
}

// Block = up to kMaxRows row genomes x 256 column genomes; LDS per row: the
// node hash [HN] and the connection hash [HC] (keys, then attributes).
__global__ __launch_bounds__(kPairBlock) void pair_nodes_kernel(WsN ws, int P, int HN, int HC,
                                                                 int R, float c_d, float c_h,
                                                                 float* dist, int32_t* DN_out,
                                                                 int32_t* DC_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  long long* nk_all = (long long*)smem;                         // [R][HN]
  long long* ck_all = nk_all + (size_t)R * HN;                  // [R][HC]
  Gene* nv_all = (Gene*)(ck_all + (size_t)R * HC);              // [R][HN]
  Gene* cv_all = nv_all + (size_t)R * HN;                       // [R][HC]
  const int i0 = blockIdx.y * R;
  const int j = blockIdx.x * kPairBlock + threadIdx.x;
  const int nr = min(R, P - i0);
  if ((int)(blockIdx.x * kPairBlock + kPairBlock - 1) < i0) return;  // all below the diagonal
  for (int h = threadIdx.x; h < nr * HN; h += kPairBlock) nk_all[h] = -1;
  for (int h = threadIdx.x; h < nr * HC; h += kPairBlock) ck_all[h] = -1;
  __syncthreads();
  for (int r = 0; r < nr; ++r) {
    const int i = i0 + r;
    const int nn = ws.cnt_n[i], nc = ws.cnt_c[i];
    fill_hash(ws.nodes, P, i, nn, HN, nk_all + (size_t)r * HN, nv_all + (size_t)r * HN);
    fill_hash(ws.conns, P, i, nc, HC, ck_all + (size_t)r * HC, cv_all + (size_t)r * HC);
  }
  __syncthreads();
  if (j >= P) return;
  const int nj_n = ws.cnt_n[j], nj_c = ws.cnt_c[j];
  int ni_n[kMaxRows], ni_c[kMaxRows], hom_n[kMaxRows], hom_c[kMaxRows];
  float H_n[kMaxRows], H_c[kMaxRows];
#pragma unroll
  for (int r = 0; r < kMaxRows; ++r) {
    ni_n[r] = r < nr ? ws.cnt_n[i0 + r] : 0;
    ni_c[r] = r < nr ? ws.cnt_c[i0 + r] : 0;
    hom_n[r] = hom_c[r] = 0;
    H_n[r] = H_c[r] = 0.0f;
  }
  walk_genes(ws.nodes, P, j, max(nj_n, 0), nr, i0, ni_n, HN, nk_all, nv_all, hom_n, H_n);
  walk_genes(ws.conns, P, j, max(nj_c, 0), nr, i0, ni_c, HC, ck_all, cv_all, hom_c, H_c);
#pragma unroll
  for (int r = 0; r < kMaxRows; ++r) {
    if (r >= nr || j < i0 + r) continue;
    const int64_t o = (int64_t)(i0 + r) * P + j;
    const int64_t ot = (int64_t)j * P + (i0 + r);
    float d;
    int dn, dc;
    if (ni_n[r] < 0 || nj_n < 0) {
      d = __builtin_nanf("");
      dn = dc = -1;
    } else {
      d = kind_term(ni_n[r], nj_n, hom_n[r], H_n[r], c_d, c_h) +
          kind_term(ni_c[r], nj_c, hom_c[r], H_c[r], c_d, c_h);
      dn = ni_n[r] + nj_n - 2 * hom_n[r];
      dc = ni_c[r] + nj_c - 2 * hom_c[r];
    }
    dist[o] = d;
    dist[ot] = d;
    if (DN_out) {
      DN_out[o] = dn;
      DC_out[o] = dc;
      DN_out[ot] = dn;
      DC_out[ot] = dc;
    }
  }
}

}  // namespace

size_t distance_workspace_bytes(int P, int C_max) { return ws_bytes(P, C_max); }

// ------------------------------------------------ allocation-free variant

// Workspace of tn_distance_noalloc: a fixed device array instead of a caller
// buffer. Each device holds its own copy for the life of the process; every
// call on a device reuses it (the prep kernel rewrites every entry the pair
// kernel reads, so nothing needs clearing between calls).
static __device__ __align__(256) unsigned char scratch[TN_DISTANCE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (host code must never use the array's name as an address).
int noalloc_scratch(void** out) {
  int dev = 0;
  int rc = record_hip(hipGetDevice(&dev));
  if (rc != TN_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return TN_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    rc = record_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (rc != TN_OK) return rc;
    if (!ptr) return record_hip(hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TN_OK;
}

int launch_distance(const tn_population& p, float c1, float c2, float c3, void* workspace,
                    float* dist, int32_t* E, int32_t* D, hipStream_t stream) {
  const int S = next_pow2(p.C_max);
  const size_t prep_lds = (sizeof(long long) + sizeof(float)) * (size_t)S;
  const int HC = next_pow2(2 * p.C_max);
  const size_t per_row = (sizeof(long long) + sizeof(float)) * (size_t)HC +
                         sizeof(long long) * (size_t)p.C_max;
  // row genomes per block: as many as fit 64 KB of LDS (two blocks per CU), >= 1
  const int R = (int)std::max<size_t>(1, std::min<size_t>(kMaxRows, (64 * 1024) / per_row));
  const size_t pair_lds = per_row * R;
  int rc = allow_lds((const void*)prep_kernel, prep_lds);
  if (rc == TN_OK) rc = allow_lds((const void*)pair_kernel, pair_lds);
  if (rc != TN_OK || p.P == 0) return rc;
  Ws ws = carve(workspace, p.P, p.C_max);
  hipLaunchKernelGGL(prep_kernel, dim3(p.P), dim3(kWave), prep_lds, stream, make_view(p), ws, S);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  dim3 grid((p.P + kPairBlock - 1) / kPairBlock, (p.P + R - 1) / R);
  hipLaunchKernelGGL(pair_kernel, grid, dim3(kPairBlock), pair_lds, stream, ws, p.P, HC,
                     p.C_max, R, c1, c2, c3, dist, E, D);
  return check_launch();
}

size_t distance_nodes_workspace_bytes(int P, int N_max, int C_max) {
  return ws_nodes_bytes(P, N_max, C_max);
}

int launch_distance_nodes(const tn_population& p, float c_d, float c_h, void* workspace,
                          float* dist, int32_t* DN, int32_t* DC, hipStream_t stream) {
  const int S = next_pow2(std::max(p.N_max, p.C_max));
  const size_t prep_lds = (sizeof(long long) + sizeof(int32_t)) * (size_t)S;
  const int HN = next_pow2(2 * p.N_max), HC = next_pow2(2 * p.C_max);
  const size_t per_row = (sizeof(long long) + sizeof(Gene)) * (size_t)(HN + HC);
  const int R = (int)std::max<size_t>(1, std::min<size_t>(kMaxRows, (64 * 1024) / per_row));
  const size_t pair_lds = per_row * R;
  int rc = allow_lds((const void*)prep_nodes_kernel, prep_lds);
  if (rc == TN_OK) rc = allow_lds((const void*)pair_nodes_kernel, pair_lds);
  if (rc != TN_OK || p.P == 0) return rc;
  WsN ws = carve_nodes(workspace, p.P, p.N_max, p.C_max);
  hipLaunchKernelGGL(prep_nodes_kernel, dim3(p.P), dim3(kWave), prep_lds, stream, make_view(p),
                     ws, S);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  dim3 grid((p.P + kPairBlock - 1) / kPairBlock, (p.P + R - 1) / R);
  hipLaunchKernelGGL(pair_nodes_kernel, grid, dim3(kPairBlock), pair_lds, stream, ws, p.P, HN,
                     HC, R, c_d, c_h, dist, DN, DC);
  return check_launch();
}

}  // namespace tn
