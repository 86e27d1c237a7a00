// Forward pass of recurrent networks (network type "recurrent" of Appendix
// A). The paper details the calculation only for feedforward networks
// (Section 3.3); a recurrent one has no topological order, so it is evaluated
// by T synchronous sweeps: input nodes hold the observation, every other node
// starts at 0, and sweep t computes every non-input node with the Section 3.3
// node rule (response scaling the aggregate) from the values of sweep t - 1.
//
// One workgroup of four wavefronts per genome:
//   1. checks: node keys and markings hashed in LDS (repeats), input / output
//      keys present, enabled connections' endpoints present and not ending at
//      an input, attribute codes in range; any failure: NaN outputs;
//   2. the enabled in-edges grouped by destination node row in ascending
//      connection row (one bitonic sort of dst_row << 12 | conn_row in LDS),
//      each as one 8-byte record (source row offset, weight); one 16-byte
//      record per computed (non-input) row: function word with the row, its
//      in-edge range, bias, response;
//   3. tiles of 64 observations (one per lane): two LDS value buffers of
//      N_max rows x 64, read from one and written to the other each sweep; the
//      computed rows' records are dealt round-robin to the four wavefronts,
//      one barrier per sweep.
// The sum aggregation accumulates with fused multiply-adds in ascending
// in-edge order and z = fma(response, aggregate, bias), as in the feedforward
// engines, so on an acyclic sum-aggregation genome T sweeps past its largest
// level reproduce the feedforward outputs bit for bit.
#include <algorithm>

#include "fwd_core.hpp"
#include "tn_internal.hpp"

namespace tn {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int32_t kRowEmpty = 0x40000000;  // node function word of an empty row
constexpr int32_t kSortPad = 0x7fffffff;

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

struct Layout {
  int HN, HM, S;          // key hash, marking hash, sort entries (powers of two)
  size_t phase1, vals;    // bytes of the two aliased regions
  size_t persist;         // bytes of the kept tables
  size_t total;
};

Layout layout(int N, int C, int nio) {
  Layout l;
  l.HN = next_pow2(2 * N);
  l.HM = next_pow2(2 * C);
  l.S = next_pow2(C);
  l.phase1 = 8 * (size_t)l.HN + 8 * (size_t)l.HM + 4 * (size_t)l.S;
  l.vals = 2 * (size_t)N * kWave * sizeof(float);
  const size_t p = 16 * (size_t)N + 8 * (size_t)C + 4 * (size_t)N + 4 * (size_t)nio;
  l.persist = (p + 15) & ~size_t(15);
  l.total = l.persist + std::max(l.phase1, l.vals);
  return l;
}

__global__ __launch_bounds__(kBlock) void recurrent_kernel(PopView pop, const float* obs,
                                                           int64_t obs_stride, int B, int T,
                                                           float* out, int32_t* status_out,
                                                           int HN, int HM, int S,
                                                           size_t persist) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int status;
  __shared__ int n_act;  // entries of crec
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = lane_id(), wv = wave_id();
  const int N = pop.N_max, C = pop.C_max, n_in = pop.n_in, n_out = pop.n_out;
  const int nio = n_in + n_out;
  // kept tables
  int4* crec = (int4*)smem;                     // [N] computed row: act | agg << 8 | row << 16,
                                                //     e0 | e1 << 16, bias bits, response bits
  int2* edge = (int2*)(crec + N);               // [C] in-edge: source row * 64, weight bits
  int32_t* nfn = (int32_t*)(edge + C);          // [N] act | agg << 8; input: bit 31 | index
  int32_t* iorow = nfn + N;                     // [n_in + n_out] node row of key k
  unsigned char* region = smem + persist;
  // phase 1 region
  int32_t* hk = (int32_t*)region;               // [HN] node keys
  int32_t* hr = hk + HN;                        // [HN] first row holding the key
  long long* mk = (long long*)(hr + HN);        // [HM] markings
  int32_t* skey = (int32_t*)(mk + HM);          // [S] dst_row << 12 | conn_row
  // phase 2 region
  float* vals = (float*)region;                 // [2][N][64]

  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g);
  const int64_t nrows = pop.node_rows(g), crows = pop.conn_rows(g);
  if (tid == 0) {
    status = 0;
    n_act = 0;
  }
  for (int h = tid; h < HN; h += kBlock) {
    hk[h] = -1;
    hr[h] = 0x7fffffff;
  }
  for (int h = tid; h < HM; h += kBlock) mk[h] = -1;
  __syncthreads();
  const bool oversize = nrows > N || crows > C || nrows < 0 || crows < 0;
  if (oversize) {
    if (tid == 0) status = TN_OVERSIZE;
  } else {
    // node rows: key hash (first row of each key), repeats, attribute codes
    for (int r = tid; r < N; r += kBlock) {
      const int32_t k = r < nrows ? pop.node_key[nb + r] : -1;
      if (k < 0) continue;
      const int act = pop.node_act[nb + r], agg = pop.node_agg[nb + r];
      int bits = (act > TN_ACT_ABS || agg > TN_AGG_MAXABS) ? TN_BAD_ATTR : 0;
      uint32_t h = hash32((uint32_t)k) & (uint32_t)(HN - 1);
      while (true) {
        const int32_t prev = atomicCAS(&hk[h], -1, k);
        if (prev == -1) break;
        if (prev == k) {
          bits |= TN_DUP_NODE;
          break;
        }
        h = (h + 1) & (uint32_t)(HN - 1);
      }
      atomicMin(&hr[h], r);
      if (bits) atomicOr(&status, bits);
    }
    // connection rows: repeated markings (enabled or not)
    for (int r = tid; r < (int)crows; r += kBlock) {
      const int32_t a = pop.conn_in[cb + r], b = pop.conn_out[cb + r];
      if (a < 0 || b < 0) continue;
      const long long m = ((long long)a << 32) | (long long)(uint32_t)b;
      uint32_t h = hash32((uint32_t)a ^ hash32((uint32_t)b)) & (uint32_t)(HM - 1);
      while (true) {
        const long long prev = (long long)atomicCAS((unsigned long long*)&mk[h], ~0ull,
                                                    (unsigned long long)m);
        if (prev == -1) break;
        if (prev == m) {
          atomicOr(&status, TN_DUP_CONN);
          break;
        }
        h = (h + 1) & (uint32_t)(HM - 1);
      }
    }
  }
  __syncthreads();
  auto row_of = [&](int32_t k) -> int {
    uint32_t h = hash32((uint32_t)k) & (uint32_t)(HN - 1);
    while (true) {
      const int32_t kk = hk[h];
      if (kk == k) return hr[h];
      if (kk == -1) return -1;
      h = (h + 1) & (uint32_t)(HN - 1);
    }
  };
  if (!oversize) {
    for (int k = tid; k < nio; k += kBlock) {
      const int r = row_of(k);
      iorow[k] = r;
      if (r < 0) atomicOr(&status, TN_MISSING_IO);
    }
    // enabled connections: endpoints present, not ending at an input; sort keys
    for (int r = tid; r < S; r += kBlock) {
      int32_t key = kSortPad;
      if (r < crows) {
        const int32_t a = pop.conn_in[cb + r], b = pop.conn_out[cb + r];
        if (a >= 0 && b >= 0 && pop.conn_en[cb + r]) {
          const int ra = row_of(a), rb = row_of(b);
          int bits = 0;
          if (ra < 0 || rb < 0) bits |= TN_DANGLING;
          if (b < n_in) bits |= TN_INPUT_DST;
          if (bits) atomicOr(&status, bits);
          else key = (rb << 12) | r;
        }
      }
      skey[r] = key;
    }
  }
  __syncthreads();
  const int st = status;
  if (st != 0) {
    const float nan = __builtin_nanf("");
    for (int64_t i = tid; i < (int64_t)B * n_out; i += kBlock) out[(int64_t)g * B * n_out + i] = nan;
    if (status_out && tid == 0) status_out[g] = st;
    return;
  }
  // bitonic sort of the S keys (ascending): in-edges by destination row,
  // then connection row
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < S; i += kBlock) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int32_t a = skey[i], b = skey[ixj];
          if ((a > b) == ((i & k) == 0)) {
            skey[i] = b;
            skey[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < S && i < C; i += kBlock) {
    const int32_t key = skey[i];
    if (key == kSortPad) continue;
    const int row = key & 0xfff;
    edge[i] = make_int2(row_of(pop.conn_in[cb + row]) * kWave,
                        __float_as_int(pop.conn_w[cb + row]));
  }
  for (int r = tid; r < N; r += kBlock) {
    const int32_t k = r < nrows ? pop.node_key[nb + r] : -1;
    int32_t f = kRowEmpty;
    if (k >= 0 && k < n_in) f = (int32_t)(kFnInput | (uint32_t)k);
    else if (k >= 0) f = pop.node_act[nb + r] | (pop.node_agg[nb + r] << 8);
    nfn[r] = f;
    // the computed rows' records, in any order (the rows of a sweep are
    // independent); in-edges e0 .. e1-1 from the sorted keys
    if (f >= 0 && f != kRowEmpty) {
      auto first = [&](int32_t want) {
        int lo = 0, hi = S;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (skey[mid] < want) lo = mid + 1;
          else hi = mid;
        }
        return lo;
      };
      const int e0 = first(r << 12), e1 = first((r + 1) << 12);
      crec[atomicAdd(&n_act, 1)] =
          make_int4(f | (r << 16), e0 | (e1 << 16), __float_as_int(pop.node_bias[nb + r]),
                    __float_as_int(pop.node_resp[nb + r]));
    }
  }
  if (status_out && tid == 0) status_out[g] = 0;
  __syncthreads();  // phase 1 region is reused for the values from here on

  const int na = __builtin_amdgcn_readfirstlane(n_act);
  const float* x_g = obs + (int64_t)g * obs_stride;
  float* out_g = out + (int64_t)g * B * n_out;
  for (int b0 = 0; b0 < B; b0 += kWave) {
    const int b = b0 + lane;
    const bool active = b < B;
    for (int r = wv; r < N; r += kWaves) {
      const int32_t f = nfn[r];
      if (f == kRowEmpty) continue;
      float v = 0.0f;
      if (f < 0) v = active ? x_g[(int64_t)b * n_in + (f & 0xffff)] : 0.0f;
      vals[r * kWave + lane] = v;
      vals[(N + r) * kWave + lane] = v;
    }
    __syncthreads();
    for (int t = 0; t < T; ++t) {
      const float* cur = vals + (size_t)(t & 1) * N * kWave;
      float* nxt = vals + (size_t)((t + 1) & 1) * N * kWave;
      // the computed rows, dealt round-robin to the wavefronts; the row, its
      // function word and in-edge range as wavefront-uniform values (scalar
      // loop control and branches)
      for (int i = wv; i < na; i += kWaves) {
        const int4 q = crec[i];  // one 16-byte read
        const int fr = __builtin_amdgcn_readfirstlane(q.x);
        const int er = __builtin_amdgcn_readfirstlane(q.y);
        const int32_t f = fr & 0xffff;
        const int r = fr >> 16;
        const int e0 = er & 0xffff, e1 = er >> 16;
        const int agg = (f >> 8) & 0xff;
        float s;
        if (agg == TN_AGG_SUM) {
          s = 0.0f;
          int e = e0;
          for (; e + 2 <= e1; e += 2) {  // two in-edges' records, then both values
            const int2 q0 = edge[e], q1 = edge[e + 1];
            const float x0 = cur[q0.x + lane], x1 = cur[q1.x + lane];
            s = fmaf(__int_as_float(q0.y), x0, s);
            s = fmaf(__int_as_float(q1.y), x1, s);
          }
          if (e < e1) {
            const int2 q = edge[e];
            s = fmaf(__int_as_float(q.y), cur[q.x + lane], s);
          }
        } else if (e0 == e1) {
          s = 0.0f;
        } else {
          s = __int_as_float(edge[e0].y) * cur[edge[e0].x + lane];
          for (int e = e0 + 1; e < e1; ++e) {
            const float q = __int_as_float(edge[e].y) * cur[edge[e].x + lane];
            switch (agg) {
              case TN_AGG_PRODUCT: s = s * q; break;
              case TN_AGG_MAX: s = fmaxf(s, q); break;
              case TN_AGG_MIN: s = fminf(s, q); break;
              case TN_AGG_MEAN: s = s + q; break;
              default: s = fabsf(q) > fabsf(s) ? q : s; break;  // maxabs
            }
          }
          if (agg == TN_AGG_MEAN) s = s / (float)(e1 - e0);
        }
        float z[1] = {fmaf(__int_as_float(q.w), s, __int_as_float(q.z))}, v[1];
        activate_all<1>(f & 7, z, v);  // codes below 7: checked above
        nxt[r * kWave + lane] = v[0];
      }
      __syncthreads();
    }
    const float* fin = vals + (size_t)(T & 1) * N * kWave;
    if (active)
      for (int j = wv; j < n_out; j += kWaves)
        out_g[(int64_t)b * n_out + j] = fin[iorow[n_in + j] * kWave + lane];
    __syncthreads();
  }
}

}  // namespace

int recurrent_lds_check(const tn_population& p, size_t* bytes) {
  const Layout l = layout(p.N_max, p.C_max, p.n_in + p.n_out);
  *bytes = l.total;
  return l.total > max_dynamic_lds() ? TN_EUNSUPPORTED : TN_OK;
}

int launch_forward_recurrent(const tn_population& p, const float* obs, int64_t obs_stride, int B,
                             int T, float* out, int32_t* status, hipStream_t stream) {
  const Layout l = layout(p.N_max, p.C_max, p.n_in + p.n_out);
  int rc = allow_lds((const void*)recurrent_kernel, l.total);
  if (rc != TN_OK || p.P == 0) return rc;
  hipLaunchKernelGGL(recurrent_kernel, dim3(p.P), dim3(kBlock), l.total, stream, make_view(p), obs,
                     obs_stride, B, T, out, status, l.HN, l.HM, l.S, l.persist);
  return check_launch();
}

}  // namespace tn
