// Calculation stage of tensorized inference (TensorNEAT Section 3.3), batched
// over the whole population and a batch of observations.
//
// Mapping: a workgroup of W wavefronts evaluates one genome on a tile of
// 64*K observations at a time (lane = K consecutive observations). Node values
// live in LDS as vals[position][observation of the tile], one copy per
// workgroup. The tile is evaluated level by level: the positions of one level
// of the topological order are independent, so the W wavefronts take them
// round-robin and meet at a barrier before the next level. The genome's
// program (per-position in-edge range, node function, bias, response and the
// in-edge list) is identical for every lane: it is staged in LDS once per
// workgroup when it fits (global scalar loads otherwise), all loops over it are
// wavefront uniform and every value read is one conflict-free row access.
// Observations are read with consecutive threads on consecutive floats and
// scattered into the input rows; outputs are gathered the same way, so global
// traffic is coalesced.
#include <algorithm>

#include "fwd_core.hpp"

namespace tn {

namespace {

struct FwdArgs {
  int64_t obs_stride;
  int B;
  int64_t target_stride;
  float scale, offset;
  int n_tiles;   // tiles of 64*K observations per genome
  int n_groups;  // workgroups per genome
  int per_wg;    // consecutive tiles per workgroup
};

// LDS of one workgroup: level starts, io positions, [staged program], rows.
// A row holds the tile's 64*K values plus K floats of padding, so that the
// observation scatter (consecutive threads on consecutive input rows) spreads
// over the LDS banks.
struct FwdLds {
  size_t lvl_off, io_off, rec_off, edge_off, rows_off, bytes;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline FwdLds fwd_lds(int N_max, int C_max, int nio, int K, bool prog_lds) {
  FwdLds L;
  L.lvl_off = 0;
  L.io_off = align16(L.lvl_off + sizeof(int32_t) * (size_t)(N_max + 2));
  L.rec_off = align16(L.io_off + sizeof(int32_t) * (size_t)nio);
  L.edge_off = L.rec_off + (prog_lds ? sizeof(NodeRec) * (size_t)N_max : 0);
  L.rows_off = align16(L.edge_off + (prog_lds ? sizeof(EdgeRec) * (size_t)C_max : 0));
  L.bytes = L.rows_off + sizeof(float) * (size_t)N_max * (kWave + 1) * K;
  return L;
}

// Consecutive workgroups go to the 8 XCDs in turn; this keeps a genome's
// workgroups on one XCD so its program is fetched into one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  const int full = per * kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * per + bid / kXcd;
}

template <int K, bool kLoss, bool kProgLds>
__global__ __launch_bounds__(kWave * 8) void forward_kernel(
    PopView pop, const int32_t* __restrict__ status, const int32_t* __restrict__ n_valid,
    const int32_t* __restrict__ level, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ src, const int32_t* __restrict__ w_bits,
    const int32_t* __restrict__ fn, const int32_t* __restrict__ bias_bits,
    const int32_t* __restrict__ resp_bits, const int32_t* __restrict__ io_pos,
    const float* __restrict__ obs, float* __restrict__ out, const float* __restrict__ target,
    float* __restrict__ loss, FwdArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int n_lvl_sh;
  __shared__ float part[16];
  constexpr int kTile = kWave * K;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int W = blockDim.x / kWave;
  const int T = blockDim.x;
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  const FwdLds L = fwd_lds(pop.N_max, pop.C_max, nio, K, kProgLds);
  int32_t* lvl = reinterpret_cast<int32_t*>(lds + L.lvl_off);
  int32_t* io_l = reinterpret_cast<int32_t*>(lds + L.io_off);
  NodeRec* recs = reinterpret_cast<NodeRec*>(lds + L.rec_off);
  EdgeRec* edges = reinterpret_cast<EdgeRec*>(lds + L.edge_off);
  float* vals = reinterpret_cast<float*>(lds + L.rows_off);

  int g, t_begin, t_end;
  if (kLoss) {
    g = blockIdx.x;
    t_begin = 0;
    t_end = a.n_tiles;
  } else {
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    g = item / a.n_groups;
    t_begin = (item - g * a.n_groups) * a.per_wg;
    t_end = min(t_begin + a.per_wg, a.n_tiles);
  }
  const int st = status[g];
  const int n = n_valid[g];
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g), rb = pop.rowptr_base(g);

  // stage: level starts (wavefront 0), io positions and the program (all)
  if (!st) {
    if (wave == 0) {
      int cnt = 0;
      for (int base = 0; base < n; base += kWave) {
        const int p = base + lane;
        const bool start = p < n && (p == 0 || level[nb + p] != level[nb + p - 1]);
        const uint64_t m = __ballot(start);
        if (start) lvl[cnt + mbcnt(m)] = p;
        cnt += __popcll(m);
      }
      if (lane == 0) {
        lvl[cnt] = n;
        n_lvl_sh = cnt;
      }
    }
    for (int k = threadIdx.x; k < nio; k += T) io_l[k] = io_pos[(int64_t)g * nio + k];
    if (kProgLds) {
      for (int p = threadIdx.x; p < n; p += T) {
        NodeRec r;
        r.erange = row_ptr[rb + p] | (row_ptr[rb + p + 1] << 16);
        r.fn = fn[nb + p];
        r.bias = __int_as_float(bias_bits[nb + p]);
        r.resp = __int_as_float(resp_bits[nb + p]);
        recs[p] = r;
      }
      const int n_edges = row_ptr[rb + n];
      for (int e = threadIdx.x; e < n_edges; e += T) {
        EdgeRec q;
        q.src = src[cb + e];
        q.w = __int_as_float(w_bits[cb + e]);
        edges[e] = q;
      }
    }
  }
  __syncthreads();
  const int n_lvl = st ? 0 : n_lvl_sh;
  LdsProg lp{recs, edges};
  GlobalProg gp{row_ptr + rb, fn + nb, bias_bits + nb, resp_bits + nb, src + cb, w_bits + cb};

  constexpr int kRow = (kWave + 1) * K;  // floats per LDS row
  float* mine = vals + lane * K;

  // Offsets of this thread's elements in a full tile, computed once: input
  // element i = tid + j*T (observation b, component c) goes to row io[c],
  // column b; output element i = tid + j*T comes from row io[I + c].
  constexpr int kMaxIn = K == 1 ? 8 : 16, kMaxOut = K == 1 ? 4 : 8;
  const int n_in_el = kTile * I, n_out_el = kTile * O;
  const int J_in = (n_in_el + T - 1) / T, J_out = (n_out_el + T - 1) / T;
  const bool fast_in = J_in <= kMaxIn, fast_out = J_out <= kMaxOut;
  int in_off[kMaxIn], out_off[kMaxOut];
  if (!st) {
    DivWalk di(threadIdx.x, I > 0 ? I : 1, T);
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j) {
      in_off[j] = (I > 0 && threadIdx.x + j * T < n_in_el) ? io_l[di.c] * kRow + di.b : -1;
      di.step();
    }
    DivWalk dq(threadIdx.x, O, T);
#pragma unroll
    for (int j = 0; j < kMaxOut; ++j) {
      out_off[j] = (threadIdx.x + j * T < n_out_el) ? io_l[I + dq.c] * kRow + dq.b : -1;
      dq.step();
    }
  }

  float sse = 0.0f;
  // Observations of the next full tile are loaded into registers while the
  // current tile is evaluated (one tile of lookahead).
  float pre[kMaxIn];
  auto load_full = [&](int tt) {
    const float* xq = obs + (int64_t)g * a.obs_stride + (int64_t)tt * kTile * I;
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j)
      if (j < J_in) pre[j] = xq[in_off[j] >= 0 ? threadIdx.x + j * T : 0];
  };
  auto is_full = [&](int tt) { return tt < t_end && min(kTile, a.B - tt * kTile) == kTile; };
  if (!st && fast_in && I > 0 && is_full(t_begin)) load_full(t_begin);
  for (int t = t_begin; t < t_end; ++t) {
    const int b0 = t * kTile;
    const int nbat = min(kTile, a.B - b0);
    float* outp = out ? out + ((int64_t)g * a.B + b0) * O : nullptr;
    if (st) {
      if (outp)
        for (int i = threadIdx.x; i < nbat * O; i += T) outp[i] = __builtin_nanf("");
      continue;
    }
    const bool full = nbat == kTile;
    const float* xo = obs + (int64_t)g * a.obs_stride + (int64_t)b0 * I;
    if (full && fast_in) {
      if (I > 0) {
#pragma unroll
        for (int j = 0; j < kMaxIn; ++j)
          if (j < J_in && in_off[j] >= 0) vals[in_off[j]] = pre[j];
        if (is_full(t + 1)) load_full(t + 1);
      }
    } else if (I > 0) {
      const int total = nbat * I;
      DivWalk dw(threadIdx.x, I, T);
      for (int i = threadIdx.x; i < total; i += T, dw.step()) vals[io_l[dw.c] * kRow + dw.b] = xo[i];
    }
    __syncthreads();
    for (int l = 0; l < n_lvl; ++l) {
      const int p1 = lvl[l + 1];
      for (int p = lvl[l] + wave; p < p1; p += W) {
        if (kProgLds)
          eval_node<K, kRow>(lp, p, mine);
        else
          eval_node<K, kRow>(gp, p, mine);
      }
      __syncthreads();
    }
    const float* tg = kLoss ? target + (int64_t)g * a.target_stride + (int64_t)b0 * O : nullptr;
    if (full && fast_out) {
      float y[kMaxOut], tv[kMaxOut];
#pragma unroll
      for (int j = 0; j < kMaxOut; ++j) {
        if (j < J_out) {
          const bool ok = out_off[j] >= 0;
          y[j] = vals[ok ? out_off[j] : 0];
          if (kLoss) tv[j] = tg[ok ? threadIdx.x + j * T : 0];
        }
      }
#pragma unroll
      for (int j = 0; j < kMaxOut; ++j) {
        if (j < J_out && out_off[j] >= 0) {
          if (outp) outp[threadIdx.x + j * T] = y[j];
          if (kLoss) {
            const float d = y[j] - tv[j];
            sse = fmaf(d, d, sse);
          }
        }
      }
    } else {
      const int total = nbat * O;
      DivWalk dw(threadIdx.x, O, T);
      for (int i = threadIdx.x; i < total; i += T, dw.step()) {
        const float y = vals[io_l[I + dw.c] * kRow + dw.b];
        if (outp) outp[i] = y;
        if (kLoss) {
          const float d = y - tg[i];
          sse = fmaf(d, d, sse);
        }
      }
    }
    __syncthreads();
  }
  if (kLoss) {
    // deterministic: fixed per-thread assignment, fixed reduction order
    const float total = wave_sum(sse);
    if (lane == 0) part[wave] = total;
    __syncthreads();
    if (threadIdx.x == 0) {
      float acc = 0.0f;
      for (int v = 0; v < W; ++v) acc += part[v];
      loss[g] = st ? __builtin_nanf("") : fmaf(a.scale, acc, a.offset);
    }
  }
}

template <int K, bool kLoss, bool kProgLds>
int launch_k(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
             const float* target, float* loss, const FwdArgs& a, int grid, int waves,
             hipStream_t stream) {
  const size_t lds = fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, kProgLds).bytes;
  int rc = allow_lds((const void*)forward_kernel<K, kLoss, kProgLds>, lds);
  if (rc != TN_OK || grid == 0) return rc;
  hipLaunchKernelGGL((forward_kernel<K, kLoss, kProgLds>), dim3((unsigned)grid),
                     dim3(kWave * waves), lds, stream, make_view(p), t.status, t.n_valid,
                     t.level, t.row_ptr, t.edge_src, reinterpret_cast<const int32_t*>(t.edge_w),
                     t.pos_fn, reinterpret_cast<const int32_t*>(t.pos_bias),
                     reinterpret_cast<const int32_t*>(t.pos_resp), t.io_pos, obs, out, target,
                     loss, a);
  return check_launch();
}

// Program in LDS if it fits beside the rows, else read from global memory.
bool prog_fits(const tn_population& p, int K) {
  return fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, true).bytes <= max_dynamic_lds();
}

template <bool kLoss>
int dispatch(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
             const float* target, float* loss, const FwdArgs& a, int grid, int K, int waves,
             hipStream_t stream) {
  const bool in_lds = prog_fits(p, K);
  if (!in_lds && fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, false).bytes > max_dynamic_lds())
    return TN_EUNSUPPORTED;
#define TN_FWD_CASE(KK)                                                                     \
  case KK:                                                                                  \
    return in_lds ? launch_k<KK, kLoss, true>(p, t, obs, out, target, loss, a, grid, waves, \
                                              stream)                                       \
                  : launch_k<KK, kLoss, false>(p, t, obs, out, target, loss, a, grid,       \
                                               waves, stream);
  switch (K) {
    TN_FWD_CASE(1)
    TN_FWD_CASE(2)
    TN_FWD_CASE(4)
    default: return TN_EINVAL;
  }
#undef TN_FWD_CASE
}

}  // namespace

size_t forward_lds_bytes(int N_max, int C_max, int nio, int K) {
  return fwd_lds(N_max, C_max, nio, K, true).bytes;
}

int launch_forward(const tn_population& p, const tn_transformed& t, const float* obs,
                   int64_t obs_stride, int B, float* out, int K, int waves, hipStream_t stream) {
  if (K == 0) K = 1;
  if (waves <= 0) waves = 4;
  const int tile = kWave * K;
  const int n_tiles = (B + tile - 1) / tile;
  // enough workgroups to fill the chip; each takes consecutive tiles of a genome
  const int want = std::max(1, std::min(n_tiles, (2048 + p.P - 1) / std::max(1, p.P)));
  const int per_wg = (n_tiles + want - 1) / want;
  const int n_groups = (n_tiles + per_wg - 1) / per_wg;
  FwdArgs a{obs_stride, B, 0, 0.0f, 0.0f, n_tiles, n_groups, per_wg};
  const int64_t grid = (int64_t)p.P * n_groups;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  return dispatch<false>(p, t, obs, out, nullptr, nullptr, a, (int)grid, K, waves, stream);
}

int launch_forward_loss(const tn_population& p, const tn_transformed& t, const float* obs,
                        int64_t obs_stride, int B, const float* target, int64_t target_stride,
                        float scale, float offset, float* out, float* loss, hipStream_t stream) {
  const int n_tiles = (B + kWave - 1) / kWave;
  FwdArgs a{obs_stride, B, target_stride, scale, offset, n_tiles, 1, n_tiles};
  return dispatch<true>(p, t, obs, out, target, loss, a, p.P, 1, 4, stream);
}

}  // namespace tn
