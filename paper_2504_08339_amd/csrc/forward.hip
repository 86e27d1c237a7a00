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
#include "fwd_launch.hpp"

namespace tn {

namespace {

struct FwdArgs {
  int64_t obs_stride;
  int B;
  int64_t target_stride;
  float scale, offset;
  int n_tiles;   // tiles of 64*K observations per genome
  int n_groups;  // workgroups per genome
  int per_wg;    // grid form: consecutive tiles per workgroup; persistent: genomes per grab
  int rows;      // value rows per tile in LDS (>= every genome's n_rows)
  int skip_le;   // genomes with prog_rows <= skip_le are left to another launch (-1: none)
  const int32_t* genomes;  // genome list (nullptr: every genome, in order)
  int32_t* queue;          // persistent launch: next list entry to take
  int n_items;             // persistent launch: list length
};

// LDS of one workgroup: level starts, io positions, [staged program], rows.
// A row holds the tile's 64*K values plus K floats of padding, so that the
// observation scatter (consecutive threads on consecutive input rows) spreads
// over the LDS banks.
struct FwdLds {
  size_t lvl_off, io_off, rec_off, edge_off, rows_off, bytes;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline FwdLds fwd_lds(int N_max, int C_max, int nio, int K, bool prog_lds,
                                          int rows) {
  FwdLds L;
  L.lvl_off = 0;
  L.io_off = align16(L.lvl_off + sizeof(int32_t) * (size_t)(N_max + 2));
  L.rec_off = align16(L.io_off + sizeof(int32_t) * (size_t)nio);
  L.edge_off = L.rec_off + (prog_lds ? sizeof(NodeRec) * (size_t)N_max : 0);
  L.rows_off = align16(L.edge_off + (prog_lds ? sizeof(EdgeRec) * (size_t)C_max : 0));
  L.bytes = L.rows_off + sizeof(float) * (size_t)rows * (kWave + 1) * K;
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

// Whole evaluation of genome g on tiles t_begin .. t_end-1 by one workgroup.
// Starts and ends with the workgroup's LDS free (every path ends at a
// barrier), so a persistent workgroup can run it for genome after genome.
template <int K, bool kLoss, bool kProgLds>
__device__ __forceinline__ void lds_genome(
    const PopView& pop, const int32_t* __restrict__ status, const int32_t* __restrict__ n_valid,
    const int32_t* __restrict__ level, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ src, const int32_t* __restrict__ w_bits,
    const int32_t* __restrict__ fn, const int32_t* __restrict__ bias_bits,
    const int32_t* __restrict__ resp_bits, const int32_t* __restrict__ io_pos,
    const int32_t* __restrict__ pos_row, const int32_t* __restrict__ n_rows,
    const int32_t* __restrict__ prog_rows, const float* __restrict__ obs,
    float* __restrict__ out, const float* __restrict__ target, float* __restrict__ loss,
    const FwdArgs& a, int g, int t_begin, int t_end) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int n_lvl_sh;
  __shared__ float part[16];
  constexpr int kTile = kWave * K;
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x / kWave;
  const int T = blockDim.x;
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  const FwdLds L = fwd_lds(pop.N_max, pop.C_max, nio, K, kProgLds, a.rows);
  int32_t* lvl = reinterpret_cast<int32_t*>(lds + L.lvl_off);
  int32_t* io_l = reinterpret_cast<int32_t*>(lds + L.io_off);
  NodeRec* recs = reinterpret_cast<NodeRec*>(lds + L.rec_off);
  EdgeRec* edges = reinterpret_cast<EdgeRec*>(lds + L.edge_off);
  float* vals = reinterpret_cast<float*>(lds + L.rows_off);

  if (prog_rows[g] <= a.skip_le) return;  // uniform per workgroup
  // a genome needing more rows than the launch provides is reported as NaN
  const int st = status[g] ? status[g] : (n_rows[g] > a.rows ? -1 : 0);
  const int n = n_valid[g];
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g), rb = pop.rowptr_base(g);

  constexpr int kMaxIn = K == 1 ? 8 : 16, kMaxOut = K == 1 ? 4 : 8;
  const int n_in_el = kTile * I, n_out_el = kTile * O;
  const int J_in = (n_in_el + T - 1) / T, J_out = (n_out_el + T - 1) / T;
  const bool fast_in = J_in <= kMaxIn, fast_out = J_out <= kMaxOut;
  float sse = 0.0f;
  // Observations of the next full tile are loaded into registers while the
  // current tile is evaluated (one tile of lookahead); the first tile's are
  // requested before the program is staged.
  float pre[kMaxIn];
  auto load_full = [&](int tt) {
    const float* xq = obs + (int64_t)g * a.obs_stride + (int64_t)tt * kTile * I;
#pragma unroll
    for (int j = 0; j < kMaxIn; ++j)
      if (j < J_in) pre[j] = xq[threadIdx.x + j * T < n_in_el ? threadIdx.x + j * T : 0];
  };
  auto is_full = [&](int tt) { return tt < t_end && min(kTile, a.B - tt * kTile) == kTile; };
  if (!st && fast_in && I > 0 && is_full(t_begin)) load_full(t_begin);

  // stage: level starts, io positions and the program, every thread a share.
  // Levels are the Kahn rounds 0, 1, ..., each non-empty, and positions are
  // in level order, so the start of level L is the one position p with
  // level L whose predecessor has a lower level: one independent pass.
  if (!st) {
    for (int p = threadIdx.x; p < n; p += T) {
      const int lv = level[nb + p];
      if (p == 0 || level[nb + p - 1] != lv) lvl[lv] = p;
    }
    if (threadIdx.x == 0) {
      const int cnt = n > 0 ? level[nb + n - 1] + 1 : 0;
      lvl[cnt] = n;
      n_lvl_sh = cnt;
    }
    for (int k = threadIdx.x; k < nio; k += T)
      io_l[k] = pos_row[nb + io_pos[(int64_t)g * nio + k]];
    if (kProgLds) {
      constexpr int kRowBytes = (int)(sizeof(float) * (kWave + 1) * K);
      for (int p = threadIdx.x; p < n; p += T) {
        NodeRec r;
        r.erange = row_ptr[rb + p] | (row_ptr[rb + p + 1] << 16);
        // act | agg << 3 | byte offset of the value row << 6 (LdsProgT<true>)
        const int f0 = fn[nb + p];
        r.fn = f0 < 0 ? f0
                      : (f0 & 0xff) | (((f0 >> 8) & 0xff) << 3) | ((pos_row[nb + p] * kRowBytes) << 6);
        r.bias = __int_as_float(bias_bits[nb + p]);
        r.resp = __int_as_float(resp_bits[nb + p]);
        recs[p] = r;
      }
      // two in-edges per thread and step, both sources' row loads in flight
      // together
      const int n_edges = row_ptr[rb + n];
      for (int e = threadIdx.x; e < n_edges; e += 2 * T) {
        const int e2 = e + T;
        const bool two = e2 < n_edges;
        const int s1 = src[cb + e], s2 = two ? src[cb + e2] : 0;
        const int w1 = w_bits[cb + e], w2 = two ? w_bits[cb + e2] : 0;
        const int r1 = pos_row[nb + s1], r2 = two ? pos_row[nb + s2] : 0;
        edges[e] = EdgeRec{r1 * kRowBytes, __int_as_float(w1)};
        if (two) edges[e2] = EdgeRec{r2 * kRowBytes, __int_as_float(w2)};
      }
    }
  }
  __syncthreads();
  const int n_lvl = st ? 0 : n_lvl_sh;
  LdsProgT<true> lp{recs, edges};
  GlobalProg gp{row_ptr + rb, fn + nb,     bias_bits + nb, resp_bits + nb,
                src + cb,    w_bits + cb, pos_row + nb};

  constexpr int kRow = (kWave + 1) * K;  // floats per LDS row
  float* mine = vals + lane * K;

  // Offsets of this thread's elements in a full tile, computed once: input
  // element i = tid + j*T (observation b, component c) goes to row io[c],
  // column b; output element i = tid + j*T comes from row io[I + c].
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
    __syncthreads();
  }
}

#define TN_FWD_PARAMS                                                                           \
  PopView pop, const int32_t *__restrict__ status, const int32_t *__restrict__ n_valid,         \
      const int32_t *__restrict__ level, const int32_t *__restrict__ row_ptr,                   \
      const int32_t *__restrict__ src, const int32_t *__restrict__ w_bits,                      \
      const int32_t *__restrict__ fn, const int32_t *__restrict__ bias_bits,                    \
      const int32_t *__restrict__ resp_bits, const int32_t *__restrict__ io_pos,                \
      const int32_t *__restrict__ pos_row, const int32_t *__restrict__ n_rows,                  \
      const int32_t *__restrict__ prog_rows, const float *__restrict__ obs,                     \
      float *__restrict__ out, const float *__restrict__ target, float *__restrict__ loss,      \
      FwdArgs a
#define TN_FWD_ARGS                                                                             \
  pop, status, n_valid, level, row_ptr, src, w_bits, fn, bias_bits, resp_bits, io_pos, pos_row, \
      n_rows, prog_rows, obs, out, target, loss, a

// One workgroup per (genome, group of consecutive tiles).
template <int K, bool kLoss, bool kProgLds>
__global__ __launch_bounds__(kWave * lds_max_waves(K)) void forward_kernel(TN_FWD_PARAMS) {
  int item, t_begin, t_end;
  if (kLoss) {
    item = blockIdx.x;
    t_begin = 0;
    t_end = a.n_tiles;
  } else {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    item = b / a.n_groups;
    t_begin = (b - item * a.n_groups) * a.per_wg;
    t_end = min(t_begin + a.per_wg, a.n_tiles);
  }
  const int g = a.genomes ? a.genomes[item] : item;
  lds_genome<K, kLoss, kProgLds>(TN_FWD_ARGS, g, t_begin, t_end);
}

// Persistent form: each workgroup takes the next per_wg genomes of the list
// (longest first) from a counter, one atomic per grab, until the list is
// exhausted; the counter must be 0 at launch.
template <int K, bool kProgLds>
__global__ __launch_bounds__(kWave * lds_max_waves(K)) void forward_queue_kernel(TN_FWD_PARAMS) {
  __shared__ int item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(a.queue, a.per_wg);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_sh);
    __syncthreads();
    if (item >= a.n_items) break;
    const int end = min(item + a.per_wg, a.n_items);
    for (int i = item; i < end; ++i)
      lds_genome<K, false, kProgLds>(TN_FWD_ARGS, a.genomes[i], 0, a.n_tiles);
  }
}

template <int K, bool kLoss, bool kProgLds>
int launch_k(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
             const float* target, float* loss, const FwdArgs& a, int grid, int waves,
             hipStream_t stream) {
  const size_t lds = fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, kProgLds, a.rows).bytes;
  const bool queue = !kLoss && a.queue;
  const void* kern = queue ? (const void*)forward_queue_kernel<K, kProgLds>
                           : (const void*)forward_kernel<K, kLoss, kProgLds>;
  int rc = allow_lds(kern, lds);
  if (rc != TN_OK || grid == 0) return rc;
#define TN_FWD_LAUNCH_ARGS                                                                   \
  make_view(p), t.status, t.n_valid, t.level, t.row_ptr, t.edge_src,                         \
      reinterpret_cast<const int32_t*>(t.edge_w), t.pos_fn,                                  \
      reinterpret_cast<const int32_t*>(t.pos_bias), reinterpret_cast<const int32_t*>(t.pos_resp), \
      t.io_pos, t.pos_row, t.n_rows, t.prog_rows, obs, out, target, loss, a
  if (queue)
    hipLaunchKernelGGL((forward_queue_kernel<K, kProgLds>), dim3((unsigned)grid),
                       dim3(kWave * waves), lds, stream, TN_FWD_LAUNCH_ARGS);
  else
    hipLaunchKernelGGL((forward_kernel<K, kLoss, kProgLds>), dim3((unsigned)grid),
                       dim3(kWave * waves), lds, stream, TN_FWD_LAUNCH_ARGS);
#undef TN_FWD_LAUNCH_ARGS
  return check_launch();
}

// Program in LDS if it fits beside the rows, else read from global memory.
bool prog_fits(const tn_population& p, int K, int rows) {
  return fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, true, rows).bytes <= max_dynamic_lds();
}

template <bool kLoss>
int dispatch(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
             const float* target, float* loss, const FwdArgs& a, int grid, int K, int waves,
             hipStream_t stream) {
  const bool in_lds = prog_fits(p, K, a.rows);
  if (!in_lds &&
      fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, K, false, a.rows).bytes > max_dynamic_lds())
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

int lds_rows_cap(const tn_population& p) {
  // largest row count the level-parallel kernel holds at one observation per lane
  int lo = 1, hi = p.N_max;
  if (fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, 1, false, hi).bytes <= max_dynamic_lds())
    return hi;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (fwd_lds(p.N_max, p.C_max, p.n_in + p.n_out, 1, false, mid).bytes <= max_dynamic_lds())
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

size_t forward_lds_bytes(int N_max, int C_max, int nio, int K) {
  return fwd_lds(N_max, C_max, nio, K, true, N_max).bytes;
}

size_t lds_tile_bytes(const tn_population& p, int K, int rows) {
  const int nio = p.n_in + p.n_out;
  const size_t with = fwd_lds(p.N_max, p.C_max, nio, K, true, rows).bytes;
  if (with <= max_dynamic_lds()) return with;
  const size_t without = fwd_lds(p.N_max, p.C_max, nio, K, false, rows).bytes;
  return without <= max_dynamic_lds() ? without : 0;
}

int lds_queue_grid(const tn_population& p, int K, int waves, int rows) {
  const size_t lds = lds_tile_bytes(p, K, rows);
  if (lds == 0) return 0;
  const bool in_lds = prog_fits(p, K, rows);
  const void* k = nullptr;
  switch (K * 2 + (in_lds ? 1 : 0)) {
    case 2: k = (const void*)forward_queue_kernel<1, false>; break;
    case 3: k = (const void*)forward_queue_kernel<1, true>; break;
    case 4: k = (const void*)forward_queue_kernel<2, false>; break;
    case 5: k = (const void*)forward_queue_kernel<2, true>; break;
    case 8: k = (const void*)forward_queue_kernel<4, false>; break;
    case 9: k = (const void*)forward_queue_kernel<4, true>; break;
    default: return 0;
  }
  int dev = 0, cus = 0, per_cu = 0;
  if (allow_lds(k, lds) != TN_OK) return 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kWave * waves, lds);
  if (record_hip(e) != TN_OK) return 0;
  return std::max(1, per_cu) * cus;
}

int launch_forward(const tn_population& p, const tn_transformed& t, const float* obs,
                   int64_t obs_stride, int B, float* out, const LdsTile& tile,
                   const FwdWork& work, hipStream_t stream) {
  const int K = tile.K == 0 ? 1 : tile.K;
  const int waves = tile.waves <= 0 ? 4 : tile.waves;
  const int rows = tile.rows <= 0 || tile.rows > p.N_max ? p.N_max : tile.rows;
  if (waves > lds_max_waves(K)) return TN_EINVAL;
  const int n_list = work.genomes ? work.n_genomes : p.P;
  const int ktile = kWave * K;
  const int n_tiles = (B + ktile - 1) / ktile;
  FwdArgs a{obs_stride, B,   0,     0.0f, 0.0f, n_tiles, 1, n_tiles, rows, tile.skip_le,
            work.genomes, work.queue, n_list};
  int grid = work.grid;
  if (work.queue) {
    a.per_wg = std::max(1, n_list / (4 * std::max(1, grid)));  // about 4 grabs per workgroup
  } else {
    // enough workgroups to fill the chip; each takes consecutive tiles of a genome
    const int want = std::max(1, std::min(n_tiles, (2048 + n_list - 1) / std::max(1, n_list)));
    a.per_wg = (n_tiles + want - 1) / want;
    a.n_groups = (n_tiles + a.per_wg - 1) / a.per_wg;
    const int64_t g64 = (int64_t)n_list * a.n_groups;
    if (g64 > 0x7fffffff) return TN_EUNSUPPORTED;
    grid = (int)g64;
  }
  return dispatch<false>(p, t, obs, out, nullptr, nullptr, a, grid, K, waves, stream);
}

int launch_forward_loss(const tn_population& p, const tn_transformed& t, const float* obs,
                        int64_t obs_stride, int B, const float* target, int64_t target_stride,
                        float scale, float offset, float* out, float* loss, int skip_le,
                        hipStream_t stream) {
  const int n_tiles = (B + kWave - 1) / kWave;
  const int rows = std::min(p.N_max, lds_rows_cap(p));
  FwdArgs a{obs_stride, B, target_stride, scale, offset, n_tiles, 1, n_tiles, rows, skip_le,
            nullptr, nullptr, 0};
  return dispatch<true>(p, t, obs, out, target, loss, a, p.P, 1, 4, stream);
}

}  // namespace tn
