// Calculation stage (TensorNEAT Section 3.3) for genomes whose forward pass
// needs at most 200 value rows, with every node value held in registers.
//
// Mapping: one wavefront per unit of 64, 128 or 256 observations of one genome
// (lane = observation of each tile of the unit); a workgroup holds W
// wavefronts. A lane's node values live in an explicit register file (rows at
// fixed VGPRs, fwd_reg.hpp) addressed with a uniform index window, so an
// in-edge is one indexed fused multiply-add: no LDS traffic and no barrier in
// the evaluation. The value rows are the packed program's rows (freed right
// after their last read; input k sits in row k). Observations are staged
// through a small per-wavefront LDS buffer (LDS-direct loads); outputs leave
// through it or straight from the registers. With a loss, one workgroup per
// genome shares its units and reduces the squared error in a fixed order.
#include <algorithm>

#include "fwd_launch.hpp"
#include "fwd_reg.hpp"

namespace tn {

namespace {

struct RegArgs {
  int64_t obs_stride;
  int B;
  int64_t target_stride;
  float scale, offset;
  int n_tiles;     // units per genome: runs of rf_tiles(variant) tiles of 64 observations
  int n_groups;    // tile chunks per list entry (grid form without loss)
  int per_wave;    // grid form: tiles per chunk; persistent: items per wavefront per grab
  int rows;        // value rows in registers: 32 or 64
  int rows_lo;     // genomes with prog_rows <= rows_lo are left to another launch (-1: none)
  int skip_above;  // genomes needing more than `rows` rows are left to another launch
  const int32_t* genomes;  // genome list (nullptr: every genome, in order)
  int32_t* queue;          // persistent form: next item to take
  int n_items;             // grid form: list length * n_groups; persistent: * n_tiles
  int in_phase;            // tiles of inputs staged per LDS-direct round
  int stage_stride;        // floats of LDS staging per wavefront
  int n_list;              // persistent form: list length
};

// Persistent form, XCD-aware: workgroup b runs on XCD b % 8 (the round-robin
// dispatch of MI355X's 8 XCDs); the list entries e with e % 8 == x form XCD
// x's share, taken from counter x, so that the units of one genome run under
// one L2 and its program is fetched from HBM once. The placement matters for
// speed only: share x is drained by the workgroups with b % 8 == x wherever
// they run, and the launcher rounds the grid up to a multiple of 8 so every
// share has some. Entry and unit of item i of share x (items: entry-major,
// units consecutive).
constexpr int kXcds = 8;
__device__ __forceinline__ int share_items(int n_list, int x, int units) {
  return n_list > x ? ((n_list - x + kXcds - 1) / kXcds) * units : 0;
}

// Observations and outputs pass through LDS in chunks of up to kChunk
// components per observation; a row of the chunk has an odd stride, so the
// per-lane row accesses are free of bank conflicts.
constexpr int kChunk = 8;
constexpr int kStage = kWave * (kChunk + 1);  // floats per tile
// staging regions per wavefront of variant V (its tiles per unit)
constexpr int stage_tiles(int V) { return rf_tiles(V); }

// The register-file form stages a unit's observations with LDS-direct loads
// (global_load_lds: memory to LDS without passing through registers, so a
// whole round is in flight at once and waited for once; 16 bytes per lane
// when the source is aligned, which measured several times faster per byte
// than one float per lane), in rounds of as many
// of the unit's tiles as fit this many bytes per wavefront (two wavefronts per
// SIMD then still fit the compute unit's LDS), one tile per round at least.
constexpr int kDmaBytes = 20 * 1024;

// Tiles per LDS-direct round for variant V and I inputs.
int dma_phase(int V, int I) {
  int P = rf_tiles(V);
  while (P > 1 && (int64_t)P * kWave * I * 4 > kDmaBytes) P /= 2;
  return P;
}
// LDS staging floats per wavefront.
int stage_floats(int V, int I) {
  const int P = dma_phase(V, I);
  return std::max(kStage * stage_tiles(V), P * kWave * I);
}

// Rows r of register files f0 .. f0 + P - 1 := x[0 .. P-1] (P = K: one window
// for all; two of four: one window for the pair; else one window each).
template <int R>
__device__ __forceinline__ void rf_set_part(int P, int f0, int r, const float (&x)[rf_tiles(R)]) {
  constexpr int K = rf_tiles(R);
  if (P == K) {
    rfk_set<R>(r, x);
  } else if (K == 4 && P == 2) {
    if (f0 == 0)
      asm volatile("s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v56, %0\n\t"
                   "v_mov_b32 v106, %1\n\ts_set_gpr_idx_off" ::"v"(x[0]),
                   "v"(x[1]), "s"(r) : "m0");
    else
      asm volatile("s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v156, %0\n\t"
                   "v_mov_b32 v206, %1\n\ts_set_gpr_idx_off" ::"v"(x[0]),
                   "v"(x[1]), "s"(r) : "m0");
  } else {
    for (int p = 0; p < P; ++p) rf_set((f0 + p) * R + r, x[p]);
  }
}

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  const int full = per * kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * per + bid / kXcd;
}

// One unit of the register-file engine: rf_tiles(R) consecutive tiles of 64
// observations (obs b0 ...), tile k in register file k. Inputs arrive through
// the staging buffer (one region of kStage floats per tile) and are written
// to all tiles under one window per input; outputs leave the same way.
template <int R, bool kLoss>
__device__ __forceinline__ float run_unit(const int32_t* __restrict__ rec,
                                          const int2* __restrict__ pe, int nn, int in_phase,
                                          const int4* __restrict__ pn,
                                          const int32_t* __restrict__ out_pos, int orow_first,
                                          int I, int O, int b0, int B,
                                          const float* __restrict__ xg, float* __restrict__ yg,
                                          const float* __restrict__ tg, float* stg, int lane) {
  constexpr int K = rf_tiles(R);
  int nbat[K];
#pragma unroll
  for (int k = 0; k < K; ++k) nbat[k] = max(0, min(kWave, B - b0 - k * kWave));
  {
    // rounds of in_phase tiles: the tiles' observations are contiguous in
    // memory (64 * in_phase * I floats), copied verbatim into LDS with one
    // LDS-direct load per 64 floats, waited for once, then read back one
    // column per row (stride I per lane)
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // earlier LDS use is done
    for (int f0 = 0; f0 < K; f0 += in_phase) {
      const int nobs = max(0, min(in_phase * kWave, B - b0 - f0 * kWave));
      const int total = nobs * I;
      const float* src = xg + (int64_t)(b0 + f0 * kWave) * I;
      // 16 bytes per lane (global_load_lds_dwordx4: lane i's four floats land
      // at M0 + 16 i) while the source is 16-byte aligned, one float per lane
      // for the rest
      int j = 0;
      if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const int full = total & ~(4 * kWave - 1);
        const int voff = lane * 16;
        for (; j < full; j += 4 * kWave) {
          const uint32_t at = __builtin_amdgcn_readfirstlane(
              (uint32_t)reinterpret_cast<uintptr_t>(stg + j));
          asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(voff),
                       "s"(src + j), "s"(at)
                       : "memory", "m0");
        }
      }
      for (; j < total; j += kWave)
        if (j + lane < total) __builtin_amdgcn_global_load_lds(src + j + lane, stg + j, 4, 0, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      for (int c = 0; c < I; ++c) {
        float x[K];
#pragma unroll
        for (int p = 0; p < K; ++p) x[p] = p < in_phase ? stg[(p * kWave + lane) * I + c] : 0.0f;
        rf_set_part<R>(in_phase, f0, c, x);
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // reads done before the next round
    }
  }
  walk_records<R>(rec, pe, nn, lane);
  float sse = 0.0f;
  if constexpr (!kLoss && K == 1) {
    // one tile: outputs straight from the register file, lane l writing the O
    // values of its observation four at a time when O is a multiple of 4 and
    // the rows are 16-byte aligned (the stores of one group of four outputs
    // together cover the tile's rows); with several tiles per wavefront the
    // LDS transpose below is faster
    if (!yg) return 0.0f;
    const bool vec = (O & 3) == 0 && (reinterpret_cast<uintptr_t>(yg) & 15) == 0;
    for (int c0 = 0; c0 < O; c0 += vec ? 4 : 1) {
      float x[4][1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u > 0 && !vec) break;
        const int c = c0 + u;
        const int orow = c < kChunk ? __builtin_amdgcn_readlane(orow_first, c)
                                    : __builtin_amdgcn_readfirstlane(prog_row(pn, out_pos[c]));
        rfk_get<R>(orow, x[u]);
      }
      if (lane < nbat[0]) {
        float* dst = yg + (int64_t)(b0 + lane) * O + c0;
        if (vec)
          *reinterpret_cast<float4*>(dst) = make_float4(x[0][0], x[1][0], x[2][0], x[3][0]);
        else
          *dst = x[0][0];
      }
    }
    return 0.0f;
  }
  for (int c0 = 0; c0 < O; c0 += kChunk) {
    const int ch = min(kChunk, O - c0);
    const int sr = ch | 1;
    const int orow = c0 == 0 ? orow_first : (lane < ch ? prog_row(pn, out_pos[c0 + lane]) : 0);
    for (int j = 0; j < ch; ++j) {
      float x[K];
      rfk_get<R>(__builtin_amdgcn_readlane(orow, j), x);
#pragma unroll
      for (int k = 0; k < K; ++k) stg[k * kStage + lane * sr + j] = x[k];
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int tot = nbat[k] * ch;
      const float* sk = stg + k * kStage;
      const int64_t ob = (int64_t)(b0 + k * kWave) * O;
      DivWalk dw(lane, ch, kWave);
      for (int i = lane; i < tot; i += kWave) {
        const float y = sk[dw.b * sr + dw.c];
        const int64_t at = ob + (int64_t)dw.b * O + c0 + dw.c;
        if (yg) yg[at] = y;
        if (kLoss) {
          const float d = y - tg[at];
          sse = fmaf(d, d, sse);
        }
        dw.step();
      }
    }
    wave_sync();
  }
  return sse;
}

#define TN_REG_PARAMS                                                                        \
  PopView pop, const int32_t *__restrict__ status, const int32_t *__restrict__ prog_rows,     \
      const int32_t *__restrict__ n_valid, const int4 *__restrict__ prog_node,               \
      const int2 *__restrict__ prog_edge, const int32_t *__restrict__ prog_rec,              \
      const int32_t *__restrict__ io_pos, const float *__restrict__ obs,                     \
      float *__restrict__ out, const float *__restrict__ target, RegArgs a
#define TN_REG_ARGS \
  pop, status, prog_rows, n_valid, prog_node, prog_edge, prog_rec, io_pos, obs, out, target, a

// Tiles t_begin, t_begin + t_step, ... < t_end of genome g by this wavefront;
// returns its part of the squared error (kLoss). *st_out: the genome's
// status as the launch sees it (0: evaluated; -2: left to another launch).
template <int NB, bool kLoss>
__device__ __forceinline__ float reg_genome(TN_REG_PARAMS, int g, int t_begin, int t_end,
                                            int t_step, float* stg, int* st_out) {
  const int lane = lane_id();
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  const int rows = prog_rows[g];
  if (rows <= a.rows_lo || (a.skip_above && rows > a.rows)) {
    *st_out = -2;
    return 0.0f;
  }
  // a flagged genome, or one needing more rows than the launch holds, is NaN
  const int st = status[g] ? status[g] : (rows > a.rows ? -1 : 0);
  *st_out = st;
  const int n = n_valid[g];
  const int64_t nb = uniform64(pop.node_base(g)), cb = uniform64(pop.conn_base(g));
  const int4* pn = prog_node + nb;
  const int2* pe = prog_edge + cb;
  const int32_t* rec = prog_rec + nb * 16;
  const int nn = n - I;
  const int32_t* out_pos = io_pos + (int64_t)g * nio + I;
  const int orow_first = !st && lane < min(O, kChunk) ? prog_row(pn, out_pos[lane]) : 0;
  constexpr int K = rf_tiles(NB);
  float sse = 0.0f;
  for (int t = t_begin; t < t_end; t += t_step) {
    const int b0 = t * K * kWave;
    const int nobs = min(K * kWave, a.B - b0);
    float* yg = out ? out + (int64_t)g * a.B * O : nullptr;
    if (st) {
      if (yg)
        for (int i = lane; i < nobs * O; i += kWave) yg[(int64_t)b0 * O + i] = __builtin_nanf("");
      continue;
    }
    const float* xg = obs + (int64_t)g * a.obs_stride;
    const float* tg = kLoss ? target + (int64_t)g * a.target_stride : nullptr;
    sse += run_unit<NB, kLoss>(rec, pe, nn, a.in_phase, pn, out_pos, orow_first, I, O, b0, a.B, xg,
                               yg, tg, stg, lane);
  }
  return sse;
}

// Grid form: wavefront i of the launch takes item i = (list entry, chunk of
// per_wave consecutive tiles), chunks of one entry being consecutive (so the
// wavefronts of a workgroup mostly share a genome). With kLoss, one workgroup
// per list entry whose wavefronts share its tiles and reduce the squared error
// in a fixed order.
// The register file has R rows per tile at v[kRfBase ..]; the compiler gets
// the VGPRs below kRfBase.
template <int R, bool kLoss>
__global__ __launch_bounds__(kWave * 8) __attribute__((amdgpu_num_vgpr(TN_RF_BASE))) void
forward_rf_kernel(TN_REG_PARAMS, float* __restrict__ loss) {
  rf_reserve<R>();
  extern __shared__ __align__(16) float stage_all[];
  __shared__ float part[8];
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x / kWave;
  float* stg = stage_all + wave * a.stage_stride;
  int entry, t_begin, t_end, t_step;
  if (kLoss) {
    entry = blockIdx.x;
    t_begin = wave;
    t_end = a.n_tiles;
    t_step = W;
  } else {
    const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * W + wave;
    if (item >= a.n_items) return;
    entry = (int)(item / a.n_groups);
    t_begin = (int)(item - (int64_t)entry * a.n_groups) * a.per_wave;
    t_end = min(t_begin + a.per_wave, a.n_tiles);
    t_step = 1;
  }
  const int g = a.genomes ? a.genomes[entry] : entry;
  int st;
  const float sse = reg_genome<R, kLoss>(TN_REG_ARGS, g, t_begin, t_end, t_step, stg, &st);
  if (kLoss && st != -2) {
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

// Persistent form: the workgroup takes the next W * chunk (list entry, unit)
// items of its XCD's share from that share's counter (one atomic per grab) and
// wavefront w runs items base + w, base + w + W, ...; list entries are ordered
// longest first. The kXcds counters must be 0 at launch.
template <int R>
__global__ __launch_bounds__(kWave * 8) __attribute__((amdgpu_num_vgpr(TN_RF_BASE))) void
forward_rf_queue_kernel(TN_REG_PARAMS) {
  rf_reserve<R>();
  extern __shared__ __align__(16) float stage_all[];
  __shared__ int base_sh;
  const int wave = wave_id();
  const int W = blockDim.x / kWave;
  float* stg = stage_all + wave * a.stage_stride;
  const int x = blockIdx.x % kXcds;
  const int n_share = share_items(a.n_list, x, a.n_tiles);
  for (;;) {
    if (threadIdx.x == 0) base_sh = atomicAdd(a.queue + x, W * a.per_wave);
    __syncthreads();
    const int base = __builtin_amdgcn_readfirstlane(base_sh);
    __syncthreads();
    if (base >= n_share) break;
    for (int c = 0; c < a.per_wave; ++c) {
      const int item = base + c * W + wave;
      if (item >= n_share) break;
      const int le = item / a.n_tiles, t = item - le * a.n_tiles;
      int st;
      reg_genome<R, false>(TN_REG_ARGS, a.genomes[le * kXcds + x], t, t + 1, 1, stg, &st);
    }
  }
}

// Variants: register files of V rows per tile (50: four tiles per wavefront,
// 100: two, the others one).
#define TN_REG_VARIANTS(X) X(32) X(50) X(64) X(96) X(100) X(128) X(160) X(200)

template <int V, bool kLoss>
int launch_grid(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
                const float* target, float* loss, const RegArgs& a, int grid, int waves,
                hipStream_t stream) {
  if (grid == 0) return TN_OK;
  const size_t lds = sizeof(float) * (size_t)a.stage_stride * waves;
#define TN_REG_LAUNCH(K)                                                                    \
  hipLaunchKernelGGL((K), dim3((unsigned)grid), dim3(kWave * waves), lds, stream, make_view(p), \
                     t.status, t.prog_rows, t.n_valid,                                        \
                     reinterpret_cast<const int4*>(t.prog_node),                             \
                     reinterpret_cast<const int2*>(t.prog_edge), t.prog_rec, t.io_pos, obs, out, \
                     target, a,                                                              \
                     loss)
  TN_REG_LAUNCH((forward_rf_kernel<V, kLoss>));
#undef TN_REG_LAUNCH
  return check_launch();
}

template <int V>
const void* queue_kernel() {
  return (const void*)forward_rf_queue_kernel<V>;
}

template <int V>
int launch_queue(const tn_population& p, const tn_transformed& t, const float* obs, float* out,
                 const RegArgs& a, int grid, int waves, hipStream_t stream) {
  if (grid == 0) return TN_OK;
  grid = (grid + kXcds - 1) / kXcds * kXcds;  // every XCD's share gets workgroups
  const size_t lds = sizeof(float) * (size_t)a.stage_stride * waves;
#define TN_REG_LAUNCH(K)                                                                    \
  hipLaunchKernelGGL((K), dim3((unsigned)grid), dim3(kWave * waves), lds, stream, make_view(p), \
                     t.status, t.prog_rows, t.n_valid,                                        \
                     reinterpret_cast<const int4*>(t.prog_node),                             \
                     reinterpret_cast<const int2*>(t.prog_edge), t.prog_rec, t.io_pos, obs,  \
                     out,                                                                    \
                     (const float*)nullptr, a)
  TN_REG_LAUNCH((forward_rf_queue_kernel<V>));
#undef TN_REG_LAUNCH
  return check_launch();
}

bool valid_variant(int v) {
  switch (v) {
#define TN_CASE(V) case V:
    TN_REG_VARIANTS(TN_CASE)
#undef TN_CASE
    return true;
    default: return false;
  }
}

}  // namespace

int launch_forward_reg(const tn_population& p, const tn_transformed& t, const float* obs,
                       int64_t obs_stride, int B, float* out, const RegTile& tile,
                       const FwdWork& work, hipStream_t stream) {
  const int waves = tile.waves <= 0 ? 4 : tile.waves;
  const int rows = tile.rf;
  const int variant = tile.rf;
  if (waves > 8 || !valid_variant(variant)) return TN_EINVAL;
  const int n_list = work.genomes ? work.n_genomes : p.P;
  // units of stage_tiles(variant) tiles of 64 observations per genome
  const int kt = stage_tiles(variant);
  const int n_tiles = ((B + kWave - 1) / kWave + kt - 1) / kt;
  RegArgs a{obs_stride, B,  0, 0.0f, 0.0f, n_tiles, 1, n_tiles, rows, tile.rows_lo,
            tile.skip_above ? 1 : 0, work.genomes, work.queue, 0, dma_phase(variant, p.n_in),
            stage_floats(variant, p.n_in), n_list};
  if (work.queue) {
    if (!work.genomes) return TN_EINVAL;  // the persistent form takes a list
    a.n_items = n_list * n_tiles;
    // items per wavefront per grab: about 4 grabs per resident workgroup
    a.per_wave = std::max(1, (int)((int64_t)a.n_items / (4LL * waves * std::max(1, work.grid))));
    switch (variant) {
#define TN_CASE(V) \
  case V: return launch_queue<V>(p, t, obs, out, a, work.grid, waves, stream);
      TN_REG_VARIANTS(TN_CASE)
#undef TN_CASE
      default: return TN_EINVAL;
    }
  }
  // enough wavefronts to fill the chip; each takes consecutive tiles of a genome
  const int want = std::max(1, std::min(n_tiles, (8192 + n_list - 1) / std::max(1, n_list)));
  a.per_wave = (n_tiles + want - 1) / want;
  a.n_groups = (n_tiles + a.per_wave - 1) / a.per_wave;  // chunks per list entry
  a.n_items = (int)std::min<int64_t>((int64_t)n_list * a.n_groups, 0x7fffffff);
  const int64_t grid = ((int64_t)n_list * a.n_groups + waves - 1) / waves;
  if (grid > 0x7fffffff || (int64_t)n_list * a.n_groups > 0x7fffffff) return TN_EUNSUPPORTED;
  switch (variant) {
#define TN_CASE(V)                                                                          \
  case V:                                                                                   \
    return launch_grid<V, false>(p, t, obs, out, nullptr, nullptr, a, (int)grid, waves, stream);
    TN_REG_VARIANTS(TN_CASE)
#undef TN_CASE
    default: return TN_EINVAL;
  }
}

// The loss form of the register-file variant V: one workgroup of `waves`
// wavefronts per genome (grid P), sharing its units; genomes outside
// (rows_lo, V] are left to another launch when skip_above (else NaN above V).
template <int V>
int loss_rf(const tn_population& p, const tn_transformed& t, const float* obs,
            int64_t obs_stride, int B, const float* target, int64_t target_stride, float scale,
            float offset, float* out, float* loss, int waves, int rows_lo, bool skip_above,
            hipStream_t stream) {
  const int kt = stage_tiles(V);
  const int n_units = ((B + kWave - 1) / kWave + kt - 1) / kt;
  RegArgs a{obs_stride, B, target_stride, scale, offset, n_units, 1, n_units, V, rows_lo,
            skip_above ? 1 : 0, nullptr, nullptr, 0, dma_phase(V, p.n_in),
            stage_floats(V, p.n_in), p.P};
  return launch_grid<V, true>(p, t, obs, out, target, loss, a, p.P, waves, stream);
}

int launch_forward_loss_reg(const tn_population& p, const tn_transformed& t, const float* obs,
                            int64_t obs_stride, int B, const float* target,
                            int64_t target_stride, float scale, float offset, float* out,
                            float* loss, int waves, int rf, int rows_lo, bool skip_above,
                            hipStream_t stream) {
  if (waves <= 0) waves = 4;
  if (waves > 8) return TN_EINVAL;
  switch (rf) {
#define TN_CASE(V)                                                                           \
  case V:                                                                                    \
    return loss_rf<V>(p, t, obs, obs_stride, B, target, target_stride, scale, offset, out, loss, \
                      waves, rows_lo, skip_above, stream);
    TN_REG_VARIANTS(TN_CASE)
#undef TN_CASE
    default: return TN_EINVAL;
  }
}

int reg_queue_grid(int variant, int waves, int n_in) {
  int dev = 0, cus = 0, per_cu = 0;
  const size_t lds = sizeof(float) * (size_t)stage_floats(variant, n_in) * waves;
  const void* k = nullptr;
  switch (variant) {
#define TN_CASE(V) \
  case V: k = queue_kernel<V>(); break;
    TN_REG_VARIANTS(TN_CASE)
#undef TN_CASE
    default: return 0;
  }
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kWave * waves, lds);
  if (record_hip(e) != TN_OK) return 0;
  return std::max(1, per_cu) * cus;
}

}  // namespace tn
