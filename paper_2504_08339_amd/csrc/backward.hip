// Reverse-mode derivative of the calculation stage (TensorNEAT Section 3.3)
// with respect to connection weights and node biases, for gradient refinement
// of weights.
//
// Mapping: one wavefront per genome walks the genome's tiles of 64
// observations in order (lane = observation). Per tile, in LDS:
//   1. forward pass, keeping the value row v[p][.] of every position;
//   2. upstream gradient rows g[p][.]: dL/dy at the outputs (given, or the
//      fused mean-squared error 2 (y - t) * scale), 0 elsewhere;
//   3. reverse sweep over the topological order: delta_p = g_p * act'(z_p)
//      replaces g_p in place and is pushed to the sources through
//      g_src += delta_p * resp_p * d agg / d t_e * w_e;
//   4. lanes switch to edges: dW_e += resp_k * sum_b delta_k[b] * d agg/d t_e[b]
//      * v_src[b] and db_k += sum_b delta_k[b], as 64-term dot products over
//      the tile's rows, added to per-edge / per-position accumulators.
// The tile order and the in-tile summation order are fixed, so results are
// deterministic. act' comes from the stored value for identity, sigmoid, tanh
// and relu; sin, gaussian and abs re-evaluate z from the in-edges. Non-sum
// aggregations re-evaluate their terms in both phases.
#include <algorithm>

#include "fwd_core.hpp"

namespace tn {

namespace {

constexpr int kRow = kWave + 1;  // floats per LDS row (1 float of padding)

struct BwdArgs {
  int64_t obs_stride;
  int B;
  const float* dY;  // [P][B][O] upstream gradient, or null for the fused MSE
  int64_t dY_stride;
  const float* target;  // fused MSE targets (when dY is null)
  int64_t target_stride;
  float scale;  // MSE: loss = scale * sum (y - t)^2, dL/dy = 2 scale (y - t)
  float* loss;  // may be null
  float* dW;    // conn block
  float* db;    // node block
};

struct BwdLds {
  size_t rec_off, edge_off, edst_off, io_off, dw_off, db_off, v_off, g_off, bytes;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline BwdLds bwd_lds(int N, int C, int nio) {
  BwdLds L;
  L.rec_off = 0;
  L.edge_off = al16(L.rec_off + sizeof(NodeRec) * (size_t)N);
  L.edst_off = al16(L.edge_off + sizeof(EdgeRec) * (size_t)C);
  L.io_off = al16(L.edst_off + sizeof(int32_t) * (size_t)C);
  L.dw_off = al16(L.io_off + sizeof(int32_t) * (size_t)nio);
  L.db_off = al16(L.dw_off + sizeof(float) * (size_t)C);
  L.v_off = al16(L.db_off + sizeof(float) * (size_t)N);
  L.g_off = al16(L.v_off + sizeof(float) * std::max((size_t)N * kRow, (size_t)(C + N)));
  L.bytes = al16(L.g_off + sizeof(float) * (size_t)N * kRow);
  return L;
}

// z of position p for this lane (re-evaluated from the in-edges).
__device__ float node_z(const NodeRec& rec, int f, const EdgeRec* edges, const float* v,
                        int lane) {
  const int er = __builtin_amdgcn_readfirstlane(rec.erange);
  const int e0 = er & 0xffff, e1 = (er >> 16) & 0xffff;
  const int agg = (f >> 8) & 0xff;
  float s = 0.0f;
  if (agg == TN_AGG_SUM) {
    for (int e = e0; e < e1; ++e) s = fmaf(edges[e].w, v[edges[e].src * kRow + lane], s);
  } else if (e1 > e0) {
    s = edges[e0].w * v[edges[e0].src * kRow + lane];
    for (int e = e0 + 1; e < e1; ++e) {
      const float t = edges[e].w * v[edges[e].src * kRow + lane];
      switch (agg) {
        case TN_AGG_PRODUCT: s = s * t; break;
        case TN_AGG_MAX: s = fmaxf(s, t); break;
        case TN_AGG_MIN: s = fminf(s, t); break;
        case TN_AGG_MEAN: s = s + t; break;
        default: s = fabsf(t) > fabsf(s) ? t : s; break;
      }
    }
    if (agg == TN_AGG_MEAN) s = s / (float)(e1 - e0);
  }
  return fmaf(rec.resp, s, rec.bias);
}

// d act / dz at this lane, from the stored value v (and z when needed).
__device__ __forceinline__ float act_slope(int act, float v, float z) {
  switch (act) {
    case TN_ACT_IDENTITY: return 1.0f;
    case TN_ACT_SIGMOID: return v * (1.0f - v);
    case TN_ACT_TANH: return fmaf(-v, v, 1.0f);
    case TN_ACT_RELU: return v > 0.0f ? 1.0f : 0.0f;
    case TN_ACT_SIN: return cosf(z);
    case TN_ACT_GAUSSIAN: return -2.0f * z * v;
    default: return z > 0.0f ? 1.0f : (z < 0.0f ? -1.0f : 0.0f);  // abs
  }
}

__device__ __forceinline__ bool slope_needs_z(int act) {
  return act == TN_ACT_SIN || act == TN_ACT_GAUSSIAN || act == TN_ACT_ABS;
}

// d agg / d t_e for in-edge e of a node with a non-sum aggregation, this lane.
__device__ float agg_partial(int agg, int e, int e0, int e1, const EdgeRec* edges, const float* v,
                             int lane) {
  if (agg == TN_AGG_MEAN) return 1.0f / (float)(e1 - e0);
  if (agg == TN_AGG_PRODUCT) {
    float p = 1.0f;
    for (int x = e0; x < e1; ++x)
      if (x != e) p *= edges[x].w * v[edges[x].src * kRow + lane];
    return p;
  }
  // max / min / maxabs: the first extreme term in row order takes it
  int best = e0;
  float bv = edges[e0].w * v[edges[e0].src * kRow + lane];
  for (int x = e0 + 1; x < e1; ++x) {
    const float t = edges[x].w * v[edges[x].src * kRow + lane];
    const bool take = agg == TN_AGG_MAX ? t > bv : (agg == TN_AGG_MIN ? t < bv : fabsf(t) > fabsf(bv));
    if (take) {
      best = x;
      bv = t;
    }
  }
  return best == e ? 1.0f : 0.0f;
}

// Genomes the register-file adjoint (backward_rf_kernel, below) takes.
constexpr int kRfPos = 48, kRfEdges = 64, kRfSlots = kRfEdges + kRfPos, kSlotRow = kWave + 1;
// Its register file starts at v64 (the compiler keeps v0..v63: sin's argument
// reduction needs the room): tile 0 at v64..v159, tile 1 at v160..v255, each
// 96 rows, values at rows 0..47 and upstream gradients at rows 48..95.
#define TN_BW_RF_BASE 64

__device__ __forceinline__ bool rf_bwd_eligible(int st, int n, int n_edges, const int32_t* fnp) {
  if (st || n > kRfPos || n_edges > kRfEdges) return false;
  for (int p = 0; p < n; ++p) {
    const int f = fnp[p];
    const int agg = (f >> 8) & 0xff;
    if (f >= 0 && agg != TN_AGG_SUM && agg != TN_AGG_MEAN) return false;
  }
  return true;
}

__global__ __launch_bounds__(kWave) void backward_kernel(
    PopView pop, const int32_t* __restrict__ status, const int32_t* __restrict__ n_valid,
    const int32_t* __restrict__ order, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ src, const int32_t* __restrict__ w_bits,
    const int32_t* __restrict__ edge_row, const int32_t* __restrict__ fn,
    const int32_t* __restrict__ bias_bits, const int32_t* __restrict__ resp_bits,
    const int32_t* __restrict__ io_pos, const float* __restrict__ obs, BwdArgs a, int lds_ok) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int g = blockIdx.x;
  const int lane = lane_id();
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g), rb = pop.rowptr_base(g);
  const int64_t nrows = pop.node_rows(g), crows = pop.conn_rows(g);
  const int st = status[g];
  const BwdLds L = bwd_lds(pop.N_max, pop.C_max, nio);
  NodeRec* recs = reinterpret_cast<NodeRec*>(lds + L.rec_off);
  EdgeRec* edges = reinterpret_cast<EdgeRec*>(lds + L.edge_off);
  int32_t* edst = reinterpret_cast<int32_t*>(lds + L.edst_off);
  int32_t* io_l = reinterpret_cast<int32_t*>(lds + L.io_off);
  float* dwacc = reinterpret_cast<float*>(lds + L.dw_off);
  float* dbacc = reinterpret_cast<float*>(lds + L.db_off);
  float* v = reinterpret_cast<float*>(lds + L.v_off);
  float* gr = reinterpret_cast<float*>(lds + L.g_off);

  {
    const int n0 = n_valid[g];
    if (rf_bwd_eligible(st, n0, st ? 0 : row_ptr[rb + n0], fn + nb)) return;  // backward_rf_kernel's
  }
  // flagged genomes, and (when N_max rows of values and gradients exceed the
  // device's LDS) every genome the register-file adjoint could not take
  if (st || !lds_ok) {
    const float nan = __builtin_nanf("");
    for (int64_t r = lane; r < crows; r += kWave) a.dW[cb + r] = nan;
    for (int64_t r = lane; r < nrows; r += kWave) a.db[nb + r] = nan;
    if (a.loss && lane == 0) a.loss[g] = nan;
    return;
  }
  const int n = n_valid[g];
  const int n_edges = row_ptr[rb + n];
  // stage the program; destination position of every edge
  for (int p = lane; p < n; p += kWave) {
    NodeRec r;
    const int e0 = row_ptr[rb + p], e1 = row_ptr[rb + p + 1];
    r.erange = e0 | (e1 << 16);
    r.fn = fn_with_row(fn[nb + p], p);  // one value row per position here
    r.bias = __int_as_float(bias_bits[nb + p]);
    r.resp = __int_as_float(resp_bits[nb + p]);
    recs[p] = r;
    for (int e = e0; e < e1; ++e) edst[e] = p;
    dbacc[p] = 0.0f;
  }
  for (int e = lane; e < n_edges; e += kWave) {
    EdgeRec q;
    q.src = src[cb + e];
    q.w = __int_as_float(w_bits[cb + e]);
    edges[e] = q;
    dwacc[e] = 0.0f;
  }
  for (int k = lane; k < nio; k += kWave) io_l[k] = io_pos[(int64_t)g * nio + k];
  wave_sync();

  float sse = 0.0f;
  const int n_tiles = (a.B + kWave - 1) / kWave;
  for (int t = 0; t < n_tiles; ++t) {
    const int b0 = t * kWave;
    const int nbat = min(kWave, a.B - b0);
    const bool live = lane < nbat;
    // 1. inputs and forward
    const float* xo = obs + (int64_t)g * a.obs_stride + (int64_t)b0 * I;
    for (int c = 0; c < I; ++c) v[io_l[c] * kRow + lane] = live ? xo[(int64_t)lane * I + c] : 0.0f;
    wave_sync();
    LdsProg lp{recs, edges};
    for (int p = 0; p < n; ++p) eval_node<1, kRow>(lp, p, v + lane);
    // 2. upstream gradient rows
    for (int p = 0; p < n; ++p) gr[p * kRow + lane] = 0.0f;
    wave_sync();
    for (int j = 0; j < O; ++j) {
      const int pj = io_l[I + j];
      float gy = 0.0f;
      if (live) {
        const int64_t o = (int64_t)lane * O + j;
        const float y = v[pj * kRow + lane];
        if (a.dY) {
          gy = a.dY[(int64_t)g * a.dY_stride + (int64_t)b0 * O + o];
        } else {
          const float d = y - a.target[(int64_t)g * a.target_stride + (int64_t)b0 * O + o];
          sse = fmaf(d, d, sse);
          gy = 2.0f * a.scale * d;
        }
      }
      gr[pj * kRow + lane] += gy;
    }
    wave_sync();
    // 3. reverse sweep: g_p -> delta_p, pushed to the sources
    for (int p = n - 1; p >= 0; --p) {
      const NodeRec rec = recs[p];
      const int f = __builtin_amdgcn_readfirstlane(rec.fn);
      if (f < 0) continue;
      const int act = f & 7, agg = (f >> 8) & 0xff;  // codes below 7: transformed genomes
      const float vp = v[p * kRow + lane];
      const float z = slope_needs_z(act) ? node_z(rec, f, edges, v, lane) : 0.0f;
      const float delta = live ? gr[p * kRow + lane] * act_slope(act, vp, z) : 0.0f;
      gr[p * kRow + lane] = delta;
      const int er = __builtin_amdgcn_readfirstlane(rec.erange);
      const int e0 = er & 0xffff, e1 = (er >> 16) & 0xffff;
      const float dr = delta * rec.resp;
      for (int e = e0; e < e1; ++e) {
        const EdgeRec q = edges[e];
        const float part = agg == TN_AGG_SUM ? 1.0f : agg_partial(agg, e, e0, e1, edges, v, lane);
        gr[q.src * kRow + lane] = fmaf(dr * part, q.w, gr[q.src * kRow + lane]);
      }
    }
    wave_sync();
    // 4. lanes over edges / positions: dot products over the tile
    for (int e = lane; e < n_edges; e += kWave) {
      const int k = edst[e];
      const NodeRec rk = recs[k];
      const int agg = (rk.fn >> 8) & 0xff;
      const int s = edges[e].src;
      float acc = 0.0f;
      if (agg == TN_AGG_SUM) {
        for (int b = 0; b < kWave; ++b) acc = fmaf(gr[k * kRow + b], v[s * kRow + b], acc);
      } else {
        const int e0 = rk.erange & 0xffff, e1 = (rk.erange >> 16) & 0xffff;
        for (int b = 0; b < kWave; ++b)
          acc = fmaf(gr[k * kRow + b] * agg_partial(agg, e, e0, e1, edges, v, b), v[s * kRow + b],
                     acc);
      }
      dwacc[e] = fmaf(rk.resp, acc, dwacc[e]);
    }
    for (int p = lane; p < n; p += kWave) {
      if (recs[p].fn < 0) continue;
      float acc = 0.0f;
      for (int b = 0; b < kWave; ++b) acc += gr[p * kRow + b];
      dbacc[p] += acc;
    }
    wave_sync();
  }
  // write out: every row of the genome's blocks exactly once, through
  // row -> edge / row -> position maps built in the (now free) value rows
  int32_t* row_edge = reinterpret_cast<int32_t*>(v);
  int32_t* row_pos = row_edge + pop.C_max;
  for (int64_t r = lane; r < crows; r += kWave) row_edge[r] = -1;
  for (int64_t r = lane; r < nrows; r += kWave) row_pos[r] = -1;
  wave_sync();
  for (int e = lane; e < n_edges; e += kWave) row_edge[edge_row[cb + e]] = e;
  for (int p = lane; p < n; p += kWave)
    if (recs[p].fn >= 0) row_pos[order[nb + p]] = p;
  wave_sync();
  for (int64_t r = lane; r < crows; r += kWave) {
    const int e = row_edge[r];
    a.dW[cb + r] = e >= 0 ? dwacc[e] : 0.0f;
  }
  for (int64_t r = lane; r < nrows; r += kWave) {
    const int p = row_pos[r];
    a.db[nb + r] = p >= 0 ? dbacc[p] : 0.0f;
  }
  if (a.loss) {
    const float total = wave_sum(sse);
    if (lane == 0) a.loss[g] = a.scale * total;
  }
}

// ------------------------------------------------ register-file adjoint
//
// The same derivative for the genomes that fit it (tn_backward runs both
// kernels; each takes the genomes the other leaves): at most kRfPos positions
// and kRfEdges in-edges, sum or mean aggregation only, not flagged. One
// wavefront per genome, lane = observation, two tiles of 64 observations per
// step. Values and upstream gradients live in registers indexed by position
// (two files of 96 rows, values at rows 0..47 and gradients at rows 48..95);
// the genome's program is held across the lanes (read with v_readlane). Per
// step:
//   forward: v_p = act(bias + resp * agg(w_e v_src)) at every non-input
//     position (gradient row cleared in the same window);
//   outputs: gbar_out += dL/dy;
//   reverse: delta_p = gbar_p act'(z_p) (z re-evaluated for sin, gaussian,
//     abs); db_p += delta_p; dt = delta_p resp (/ n for mean); per in-edge
//     dW_e += dt v_src and gbar_src += dt w_e (one indexed read-modify-write).
// The per-observation terms (both tiles added first) accumulate per lane in
// LDS slots (row stride 65: conflict free), each in program order; at the end
// lane s sums slot s over the 64 lanes in lane order. Deterministic.
// V[p] := v{0,1}, G[p] := 0
__device__ __forceinline__ void bw_set_v(int p, float v0, float v1) {
  asm volatile(
      "s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v64, %0\n\t"
      "v_mov_b32 v160, %1\n\tv_mov_b32 v112, 0\n\tv_mov_b32 v208, 0\n\ts_set_gpr_idx_off" ::"v"(v0),
      "v"(v1), "s"(p)
      : "m0");
}
// t{0,1} := V[j]
__device__ __forceinline__ void bw_get_v(int j, float& t0, float& t1) {
  asm volatile(
      "s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v64\n\t"
      "v_mov_b32 %1, v160\n\ts_set_gpr_idx_off"
      : "=v"(t0), "=v"(t1)
      : "s"(j)
      : "m0");
}
// s{0,1} += w * V[j]
__device__ __forceinline__ void bw_fma_v(float& s0, float& s1, float w, int j) {
  asm volatile(
      "s_set_gpr_idx_on %3, gpr_idx(SRC1)\n\ts_nop 1\n\tv_fmac_f32 %0, %2, v64\n\t"
      "v_fmac_f32 %1, %2, v160\n\ts_set_gpr_idx_off"
      : "+v"(s0), "+v"(s1)
      : "s"(w), "s"(j)
      : "m0");
}
// G[p], V[p] of both files
__device__ __forceinline__ void bw_get_gv(int p, float& g0, float& g1, float& v0, float& v1) {
  asm volatile(
      "s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v112\n\t"
      "v_mov_b32 %1, v208\n\tv_mov_b32 %2, v64\n\tv_mov_b32 %3, v160\n\ts_set_gpr_idx_off"
      : "=v"(g0), "=v"(g1), "=v"(v0), "=v"(v1)
      : "s"(p)
      : "m0");
}
// G[j] += a{0,1} * w (one indexed read-modify-write per file)
__device__ __forceinline__ void bw_fma_g(int j, float a0, float a1, float w) {
  asm volatile(
      "s_set_gpr_idx_on %3, gpr_idx(SRC2,DST)\n\ts_nop 1\n\tv_fma_f32 v112, %0, %2, v112\n\t"
      "v_fma_f32 v208, %1, %2, v208\n\ts_set_gpr_idx_off" ::"v"(a0),
      "v"(a1), "v"(w), "s"(j)
      : "m0");
}

__global__ __launch_bounds__(kWave) __attribute__((amdgpu_num_vgpr(TN_BW_RF_BASE))) void
backward_rf_kernel(PopView pop, const int32_t* __restrict__ status,
                   const int32_t* __restrict__ n_valid, const int32_t* __restrict__ order,
                   const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ src,
                   const int32_t* __restrict__ w_bits, const int32_t* __restrict__ edge_row,
                   const int32_t* __restrict__ fn, const int32_t* __restrict__ bias_bits,
                   const int32_t* __restrict__ resp_bits, const int32_t* __restrict__ io_pos,
                   const float* __restrict__ obs, BwdArgs a) {
  asm volatile("" ::: "v255");  // the register file counts in the allocation
  __shared__ float slots[kRfSlots * kSlotRow];
  __shared__ int32_t maps[2 * kWave];
  const int g = blockIdx.x;
  const int lane = lane_id();
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  const int64_t nb = uniform64(pop.node_base(g)), cb = uniform64(pop.conn_base(g)),
                rb = uniform64(pop.rowptr_base(g));
  const int64_t nrows = pop.node_rows(g), crows = pop.conn_rows(g);
  const int n = n_valid[g];
  const int n_edges = status[g] ? 0 : row_ptr[rb + n];
  if (!rf_bwd_eligible(status[g], n, n_edges, fn + nb)) return;  // the LDS kernel's genome
  // the program across the lanes
  const int l_fn = lane < n ? fn[nb + lane] : 0;
  const int l_bias = lane < n ? bias_bits[nb + lane] : 0;
  const int l_resp = lane < n ? resp_bits[nb + lane] : 0;
  const int l_rp = lane <= n ? row_ptr[rb + lane] : 0;
  const int l_src = lane < n_edges ? src[cb + lane] : 0;
  const int l_w = lane < n_edges ? w_bits[cb + lane] : 0;
  const int l_io = lane < nio ? io_pos[(int64_t)g * nio + lane] : 0;
  float* my = slots + lane;  // slot s of this lane at my[s * kSlotRow]
#pragma unroll 1
  for (int s = 0; s < kRfSlots; ++s) my[s * kSlotRow] = 0.0f;
  float sse = 0.0f;
  const int n_steps = (a.B + 2 * kWave - 1) / (2 * kWave);
  for (int t = 0; t < n_steps; ++t) {
    int bk[2];
    bool live[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      bk[k] = t * 2 * kWave + k * kWave + lane;
      live[k] = bk[k] < a.B;
    }
    const float* xg = obs + (int64_t)g * a.obs_stride;
    // inputs (gradient rows cleared with them)
    for (int c = 0; c < I; ++c) {
      const int p = __builtin_amdgcn_readlane(l_io, c);
      const float x0 = live[0] ? xg[(int64_t)bk[0] * I + c] : 0.0f;
      const float x1 = live[1] ? xg[(int64_t)bk[1] * I + c] : 0.0f;
      bw_set_v(p, x0, x1);
    }
    // forward
    for (int p = 0; p < n; ++p) {
      const int f = __builtin_amdgcn_readlane(l_fn, p);
      if (f < 0) continue;
      const int e0 = __builtin_amdgcn_readlane(l_rp, p), e1 = __builtin_amdgcn_readlane(l_rp, p + 1);
      float sum[2] = {0.0f, 0.0f};
      for (int e = e0; e < e1; ++e) {
        const int j = __builtin_amdgcn_readlane(l_src, e);
        bw_fma_v(sum[0], sum[1], __int_as_float(__builtin_amdgcn_readlane(l_w, e)), j);
      }
      if (((f >> 8) & 0xff) == TN_AGG_MEAN && e1 > e0) {
        sum[0] = sum[0] / (float)(e1 - e0);
        sum[1] = sum[1] / (float)(e1 - e0);
      }
      const float rho = __int_as_float(__builtin_amdgcn_readlane(l_resp, p));
      const float bias = __int_as_float(__builtin_amdgcn_readlane(l_bias, p));
      // one tile at a time (the empty asm keeps the compiler from
      // interleaving them: less register pressure in sin's reduction)
      const float z0[1] = {fmaf(rho, sum[0], bias)}, z1[1] = {fmaf(rho, sum[1], bias)};
      float v0[1], v1[1];
      activate_all<1>(f & 7, z0, v0);  // codes below 7: transformed genomes
      asm volatile("" : "+v"(v0[0]));
      activate_all<1>(f & 7, z1, v1);
      bw_set_v(p, v0[0], v1[0]);
    }
    // upstream gradient at the outputs
    for (int jo = 0; jo < O; ++jo) {
      const int pj = __builtin_amdgcn_readlane(l_io, I + jo);
      float y[2];
      bw_get_v(pj, y[0], y[1]);
      float gy[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        gy[k] = 0.0f;
        if (live[k]) {
          const int64_t o = (int64_t)bk[k] * O + jo;
          if (a.dY) {
            gy[k] = a.dY[(int64_t)g * a.dY_stride + o];
          } else {
            const float d = y[k] - a.target[(int64_t)g * a.target_stride + o];
            sse = fmaf(d, d, sse);
            gy[k] = 2.0f * a.scale * d;
          }
        }
      }
      bw_fma_g(pj, gy[0], gy[1], 1.0f);
    }
    // reverse sweep
    for (int p = n - 1; p >= 0; --p) {
      const int f = __builtin_amdgcn_readlane(l_fn, p);
      if (f < 0) continue;
      const int act = f & 7;
      const int e0 = __builtin_amdgcn_readlane(l_rp, p), e1 = __builtin_amdgcn_readlane(l_rp, p + 1);
      const bool mean = ((f >> 8) & 0xff) == TN_AGG_MEAN && e1 > e0;
      const float rho = __int_as_float(__builtin_amdgcn_readlane(l_resp, p));
      float g0, g1, v0, v1;
      bw_get_gv(p, g0, g1, v0, v1);
      float z[2] = {0.0f, 0.0f};
      if (slope_needs_z(act)) {
        float sum[2] = {0.0f, 0.0f};
        for (int e = e0; e < e1; ++e) {
          const int j = __builtin_amdgcn_readlane(l_src, e);
          bw_fma_v(sum[0], sum[1], __int_as_float(__builtin_amdgcn_readlane(l_w, e)), j);
        }
        if (mean) {
          sum[0] = sum[0] / (float)(e1 - e0);
          sum[1] = sum[1] / (float)(e1 - e0);
        }
        const float bias = __int_as_float(__builtin_amdgcn_readlane(l_bias, p));
        z[0] = fmaf(rho, sum[0], bias);
        z[1] = fmaf(rho, sum[1], bias);
      }
      float d0 = live[0] ? g0 * act_slope(act, v0, z[0]) : 0.0f;
      asm volatile("" : "+v"(d0));
      const float d1 = live[1] ? g1 * act_slope(act, v1, z[1]) : 0.0f;
      my[(kRfEdges + p) * kSlotRow] += d0 + d1;
      float dt0 = d0 * rho, dt1 = d1 * rho;
      if (mean) {
        dt0 = dt0 / (float)(e1 - e0);
        dt1 = dt1 / (float)(e1 - e0);
      }
      for (int e = e0; e < e1; ++e) {
        const float old = my[e * kSlotRow];
        const int j = __builtin_amdgcn_readlane(l_src, e);
        float t[2];
        bw_get_v(j, t[0], t[1]);
        bw_fma_g(j, dt0, dt1, __int_as_float(__builtin_amdgcn_readlane(l_w, e)));
        my[e * kSlotRow] = old + fmaf(dt1, t[1], dt0 * t[0]);
      }
    }
  }
  wave_sync();
  // slot s (edge s, or position s - kRfEdges) summed by lane s in lane order
  float sums[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = h * kWave + lane;
    float acc = 0.0f;
    if (s < kRfSlots)
#pragma unroll 8
      for (int b = 0; b < kWave; ++b) acc += slots[s * kSlotRow + b];
    sums[h] = acc;
  }
  // write every row of the genome's blocks once: row -> edge / position maps
  int32_t* row_edge = maps;
  int32_t* row_pos = maps + kWave;
  wave_sync();
  for (int64_t r0 = 0; r0 < crows; r0 += kWave) {
    row_edge[lane] = -1;
    wave_sync();
    if (lane < n_edges) {
      const int64_t r = edge_row[cb + lane] - r0;
      if (r >= 0 && r < kWave) row_edge[r] = lane;
    }
    wave_sync();
    const int e = row_edge[lane];
    const float dwv = __shfl(sums[0], e < 0 ? 0 : e, kWave);
    if (r0 + lane < crows) a.dW[cb + r0 + lane] = e >= 0 ? dwv : 0.0f;
    wave_sync();
  }
  for (int64_t r0 = 0; r0 < nrows; r0 += kWave) {
    row_pos[lane] = -1;
    wave_sync();
    if (lane < n && l_fn >= 0) {
      const int64_t r = order[nb + lane] - r0;
      if (r >= 0 && r < kWave) row_pos[r] = lane;
    }
    wave_sync();
    const int p = row_pos[lane];
    // position p's sum is slot kRfEdges + p: lane p of sums[0] for p < 0,
    // i.e. lane (kRfEdges + p) - 64 of sums[1]
    const int sl = kRfEdges + (p < 0 ? 0 : p);
    const float lo = __shfl(sums[0], sl & (kWave - 1), kWave);
    const float hi = __shfl(sums[1], sl & (kWave - 1), kWave);
    const float dbv = sl < kWave ? lo : hi;
    if (r0 + lane < nrows) a.db[nb + r0 + lane] = p >= 0 ? dbv : 0.0f;
    wave_sync();
  }
  if (a.loss) {
    const float total = wave_sum(sse);
    if (lane == 0) a.loss[g] = a.scale * total;
  }
}

}  // namespace

int launch_backward(const tn_population& p, const tn_transformed& t, const float* obs,
                    int64_t obs_stride, int B, const float* dY, int64_t dY_stride,
                    const float* target, int64_t target_stride, float scale, float* loss,
                    float* dW, float* db, hipStream_t stream) {
  // The LDS adjoint holds N_max rows of values and of gradients; above the
  // device's LDS (N_max beyond about 300) it only writes NaN for the genomes
  // the register-file adjoint leaves to it, and the call still succeeds.
  size_t lds = bwd_lds(p.N_max, p.C_max, p.n_in + p.n_out).bytes;
  int rc = allow_lds((const void*)backward_kernel, lds);
  const int lds_ok = rc == TN_OK;
  if (rc == TN_EUNSUPPORTED) {
    lds = 0;
    rc = TN_OK;
  }
  if (rc != TN_OK || p.P == 0) return rc;
  BwdArgs a{obs_stride, B, dY, dY_stride, target, target_stride, scale, loss, dW, db};
  hipLaunchKernelGGL(backward_rf_kernel, dim3(p.P), dim3(kWave), 0, stream, make_view(p),
                     t.status, t.n_valid, t.order, t.row_ptr, t.edge_src,
                     reinterpret_cast<const int32_t*>(t.edge_w), t.edge_row, t.pos_fn,
                     reinterpret_cast<const int32_t*>(t.pos_bias),
                     reinterpret_cast<const int32_t*>(t.pos_resp), t.io_pos, obs, a);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(backward_kernel, dim3(p.P), dim3(kWave), lds, stream, make_view(p), t.status,
                     t.n_valid, t.order, t.row_ptr, t.edge_src,
                     reinterpret_cast<const int32_t*>(t.edge_w), t.edge_row, t.pos_fn,
                     reinterpret_cast<const int32_t*>(t.pos_bias),
                     reinterpret_cast<const int32_t*>(t.pos_resp), t.io_pos, obs, a, lds_ok);
  return check_launch();
}

}  // namespace tn
