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

__global__ __launch_bounds__(kWave) void backward_kernel(
    PopView pop, const int32_t* __restrict__ status, const int32_t* __restrict__ n_valid,
    const int32_t* __restrict__ order, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ src, const int32_t* __restrict__ w_bits,
    const int32_t* __restrict__ edge_row, const int32_t* __restrict__ fn,
    const int32_t* __restrict__ bias_bits, const int32_t* __restrict__ resp_bits,
    const int32_t* __restrict__ io_pos, const float* __restrict__ obs, BwdArgs a) {
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

  if (st) {
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
      const int act = f & 0xff, agg = (f >> 8) & 0xff;
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

}  // namespace

int launch_backward(const tn_population& p, const tn_transformed& t, const float* obs,
                    int64_t obs_stride, int B, const float* dY, int64_t dY_stride,
                    const float* target, int64_t target_stride, float scale, float* loss,
                    float* dW, float* db, hipStream_t stream) {
  const size_t lds = bwd_lds(p.N_max, p.C_max, p.n_in + p.n_out).bytes;
  int rc = allow_lds((const void*)backward_kernel, lds);
  if (rc != TN_OK || p.P == 0) return rc;
  BwdArgs a{obs_stride, B, dY, dY_stride, target, target_stride, scale, loss, dW, db};
  hipLaunchKernelGGL(backward_kernel, dim3(p.P), dim3(kWave), lds, stream, make_view(p), t.status,
                     t.n_valid, t.order, t.row_ptr, t.edge_src,
                     reinterpret_cast<const int32_t*>(t.edge_w), t.edge_row, t.pos_fn,
                     reinterpret_cast<const int32_t*>(t.pos_bias),
                     reinterpret_cast<const int32_t*>(t.pos_resp), t.io_pos, obs, a);
  return check_launch();
}

}  // namespace tn
