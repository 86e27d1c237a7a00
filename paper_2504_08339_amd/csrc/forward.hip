// Calculation stage of tensorized inference (TensorNEAT Section 3.3), batched
// over the whole population and a batch of observations.
//
// Mapping: one wavefront per (genome, tile of 64 observations); lane = one
// observation. The genome's topology is identical for every lane, so the
// position loop, the in-edge loop and the activation switch are wavefront
// uniform (scalar loads of row_ptr / edge_src / edge_w, scalar branches).
// Node values live in LDS as vals[position][lane]: every lane reads the same
// row, so each access touches 64 consecutive dwords (no bank conflicts).
// Observations are loaded with consecutive lanes on consecutive floats and
// scattered into the input rows; outputs are gathered the same way so that
// the global stores are coalesced.
#include "tn_internal.hpp"

namespace tn {

namespace {

// Walks (b, c) = divmod(i, d) for i = lane, lane + 64, ... without dividing
// in the loop.
struct DivWalk {
  int b, c, qb, qc, d;
  __device__ DivWalk(int i, int d_) : d(d_) {
    b = i / d;
    c = i - b * d;
    qb = kWave / d;
    qc = kWave - qb * d;
  }
  __device__ __forceinline__ void step() {
    b += qb;
    c += qc;
    if (c >= d) {
      c -= d;
      ++b;
    }
  }
};

// Evaluates positions 0..n-1 for this lane's observation; inputs are already
// in vals. Returns nothing: results stay in vals.
__device__ __forceinline__ void eval_nodes(const TrView& tr, int64_t nb, int64_t cb, int64_t rb,
                                           int n, float* vals, int lane) {
  const int32_t* __restrict__ row_ptr = tr.row_ptr + rb;
  const int32_t* __restrict__ esrc = tr.edge_src + cb;
  const float* __restrict__ ew = tr.edge_w + cb;
  const int32_t* __restrict__ fnp = tr.pos_fn + nb;
  const float* __restrict__ bias = tr.pos_bias + nb;
  const float* __restrict__ resp = tr.pos_resp + nb;
  for (int p = 0; p < n; ++p) {
    const int32_t fn = fnp[p];
    if (fn < 0) continue;  // input node: value is the observation
    const int e0 = row_ptr[p], e1 = row_ptr[p + 1];
    const int agg = (fn >> 8) & 0xff;
    float s;
    if (agg == TN_AGG_SUM) {
      float acc = 0.0f;
      for (int e = e0; e < e1; ++e) acc = fmaf(ew[e], vals[esrc[e] * kWave + lane], acc);
      s = acc;
    } else if (e0 == e1) {
      s = 0.0f;
    } else {
      float first = ew[e0] * vals[esrc[e0] * kWave + lane];
      s = first;
      for (int e = e0 + 1; e < e1; ++e) {
        const float t = ew[e] * vals[esrc[e] * kWave + lane];
        switch (agg) {
          case TN_AGG_PRODUCT: s = s * t; break;
          case TN_AGG_MAX: s = fmaxf(s, t); break;
          case TN_AGG_MIN: s = fminf(s, t); break;
          case TN_AGG_MEAN: s = s + t; break;
          case TN_AGG_MAXABS: s = fabsf(t) > fabsf(s) ? t : s; break;
          default: break;
        }
      }
      if (agg == TN_AGG_MEAN) s = s / (float)(e1 - e0);
    }
    const float z = fmaf(resp[p], s, bias[p]);
    vals[p * kWave + lane] = activate(fn & 0xff, z);
  }
}

struct FwdArgs {
  const float* obs;
  int64_t obs_stride;
  int B;
  float* out;
  const float* target;
  int64_t target_stride;
  float scale, offset;
  float* loss;
  int n_tiles;
};

// XCD-aware block order: hardware hands consecutive workgroups to the 8 XCDs
// in turn; remapping keeps a genome's consecutive tiles on one XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd;
  const int full = per * kXcd;
  if (bid >= full) return bid;
  return (bid % kXcd) * per + bid / kXcd;
}

template <bool kLoss>
__global__ __launch_bounds__(kWave) void forward_kernel(PopView pop, TrView tr, FwdArgs a) {
  extern __shared__ float vals[];
  const int lane = lane_id();
  const int I = pop.n_in, O = pop.n_out, nio = I + O;
  int g, t_begin, t_end;
  if (kLoss) {
    g = blockIdx.x;
    t_begin = 0;
    t_end = a.n_tiles;
  } else {
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    g = item / a.n_tiles;
    t_begin = item - g * a.n_tiles;
    t_end = t_begin + 1;
  }
  const int st = tr.status[g];
  const int n = tr.n_valid[g];
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g), rb = pop.rowptr_base(g);
  const int32_t* io = tr.io_pos + (int64_t)g * nio;
  float sse = 0.0f;
  for (int t = t_begin; t < t_end; ++t) {
    const int b0 = t * kWave;
    const int nbat = min(kWave, a.B - b0);
    float* outp = a.out ? a.out + ((int64_t)g * a.B + b0) * O : nullptr;
    if (st) {
      if (outp)
        for (int i = lane; i < nbat * O; i += kWave) outp[i] = __builtin_nanf("");
      continue;
    }
    const float* xo = a.obs + (int64_t)g * a.obs_stride + (int64_t)b0 * I;
    if (I > 0) {
      DivWalk w(lane, I);
      for (int i = lane; i < nbat * I; i += kWave, w.step())
        vals[io[w.c] * kWave + w.b] = xo[i];
    }
    __syncthreads();
    eval_nodes(tr, nb, cb, rb, n, vals, lane);
    __syncthreads();
    {
      const float* tg = kLoss ? a.target + (int64_t)g * a.target_stride + (int64_t)b0 * O : nullptr;
      DivWalk w(lane, O);
      for (int i = lane; i < nbat * O; i += kWave, w.step()) {
        const float y = vals[io[I + w.c] * kWave + w.b];
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
    const float total = wave_sum(sse);
    if (lane == 0) a.loss[g] = st ? __builtin_nanf("") : fmaf(a.scale, total, a.offset);
  }
}

template <bool kLoss>
int launch(const tn_population& p, const tn_transformed& t, const FwdArgs& a, int grid) {
  return allow_lds((const void*)forward_kernel<kLoss>, (size_t)p.N_max * kWave * sizeof(float));
}

}  // namespace

size_t forward_lds_bytes(int N_max) { return (size_t)N_max * kWave * sizeof(float); }

int launch_forward(const tn_population& p, const tn_transformed& t, const float* obs,
                   int64_t obs_stride, int B, float* out, hipStream_t stream) {
  FwdArgs a{obs, obs_stride, B, out, nullptr, 0, 0.0f, 0.0f, nullptr, (B + kWave - 1) / kWave};
  const int64_t grid = (int64_t)p.P * a.n_tiles;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  int rc = launch<false>(p, t, a, (int)grid);
  if (rc != TN_OK || grid == 0) return rc;
  hipLaunchKernelGGL(forward_kernel<false>, dim3((unsigned)grid), dim3(kWave),
                     forward_lds_bytes(p.N_max), stream, make_view(p), make_view(t), a);
  return check_launch();
}

int launch_forward_loss(const tn_population& p, const tn_transformed& t, const float* obs,
                        int64_t obs_stride, int B, const float* target, int64_t target_stride,
                        float scale, float offset, float* out, float* loss, hipStream_t stream) {
  FwdArgs a{obs, obs_stride, B, out, target, target_stride, scale, offset, loss,
            (B + kWave - 1) / kWave};
  int rc = launch<true>(p, t, a, p.P);
  if (rc != TN_OK || p.P == 0) return rc;
  hipLaunchKernelGGL(forward_kernel<true>, dim3(p.P), dim3(kWave), forward_lds_bytes(p.N_max),
                     stream, make_view(p), make_view(t), a);
  return check_launch();
}

}  // namespace tn
