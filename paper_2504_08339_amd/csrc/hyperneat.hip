// HyperNEAT over a grid substrate (the indirect encoding among TensorNEAT's
// algorithms, Section 4.4): every CPPN genome is queried at all source /
// target pairs of a grid substrate, the result is thresholded and rounded to
// bfloat16, and the substrate then runs as a dense two-layer network on the
// matrix cores.
//
//   query    one lane = one substrate connection (s -> t): the CPPN's inputs
//            (x_s, y_s, x_t, y_t, 1) are computed from the indices and its
//            packed program runs in registers (the register engine's walk);
//            weights are stored transposed, w1t[t][s] and w2t[j][s], so that
//            both GEMM operands are contiguous along the reduction index.
//   hidden   H = tanh(X W1): v_mfma_f32_16x16x32_bf16, one wavefront per
//            64 x 64 tile of H, fp32 accumulation, tanh in the epilogue.
//   output   Y = bf16(H) W2 with fp32 accumulation in a fixed order.
// Geometry: an n x n grid layer has node n*r + c at (-1 + 2c/(n-1),
// -1 + 2r/(n-1)); output j of m sits at (-1 + 2j/(m-1), 0).
#include <algorithm>

#include "fwd_reg.hpp"
#include "tn_internal.hpp"

namespace tn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct SubGeom {
  int grid;    // n: the grid layers are n x n
  int S;       // n * n
  int n_out;   // m
  float thr;   // |w| < thr -> 0
  float step;  // 2 / (n - 1)
  float ostep; // 2 / (m - 1)
};

// float32 -> bfloat16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ------------------------------------------------------------------ query

template <int NB>
__device__ __forceinline__ float cppn_eval(const int4* __restrict__ pn, const int2* __restrict__ pe,
                                           int n, int out_row, float xs, float ys, float xt,
                                           float yt) {
  f32x32 lo = 0.0f, hi = 0.0f;
  asm volatile("" : "+v"(lo));
  if (NB == 2) asm volatile("" : "+v"(hi));
  vset<NB>(lo, hi, 0, xs);
  vset<NB>(lo, hi, 1, ys);
  vset<NB>(lo, hi, 2, xt);
  vset<NB>(lo, hi, 3, yt);
  vset<NB>(lo, hi, 4, 1.0f);
  walk_program<NB>(lo, hi, pn, pe, n);
  return vget<NB>(lo, hi, out_row);
}

// Workgroups over (genome, chunk of query tiles); each wavefront takes
// `per_wave` consecutive tiles of 64 queries. Queries 0 .. S*S-1 fill w1t
// (t = q / S, s = q % S), the next S*m fill w2t (j, s).
__global__ __launch_bounds__(256) void cppn_query_kernel(
    PopView pop, const int32_t* __restrict__ status, const int32_t* __restrict__ prog_rows,
    const int32_t* __restrict__ n_valid, const int4* __restrict__ prog_node,
    const int2* __restrict__ prog_edge, const int32_t* __restrict__ io_pos, SubGeom sg,
    int n_chunks, int per_wave, uint16_t* __restrict__ w1t, uint16_t* __restrict__ w2t,
    float* __restrict__ raw1, float* __restrict__ raw2) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int W = blockDim.x / kWave;
  const int g = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - g * n_chunks;
  const int Q1 = sg.S * sg.S, Q = Q1 + sg.S * sg.n_out;  // < 2^31 (checked on the host)
  const int n_tiles = (Q + kWave - 1) / kWave;
  const int t0 = (chunk * W + wave) * per_wave;
  const int t1 = min(t0 + per_wave, n_tiles);
  const int rows = prog_rows[g];
  const bool bad = status[g] != 0 || rows > 64;
  const int n = n_valid[g];
  const int4* pn = prog_node + pop.node_base(g);
  const int2* pe = prog_edge + pop.conn_base(g);
  const int nio = pop.n_in + pop.n_out;
  const int out_row = bad ? 0 : ((pn[io_pos[(int64_t)g * nio + pop.n_in]].y >> 16) & 0x7fff);
  uint16_t* W1 = w1t + (int64_t)g * Q1;
  uint16_t* W2 = w2t + (int64_t)g * sg.S * sg.n_out;
  float* R1 = raw1 ? raw1 + (int64_t)g * Q1 : nullptr;
  float* R2 = raw2 ? raw2 + (int64_t)g * sg.S * sg.n_out : nullptr;
  for (int t = t0; t < t1; ++t) {
    const int q = t * kWave + lane;
    const bool live = q < Q;
    const bool first = q < Q1;
    const int qq = first ? q : q - Q1;
    const int tgt = qq / sg.S;
    const int src = qq - tgt * sg.S;
    const int rs = src / sg.grid, cs = src - rs * sg.grid;
    const float xs = fmaf((float)cs, sg.step, -1.0f), ys = fmaf((float)rs, sg.step, -1.0f);
    float xt, yt;
    if (first) {
      const int rt = tgt / sg.grid, ct = tgt - rt * sg.grid;
      xt = fmaf((float)ct, sg.step, -1.0f);
      yt = fmaf((float)rt, sg.step, -1.0f);
    } else {
      xt = sg.n_out > 1 ? fmaf((float)tgt, sg.ostep, -1.0f) : 0.0f;
      yt = 0.0f;
    }
    float y;
    if (bad)
      y = __builtin_nanf("");
    else if (rows <= 32)
      y = cppn_eval<1>(pn, pe, n, out_row, xs, ys, xt, yt);
    else
      y = cppn_eval<2>(pn, pe, n, out_row, xs, ys, xt, yt);
    const uint16_t wb = bf16_bits(fabsf(y) < sg.thr ? 0.0f : y);
    if (live) {
      if (first) {
        W1[qq] = wb;
        if (R1) R1[qq] = y;
      } else {
        W2[qq] = wb;
        if (R2) R2[qq] = y;
      }
    }
  }
}

// ----------------------------------------------------------------- hidden

// One wavefront per 64 x 64 tile of H (rows b, columns t) of one genome:
// Z[b][t] = sum_s X[b][s] w1t[t][s] over K steps of 32 with 16 MFMA
// 16x16x32 per step, then H = tanh(Z) in fp32. Operand fragments are loaded
// straight from global memory (16 bytes per lane: 8 consecutive s of one row),
// the same k-ordering on both operands. Rows b >= B read zeros and are not
// stored.
__global__ __launch_bounds__(256) void substrate_hidden_kernel(
    const uint16_t* __restrict__ x, int64_t x_stride, const uint16_t* __restrict__ w1t, int S,
    int B, int m_tiles, int n_tiles, int64_t n_items, float* __restrict__ h) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
  if (item >= n_items) return;  // wavefront-uniform; the kernel has no barrier
  const int per_g = m_tiles * n_tiles;
  const int g = (int)(item / per_g);
  const int r = (int)(item - (int64_t)g * per_g);
  const int mt = r / n_tiles, nt = r - mt * n_tiles;
  const int m0 = mt * 64, n0 = nt * 64;
  const uint16_t* X = x + (int64_t)g * x_stride;
  const uint16_t* Wt = w1t + (int64_t)g * S * S;
  const int li = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  const bf16x8 zero8 = {};
  for (int k0 = 0; k0 < S; k0 += 32) {
    bf16x8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = m0 + 16 * i + li;
      a[i] = row < B ? *reinterpret_cast<const bf16x8*>(X + (int64_t)row * S + k0 + kq) : zero8;
      b[i] = *reinterpret_cast<const bf16x8*>(Wt + (int64_t)(n0 + 16 * i + li) * S + k0 + kq);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  float* Hg = h + (int64_t)g * B * S;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // D[16x16] fragment: lane holds rows 4*(lane/16) + e, column lane % 16
        const int row = m0 + 16 * i + (lane >> 4) * 4 + e;
        const int col = n0 + 16 * j + li;
        if (row < B) Hg[(int64_t)row * S + col] = act_tanh(acc[i][j][e]);
      }
}

// ----------------------------------------------------------------- output

// Y[b][j] = sum_t bf16(H[b][t]) w2t[j][t], fp32 accumulation in ascending t.
// One thread per (b, j); the weights of one genome are staged in LDS.
__global__ __launch_bounds__(256) void substrate_output_kernel(
    const float* __restrict__ h, const uint16_t* __restrict__ w2t, int S, int B, int m,
    int rows_per_wg, int wg_per_g, float* __restrict__ y) {
  extern __shared__ __align__(16) uint16_t w2s[];
  const int g = blockIdx.x / wg_per_g;
  const int part = blockIdx.x - g * wg_per_g;
  const uint16_t* W = w2t + (int64_t)g * S * m;
  for (int i = threadIdx.x; i < S * m; i += blockDim.x) w2s[i] = W[i];
  __syncthreads();
  const int b0 = part * rows_per_wg;
  for (int i = threadIdx.x; i < rows_per_wg * m; i += blockDim.x) {
    const int b = b0 + i / m, j = i - (i / m) * m;
    if (b >= B) continue;
    const float* hr = h + ((int64_t)g * B + b) * S;
    const uint16_t* wr = w2s + j * S;
    float acc = 0.0f;
    for (int t = 0; t < S; ++t) acc = fmaf(bf16_float(bf16_bits(hr[t])), bf16_float(wr[t]), acc);
    y[((int64_t)g * B + b) * m + j] = acc;
  }
}

}  // namespace

int check_substrate(const tn_substrate* sub) {
  if (!sub) return TN_EINVAL;
  if (sub->grid < 2 || sub->n_out < 1 || !(sub->threshold >= 0.0f)) return TN_EINVAL;
  const int64_t S = (int64_t)sub->grid * sub->grid;
  // MFMA tiles of 64 along S; the output weights of one genome fit in LDS
  if (S % 64 != 0 || S > 16384 || S * sub->n_out * 2 > 64 * 1024) return TN_EUNSUPPORTED;
  return TN_OK;
}

int launch_cppn_query(const tn_population& p, const tn_transformed& t, const tn_substrate& sub,
                      uint16_t* w1t, uint16_t* w2t, float* raw1, float* raw2,
                      hipStream_t stream) {
  SubGeom sg;
  sg.grid = sub.grid;
  sg.S = sub.grid * sub.grid;
  sg.n_out = sub.n_out;
  sg.thr = sub.threshold;
  sg.step = 2.0f / (float)(sub.grid - 1);
  sg.ostep = sub.n_out > 1 ? 2.0f / (float)(sub.n_out - 1) : 0.0f;
  const int64_t Q = (int64_t)sg.S * sg.S + (int64_t)sg.S * sg.n_out;  // < 2^31 by check_substrate
  const int64_t n_tiles = (Q + kWave - 1) / kWave;
  const int waves = 4, per_wave = 16;
  const int n_chunks = (int)((n_tiles + (int64_t)waves * per_wave - 1) / ((int64_t)waves * per_wave));
  const int64_t grid = (int64_t)p.P * n_chunks;
  if (grid == 0) return TN_OK;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  hipLaunchKernelGGL(cppn_query_kernel, dim3((unsigned)grid), dim3(kWave * waves), 0, stream,
                     make_view(p), t.status, t.prog_rows, t.n_valid,
                     reinterpret_cast<const int4*>(t.prog_node),
                     reinterpret_cast<const int2*>(t.prog_edge), t.io_pos, sg, n_chunks, per_wave,
                     w1t, w2t, raw1, raw2);
  return check_launch();
}

int launch_substrate_forward(const tn_substrate& sub, int P, const uint16_t* w1t,
                             const uint16_t* w2t, const uint16_t* x, int64_t x_stride, int B,
                             float* h, float* y, hipStream_t stream) {
  const int S = sub.grid * sub.grid;
  const int m_tiles = (B + 63) / 64, n_tiles = S / 64;
  const int64_t waves = (int64_t)P * m_tiles * n_tiles;
  if (waves == 0) return TN_OK;
  const int64_t grid = (waves + 3) / 4;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  hipLaunchKernelGGL(substrate_hidden_kernel, dim3((unsigned)grid), dim3(256), 0, stream, x,
                     x_stride, w1t, S, B, m_tiles, n_tiles, waves, h);
  int rc = check_launch();
  if (rc != TN_OK) return rc;
  const int rows_per_wg = std::max(1, 256 / sub.n_out);
  const int wg_per_g = (B + rows_per_wg - 1) / rows_per_wg;
  const size_t lds = sizeof(uint16_t) * (size_t)S * sub.n_out;
  rc = allow_lds((const void*)substrate_output_kernel, lds);
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(substrate_output_kernel, dim3((unsigned)(P * wg_per_g)), dim3(256), lds,
                     stream, h, w2t, S, B, sub.n_out, rows_per_wg, wg_per_g, y);
  return check_launch();
}

}  // namespace tn
