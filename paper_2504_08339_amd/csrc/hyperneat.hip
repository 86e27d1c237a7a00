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
//   hidden   H = tanh(X W1): v_mfma_f32_16x16x32_bf16, a workgroup of four
//            wavefronts per 128 x 128 tile of H with K staged through LDS,
//            fp32 accumulation, tanh in the epilogue.
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

// Workgroups over (genome, chunk of query units); each wavefront takes
// `per_wave` consecutive units of 4 x 64 queries and runs the CPPN's packed
// program on them with the register engine's walk (a register file of 50 rows
// per tile, four tiles under each index window). Queries 0 .. S*S-1 fill w1t
// (t = q / S, s = q % S), the next S*m fill w2t (j, s); S*S is a multiple of
// 4096, so a unit lies in one of the two.
constexpr int kQueryRows = 50;

__global__ __launch_bounds__(256) __attribute__((amdgpu_num_vgpr(TN_RF_BASE))) void
cppn_query_kernel(PopView pop, const int32_t* __restrict__ status,
                  const int32_t* __restrict__ prog_rows, const int32_t* __restrict__ n_valid,
                  const int4* __restrict__ prog_node, const int2* __restrict__ prog_edge,
                  const int32_t* __restrict__ prog_rec, const int32_t* __restrict__ io_pos,
                  SubGeom sg, int n_chunks, int per_wave, uint16_t* __restrict__ w1t,
                  uint16_t* __restrict__ w2t, float* __restrict__ raw1, float* __restrict__ raw2) {
  constexpr int R = kQueryRows, K = rf_tiles(kQueryRows), kUnit = K * kWave;
  rf_reserve<R>();
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x / kWave;
  const int g = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - g * n_chunks;
  const int Q1 = sg.S * sg.S, Q = Q1 + sg.S * sg.n_out;  // < 2^31 (checked on the host)
  const int n_units = (Q + kUnit - 1) / kUnit;
  const int u0 = (chunk * W + wave) * per_wave;
  const int u1 = min(u0 + per_wave, n_units);
  const bool bad = status[g] != 0 || prog_rows[g] > R;
  const int nn = n_valid[g] - pop.n_in;
  const int64_t nb = uniform64(pop.node_base(g)), cb = uniform64(pop.conn_base(g));
  const int32_t* rec = prog_rec + nb * 16;
  const int2* pe = prog_edge + cb;
  const int nio = pop.n_in + pop.n_out;
  const int out_row =
      bad ? 0 : ((prog_node[nb + io_pos[(int64_t)g * nio + pop.n_in]].y >> 16) & 0x7fff);
  uint16_t* W1 = w1t + (int64_t)g * Q1;
  uint16_t* W2 = w2t + (int64_t)g * sg.S * sg.n_out;
  float* R1 = raw1 ? raw1 + (int64_t)g * Q1 : nullptr;
  float* R2 = raw2 ? raw2 + (int64_t)g * sg.S * sg.n_out : nullptr;
  const int step_r = kWave / sg.grid, step_c = kWave - step_r * sg.grid;  // 64 = step_r grid + step_c
  for (int u = u0; u < u1; ++u) {
    const bool first = u * kUnit < Q1;
    const int base = first ? u * kUnit : u * kUnit - Q1;
    float y[K];
    if (bad) {
#pragma unroll
      for (int k = 0; k < K; ++k) y[k] = __builtin_nanf("");
    } else {
      // the CPPN's inputs (x_s, y_s, x_t, y_t, 1) at rows 0..4 of every tile
      // query qq = tgt * S + src, src = rs * grid + cs, tgt = rt * grid + ct:
      // divided once for the unit's first tile, then stepped by 64 queries
      // per tile (S is a multiple of 64, so src wraps at most once a step)
      float xs[K], ys[K], xt[K], yt[K], one[K];
      const int q0 = base + lane;
      int tgt = q0 / sg.S;
      int src = q0 - tgt * sg.S;
      int rs = src / sg.grid, cs = src - rs * sg.grid;
      int rt = tgt / sg.grid, ct = tgt - rt * sg.grid;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        xs[k] = fmaf((float)cs, sg.step, -1.0f);
        ys[k] = fmaf((float)rs, sg.step, -1.0f);
        if (first) {
          xt[k] = fmaf((float)ct, sg.step, -1.0f);
          yt[k] = fmaf((float)rt, sg.step, -1.0f);
        } else {
          xt[k] = sg.n_out > 1 ? fmaf((float)tgt, sg.ostep, -1.0f) : 0.0f;
          yt[k] = 0.0f;
        }
        one[k] = 1.0f;
        src += kWave;
        rs += step_r;
        cs += step_c;
        if (cs >= sg.grid) {
          cs -= sg.grid;
          ++rs;
        }
        if (src >= sg.S) {
          src -= sg.S;
          rs -= sg.grid;
          ++tgt;
          if (++ct == sg.grid) {
            ct = 0;
            ++rt;
          }
        }
      }
      rfk_set<R>(0, xs);
      rfk_set<R>(1, ys);
      rfk_set<R>(2, xt);
      rfk_set<R>(3, yt);
      rfk_set<R>(4, one);
      walk_records<R>(rec, pe, nn, lane);
      rfk_get<R>(out_row, y);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int qq = base + k * kWave + lane;
      const uint16_t wb = bf16_bits(fabsf(y[k]) < sg.thr ? 0.0f : y[k]);
      if (first) {
        W1[qq] = wb;
        if (R1) R1[qq] = y[k];
      } else if (qq < sg.S * sg.n_out) {
        W2[qq] = wb;
        if (R2) R2[qq] = y[k];
      }
    }
  }
}

// ----------------------------------------------------------------- hidden

// Batched C[g][m][n] = sum_k A[g][m][k] * B[g][n][k] (bfloat16 operands, both
// contiguous along k; float32 accumulation). A workgroup of four wavefronts
// computes a 128 x 128 tile of C, each wavefront a 64 x 64 quarter with MFMA
// 16x16x32. K runs in stages of 64: while the wavefronts multiply from one LDS
// buffer, every thread fetches its 16-byte chunks of the next stage's A and B
// rows into registers and then writes them to the other buffer, one barrier
// per stage. Rows m >= M, n >= N and columns k >= K read zeros and are not
// stored; K is a multiple of 32. kTanh applies tanh in the epilogue (the
// substrate's hidden layer). The tiles of one batch entry are consecutive
// workgroups kept on one XCD, so its operands come from HBM once.
struct GemmArgs {
  const uint16_t* a;
  int64_t lda, a_batch;
  const uint16_t* b;
  int64_t ldb, b_batch;
  float* c;
  int64_t ldc, c_batch;
  int M, N, K;
  int m_tiles, n_tiles;
  int64_t n_items;
};

constexpr int kGemmTile = 128;              // rows of C per workgroup, both ways
constexpr int kGemmKs = 64;                 // k per stage
constexpr int kGemmRow = kGemmKs + 8;       // bf16 per LDS row (16 bytes of padding)
constexpr int kGemmBuf = kGemmTile * kGemmRow;  // bf16 per operand buffer
constexpr size_t kGemmLds = sizeof(uint16_t) * 4 * kGemmBuf;  // A and B, two buffers each

// Workgroup b of n runs on XCD b mod 8; returns the item it takes so that
// consecutive items share an XCD (the last n mod 8 in order).
__device__ __forceinline__ int64_t gemm_item(int64_t b, int64_t n) {
  constexpr int kXcd = 8;
  const int64_t per = n / kXcd, full = per * kXcd;
  if (b >= full) return b;
  return (b % kXcd) * per + b / kXcd;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// 16 bytes from global memory (the operands arrive as pointers in a struct
// argument, whose address space the compiler cannot infer)
__device__ __forceinline__ u32x4 load_global16(const uint16_t* q) {
  return *(const __attribute__((address_space(1))) u32x4*)q;
}
__device__ __forceinline__ void store_global(float* q, float v) {
  *(__attribute__((address_space(1))) float*)q = v;
}

template <bool kTanh>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs p) {
  extern __shared__ __align__(16) uint16_t gemm_lds[];
  const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
  const int64_t item = gemm_item(blockIdx.x, gridDim.x);
  const int per_g = p.m_tiles * p.n_tiles;
  const int g = (int)(item / per_g);
  const int r = (int)(item - (int64_t)g * per_g);
  const int nt = r / p.m_tiles, mt = r - nt * p.m_tiles;
  const int m0 = mt * kGemmTile, n0 = nt * kGemmTile;
  const uint16_t* A = p.a + (int64_t)g * p.a_batch;
  const uint16_t* Bm = p.b + (int64_t)g * p.b_batch;
  uint16_t* sa = gemm_lds;                 // [2][kGemmBuf]
  uint16_t* sb = gemm_lds + 2 * kGemmBuf;  // [2][kGemmBuf]

  // this thread's chunks of a stage: chunk c = tid + 256 u is row c / 8,
  // k (c % 8) * 8 .. + 7 of the stage
  constexpr int kChunks = kGemmTile * kGemmKs / 8 / 256;
  struct Regs {
    u32x4 a[kChunks], b[kChunks];
  };
  const u32x4 zero4 = {0u, 0u, 0u, 0u};
  auto fetch = [&](int st, Regs& r) {
    const int k0 = st * kGemmKs;
#pragma unroll
    for (int u = 0; u < kChunks; ++u) {
      const int c = tid + 256 * u, row = c >> 3, k = k0 + (c & 7) * 8;
      const bool kin = k < p.K;
      r.a[u] = m0 + row < p.M && kin ? load_global16(A + (int64_t)(m0 + row) * p.lda + k) : zero4;
      r.b[u] = n0 + row < p.N && kin ? load_global16(Bm + (int64_t)(n0 + row) * p.ldb + k) : zero4;
    }
  };
  auto stash = [&](int buf, const Regs& r) {
#pragma unroll
    for (int u = 0; u < kChunks; ++u) {
      const int c = tid + 256 * u, at = (c >> 3) * kGemmRow + (c & 7) * 8;
      *reinterpret_cast<u32x4*>(sa + buf * kGemmBuf + at) = r.a[u];
      *reinterpret_cast<u32x4*>(sb + buf * kGemmBuf + at) = r.b[u];
    }
  };

  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;  // this wavefront's quarter
  const int li = lane & 15, kq = (lane >> 4) * 8;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
  auto multiply = [&](int buf) {
    const uint16_t* pa = sa + buf * kGemmBuf + (wm + li) * kGemmRow + kq;
    const uint16_t* pb = sb + buf * kGemmBuf + (wn + li) * kGemmRow + kq;
#pragma unroll
    for (int kk = 0; kk < kGemmKs; kk += 32) {
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        fa[i] = *reinterpret_cast<const bf16x8*>(pa + 16 * i * kGemmRow + kk);
        fb[i] = *reinterpret_cast<const bf16x8*>(pb + 16 * i * kGemmRow + kk);
      }
      // B as the first operand: the fragment is the 16 x 16 block of C
      // transposed, so a lane ends up with four consecutive columns of a row
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[j], fa[i], acc[i][j], 0, 0, 0);
    }
  };
  // Stage st sits in LDS buffer st % 2 while the wavefronts multiply it; the
  // next stage is requested to registers before the multiply and written to
  // the other buffer after it, which was last read before the previous
  // barrier. (Two stages in flight need a second register set: 352 registers,
  // one wavefront per SIMD, or spills when held to two.)
  const int n_stages = (p.K + kGemmKs - 1) / kGemmKs;
  Regs rg;
  fetch(0, rg);
  stash(0, rg);
  __syncthreads();
  for (int st = 0; st < n_stages; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < n_stages;
    if (more) fetch(st + 1, rg);
    multiply(buf);
    if (more) stash(buf ^ 1, rg);
    __syncthreads();
  }
  float* C = p.c + (int64_t)g * p.c_batch;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // the fragment of D = C^T holds rows 4 (lane / 16) + e, column lane % 16:
      // C row lane % 16, columns 4 (lane / 16) + e of the block
      const int row = m0 + wm + 16 * i + li;
      const int col = n0 + wn + 16 * j + (lane >> 4) * 4;
      if (row >= p.M) continue;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = kTanh ? act_tanh(acc[i][j][e]) : acc[i][j][e];
      float* q = C + (int64_t)row * p.ldc + col;
      if (col + 3 < p.N && (p.ldc & 3) == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0) {
        f32x4 w = {v[0], v[1], v[2], v[3]};
        *(__attribute__((address_space(1))) f32x4*)q = w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (col + e < p.N) store_global(q + e, v[e]);
      }
    }
}

template <bool kTanh>
int launch_gemm(GemmArgs p, int batch, hipStream_t stream) {
  p.m_tiles = (p.M + kGemmTile - 1) / kGemmTile;
  p.n_tiles = (p.N + kGemmTile - 1) / kGemmTile;
  p.n_items = (int64_t)batch * p.m_tiles * p.n_tiles;
  const int rc = allow_lds((const void*)gemm_nt_kernel<kTanh>, kGemmLds);
  if (rc != TN_OK || p.n_items == 0) return rc;
  if (p.n_items > 0x7fffffff) return TN_EUNSUPPORTED;
  hipLaunchKernelGGL((gemm_nt_kernel<kTanh>), dim3((unsigned)p.n_items), dim3(256), kGemmLds,
                     stream, p);
  return check_launch();
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

// ---------------------------------------------------------------- backward

constexpr int kMaxOutBwd = 32;

// For L = sum(dY * Y), per hidden unit t of genome g (one thread each):
//   dw2t[j][t] = sum_b H[b][t] dY[b][j]                  (ascending b)
//   dz[b][t]   = (sum_j dY[b][j] w2t[j][t]) (1 - H[b][t]^2)
// dz is stored transposed and rounded to bfloat16, dzt[t][b], rows padded
// with zeros to Kp (a multiple of 32) for the weight-gradient GEMM.
__global__ __launch_bounds__(256) void substrate_grad_out_kernel(
    const float* __restrict__ h, const uint16_t* __restrict__ w2t, const float* __restrict__ dy,
    int S, int B, int Kp, int m, int wg_per_g, uint16_t* __restrict__ dzt,
    float* __restrict__ dw2t) {
  extern __shared__ __align__(16) float dys[];
  const int g = blockIdx.x / wg_per_g;
  const int t = (blockIdx.x - g * wg_per_g) * blockDim.x + threadIdx.x;
  const float* D = dy + (int64_t)g * B * m;
  for (int i = threadIdx.x; i < B * m; i += blockDim.x) dys[i] = D[i];
  __syncthreads();
  if (t >= S) return;
  float w2[kMaxOutBwd], acc[kMaxOutBwd];
#pragma unroll
  for (int j = 0; j < kMaxOutBwd; ++j) {
    w2[j] = j < m ? bf16_float(w2t[((int64_t)g * m + j) * S + t]) : 0.0f;
    acc[j] = 0.0f;
  }
  const float* H = h + (int64_t)g * B * S + t;
  uint16_t* Z = dzt + ((int64_t)g * S + t) * Kp;
  for (int b0 = 0; b0 < Kp; b0 += 8) {
    uint16_t pack[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u;
      float dz = 0.0f;
      if (b < B) {
        const float hb = H[(int64_t)b * S];
        const float* d = dys + b * m;
        float up = 0.0f;
#pragma unroll
        for (int j = 0; j < kMaxOutBwd; ++j)
          if (j < m) {
            up = fmaf(d[j], w2[j], up);
            acc[j] = fmaf(hb, d[j], acc[j]);
          }
        dz = up * fmaf(-hb, hb, 1.0f);
      }
      pack[u] = bf16_bits(dz);
    }
    uint4 v;
    v.x = pack[0] | ((uint32_t)pack[1] << 16);
    v.y = pack[2] | ((uint32_t)pack[3] << 16);
    v.z = pack[4] | ((uint32_t)pack[5] << 16);
    v.w = pack[6] | ((uint32_t)pack[7] << 16);
    *reinterpret_cast<uint4*>(Z + b0) = v;
  }
  for (int j = 0; j < m; ++j) dw2t[((int64_t)g * m + j) * S + t] = acc[j];
}

// xt[g][s][b] = x[g][b][s] (bfloat16 bits), rows padded with zeros to Kp.
__global__ __launch_bounds__(256) void transpose_x_kernel(const uint16_t* __restrict__ x,
                                                          int64_t x_stride, int S, int B, int Kp,
                                                          int wg_per_g, uint16_t* __restrict__ xt) {
  const int g = blockIdx.x / wg_per_g;
  const int s = (blockIdx.x - g * wg_per_g) * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint16_t* X = x + (int64_t)g * x_stride + s;
  uint16_t* T = xt + ((int64_t)g * S + s) * Kp;
  for (int b0 = 0; b0 < Kp; b0 += 8) {
    uint16_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = b0 + u < B ? X[(int64_t)(b0 + u) * S] : (uint16_t)0;
    uint4 q;
    q.x = v[0] | ((uint32_t)v[1] << 16);
    q.y = v[2] | ((uint32_t)v[3] << 16);
    q.z = v[4] | ((uint32_t)v[5] << 16);
    q.w = v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4*>(T + b0) = q;
  }
}

// ----------------------------------------------------------- CPPN adjoint

// Limits of the CPPN adjoint: node values, pre-activations and upstream
// gradients live in registers indexed by topological position (no row reuse:
// the reverse sweep needs every value).
constexpr int kCppnNodes = 32, kCppnEdges = 64;
constexpr int kCppnPart = kCppnEdges + kCppnNodes;  // partial sums per wavefront

// Register file of the adjoint, per tile of 64 queries: values V at rows
// 0..31, pre-activations Z at 32..63, upstream gradients G at 64..95; two
// tiles per wavefront, tile 0 at v56, tile 1 at v152 (v56..v247 in all, the
// compiler keeping v0..v55). Windows wait two cycles after s_set_gpr_idx_on
// (see fwd_reg.hpp).
__device__ __forceinline__ void adj_reserve() { asm volatile("" ::: "v247"); }

// s{0,1} += w * V[j] of tiles 0 and 1.
__device__ __forceinline__ void adj_fma_v(float& s0, float& s1, float w, int j) {
  asm volatile(
      "s_set_gpr_idx_on %3, gpr_idx(SRC1)\n\ts_nop 1\n\tv_fmac_f32 %0, %2, v56\n\t"
      "v_fmac_f32 %1, %2, v152\n\ts_set_gpr_idx_off"
      : "+v"(s0), "+v"(s1)
      : "s"(w), "s"(j) : "m0");
}
// V[p] := v{0,1}
__device__ __forceinline__ void adj_set_v(int p, float v0, float v1) {
  asm volatile(
      "s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v56, %0\n\t"
      "v_mov_b32 v152, %1\n\ts_set_gpr_idx_off" ::"v"(v0),
      "v"(v1), "s"(p) : "m0");
}
// V[p] := v{0,1}, Z[p] := z{0,1}
__device__ __forceinline__ void adj_set_vz(int p, float v0, float v1, float z0, float z1) {
  asm volatile(
      "s_set_gpr_idx_on %4, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v56, %0\n\t"
      "v_mov_b32 v152, %1\n\tv_mov_b32 v88, %2\n\tv_mov_b32 v184, %3\n\ts_set_gpr_idx_off" ::"v"(v0),
      "v"(v1), "v"(z0), "v"(z1), "s"(p) : "m0");
}
// G[p] := g{0,1}
__device__ __forceinline__ void adj_set_g(int p, float g0, float g1) {
  asm volatile(
      "s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v120, %0\n\t"
      "v_mov_b32 v216, %1\n\ts_set_gpr_idx_off" ::"v"(g0),
      "v"(g1), "s"(p) : "m0");
}
// t{0,1} := V[j]
__device__ __forceinline__ void adj_get_v(int j, float& t0, float& t1) {
  asm volatile(
      "s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v56\n\t"
      "v_mov_b32 %1, v152\n\ts_set_gpr_idx_off"
      : "=v"(t0), "=v"(t1)
      : "s"(j) : "m0");
}
// G[p], V[p], Z[p] of both tiles
__device__ __forceinline__ void adj_get_gvz(int p, float& g0, float& g1, float& v0, float& v1,
                                            float& z0, float& z1) {
  asm volatile(
      "s_set_gpr_idx_on %6, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v120\n\t"
      "v_mov_b32 %1, v216\n\tv_mov_b32 %2, v56\n\tv_mov_b32 %3, v152\n\t"
      "v_mov_b32 %4, v88\n\tv_mov_b32 %5, v184\n\ts_set_gpr_idx_off"
      : "=v"(g0), "=v"(g1), "=v"(v0), "=v"(v1), "=v"(z0), "=v"(z1)
      : "s"(p) : "m0");
}
// G[j] += dt{0,1} * w, one indexed read-modify-write per tile
__device__ __forceinline__ void adj_fma_g(int j, float dt0, float dt1, float w) {
  asm volatile(
      "s_set_gpr_idx_on %3, gpr_idx(SRC2,DST)\n\ts_nop 1\n\tv_fma_f32 v120, %0, %2, v120\n\t"
      "v_fma_f32 v216, %1, %2, v216\n\ts_set_gpr_idx_off" ::"v"(dt0),
      "v"(dt1), "s"(w), "s"(j) : "m0");
}
// G := 0 for both tiles (fixed registers, no window)
__device__ __forceinline__ void adj_zero_g() {
  asm volatile(
#define TN_Z4(a, b, c, d) "v_mov_b32 v" #a ", 0\n\tv_mov_b32 v" #b ", 0\n\tv_mov_b32 v" #c \
                          ", 0\n\tv_mov_b32 v" #d ", 0\n\t"
      TN_Z4(120, 121, 122, 123) TN_Z4(124, 125, 126, 127) TN_Z4(128, 129, 130, 131)
      TN_Z4(132, 133, 134, 135) TN_Z4(136, 137, 138, 139) TN_Z4(140, 141, 142, 143)
      TN_Z4(144, 145, 146, 147) TN_Z4(148, 149, 150, 151) TN_Z4(216, 217, 218, 219)
      TN_Z4(220, 221, 222, 223) TN_Z4(224, 225, 226, 227) TN_Z4(228, 229, 230, 231)
      TN_Z4(232, 233, 234, 235) TN_Z4(236, 237, 238, 239) TN_Z4(240, 241, 242, 243)
      TN_Z4(244, 245, 246, 247)
#undef TN_Z4
      "s_nop 0");
}

__device__ __forceinline__ float cppn_slope(int act, float v, float z) {
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

// The gradient of sum_q u_q * w(q) over every query q of the substrate with
// respect to the CPPN's connection weights and node biases, where the upstream
// u_q is dw1t / dw2t at the query when its weight survived the threshold (the
// CPPN value of this very evaluation, float32) and 0 otherwise. Each lane runs
// the CPPN forward at one query of each of the wavefront's two tiles (values
// and pre-activations kept by position), then the reverse sweep:
//   delta_k = gbar_k act'(z_k);  db_k += delta_k;
//   for in-edge e = (j -> k): dt = delta_k rho_k (/ n for mean);
//   dw_e += dt v_j;  gbar_j += dt w_e
// The per-lane sums (both tiles' terms added first) accumulate in LDS, one
// slot per lane and sum (read, add, write: a wavefront's LDS operations
// complete in order, so each sum runs in program order); at the end every
// slot is reduced over the wavefront in a fixed order and written to this
// wavefront's slot of `part`.
// Sum and mean aggregation only (the CPPN's); other genomes get NaN.
// The kernel is compiled for two slot counts and both forms are launched:
// KE = 48 in-edge slots (80 per lane with the node slots: 20 KB per
// wavefront, so eight wavefronts fit a compute unit's LDS, as many as its
// registers allow) takes the genomes with at most 48 in-edges, KE = 64 the
// others and writes the NaN partials of the genomes no form takes.
constexpr int kCppnWaves = 2, kCppnUnitsPerWave = 32, kCppnUnit = 2 * kWave;
constexpr int kCppnCompactEdges = 48;

template <int KE>
__global__ __launch_bounds__(kWave * kCppnWaves) __attribute__((amdgpu_num_vgpr(TN_RF_BASE))) void
cppn_backward_kernel(PopView pop, const int32_t* __restrict__ status,
                     const int32_t* __restrict__ n_valid, const int32_t* __restrict__ row_ptr,
                     const int32_t* __restrict__ edge_src, const int32_t* __restrict__ w_bits,
                     const int32_t* __restrict__ fn, const int32_t* __restrict__ bias_bits,
                     const int32_t* __restrict__ resp_bits, const int32_t* __restrict__ io_pos,
                     SubGeom sg, int n_chunks, const float* __restrict__ dw1t,
                     const float* __restrict__ dw2t, float* __restrict__ part) {
  adj_reserve();
  constexpr int kSlots = KE + kCppnNodes;  // LDS sums per lane: in-edges, then positions
  __shared__ float acc_all[kCppnWaves * kSlots * kWave];
  const int lane = lane_id();
  const int wave = wave_id();
  const int W = blockDim.x / kWave;
  const int g = blockIdx.x / n_chunks;
  const int chunk = blockIdx.x - g * n_chunks;
  float* out = part + ((int64_t)g * n_chunks * W + (int64_t)chunk * W + wave) * kCppnPart;
  float* acc = acc_all + wave * kSlots * kWave + lane;  // slot i at acc[i * kWave]
  const int n = n_valid[g];
  const int64_t nb = uniform64(pop.node_base(g)), cb = uniform64(pop.conn_base(g)),
                rb = uniform64(pop.rowptr_base(g));
  const int32_t* rp = row_ptr + rb;
  const int n_edges = n > 0 ? rp[n] : 0;
  const int nio = pop.n_in + pop.n_out;
  const int op = status[g] ? 0 : io_pos[(int64_t)g * nio + pop.n_in];
  bool ok = status[g] == 0 && n <= kCppnNodes && n_edges <= kCppnEdges;
  for (int p = 0; ok && p < n; ++p) {
    const int f = fn[nb + p];
    const int agg = (f >> 8) & 0xff;
    if (f >= 0 && agg != TN_AGG_SUM && agg != TN_AGG_MEAN) ok = false;
  }
  if (!ok) {
    if (KE == kCppnEdges)
      for (int i = lane; i < kCppnPart; i += kWave) out[i] = __builtin_nanf("");
    return;
  }
  if ((n_edges <= kCppnCompactEdges) != (KE == kCppnCompactEdges)) return;  // the other form's
  for (int i = 0; i < kSlots; ++i) acc[i * kWave] = 0.0f;
  // the genome's program across the wavefront, read once: lane p holds
  // position p's function word, bias, response and first in-edge (lane n the
  // end of the last), lane e edge e's source position and weight; the sweeps
  // below take every field with v_readlane instead of a memory load
  const int l_fn = lane < n ? fn[nb + lane] : 0;
  const int l_bias = lane < n ? bias_bits[nb + lane] : 0;
  const int l_resp = lane < n ? resp_bits[nb + lane] : 0;
  const int l_rp = lane <= n ? rp[lane] : 0;
  const int l_src = lane < n_edges ? edge_src[cb + lane] : 0;
  const int l_w = lane < n_edges ? w_bits[cb + lane] : 0;
  const int Q1 = sg.S * sg.S, Q2 = sg.S * sg.n_out, Q = Q1 + Q2;
  const int n_units = (Q + kCppnUnit - 1) / kCppnUnit;
  const int u0 = (chunk * W + wave) * kCppnUnitsPerWave;
  const int u1 = min(u0 + kCppnUnitsPerWave, n_units);
  const int step_r = kWave / sg.grid, step_c = kWave - step_r * sg.grid;  // 64 = step_r grid + step_c
  for (int u = u0; u < u1; ++u) {
    const bool first = u * kCppnUnit < Q1;  // S*S is a multiple of 4096
    const int base = first ? u * kCppnUnit : u * kCppnUnit - Q1;
    // coordinates divided once for the first tile, stepped by 64 queries for
    // the second (as in the query kernel)
    float in[2][5], up[2];
    int tgt = (base + lane) / sg.S;
    int src = base + lane - tgt * sg.S;
    int rs = src / sg.grid, cs = src - rs * sg.grid;
    int rt = tgt / sg.grid, ct = tgt - rt * sg.grid;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int qq = base + k * kWave + lane;
      in[k][0] = fmaf((float)cs, sg.step, -1.0f);
      in[k][1] = fmaf((float)rs, sg.step, -1.0f);
      if (first) {
        in[k][2] = fmaf((float)ct, sg.step, -1.0f);
        in[k][3] = fmaf((float)rt, sg.step, -1.0f);
        up[k] = dw1t[(int64_t)g * Q1 + qq];
      } else {
        in[k][2] = sg.n_out > 1 ? fmaf((float)tgt, sg.ostep, -1.0f) : 0.0f;
        in[k][3] = 0.0f;
        up[k] = qq < Q2 ? dw2t[(int64_t)g * Q2 + qq] : 0.0f;
      }
      in[k][4] = 1.0f;
      src += kWave;
      rs += step_r;
      cs += step_c;
      if (cs >= sg.grid) {
        cs -= sg.grid;
        ++rs;
      }
      if (src >= sg.S) {
        src -= sg.S;
        rs -= sg.grid;
        ++tgt;
        if (++ct == sg.grid) {
          ct = 0;
          ++rt;
        }
      }
    }
    // forward, values and pre-activations by position
    for (int p = 0; p < n; ++p) {
      const int f = __builtin_amdgcn_readlane(l_fn, p);
      if (f < 0) {
        const int i = (f >> 16) & 0x7fff;
        float x[2];
#pragma unroll
        for (int k = 0; k < 2; ++k)
          x[k] = i == 0 ? in[k][0] : i == 1 ? in[k][1] : i == 2 ? in[k][2] : i == 3 ? in[k][3]
                                                                                 : in[k][4];
        adj_set_v(p, x[0], x[1]);
        continue;
      }
      const int e0 = __builtin_amdgcn_readlane(l_rp, p), e1 = __builtin_amdgcn_readlane(l_rp, p + 1);
      float s0 = 0.0f, s1 = 0.0f;
      for (int e = e0; e < e1; ++e) {
        const int j = __builtin_amdgcn_readlane(l_src, e);
        adj_fma_v(s0, s1, __int_as_float(__builtin_amdgcn_readlane(l_w, e)), j);
      }
      if (((f >> 8) & 0xff) == TN_AGG_MEAN && e1 > e0) {
        s0 = s0 / (float)(e1 - e0);
        s1 = s1 / (float)(e1 - e0);
      }
      const float rho = __int_as_float(__builtin_amdgcn_readlane(l_resp, p));
      const float bias = __int_as_float(__builtin_amdgcn_readlane(l_bias, p));
      const float z[2] = {fmaf(rho, s0, bias), fmaf(rho, s1, bias)};
      float v[2];
      activate_all<2>(f & 7, z, v);  // codes below 7 (flagged genomes return above)
      adj_set_vz(p, v[0], v[1], z[0], z[1]);
    }
    float y0, y1;
    adj_get_v(op, y0, y1);
    // NaN y: no gradient
    adj_zero_g();
    adj_set_g(op, fabsf(y0) >= sg.thr ? up[0] : 0.0f, fabsf(y1) >= sg.thr ? up[1] : 0.0f);
    // reverse sweep
    for (int p = n - 1; p >= 0; --p) {
      const int f = __builtin_amdgcn_readlane(l_fn, p);
      if (f < 0) continue;
      float g0, g1, v0, v1, z0, z1;
      adj_get_gvz(p, g0, g1, v0, v1, z0, z1);
      const int act = f & 7;
      const float d0 = g0 * cppn_slope(act, v0, z0), d1 = g1 * cppn_slope(act, v1, z1);
      acc[(KE + p) * kWave] += d0 + d1;
      const int e0 = __builtin_amdgcn_readlane(l_rp, p), e1 = __builtin_amdgcn_readlane(l_rp, p + 1);
      const float rho = __int_as_float(__builtin_amdgcn_readlane(l_resp, p));
      float dt0 = d0 * rho, dt1 = d1 * rho;
      if (((f >> 8) & 0xff) == TN_AGG_MEAN && e1 > e0) {
        dt0 = dt0 / (float)(e1 - e0);
        dt1 = dt1 / (float)(e1 - e0);
      }
      // two in-edges per step (their sources differ, so the two updates of
      // G are independent); the fields of both are read before either window
      int e = e0;
      for (; e + 1 < e1; e += 2) {
        const float oa = acc[e * kWave], ob = acc[(e + 1) * kWave];  // loads issued first
        const int ja = __builtin_amdgcn_readlane(l_src, e);
        const int jb = __builtin_amdgcn_readlane(l_src, e + 1);
        const float wa = __int_as_float(__builtin_amdgcn_readlane(l_w, e));
        const float wb = __int_as_float(__builtin_amdgcn_readlane(l_w, e + 1));
        float ta0, ta1, tb0, tb1;
        adj_get_v(ja, ta0, ta1);
        adj_get_v(jb, tb0, tb1);
        adj_fma_g(ja, dt0, dt1, wa);
        adj_fma_g(jb, dt0, dt1, wb);
        acc[e * kWave] = oa + fmaf(dt1, ta1, dt0 * ta0);
        acc[(e + 1) * kWave] = ob + fmaf(dt1, tb1, dt0 * tb0);
      }
      if (e < e1) {
        const float o = acc[e * kWave];
        const int j = __builtin_amdgcn_readlane(l_src, e);
        float t0, t1;
        adj_get_v(j, t0, t1);
        adj_fma_g(j, dt0, dt1, __int_as_float(__builtin_amdgcn_readlane(l_w, e)));
        acc[e * kWave] = o + fmaf(dt1, t1, dt0 * t0);
      }
    }
  }
  // one reduction over the wavefront per sum, fixed order; partial slot
  // layout: in-edge e at e, position p at kCppnEdges + p
  for (int i = 0; i < kSlots; ++i) {
    const float t = wave_sum(acc[i * kWave]);
    if (lane == 0) out[i < KE ? i : kCppnEdges + (i - KE)] = t;
  }
}

// Sums the wavefront partials of each genome in slot order and scatters them:
// dW[connection row of in-edge e], db[node row of position p]; every other row
// of the genome (disabled, padding, inputs) is 0; NaN where the partials are.
__global__ __launch_bounds__(256) void cppn_grad_reduce_kernel(
    PopView pop, const int32_t* __restrict__ n_valid, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ edge_row, const int32_t* __restrict__ order,
    const int32_t* __restrict__ fn, const float* __restrict__ part, int slots,
    float* __restrict__ dW, float* __restrict__ db) {
  const int g = blockIdx.x;
  const int64_t nb = pop.node_base(g), cb = pop.conn_base(g), rb = pop.rowptr_base(g);
  const int nrows = (int)pop.node_rows(g), crows = (int)pop.conn_rows(g);
  const int n = n_valid[g];
  const int n_edges = n > 0 ? row_ptr[rb + n] : 0;
  const float* pg = part + (int64_t)g * slots * kCppnPart;
  const bool bad = n == 0 || pg[0] != pg[0] || n > kCppnNodes || n_edges > kCppnEdges;
  for (int r = threadIdx.x; r < crows; r += blockDim.x) dW[cb + r] = bad ? __builtin_nanf("") : 0.0f;
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) db[nb + r] = bad ? __builtin_nanf("") : 0.0f;
  __syncthreads();
  if (bad) return;
  for (int i = threadIdx.x; i < n_edges + n; i += blockDim.x) {
    const int col = i < n_edges ? i : kCppnEdges + (i - n_edges);
    float acc = 0.0f;
    for (int w = 0; w < slots; ++w) acc += pg[(int64_t)w * kCppnPart + col];
    if (i < n_edges) {
      dW[cb + edge_row[cb + i]] = acc;
    } else {
      const int p = i - n_edges;
      if (fn[nb + p] >= 0) db[nb + order[nb + p]] = acc;
    }
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
  const int64_t unit = (int64_t)rf_tiles(kQueryRows) * kWave;
  const int64_t n_units = (Q + unit - 1) / unit;
  const int waves = 4, per_wave = 4;
  const int n_chunks = (int)((n_units + (int64_t)waves * per_wave - 1) / ((int64_t)waves * per_wave));
  const int64_t grid = (int64_t)p.P * n_chunks;
  if (grid == 0) return TN_OK;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  hipLaunchKernelGGL(cppn_query_kernel, dim3((unsigned)grid), dim3(kWave * waves), 0, stream,
                     make_view(p), t.status, t.prog_rows, t.n_valid,
                     reinterpret_cast<const int4*>(t.prog_node),
                     reinterpret_cast<const int2*>(t.prog_edge), t.prog_rec, t.io_pos, sg,
                     n_chunks, per_wave, w1t, w2t, raw1, raw2);
  return check_launch();
}

int launch_substrate_forward(const tn_substrate& sub, int P, const uint16_t* w1t,
                             const uint16_t* w2t, const uint16_t* x, int64_t x_stride, int B,
                             float* h, float* y, hipStream_t stream) {
  const int S = sub.grid * sub.grid;
  GemmArgs ga{};
  ga.a = x;
  ga.lda = S;
  ga.a_batch = x_stride;
  ga.b = w1t;
  ga.ldb = S;
  ga.b_batch = (int64_t)S * S;
  ga.c = h;
  ga.ldc = S;
  ga.c_batch = (int64_t)B * S;
  ga.M = B;
  ga.N = S;
  ga.K = S;
  int rc = launch_gemm<true>(ga, P, stream);
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

size_t substrate_workspace_bytes(const tn_substrate& sub, int P, int B, int64_t x_stride) {
  const int64_t S = (int64_t)sub.grid * sub.grid;
  const int64_t Kp = ((int64_t)B + 31) / 32 * 32;
  const int64_t px = x_stride == 0 ? 1 : P;
  return (size_t)(2 * S * Kp * (P + px));
}

int launch_substrate_backward(const tn_substrate& sub, int P, const uint16_t* w2t,
                              const uint16_t* x, int64_t x_stride, int B, const float* h,
                              const float* dy, void* workspace, float* dw1t, float* dw2t,
                              hipStream_t stream) {
  const int S = sub.grid * sub.grid, m = sub.n_out;
  const int Kp = (B + 31) / 32 * 32;
  const int px = x_stride == 0 ? 1 : P;
  uint16_t* dzt = static_cast<uint16_t*>(workspace);
  uint16_t* xt = dzt + (int64_t)P * S * Kp;
  const int wg_per_g = (S + 255) / 256;
  const size_t lds = sizeof(float) * (size_t)B * m;
  int rc = allow_lds((const void*)substrate_grad_out_kernel, lds);
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(substrate_grad_out_kernel, dim3((unsigned)(P * wg_per_g)), dim3(256), lds,
                     stream, h, w2t, dy, S, B, Kp, m, wg_per_g, dzt, dw2t);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  hipLaunchKernelGGL(transpose_x_kernel, dim3((unsigned)(px * wg_per_g)), dim3(256), 0, stream, x,
                     x_stride, S, B, Kp, wg_per_g, xt);
  rc = check_launch();
  if (rc != TN_OK) return rc;
  // dw1t[t][s] = sum_b dz[b][t] x[b][s]
  GemmArgs ga{};
  ga.a = dzt;
  ga.lda = Kp;
  ga.a_batch = (int64_t)S * Kp;
  ga.b = xt;
  ga.ldb = Kp;
  ga.b_batch = x_stride == 0 ? 0 : (int64_t)S * Kp;
  ga.c = dw1t;
  ga.ldc = S;
  ga.c_batch = (int64_t)S * S;
  ga.M = S;
  ga.N = S;
  ga.K = Kp;
  return launch_gemm<false>(ga, P, stream);
}

namespace {
int cppn_chunks(const tn_substrate& sub) {
  const int64_t S = (int64_t)sub.grid * sub.grid;
  const int64_t n_units = (S * S + S * sub.n_out + kCppnUnit - 1) / kCppnUnit;
  const int64_t per_wg = (int64_t)kCppnWaves * kCppnUnitsPerWave;
  return (int)((n_units + per_wg - 1) / per_wg);
}
}  // namespace

size_t cppn_backward_workspace_bytes(const tn_population& p, const tn_substrate& sub) {
  return sizeof(float) * (size_t)p.P * cppn_chunks(sub) * kCppnWaves * kCppnPart;
}

int launch_cppn_backward(const tn_population& p, const tn_transformed& t, const tn_substrate& sub,
                         const float* dw1t, const float* dw2t, void* workspace, float* dW,
                         float* db, hipStream_t stream) {
  SubGeom sg;
  sg.grid = sub.grid;
  sg.S = sub.grid * sub.grid;
  sg.n_out = sub.n_out;
  sg.thr = sub.threshold;
  sg.step = 2.0f / (float)(sub.grid - 1);
  sg.ostep = sub.n_out > 1 ? 2.0f / (float)(sub.n_out - 1) : 0.0f;
  const int n_chunks = cppn_chunks(sub);
  const int64_t grid = (int64_t)p.P * n_chunks;
  if (grid == 0) return TN_OK;
  if (grid > 0x7fffffff) return TN_EUNSUPPORTED;
  float* part = static_cast<float*>(workspace);
  int rc = TN_OK;
#define TN_CPPN_BWD(KE)                                                                        \
  hipLaunchKernelGGL(cppn_backward_kernel<KE>, dim3((unsigned)grid), dim3(kWave * kCppnWaves), \
                     0, stream, make_view(p), t.status, t.n_valid, t.row_ptr, t.edge_src,      \
                     reinterpret_cast<const int32_t*>(t.edge_w), t.pos_fn,                    \
                     reinterpret_cast<const int32_t*>(t.pos_bias),                            \
                     reinterpret_cast<const int32_t*>(t.pos_resp), t.io_pos, sg, n_chunks,    \
                     dw1t, dw2t, part);                                                       \
  rc = check_launch();                                                                        \
  if (rc != TN_OK) return rc;
  TN_CPPN_BWD(kCppnCompactEdges)
  TN_CPPN_BWD(kCppnEdges)
#undef TN_CPPN_BWD
  hipLaunchKernelGGL(cppn_grad_reduce_kernel, dim3((unsigned)p.P), dim3(256), 0, stream,
                     make_view(p), t.n_valid, t.row_ptr, t.edge_row, t.order, t.pos_fn, part,
                     n_chunks * kCppnWaves, dW, db);
  return check_launch();
}

}  // namespace tn
