// Device building blocks of the calculation stage (TensorNEAT Section 3.3)
// shared by the forward, batched-forward and adjoint kernels.
#pragma once

#include "tn_internal.hpp"

namespace tn {

// Walks (b, c) = divmod(i, d) for i = start, start + stride, ... without a
// division per step (stride < 2^16 and d >= 1).
struct DivWalk {
  int b, c, qb, qc, d;
  __device__ DivWalk(int i, int d_, int stride) : d(d_) {
    b = i / d;
    c = i - b * d;
    qb = stride / d;
    qc = stride - qb * d;
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

// K consecutive floats of one LDS row (K = 1, 2, 4: one ds_read_b32/64/128).
template <int K> struct Vec;
template <> struct Vec<1> {
  float x[1];
  __device__ __forceinline__ void load(const float* p) { x[0] = *p; }
  __device__ __forceinline__ void store(float* p) const { *p = x[0]; }
};
template <> struct Vec<2> {
  float x[2];
  __device__ __forceinline__ void load(const float* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    x[0] = v.x;
    x[1] = v.y;
  }
  __device__ __forceinline__ void store(float* p) const {
    *reinterpret_cast<float2*>(p) = make_float2(x[0], x[1]);
  }
};
template <> struct Vec<4> {
  float x[4];
  __device__ __forceinline__ void load(const float* p) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
  __device__ __forceinline__ void store(float* p) const {
    *reinterpret_cast<float4*>(p) = make_float4(x[0], x[1], x[2], x[3]);
  }
};

// Node activations on the hardware exp2 / reciprocal (v_exp_f32, v_rcp_f32,
// about 1 ulp each). tanh switches to its odd Taylor polynomial below
// |z| = 1/4, where 1 - 2 / (1 + e^{2|z|}) would cancel; the polynomial's first
// omitted term is below 4e-11 relative there.
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float act_sigmoid(float z) {
  return rcp_hw(1.0f + exp2_hw(-kLog2e * z));
}

__device__ __forceinline__ float act_tanh(float z) {
  const float a = fabsf(z);
  // |z| >= 1/4: 1 - 2 / (1 + e^{2|z|}) with the sign of z
  const float e = exp2_hw(2.0f * kLog2e * a);
  const float big = fmaf(-2.0f, rcp_hw(1.0f + e), 1.0f);
  // |z| < 1/4: z + z^3 * (-1/3 + z^2 (2/15 + z^2 (-17/315 + z^2 (62/2835 +
  //            z^2 (-1382/155925 + z^2 * 21844/6081075)))))
  const float z2 = z * z;
  float q = 21844.0f / 6081075.0f;
  q = fmaf(q, z2, -1382.0f / 155925.0f);
  q = fmaf(q, z2, 62.0f / 2835.0f);
  q = fmaf(q, z2, -17.0f / 315.0f);
  q = fmaf(q, z2, 2.0f / 15.0f);
  q = fmaf(q, z2, -1.0f / 3.0f);
  const float small = fmaf(z * z2, q, z);
  return a < 0.25f ? small : copysignf(big, z);
}

__device__ __forceinline__ float act_gaussian(float z) { return exp2_hw(-kLog2e * (z * z)); }

template <int K>
__device__ __forceinline__ void activate_all(int act, const float (&z)[K], float (&v)[K]) {
  switch (act) {
    case TN_ACT_IDENTITY:
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = z[k];
      break;
    case TN_ACT_SIGMOID:
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = act_sigmoid(z[k]);
      break;
    case TN_ACT_TANH:
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = act_tanh(z[k]);
      break;
    case TN_ACT_RELU:
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = fmaxf(z[k], 0.0f);
      break;
    case TN_ACT_SIN:
      // one value at a time: the large-argument reduction of sinf needs
      // many registers, and K of them interleaved would not fit beside an
      // explicit register file
    {
      float zz[K];
#pragma unroll
      for (int k = 0; k < K; ++k) zz[k] = z[k];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        v[k] = sinf(zz[k]);
        if (k + 1 < K) asm volatile("" : "+v"(v[k]), "+v"(zz[(k + 1) % K]));
      }
    }
      break;
    case TN_ACT_GAUSSIAN:
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = act_gaussian(z[k]);
      break;
    default:  // TN_ACT_ABS (codes are validated by the transformation)
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = fabsf(z[k]);
      break;
  }
}

// One topological position of a genome's program.
struct NodeRec {
  int32_t erange;  // first in-edge | one-past-last in-edge << 16
  int32_t fn;      // act | agg << 8 | value row << 16; negative for an input position
  float bias;
  float resp;
};
struct EdgeRec {
  int32_t src;  // value row of the source
  float w;
};

// Node function word of a non-input position with its value row attached.
__host__ __device__ __forceinline__ int32_t fn_with_row(int32_t fn, int32_t row) {
  return fn < 0 ? fn : ((fn & 0xffff) | (row << 16));
}

// Program staged in LDS (one copy per workgroup). A record is read with one
// 16-byte load. kSrcBytes: the in-edge records hold the byte offset of the
// source row (row * kRow * 4) instead of its index, which saves a 32-bit
// multiply per in-edge.
// kBytes also changes the node's function word: act | agg << 3 | (byte offset
// of its value row) << 6 (negative for an input position), so the row's
// address needs no multiply.
template <bool kBytes>
struct LdsProgT {
  static constexpr bool kSrcBytes = kBytes;
  static constexpr bool kDstBytes = kBytes;
  const NodeRec* recs;
  const EdgeRec* edges;
  __device__ __forceinline__ NodeRec node(int p) const {
    const int4 q = reinterpret_cast<const int4*>(recs)[p];
    // all four words used here: the read is not split around the
    // input-position test that follows (inputs only, so nothing is copied)
    asm volatile("" ::"v"(q.x), "v"(q.y), "v"(q.z), "v"(q.w));
    NodeRec r;
    r.erange = q.x;
    r.fn = q.y;
    r.bias = __int_as_float(q.z);
    r.resp = __int_as_float(q.w);
    return r;
  }
  __device__ __forceinline__ EdgeRec edge(int e) const { return edges[e]; }
};
using LdsProg = LdsProgT<false>;

// Program read straight from the transformed arrays in global memory. The
// float arrays are read through int32 views, so that the kernel's float stores
// cannot alias them and the loads stay scalar.
struct GlobalProg {
  static constexpr bool kSrcBytes = false;
  static constexpr bool kDstBytes = false;
  const int32_t* rp;
  const int32_t* fn;
  const int32_t* bias;
  const int32_t* resp;
  const int32_t* src;
  const int32_t* w;
  const int32_t* row;  // value row of each position
  __device__ __forceinline__ NodeRec node(int p) const {
    NodeRec r;
    r.erange = rp[p] | (rp[p + 1] << 16);
    r.fn = fn_with_row(fn[p], row[p]);
    r.bias = __int_as_float(bias[p]);
    r.resp = __int_as_float(resp[p]);
    return r;
  }
  __device__ __forceinline__ EdgeRec edge(int e) const {
    EdgeRec q;
    q.src = row[src[e]];
    q.w = __int_as_float(w[e]);
    return q;
  }
};

// Evaluates position p of the program for this lane's K observations, whose
// floats sit at mine + row * kRow (value rows come from the program). Inputs
// are skipped (their rows hold the observation). Sum aggregation accumulates
// in ascending in-edge order with fused multiply-add.
// This lane's floats of the source row of in-edge record q.
template <int kRow, class Prog>
__device__ __forceinline__ const float* src_row(const float* mine, const EdgeRec& q) {
  if constexpr (Prog::kSrcBytes)
    return reinterpret_cast<const float*>(reinterpret_cast<const char*>(mine) + q.src);
  else
    return mine + q.src * kRow;
}

// s[k] += w * x[k] over in-edges e .. e+N-1 in ascending order, the N records
// requested first, then the N source values.
template <int N, int K, int kRow, class Prog>
__device__ __forceinline__ void sum_edges(const Prog& prog, int e, const float* mine, float (&s)[K]) {
  EdgeRec q[N];
#pragma unroll
  for (int j = 0; j < N; ++j) q[j] = prog.edge(e + j);
  Vec<K> x[N];
#pragma unroll
  for (int j = 0; j < N; ++j) x[j].load(src_row<kRow, Prog>(mine, q[j]));
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = fmaf(q[j].w, x[j].x[k], s[k]);
  }
}

template <int K, int kRow, class Prog>
__device__ __forceinline__ void eval_node(const Prog& prog, int p, float* mine) {
  const NodeRec rec = prog.node(p);
  const int f = __builtin_amdgcn_readfirstlane(rec.fn);
  if (f < 0) return;
  const int er = __builtin_amdgcn_readfirstlane(rec.erange);
  const int e0 = er & 0xffff, e1 = (er >> 16) & 0xffff;
  const int agg = Prog::kDstBytes ? (f >> 3) & 7 : (f >> 8) & 0xff;
  float s[K];
  if (agg == TN_AGG_SUM) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0f;
    // the last one to three in-edges unrolled: their records requested
    // together, then their source values; most nodes have no more than
    // three, so that case comes first (same order of terms either way)
    auto tail = [&](int e) {
      switch (e1 - e) {
        case 1: sum_edges<1, K, kRow>(prog, e, mine, s); break;
        case 2: sum_edges<2, K, kRow>(prog, e, mine, s); break;
        case 3: sum_edges<3, K, kRow>(prog, e, mine, s); break;
        default: break;
      }
    };
    if (__builtin_expect(e1 - e0 < 4, 1)) {
      tail(e0);
    } else {
      int e = e0;
      for (; e + 4 <= e1; e += 4) sum_edges<4, K, kRow>(prog, e, mine, s);
      tail(e);
    }
  } else if (e0 == e1) {
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0f;
  } else {
    {
      const EdgeRec q = prog.edge(e0);
      Vec<K> x;
      x.load(src_row<kRow, Prog>(mine, q));
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] = q.w * x.x[k];
    }
    for (int e = e0 + 1; e < e1; ++e) {
      const EdgeRec q = prog.edge(e);
      Vec<K> x;
      x.load(src_row<kRow, Prog>(mine, q));
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t = q.w * x.x[k];
        switch (agg) {
          case TN_AGG_PRODUCT: s[k] = s[k] * t; break;
          case TN_AGG_MAX: s[k] = fmaxf(s[k], t); break;
          case TN_AGG_MIN: s[k] = fminf(s[k], t); break;
          case TN_AGG_MEAN: s[k] = s[k] + t; break;
          default: s[k] = fabsf(t) > fabsf(s[k]) ? t : s[k]; break;  // maxabs
        }
      }
    }
    if (agg == TN_AGG_MEAN) {
      const float cnt = (float)(e1 - e0);
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] = s[k] / cnt;
    }
  }
  float z[K], v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) z[k] = fmaf(rec.resp, s[k], rec.bias);
  activate_all<K>(f & 7, z, v);  // codes below 7, checked by the transformation
  Vec<K> out;
#pragma unroll
  for (int k = 0; k < K; ++k) out.x[k] = v[k];
  if constexpr (Prog::kDstBytes)
    out.store(reinterpret_cast<float*>(reinterpret_cast<char*>(mine) + (f >> 6)));
  else
    out.store(mine + ((f >> 16) & 0x7fff) * kRow);
}

}  // namespace tn
