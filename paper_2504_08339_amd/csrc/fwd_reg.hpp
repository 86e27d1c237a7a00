// Register-resident evaluation of a genome's packed program (the calculation
// stage of TensorNEAT Section 3.3): one lane = one evaluation, node values in
// one or two 32-entry register banks addressed with a uniform index
// (s_set_gpr_idx), the program read with scalar loads. Shared by the forward
// engine and the CPPN query of the substrate.
#pragma once

#include "fwd_core.hpp"

namespace tn {

typedef float f32x32 __attribute__((ext_vector_type(32)));

// Node values of one lane: rows 0..31 in bank lo, rows 32..63 in bank hi
// (NB = 2). The banks are plain local vectors (a struct around them makes the
// compiler keep them in scratch memory).
template <int NB>
__device__ __forceinline__ float vget(const f32x32& lo, const f32x32& hi, int r) {
  if (NB == 1) return lo[r];
  const int r0 = r & 31;
  const float a = lo[r0], b = hi[r0];
  return r < 32 ? a : b;
}

// Both banks are written at r & 31, the untouched one with its own value: a
// write under a branch would make the compiler copy the whole bank.
template <int NB>
__device__ __forceinline__ void vset(f32x32& lo, f32x32& hi, int r, float x) {
  if (NB == 1) {
    lo[r] = x;
    return;
  }
  const int r0 = r & 31;
  const float o0 = lo[r0], o1 = hi[r0];
  lo[r0] = r < 32 ? x : o0;
  hi[r0] = r < 32 ? o1 : x;
}

// Program row of (non-input) position p: bits 16..30 of its function word.
__device__ __forceinline__ int prog_row(const int4* __restrict__ pn, int p) {
  return (pn[p].y >> 16) & 0x7fff;
}

// In-edges e .. e1-1 of one position, aggregated (Section 3.3's f_agg).
template <int NB>
__device__ __forceinline__ float aggregate(const f32x32& lo, const f32x32& hi,
                                           const int2* __restrict__ pe,
                                           int& e, int e1, int agg) {
  float s = 0.0f;
  if (agg == TN_AGG_SUM) {
    // scalar loads return out of order, so every use waits for all of them:
    // groups of 8 edges (one s_load_dwordx16) amortise that wait
    for (; e + 8 <= e1; e += 8) {
      int2 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = pe[e + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) s = fmaf(__int_as_float(q[u].y), vget<NB>(lo, hi, q[u].x), s);
    }
    if (e + 4 <= e1) {
      int2 q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = pe[e + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) s = fmaf(__int_as_float(q[u].y), vget<NB>(lo, hi, q[u].x), s);
      e += 4;
    }
    for (; e < e1; ++e) {
      const int2 q = pe[e];
      s = fmaf(__int_as_float(q.y), vget<NB>(lo, hi, q.x), s);
    }
    return s;
  }
  if (e == e1) return s;
  const int e0 = e;
  {
    const int2 q = pe[e];
    s = __int_as_float(q.y) * vget<NB>(lo, hi, q.x);
  }
  for (++e; e < e1; ++e) {
    const int2 q = pe[e];
    const float t = __int_as_float(q.y) * vget<NB>(lo, hi, q.x);
    switch (agg) {
      case TN_AGG_PRODUCT: s = s * t; break;
      case TN_AGG_MAX: s = fmaxf(s, t); break;
      case TN_AGG_MIN: s = fminf(s, t); break;
      case TN_AGG_MEAN: s = s + t; break;
      default: s = fabsf(t) > fabsf(s) ? t : s; break;  // maxabs
    }
  }
  if (agg == TN_AGG_MEAN) s = s / (float)(e1 - e0);
  return s;
}

// The program of one genome, in topological order, on this lane's banks;
// input rows must already hold the inputs. The next position's header is
// loaded before this position's edges, so one wait covers both.
template <int NB>
__device__ __forceinline__ void walk_program(f32x32& lo, f32x32& hi, const int4* __restrict__ pn,
                                             const int2* __restrict__ pe, int n) {
  int e = 0;
  int4 h = pn[0];
  for (int p = 0; p < n; ++p) {
    const int4 nx = pn[p + 1 < n ? p + 1 : p];
    const int f = h.y;
    if (f >= 0) {  // an input's row already holds its value
      const float s = aggregate<NB>(lo, hi, pe, e, h.x, (f >> 8) & 0xff);
      const float z[1] = {fmaf(__int_as_float(h.w), s, __int_as_float(h.z))};
      float a[1];
      activate_all<1>(f & 0xff, z, a);
      vset<NB>(lo, hi, (f >> 16) & 0x7fff, a[0]);
    }
    h = nx;
  }
}

}  // namespace tn
