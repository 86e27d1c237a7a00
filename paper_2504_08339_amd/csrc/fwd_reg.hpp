// Register-resident evaluation of a genome's packed program (the calculation
// stage of TensorNEAT Section 3.3): one lane = one evaluation, node values in
// registers addressed with a uniform index (s_set_gpr_idx), the program read
// with scalar loads. Shared by the forward engine and the CPPN query of the
// substrate. Two storage forms, chosen by the template parameter NB:
//   NB = 1, 2   one or two 32-entry vector banks the compiler allocates (a
//               row of the second bank costs a select);
//   NB >= 32    an explicit register file of NB rows at v[kRfBase ..
//               kRfBase + NB): the kernel limits the compiler to the VGPRs
//               below kRfBase and reserves the file with a clobber, and every
//               access is one s_set_gpr_idx window around one instruction (an
//               in-edge is a single v_fmac_f32 with an indexed operand).
#pragma once

#include "fwd_core.hpp"

namespace tn {

typedef float f32x32 __attribute__((ext_vector_type(32)));

// First VGPR of the explicit register file; kernels using it carry
// __attribute__((amdgpu_num_vgpr(kRfBase))).
#define TN_RF_BASE 48
#define TN_RF_V0 "v48"
constexpr int kRfBase = TN_RF_BASE;

// s_set_gpr_idx_on writes M0; none of these kernels keeps anything in M0.
__device__ __forceinline__ float rf_get(int r) {
  float x;
  asm volatile("s_set_gpr_idx_on %1, gpr_idx(SRC0)\n\tv_mov_b32 %0, " TN_RF_V0
               "\n\ts_set_gpr_idx_off"
               : "=v"(x)
               : "s"(r));
  return x;
}
__device__ __forceinline__ void rf_set(int r, float x) {
  asm volatile("s_set_gpr_idx_on %1, gpr_idx(DST)\n\tv_mov_b32 " TN_RF_V0
               ", %0\n\ts_set_gpr_idx_off" ::"v"(x),
               "s"(r));
}
// acc += w * row[r] in one instruction
__device__ __forceinline__ void rf_fma(float& acc, float w, int r) {
  asm volatile("s_set_gpr_idx_on %2, gpr_idx(SRC1)\n\tv_fmac_f32 %0, %1, " TN_RF_V0
               "\n\ts_set_gpr_idx_off"
               : "+v"(acc)
               : "s"(w), "s"(r));
}

// Makes the compiler count the register file in the kernel's VGPR allocation
// (a clobber of its last register); R = rows.
template <int R>
__device__ __forceinline__ void rf_reserve() {
  static_assert(R == 32 || R == 64 || R == 96 || R == 128 || R == 160 || R == 208,
                "register file sizes");
  if constexpr (R == 32) asm volatile("" ::: "v79");
  if constexpr (R == 64) asm volatile("" ::: "v111");
  if constexpr (R == 96) asm volatile("" ::: "v143");
  if constexpr (R == 128) asm volatile("" ::: "v175");
  if constexpr (R == 160) asm volatile("" ::: "v207");
  if constexpr (R == 208) asm volatile("" ::: "v255");
}

// Node values of one lane: rows 0..31 in bank lo, rows 32..63 in bank hi
// (NB = 2). The banks are plain local vectors (a struct around them makes the
// compiler keep them in scratch memory).
template <int NB>
__device__ __forceinline__ float vget(const f32x32& lo, const f32x32& hi, int r) {
  if constexpr (NB >= 32) return rf_get(r);
  if (NB == 1) return lo[r];
  const int r0 = r & 31;
  const float a = lo[r0], b = hi[r0];
  return r < 32 ? a : b;
}

// Both banks are written at r & 31, the untouched one with its own value: a
// write under a branch would make the compiler copy the whole bank.
template <int NB>
__device__ __forceinline__ void vset(f32x32& lo, f32x32& hi, int r, float x) {
  if constexpr (NB >= 32) {
    rf_set(r, x);
    return;
  }
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

// s += w * value of the edge's source row (one in-edge of the sum).
template <int NB>
__device__ __forceinline__ void edge_fma(const f32x32& lo, const f32x32& hi, float& s, int2 q) {
  if constexpr (NB >= 32)
    rf_fma(s, __int_as_float(q.y), q.x);
  else
    s = fmaf(__int_as_float(q.y), vget<NB>(lo, hi, q.x), s);
}

// In-edges e .. e1-1 of one position, aggregated (Section 3.3's f_agg); g
// holds the first 8 edge words from e on (loaded ahead). Edge words may be
// read up to 7 past e1 (tn_transformed.prog_edge is padded for that).
template <int NB>
__device__ __forceinline__ float aggregate(const f32x32& lo, const f32x32& hi,
                                           const int2* __restrict__ pe, const int2 (&g)[8],
                                           int e, int e1, int agg) {
  const int cnt = e1 - e;
  float s = 0.0f;
  if (agg == TN_AGG_SUM) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (u < cnt) edge_fma<NB>(lo, hi, s, g[u]);
    // further edges 8 at a time (one s_load_dwordx16; scalar loads return out
    // of order, so each use waits for all of them)
    for (int b = e + 8; b < e1; b += 8) {
      int2 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = pe[b + u];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (b + u < e1) edge_fma<NB>(lo, hi, s, q[u]);
    }
    return s;
  }
  if (cnt == 0) return s;
  s = __int_as_float(g[0].y) * vget<NB>(lo, hi, g[0].x);
  for (int i = e + 1; i < e1; ++i) {
    const int2 q = pe[i];
    const float t = __int_as_float(q.y) * vget<NB>(lo, hi, q.x);
    switch (agg) {
      case TN_AGG_PRODUCT: s = s * t; break;
      case TN_AGG_MAX: s = fmaxf(s, t); break;
      case TN_AGG_MIN: s = fminf(s, t); break;
      case TN_AGG_MEAN: s = s + t; break;
      default: s = fabsf(t) > fabsf(s) ? t : s; break;  // maxabs
    }
  }
  if (agg == TN_AGG_MEAN) s = s / (float)cnt;
  return s;
}

// The program of one genome, in topological order, on this lane's registers;
// input rows must already hold the inputs. Software-pipelined over positions:
// position p's in-edges are consumed first, then the header and first edge
// group of position p+1 are requested, and p's activation runs while those
// scalar loads are in flight.
template <int NB>
__device__ __forceinline__ void walk_program(f32x32& lo, f32x32& hi, const int4* __restrict__ pn,
                                             const int2* __restrict__ pe, int n) {
  int e = 0;
  int4 h = pn[0];
  int2 g[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) g[u] = pe[u];
  for (int p = 0; p < n; ++p) {
    const int f = h.y, e1 = h.x;
    float s = 0.0f;
    if (f >= 0) s = aggregate<NB>(lo, hi, pe, g, e, e1, (f >> 8) & 0xff);
    const int4 nh = pn[p + 1 < n ? p + 1 : p];
    int2 ng[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ng[u] = pe[e1 + u];
    if (f >= 0) {  // an input's row already holds its value
      const float z[1] = {fmaf(__int_as_float(h.w), s, __int_as_float(h.z))};
      float a[1];
      activate_all<1>(f & 0xff, z, a);
      vset<NB>(lo, hi, (f >> 16) & 0x7fff, a[0]);
    }
    e = e1;
    h = nh;
#pragma unroll
    for (int u = 0; u < 8; ++u) g[u] = ng[u];
  }
}

// The register-file form of the walk, over the 16-word records of the
// non-input positions (tn_transformed.prog_rec): one s_load_dwordx16 per
// node brings its header and first 6 in-edges; unused slots read the zero
// row with weight +0 (exact: the running sum starts at +0 and can never be
// -0, so adding +0 * 0 leaves it unchanged), so the sum needs no branch for
// up to 6 in-edges. The next record is requested after this node's in-edges
// and before its activation. The zero row must hold +0.
template <int R>
__device__ __forceinline__ void walk_records(const int32_t* __restrict__ rec,
                                             const int2* __restrict__ pe, int nn) {
  int w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = rec[i];
  for (int q = 0; q < nn; ++q) {
    const int d0 = w[0];
    const int agg = (d0 >> 3) & 7, ne = (d0 >> 17) & 0x7fff;
    float s = 0.0f;
    if (agg == TN_AGG_SUM) {
#pragma unroll
      for (int i = 0; i < 6; ++i) rf_fma(s, __int_as_float(w[5 + 2 * i]), w[4 + 2 * i]);
      for (int e = w[3]; e < w[3] + ne - 6; ++e) {
        const int2 qe = pe[e];
        rf_fma(s, __int_as_float(qe.y), qe.x);
      }
    } else if (ne > 0) {
      // other aggregations: terms in order, no padding
      s = __int_as_float(w[5]) * rf_get(w[4]);
      for (int i = 1; i < ne; ++i) {
        int r, wb;
        if (i < 6) {
          r = i == 1 ? w[6] : i == 2 ? w[8] : i == 3 ? w[10] : i == 4 ? w[12] : w[14];
          wb = i == 1 ? w[7] : i == 2 ? w[9] : i == 3 ? w[11] : i == 4 ? w[13] : w[15];
        } else {
          const int2 qe = pe[w[3] + i - 6];
          r = qe.x;
          wb = qe.y;
        }
        const float t = __int_as_float(wb) * rf_get(r);
        switch (agg) {
          case TN_AGG_PRODUCT: s = s * t; break;
          case TN_AGG_MAX: s = fmaxf(s, t); break;
          case TN_AGG_MIN: s = fminf(s, t); break;
          case TN_AGG_MEAN: s = s + t; break;
          default: s = fabsf(t) > fabsf(s) ? t : s; break;  // maxabs
        }
      }
      if (agg == TN_AGG_MEAN) s = s / (float)ne;
    }
    const float bias = __int_as_float(w[1]), resp = __int_as_float(w[2]);
    const int row = (d0 >> 6) & 0x7ff, act = d0 & 7;
    const int* nx = rec + 16 * (q + 1 < nn ? q + 1 : q);
    int nw[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) nw[i] = nx[i];
    const float z[1] = {fmaf(resp, s, bias)};
    float a[1];
    activate_all<1>(act, z, a);
    rf_set(row, a[0]);
    // the next record is needed from here on (and not before: the empty asm
    // keeps the compiler from waiting for it ahead of the activation)
    asm volatile(""
                 : "+s"(nw[0]), "+s"(nw[1]), "+s"(nw[2]), "+s"(nw[3]), "+s"(nw[4]), "+s"(nw[5]),
                   "+s"(nw[6]), "+s"(nw[7]), "+s"(nw[8]), "+s"(nw[9]), "+s"(nw[10]),
                   "+s"(nw[11]), "+s"(nw[12]), "+s"(nw[13]), "+s"(nw[14]), "+s"(nw[15]));
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = nw[i];
  }
}

}  // namespace tn
