// Register-resident evaluation of a genome's packed program (the calculation
// stage of TensorNEAT Section 3.3): one lane = one evaluation, node values in
// an explicit register file addressed with a uniform index (s_set_gpr_idx),
// the program read across lanes. Shared by the forward engine and the CPPN
// query of the substrate. The file of R rows per tile sits at v[kRfBase ..]:
// the kernel limits the compiler to the VGPRs below kRfBase and reserves the
// file with a clobber, and every access is one s_set_gpr_idx window around
// one instruction per tile (an in-edge is a single v_fmac_f32 with an indexed
// operand).
#pragma once

#include "fwd_core.hpp"

namespace tn {

// First VGPR of the explicit register file; kernels using it carry
// __attribute__((amdgpu_num_vgpr(kRfBase))).
#define TN_RF_BASE 56
#define TN_RF_V0 "v56"
constexpr int kRfBase = TN_RF_BASE;

// s_set_gpr_idx_on writes M0; none of these kernels keeps anything in M0.
// Every window waits two cycles after s_set_gpr_idx_on before its first
// indexed instruction: measured on MI355X, an index written to its SGPR just
// before the window (a v_readlane of a record word, or a scalar op) is
// otherwise not reliably applied to that first instruction (the wrong row is
// read), and the wait also covers the two wait states a VALU read of an SGPR
// written by a VALU (the weights) needs, which the compiler does not insert
// for inline assembly.
__device__ __forceinline__ float rf_get(int r) {
  float x;
  asm volatile("s_set_gpr_idx_on %1, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, " TN_RF_V0
               "\n\ts_set_gpr_idx_off"
               : "=v"(x)
               : "s"(r) : "m0");
  return x;
}
__device__ __forceinline__ void rf_set(int r, float x) {
  asm volatile("s_set_gpr_idx_on %1, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 " TN_RF_V0
               ", %0\n\ts_set_gpr_idx_off" ::"v"(x),
               "s"(r) : "m0");
}
// acc += w * row[r] in one instruction.
__device__ __forceinline__ void rf_fma(float& acc, float w, int r) {
  asm volatile("s_set_gpr_idx_on %2, gpr_idx(SRC1)\n\ts_nop 1\n\tv_fmac_f32 %0, %1, " TN_RF_V0
               "\n\ts_set_gpr_idx_off"
               : "+v"(acc)
               : "s"(w), "s"(r) : "m0");
}

// Observation tiles held per wavefront by a register file of R rows per tile:
// 50 rows hold four tiles (files at v56, v106, v156, v206), 100 rows two (v56,
// v156), every other size one. A window of s_set_gpr_idx costs about as much as
// the 2-4 multiply-adds it covers, so sharing one window (and one record load,
// decode and branch) between the tiles of a wavefront divides the per-edge
// and per-node cost by the tile count.
__host__ __device__ constexpr int rf_tiles(int R) { return rf_tiles_of(R); }

// Makes the compiler count the register file in the kernel's VGPR allocation
// (a clobber of its last register); R = rows per tile.
template <int R>
__device__ __forceinline__ void rf_reserve() {
  constexpr int total = R * rf_tiles(R);
  static_assert(total == 32 || total == 64 || total == 96 || total == 128 || total == 160 ||
                    total == 200,
                "register file sizes");
  if constexpr (total == 32) asm volatile("" ::: "v87");
  if constexpr (total == 64) asm volatile("" ::: "v119");
  if constexpr (total == 96) asm volatile("" ::: "v151");
  if constexpr (total == 128) asm volatile("" ::: "v183");
  if constexpr (total == 160) asm volatile("" ::: "v215");
  if constexpr (total == 200) asm volatile("" ::: "v255");
}

// acc[k] += w * (row r of tile k) for the rf_tiles(R) tiles, under one window.
template <int R>
__device__ __forceinline__ void rfk_fma(float (&acc)[rf_tiles(R)], float w, int r) {
  if constexpr (rf_tiles(R) == 1) {
    rf_fma(acc[0], w, r);
  } else if constexpr (rf_tiles(R) == 2) {
    asm volatile(
        "s_set_gpr_idx_on %3, gpr_idx(SRC1)\n\ts_nop 1\n\tv_fmac_f32 %0, %2, v56\n\t"
        "v_fmac_f32 %1, %2, v156\n\ts_set_gpr_idx_off"
        : "+v"(acc[0]), "+v"(acc[1])
        : "s"(w), "s"(r) : "m0");
  } else {
    asm volatile(
        "s_set_gpr_idx_on %5, gpr_idx(SRC1)\n\ts_nop 1\n\tv_fmac_f32 %0, %4, v56\n\t"
        "v_fmac_f32 %1, %4, v106\n\tv_fmac_f32 %2, %4, v156\n\t"
        "v_fmac_f32 %3, %4, v206\n\ts_set_gpr_idx_off"
        : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])
        : "s"(w), "s"(r) : "m0");
  }
}

// row r of tile k := x[k] for the rf_tiles(R) tiles, under one window.
template <int R>
__device__ __forceinline__ void rfk_set(int r, const float (&x)[rf_tiles(R)]) {
  if constexpr (rf_tiles(R) == 1) {
    rf_set(r, x[0]);
  } else if constexpr (rf_tiles(R) == 2) {
    asm volatile(
        "s_set_gpr_idx_on %2, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v56, %0\n\t"
        "v_mov_b32 v156, %1\n\ts_set_gpr_idx_off" ::"v"(x[0]),
        "v"(x[1]), "s"(r) : "m0");
  } else {
    asm volatile(
        "s_set_gpr_idx_on %4, gpr_idx(DST)\n\ts_nop 1\n\tv_mov_b32 v56, %0\n\t"
        "v_mov_b32 v106, %1\n\tv_mov_b32 v156, %2\n\tv_mov_b32 v206, %3\n\t"
        "s_set_gpr_idx_off" ::"v"(x[0]),
        "v"(x[1]), "v"(x[2]), "v"(x[3]), "s"(r) : "m0");
  }
}

// x[k] := row r of tile k for the rf_tiles(R) tiles, under one window.
template <int R>
__device__ __forceinline__ void rfk_get(int r, float (&x)[rf_tiles(R)]) {
  if constexpr (rf_tiles(R) == 1) {
    x[0] = rf_get(r);
  } else if constexpr (rf_tiles(R) == 2) {
    asm volatile(
        "s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v56\n\t"
        "v_mov_b32 %1, v156\n\ts_set_gpr_idx_off"
        : "=v"(x[0]), "=v"(x[1])
        : "s"(r) : "m0");
  } else {
    asm volatile(
        "s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\ts_nop 1\n\tv_mov_b32 %0, v56\n\t"
        "v_mov_b32 %1, v106\n\tv_mov_b32 %2, v156\n\tv_mov_b32 %3, v206\n\t"
        "s_set_gpr_idx_off"
        : "=v"(x[0]), "=v"(x[1]), "=v"(x[2]), "=v"(x[3])
        : "s"(r) : "m0");
  }
}

// Program row of (non-input) position p: bits 16..30 of its function word.
__device__ __forceinline__ int prog_row(const int4* __restrict__ pn, int p) {
  return (pn[p].y >> 16) & 0x7fff;
}

// One non-input position of the register-file walk, on every tile of the
// wavefront. w(i) gives word i of the node's record: {act | agg << 3 | row << 6
// | in-degree << 17, bias, response, index of the 7th in-edge, then (source
// row, weight) of the first 6 in-edges}; i is a constant at every call. Only
// the node's real in-edges are read: one window per in-edge (the tiles share
// it), a compare and a branch per slot.
template <int R, class Rec>
__device__ __forceinline__ void rf_node(const Rec& w, const int2* __restrict__ pe) {
  constexpr int K = rf_tiles(R);
  const int d0 = w(0);
  const int agg = (d0 >> 3) & 7, ne = (d0 >> 17) & 0x7fff;
  float s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.0f;
  if (ne <= 0) {
    // no in-edges: the aggregate is 0 whatever the aggregation
  } else if (agg == TN_AGG_SUM) {
    {
      rfk_fma<R>(s, __int_as_float(w(5)), w(4));
      if (ne > 1) {
        rfk_fma<R>(s, __int_as_float(w(7)), w(6));
        if (ne > 2) {
          rfk_fma<R>(s, __int_as_float(w(9)), w(8));
          if (ne > 3) {
            rfk_fma<R>(s, __int_as_float(w(11)), w(10));
            if (ne > 4) {
              rfk_fma<R>(s, __int_as_float(w(13)), w(12));
              if (ne > 5) {
                rfk_fma<R>(s, __int_as_float(w(15)), w(14));
                // further in-edges 8 at a time (prog_edge is padded for the
                // over-read past the genome's last edge)
                const int e0 = w(3), e1 = e0 + ne - 6;
                for (int b = e0; b < e1; b += 8) {
                  int2 q[8];
#pragma unroll
                  for (int u = 0; u < 8; ++u) q[u] = pe[b + u];
#pragma unroll
                  for (int u = 0; u < 8; ++u)
                    if (b + u < e1) rfk_fma<R>(s, __int_as_float(q[u].y), q[u].x);
                }
              }
            }
          }
        }
      }
    }
  } else {
    // other aggregations: terms in order
    const int r0 = w(4), w0 = w(5);
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = __int_as_float(w0) * rf_get(k * R + r0);
    const int rs[5] = {w(6), w(8), w(10), w(12), w(14)};
    const int ws[5] = {w(7), w(9), w(11), w(13), w(15)};
    const int e6 = w(3);
    for (int i = 1; i < ne; ++i) {
      int r, wb;
      if (i < 6) {
        r = i == 1 ? rs[0] : i == 2 ? rs[1] : i == 3 ? rs[2] : i == 4 ? rs[3] : rs[4];
        wb = i == 1 ? ws[0] : i == 2 ? ws[1] : i == 3 ? ws[2] : i == 4 ? ws[3] : ws[4];
      } else {
        const int2 qe = pe[e6 + i - 6];
        r = qe.x;
        wb = qe.y;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t = __int_as_float(wb) * rf_get(k * R + r);
        switch (agg) {
          case TN_AGG_PRODUCT: s[k] = s[k] * t; break;
          case TN_AGG_MAX: s[k] = fmaxf(s[k], t); break;
          case TN_AGG_MIN: s[k] = fminf(s[k], t); break;
          case TN_AGG_MEAN: s[k] = s[k] + t; break;
          default: s[k] = fabsf(t) > fabsf(s[k]) ? t : s[k]; break;  // maxabs
        }
      }
    }
    if (agg == TN_AGG_MEAN)
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] = s[k] / (float)ne;
  }
  const float bias = __int_as_float(w(1)), resp = __int_as_float(w(2));
  float z[K], a[K];
#pragma unroll
  for (int k = 0; k < K; ++k) z[k] = fmaf(resp, s[k], bias);
  activate_all<K>(d0 & 7, z, a);
  rfk_set<R>((d0 >> 6) & 0x7ff, a);
}

// Record J of a block of four held across the wavefront (lane l holds word l
// of the block): word i is read with v_readlane at the constant lane 16 J + i.
template <int J>
struct LaneRec {
  int blk;
  __device__ __forceinline__ int operator()(int i) const {
    return __builtin_amdgcn_readlane(blk, 16 * J + i);
  }
};

// The register-file walk over the 16-word records of the non-input positions
// (tn_transformed.prog_rec), in topological order, for every tile of the
// wavefront. The records come four at a time with one coalesced vector load
// (64 lanes x one word), each block requested two blocks ahead; the compiler
// waits for it where the loop moves it to the next block's register, so a
// load overlaps one block (four nodes) of work (blocks of eight records, whose
// loads overlap eight nodes, measured no faster: the walk does not wait on
// these loads). The words reach the scalar unit through v_readlane with
// constant lane indexes. Lanes past the genome's last
// record read its last word instead (no load past the genome's records).
template <int R>
__device__ __forceinline__ void walk_records(const int32_t* __restrict__ rec,
                                             const int2* __restrict__ pe, int nn, int lane) {
  if (nn <= 0) return;
  const int lim = nn * 16 - 1;
  int cur = rec[min(lane, lim)];
  int nx1 = rec[min(kWave + lane, lim)];
  for (int q = 0; q < nn; q += 4) {
    const int nx2 = rec[min(q * 16 + 2 * kWave + lane, lim)];
    rf_node<R>(LaneRec<0>{cur}, pe);
    if (q + 1 < nn) {
      rf_node<R>(LaneRec<1>{cur}, pe);
      if (q + 2 < nn) {
        rf_node<R>(LaneRec<2>{cur}, pe);
        if (q + 3 < nn) rf_node<R>(LaneRec<3>{cur}, pe);
      }
    }
    cur = nx1;
    nx1 = nx2;
  }
}

}  // namespace tn
