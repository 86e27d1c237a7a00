// Internal declarations shared by the HIP translation units of libtnhip.
// Not part of the public ABI (that is include/tensorneat_hip.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tensorneat_hip.h"

namespace tn {

// Tiles of 64 observations per wavefront of the register engine's register
// file of R rows per tile (50 rows: four, 100: two, other sizes: one).
__host__ __device__ constexpr int rf_tiles_of(int R) { return R == 50 ? 4 : R == 100 ? 2 : 1; }

constexpr int kWave = 64;

// Population descriptor passed to kernels by value.
struct PopView {
  int P, n_in, n_out, N_max, C_max;
  const int64_t* node_off;
  const int64_t* conn_off;
  const int32_t* node_key;
  const float* node_bias;
  const float* node_resp;
  const uint8_t* node_act;
  const uint8_t* node_agg;
  const int32_t* conn_in;
  const int32_t* conn_out;
  const float* conn_w;
  const uint8_t* conn_en;

  __device__ __forceinline__ int64_t node_base(int g) const {
    return node_off ? node_off[g] : (int64_t)g * N_max;
  }
  __device__ __forceinline__ int64_t conn_base(int g) const {
    return conn_off ? conn_off[g] : (int64_t)g * C_max;
  }
  // Row counts; a ragged count above the capacity is returned as is (the
  // caller flags it as oversize).
  __device__ __forceinline__ int64_t node_rows(int g) const {
    return node_off ? node_off[g + 1] - node_off[g] : (int64_t)N_max;
  }
  __device__ __forceinline__ int64_t conn_rows(int g) const {
    return conn_off ? conn_off[g + 1] - conn_off[g] : (int64_t)C_max;
  }
  __device__ __forceinline__ int64_t rowptr_base(int g) const {
    return node_off ? node_off[g] + g : (int64_t)g * (N_max + 1);
  }
};

struct TrView {
  int32_t* status;
  int32_t* n_valid;
  int32_t* order;
  int32_t* level;
  int32_t* row_ptr;
  int32_t* edge_src;
  int32_t* edge_row;
  float* edge_w;
  float* pos_bias;
  float* pos_resp;
  int32_t* pos_fn;
  int32_t* io_pos;
  int32_t* pos_row;
  int32_t* n_rows;
  int4* prog_node;
  int2* prog_edge;
  int32_t* prog_rows;
  int32_t* prog_rec;
};

inline PopView make_view(const tn_population& p) {
  PopView v;
  v.P = p.P; v.n_in = p.n_in; v.n_out = p.n_out; v.N_max = p.N_max; v.C_max = p.C_max;
  v.node_off = p.node_off; v.conn_off = p.conn_off;
  v.node_key = p.node_key; v.node_bias = p.node_bias; v.node_resp = p.node_resp;
  v.node_act = p.node_act; v.node_agg = p.node_agg;
  v.conn_in = p.conn_in; v.conn_out = p.conn_out; v.conn_w = p.conn_w; v.conn_en = p.conn_en;
  return v;
}

inline TrView make_view(const tn_transformed& t) {
  TrView v;
  v.status = t.status; v.n_valid = t.n_valid; v.order = t.order; v.level = t.level;
  v.row_ptr = t.row_ptr; v.edge_src = t.edge_src; v.edge_row = t.edge_row;
  v.edge_w = t.edge_w; v.pos_bias = t.pos_bias; v.pos_resp = t.pos_resp;
  v.pos_fn = t.pos_fn; v.io_pos = t.io_pos; v.pos_row = t.pos_row; v.n_rows = t.n_rows;
  v.prog_node = reinterpret_cast<int4*>(t.prog_node);
  v.prog_edge = reinterpret_cast<int2*>(t.prog_edge);
  v.prog_rows = t.prog_rows;
  v.prog_rec = t.prog_rec;
  return v;
}

// pos_fn encoding: act | agg << 8; inputs have bit 31 set and their input
// index in bits 16..30.
constexpr uint32_t kFnInput = 0x80000000u;

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// A 64-bit value that is the same on every lane, as a wavefront-uniform value
// (offsets computed with 64-bit vector multiplies stay in vector registers;
// made uniform, the addresses built from them stay on the scalar unit).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Index of this wavefront in its workgroup, as a wavefront-uniform value (the
// compiler cannot see that threadIdx.x / 64 is uniform; anything derived from
// it would otherwise leave the scalar unit: vector loads of the program,
// indexed register reads through a per-lane loop).
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ int mbcnt(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders this wavefront's LDS accesses before / after the call (the wavefront
// only shares the LDS rows it owns; no other wavefront is waited for).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_inclusive_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(x, off, kWave);
    if (lane >= off) x += t;
  }
  return x;
}

__device__ __forceinline__ int wave_inclusive_max(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int t = __shfl_up(x, off, kWave);
    if (lane >= off) x = max(x, t);
  }
  return x;
}

// Butterfly sum over the wave; every lane gets the same value, summed in a
// fixed order (deterministic).
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

__device__ __forceinline__ int wave_sum_int(int x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  return x;
}

// --------------------------------------------------------- node functions

__device__ __forceinline__ float activate(int act, float z) {
  switch (act) {
    case TN_ACT_IDENTITY: return z;
    case TN_ACT_SIGMOID: return 1.0f / (1.0f + expf(-z));
    case TN_ACT_TANH: return tanhf(z);
    case TN_ACT_RELU: return fmaxf(z, 0.0f);
    case TN_ACT_SIN: return sinf(z);
    case TN_ACT_GAUSSIAN: return expf(-z * z);
    case TN_ACT_ABS: return fabsf(z);
    default: return __builtin_nanf("");
  }
}

// ----------------------------------------------------------- host helpers

// Largest dynamic LDS allocation of one workgroup on the current device.
size_t max_dynamic_lds();

// Remembers a HIP error for tn_last_error(); returns TN_OK for hipSuccess,
// TN_EHIP otherwise.
int record_hip(hipError_t e);

// Error of the launch just issued (hipGetLastError), recorded.
inline int check_launch() { return record_hip(hipGetLastError()); }

// Argument checks shared by the entry points (TN_OK or the error code).
int check_population(const tn_population* p);
int check_transformed(const tn_transformed* t);
int check_obs(const tn_population* p, const float* obs, int64_t stride, int32_t B);

// Lets `kernel` take `bytes` of dynamic LDS. Only requests above 64 KiB need
// the function attribute; returns TN_EUNSUPPORTED beyond the device limit.
int allow_lds(const void* kernel, size_t bytes);

}  // namespace tn
