// The paper's own float encoding of a population (Section 3.1: P_N and P_C,
// padding rows of NaN) converted into the library's structure-of-arrays
// layout, with every row checked.
//
// One thread per row: node rows [k, bias, response, act, agg] and connection
// rows [k_in, k_out, e, w] (the enabled flag before the attributes, as the
// paper orders a connection tensor). Rows are independent, so the grid covers
// the node rows and then the connection rows of the whole population; a bad
// row sets its genome's error bits with an atomic OR and is written as an
// empty row.
#include <algorithm>

#include "tn_internal.hpp"

namespace tn {

namespace {

constexpr float kKeyLimit = 16777216.0f;  // 2^24: every integer below is exact in float32

// An exact non-negative integer below 2^24 (NaN and infinities fail both tests).
__device__ __forceinline__ bool is_key(float k) {
  return k >= 0.0f && k < kKeyLimit && truncf(k) == k;
}

__device__ __forceinline__ bool is_code(float c) {
  return c >= 0.0f && c <= 255.0f && truncf(c) == c;
}

__global__ void zero_err_kernel(int32_t* err, int P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) err[i] = 0;
}

__global__ void pack_kernel(const float* __restrict__ PN, const float* __restrict__ PC, int P,
                            int N_max, int C_max, tn_population_arrays out,
                            int32_t* __restrict__ err) {
  const int64_t n_nodes = (int64_t)P * N_max;
  const int64_t n_conns = (int64_t)P * C_max;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_nodes + n_conns;
       i += stride) {
    if (i < n_nodes) {
      const float* r = PN + 5 * i;
      const float k = r[0], b = r[1], rho = r[2], act = r[3], agg = r[4];
      int bits = 0;
      if (!__builtin_isnan(k)) {
        if (!is_key(k)) bits |= TN_PACK_NODE_KEY;
        if (!is_code(act) || !is_code(agg)) bits |= TN_PACK_NODE_CODE;
      }
      const bool keep = !__builtin_isnan(k) && bits == 0;
      out.node_key[i] = keep ? (int32_t)k : -1;
      out.node_bias[i] = keep ? b : 0.0f;
      out.node_resp[i] = keep ? rho : 0.0f;
      out.node_act[i] = keep ? (uint8_t)act : 0;
      out.node_agg[i] = keep ? (uint8_t)agg : 0;
      if (bits) atomicOr(err + i / N_max, bits);
    } else {
      const int64_t j = i - n_nodes;
      const float4 r = *reinterpret_cast<const float4*>(PC + 4 * j);
      int bits = 0;
      if (!__builtin_isnan(r.x)) {
        if (!is_key(r.x) || !is_key(r.y)) bits |= TN_PACK_CONN_KEY;
        if (!(r.z == 0.0f || r.z == 1.0f)) bits |= TN_PACK_CONN_FLAG;
      }
      const bool keep = !__builtin_isnan(r.x) && bits == 0;
      out.conn_in[j] = keep ? (int32_t)r.x : -1;
      out.conn_out[j] = keep ? (int32_t)r.y : -1;
      out.conn_en[j] = keep ? (uint8_t)r.z : 0;
      out.conn_w[j] = keep ? r.w : 0.0f;
      if (bits) atomicOr(err + j / C_max, bits);
    }
  }
}

}  // namespace

int launch_pack(const float* PN, const float* PC, int P, int N_max, int C_max,
                const tn_population_arrays& out, int32_t* err, hipStream_t stream) {
  hipLaunchKernelGGL(zero_err_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, err, P);
  int rc = check_launch();
  if (rc != TN_OK) return rc;
  const int64_t rows = (int64_t)P * (N_max + C_max);
  const int64_t blocks = std::min<int64_t>((rows + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, PN, PC, P, N_max,
                     C_max, out, err);
  return check_launch();
}

}  // namespace tn
