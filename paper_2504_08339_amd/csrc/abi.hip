// The extern "C" entry points of libtnhip: host-side argument validation and
// dispatch to the launchers of each translation unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fwd_launch.hpp"
#include "tn_internal.hpp"

namespace tn {

size_t transform_lds_bytes(int N_max, int C_max);
int launch_transform(const tn_population& p, const tn_transformed& t, hipStream_t stream);
size_t forward_lds_bytes(int N_max, int C_max, int nio, int K);
int launch_backward(const tn_population& p, const tn_transformed& t, const float* obs,
                    int64_t obs_stride, int B, const float* dY, int64_t dY_stride,
                    const float* target, int64_t target_stride, float scale, float* loss,
                    float* dW, float* db, hipStream_t stream);
int check_substrate(const tn_substrate* sub);
int launch_cppn_query(const tn_population& p, const tn_transformed& t, const tn_substrate& sub,
                      uint16_t* w1t, uint16_t* w2t, float* raw1, float* raw2,
                      hipStream_t stream);
int launch_substrate_forward(const tn_substrate& sub, int P, const uint16_t* w1t,
                             const uint16_t* w2t, const uint16_t* x, int64_t x_stride, int B,
                             float* h, float* y, hipStream_t stream);
size_t substrate_workspace_bytes(const tn_substrate& sub, int P, int B, int64_t x_stride);
int launch_substrate_backward(const tn_substrate& sub, int P, const uint16_t* w2t,
                              const uint16_t* x, int64_t x_stride, int B, const float* h,
                              const float* dy, void* workspace, float* dw1t, float* dw2t,
                              hipStream_t stream);
size_t cppn_backward_workspace_bytes(const tn_population& p, const tn_substrate& sub);
int launch_cppn_backward(const tn_population& p, const tn_transformed& t, const tn_substrate& sub,
                         const float* dw1t, const float* dw2t, void* workspace, float* dW,
                         float* db, hipStream_t stream);
int launch_pack(const float* PN, const float* PC, int P, int N_max, int C_max,
                const tn_population_arrays& out, int32_t* err, hipStream_t stream);
size_t distance_workspace_bytes(int P, int C_max);
int launch_distance(const tn_population& p, float c1, float c2, float c3, void* workspace,
                    float* dist, int32_t* E, int32_t* D, hipStream_t stream);
int noalloc_scratch(void** out);
size_t neat_workspace_bytes(int P, int S, int N, int C);
int launch_neat_init(int P, int n_in, int n_out, int N, int C, const float* Z,
                     const tn_mutation_params& m, const tn_population_arrays& out,
                     const tn_species_table* table, hipStream_t stream);
int launch_neat_generation(const tn_population& p, const float* fit, int gen,
                           const tn_neat_params& prm, const tn_species_table& table,
                           const float* sel, const float* U, const float* Z, int32_t next_key,
                           const tn_population_arrays& children, int32_t* species_of,
                           int32_t* parents, int32_t* next_key_out, void* workspace,
                           hipStream_t stream);
int recurrent_lds_check(const tn_population& p, size_t* bytes);
int launch_forward_recurrent(const tn_population& p, const float* obs, int64_t obs_stride, int B,
                             int T, float* out, int32_t* status, hipStream_t stream);
size_t reproduce_workspace_bytes(int n);
int launch_reproduce(const tn_population& p, int n, const int32_t* parents, const float* U,
                     const float* Z, const tn_mutation_params& prm, int32_t next_key,
                     const tn_population_arrays& out, int32_t* next_key_out, void* workspace,
                     hipStream_t stream);
size_t distance_nodes_workspace_bytes(int P, int N_max, int C_max);
int launch_distance_nodes(const tn_population& p, float c_d, float c_h, void* workspace,
                          float* dist, int32_t* DN, int32_t* DC, hipStream_t stream);

size_t max_dynamic_lds() {
  static size_t cached = 0;
  if (cached) return cached;
  int dev = 0;
  int bytes = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      bytes > 0)
    cached = (size_t)bytes;
  else
    cached = 64 * 1024;
  return cached;
}

namespace {
thread_local hipError_t g_last_error = hipSuccess;
}  // namespace

int record_hip(hipError_t e) {
  if (e == hipSuccess) return TN_OK;
  g_last_error = e;
  return TN_EHIP;
}

int allow_lds(const void* kernel, size_t bytes) {
  if (bytes > max_dynamic_lds()) return TN_EUNSUPPORTED;
  if (bytes <= 64 * 1024) return TN_OK;
  return record_hip(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)bytes));
}

int check_population(const tn_population* p) {
  if (!p) return TN_EINVAL;
  if (p->P < 0 || p->n_in < 0 || p->n_out < 1 || p->N_max < 1 || p->C_max < 1) return TN_EINVAL;
  if (p->N_max > TN_MAX_NODES || p->C_max > TN_MAX_CONNS || p->n_in + p->n_out > TN_MAX_IO)
    return TN_EUNSUPPORTED;
  if ((p->node_off == nullptr) != (p->conn_off == nullptr)) return TN_EINVAL;
  if (p->P == 0) return TN_OK;
  if (!p->node_key || !p->node_bias || !p->node_resp || !p->node_act || !p->node_agg ||
      !p->conn_in || !p->conn_out || !p->conn_w || !p->conn_en)
    return TN_EINVAL;
  if (p->node_off && (p->total_nodes < 0 || p->total_conns < 0)) return TN_EINVAL;
  return TN_OK;
}

namespace {
int64_t node_elems(const tn_population* p) {
  return p->node_off ? p->total_nodes : (int64_t)p->P * p->N_max;
}
int64_t conn_elems(const tn_population* p) {
  return p->node_off ? p->total_conns : (int64_t)p->P * p->C_max;
}
}  // namespace

int check_transformed(const tn_transformed* t) {
  if (!t) return TN_EINVAL;
  if (!t->status || !t->n_valid || !t->order || !t->level || !t->row_ptr || !t->edge_src ||
      !t->edge_row || !t->edge_w || !t->pos_bias || !t->pos_resp || !t->pos_fn || !t->io_pos ||
      !t->pos_row || !t->n_rows || !t->prog_node || !t->prog_edge || !t->prog_rows || !t->prog_rec)
    return TN_EINVAL;
  return TN_OK;
}

int check_obs(const tn_population* p, const float* obs, int64_t stride, int32_t B) {
  if (B < 0 || stride < 0) return TN_EINVAL;
  if (B > 0 && p->n_in > 0 && !obs) return TN_EINVAL;
  if (stride > 0 && stride < (int64_t)B * p->n_in) return TN_ESHAPE;
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

const char* tn_status_string(int status) {
  switch (status) {
    case TN_OK: return "TN_OK";
    case TN_EINVAL: return "TN_EINVAL: invalid argument";
    case TN_ESHAPE: return "TN_ESHAPE: inconsistent sizes";
    case TN_EUNSUPPORTED: return "TN_EUNSUPPORTED: above a compiled or device limit";
    case TN_EHIP: return "TN_EHIP: HIP launch or runtime error";
    case TN_ENOMEM: return "TN_ENOMEM: allocation failed";
    default: return "unknown tn_status";
  }
}

int tn_version(void) { return 100; }

const char* tn_last_error(void) {
  return g_last_error == hipSuccess ? "" : hipGetErrorString(g_last_error);
}

int tn_validate_population(const tn_population* pop) { return check_population(pop); }

int tn_transformed_size(const tn_population* pop, tn_transformed_elems* out) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (!out) return TN_EINVAL;
  out->node_elems = node_elems(pop);
  out->rowptr_elems = node_elems(pop) + pop->P;
  out->conn_elems = conn_elems(pop);
  out->genome_elems = pop->P;
  out->io_elems = (int64_t)pop->P * (pop->n_in + pop->n_out);
  return TN_OK;
}

int tn_pack_paper_layout(const float* PN, const float* PC, int32_t P, int32_t N_max,
                         int32_t C_max, const tn_population_arrays* out, int32_t* pack_err,
                         hipStream_t stream) {
  if (P < 0 || N_max < 1 || C_max < 1 || !out) return TN_EINVAL;
  if (N_max > TN_MAX_NODES || C_max > TN_MAX_CONNS) return TN_EUNSUPPORTED;
  if (P == 0) return TN_OK;
  if (!PN || !PC || !pack_err || !out->node_key || !out->node_bias || !out->node_resp ||
      !out->node_act || !out->node_agg || !out->conn_in || !out->conn_out || !out->conn_w ||
      !out->conn_en)
    return TN_EINVAL;
  if (reinterpret_cast<uintptr_t>(PC) % 16 != 0) return TN_EINVAL;
  int rc = launch_pack(PN, PC, P, N_max, C_max, *out, pack_err, stream);
  if (rc != TN_OK) return rc;
  std::vector<int32_t> err((size_t)P);
  rc = record_hip(hipMemcpyAsync(err.data(), pack_err, sizeof(int32_t) * (size_t)P,
                                 hipMemcpyDeviceToHost, stream));
  if (rc == TN_OK) rc = record_hip(hipStreamSynchronize(stream));
  if (rc != TN_OK) return rc;
  for (int32_t e : err)
    if (e) return TN_EINVAL;
  return TN_OK;
}

int tn_transform(const tn_population* pop, const tn_transformed* tr, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->P == 0) return TN_OK;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  return launch_transform(*pop, *tr, stream);
}

}  // extern "C"

namespace {

// TN_ENGINE_AUTO: the register engine for every genome whose packed program
// fits in a 200-row register file, one launch per register-file size of
// tn::reg_classes (smallest first, each skipping what an earlier one took),
// and the level-parallel LDS engine for the rest (prog_rows <= N_max, so small
// populations need fewer launches).
int forward_auto(const tn_population& p, const tn_transformed& t, const float* obs,
                 int64_t stride, int B, float* out, hipStream_t stream) {
  int cls[6];
  const int n = tn::reg_classes(B, cls);
  int lo = -1;
  for (int i = 0; i < n; ++i) {
    tn::RegTile rt;
    rt.rf = cls[i];
    rt.rows_lo = lo;
    rt.skip_above = p.N_max > cls[i];
    const int rc = tn::launch_forward_reg(p, t, obs, stride, B, out, rt, tn::FwdWork(), stream);
    if (rc != TN_OK || p.N_max <= cls[i]) return rc;
    lo = cls[i];
  }
  tn::LdsTile lt;
  lt.rows = std::min(p.N_max, tn::lds_rows_cap(p));
  lt.skip_le = tn::kRegRowsMax;
  return tn::launch_forward(p, t, obs, stride, B, out, lt, tn::FwdWork(), stream);
}

}  // namespace

extern "C" {

int tn_forward(const tn_population* pop, const tn_transformed* tr, const float* obs,
               int64_t obs_genome_stride, int32_t B, float* out, hipStream_t stream) {
  return tn_forward_tiled(pop, tr, obs, obs_genome_stride, B, out, nullptr, stream);
}

int tn_forward_tiled(const tn_population* pop, const tn_transformed* tr, const float* obs,
                     int64_t obs_genome_stride, int32_t B, float* out, const tn_tile* tile,
                     hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  const int engine = tile ? tile->engine : TN_ENGINE_AUTO;
  if (tile) {
    const int K = tile->obs_per_lane, W = tile->waves_per_genome, R = tile->rows;
    if (W < 0 || W > (engine == TN_ENGINE_LDS ? tn::lds_max_waves(K) : 8) || R < 0)
      return TN_EINVAL;
    if (engine == TN_ENGINE_LDS && K != 0 && K != 1 && K != 2 && K != 4) return TN_EINVAL;
    if (engine == TN_ENGINE_REG &&
        ((K != 0 && K != 1) ||
         (R != 0 && R != 32 && R != 50 && R != 64 && R != 96 && R != 100 && R != 128 &&
          R != 160 && R != 200)))
      return TN_EINVAL;
    if (engine != TN_ENGINE_AUTO && engine != TN_ENGINE_LDS && engine != TN_ENGINE_REG)
      return TN_EINVAL;
  }
  if (pop->P == 0) return TN_OK;
  rc = check_obs(pop, obs, obs_genome_stride, B);
  if (rc != TN_OK) return rc;
  if (B == 0) return TN_OK;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!out) return TN_EINVAL;
  if (engine == TN_ENGINE_LDS) {
    tn::LdsTile lt;
    lt.K = tile->obs_per_lane;
    lt.waves = tile->waves_per_genome;
    lt.rows = tile->rows;
    return tn::launch_forward(*pop, *tr, obs, obs_genome_stride, B, out, lt, tn::FwdWork(),
                              stream);
  }
  if (engine == TN_ENGINE_REG) {
    tn::RegTile rt;
    rt.waves = tile->waves_per_genome;
    rt.rf = tile->rows == 0 ? 64 : tile->rows;
    return tn::launch_forward_reg(*pop, *tr, obs, obs_genome_stride, B, out, rt, tn::FwdWork(),
                                  stream);
  }
  return forward_auto(*pop, *tr, obs, obs_genome_stride, B, out, stream);
}

int tn_forward_loss(const tn_population* pop, const tn_transformed* tr, const float* obs,
                    int64_t obs_genome_stride, int32_t B, const float* target,
                    int64_t target_genome_stride, float scale, float offset, float* out,
                    float* loss, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->P == 0) return TN_OK;
  rc = check_obs(pop, obs, obs_genome_stride, B);
  if (rc != TN_OK) return rc;
  if (target_genome_stride < 0) return TN_EINVAL;
  if (target_genome_stride > 0 && target_genome_stride < (int64_t)B * pop->n_out) return TN_ESHAPE;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!loss || (B > 0 && !target)) return TN_EINVAL;
  // the register files of the automatic choice, smallest first (each taking
  // the genomes the smaller ones could not; prog_rows <= N_max, so a small
  // population needs one launch), then the LDS engine above 200 rows
  int cls[6];
  const int n = tn::reg_classes(B, cls);
  int lo = -1;
  for (int i = 0; i < n; ++i) {
    rc = tn::launch_forward_loss_reg(*pop, *tr, obs, obs_genome_stride, B, target,
                                     target_genome_stride, scale, offset, out, loss, 4, cls[i],
                                     lo, pop->N_max > cls[i], stream);
    if (rc != TN_OK || pop->N_max <= cls[i]) return rc;
    lo = cls[i];
  }
  return tn::launch_forward_loss(*pop, *tr, obs, obs_genome_stride, B, target,
                                 target_genome_stride, scale, offset, out, loss, tn::kRegRowsMax,
                                 stream);
}

int tn_backward(const tn_population* pop, const tn_transformed* tr, const float* obs,
                int64_t obs_genome_stride, int32_t B, const float* dY, int64_t dY_genome_stride,
                float* dW, float* db, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->P == 0) return TN_OK;
  rc = check_obs(pop, obs, obs_genome_stride, B);
  if (rc != TN_OK) return rc;
  if (dY_genome_stride < 0) return TN_EINVAL;
  if (dY_genome_stride > 0 && dY_genome_stride < (int64_t)B * pop->n_out) return TN_ESHAPE;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!dW || !db || (B > 0 && !dY)) return TN_EINVAL;
  return launch_backward(*pop, *tr, obs, obs_genome_stride, B, dY, dY_genome_stride, nullptr, 0,
                         0.0f, nullptr, dW, db, stream);
}

int tn_forward_backward_mse(const tn_population* pop, const tn_transformed* tr, const float* obs,
                            int64_t obs_genome_stride, int32_t B, const float* target,
                            int64_t target_genome_stride, float* loss, float* dW, float* db,
                            hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->P == 0) return TN_OK;
  rc = check_obs(pop, obs, obs_genome_stride, B);
  if (rc != TN_OK) return rc;
  if (target_genome_stride < 0) return TN_EINVAL;
  if (target_genome_stride > 0 && target_genome_stride < (int64_t)B * pop->n_out) return TN_ESHAPE;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!dW || !db || (B > 0 && !target)) return TN_EINVAL;
  const float scale = B > 0 ? 1.0f / ((float)B * (float)pop->n_out) : 0.0f;
  return launch_backward(*pop, *tr, obs, obs_genome_stride, B, nullptr, 0, target,
                         target_genome_stride, scale, loss, dW, db, stream);
}

int tn_distance_workspace_size(const tn_population* pop, size_t* bytes) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (!bytes) return TN_EINVAL;
  *bytes = distance_workspace_bytes(pop->P, pop->C_max);
  return TN_OK;
}

int tn_distance(const tn_population* pop, float c1, float c2, float c3, void* workspace,
                float* dist, int32_t* excess, int32_t* disjoint, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if ((excess == nullptr) != (disjoint == nullptr)) return TN_EINVAL;
  if (pop->P > 65535) return TN_EUNSUPPORTED;
  if (pop->P == 0) return TN_OK;
  if (!workspace || !dist) return TN_EINVAL;
  return launch_distance(*pop, c1, c2, c3, workspace, dist, excess, disjoint, stream);
}

int tn_distance_noalloc(const tn_population* pop, float c1, float c2, float c3, float* dist,
                        int32_t* excess, int32_t* disjoint, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if ((excess == nullptr) != (disjoint == nullptr)) return TN_EINVAL;
  if (pop->P > 65535) return TN_EUNSUPPORTED;
  if (pop->P == 0) return TN_OK;
  if (!dist) return TN_EINVAL;
  if (distance_workspace_bytes(pop->P, pop->C_max) > (size_t)TN_DISTANCE_NOALLOC_SCRATCH_BYTES)
    return TN_EUNSUPPORTED;
  void* ws = nullptr;
  rc = noalloc_scratch(&ws);
  if (rc != TN_OK) return rc;
  return launch_distance(*pop, c1, c2, c3, ws, dist, excess, disjoint, stream);
}

int tn_distance_nodes_workspace_size(const tn_population* pop, size_t* bytes) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (!bytes) return TN_EINVAL;
  *bytes = distance_nodes_workspace_bytes(pop->P, pop->N_max, pop->C_max);
  return TN_OK;
}

int tn_distance_nodes(const tn_population* pop, float c_disjoint, float c_homologous,
                      void* workspace, float* dist, int32_t* d_nodes, int32_t* d_conns,
                      hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if ((d_nodes == nullptr) != (d_conns == nullptr)) return TN_EINVAL;
  if (pop->P > 65535) return TN_EUNSUPPORTED;
  if (pop->P == 0) return TN_OK;
  if (!workspace || !dist) return TN_EINVAL;
  return launch_distance_nodes(*pop, c_disjoint, c_homologous, workspace, dist, d_nodes, d_conns,
                               stream);
}

int tn_reproduce_draws(int32_t N_max, int32_t C_max, int32_t* n_uniform, int32_t* n_normal) {
  if (!n_uniform || !n_normal || N_max < 1 || C_max < 1) return TN_EINVAL;
  if (N_max > TN_MAX_NODES || C_max > TN_MAX_CONNS) return TN_EUNSUPPORTED;
  *n_uniform = 16 + 7 * N_max + 2 * C_max;
  *n_normal = 4 + 2 * N_max + C_max;
  return TN_OK;
}

int tn_reproduce_workspace_size(int32_t n_children, size_t* bytes) {
  if (!bytes || n_children < 0) return TN_EINVAL;
  *bytes = reproduce_workspace_bytes(n_children);
  return TN_OK;
}

namespace {
bool prob_ok(float p) { return p >= 0.0f && p <= 1.0f; }  // false for NaN

bool options_ok(int32_t n, const uint8_t* o) {
  if (n < 1 || n > 8) return false;
  for (int i = 1; i < n; ++i)
    if (o[i] <= o[i - 1]) return false;
  return true;
}

int check_params(const tn_mutation_params* m) {
  if (!m) return TN_EINVAL;
  const float probs[] = {m->node_add, m->node_delete, m->conn_add, m->conn_delete,
                         m->bias_mutate_rate, m->bias_replace_rate, m->resp_mutate_rate,
                         m->resp_replace_rate, m->weight_mutate_rate, m->weight_replace_rate,
                         m->act_replace_rate, m->agg_replace_rate};
  for (float p : probs)
    if (!prob_ok(p)) return TN_EINVAL;
  if (!options_ok(m->n_act_options, m->act_options) ||
      !options_ok(m->n_agg_options, m->agg_options))
    return TN_EINVAL;
  if (m->act_default < 0 || m->act_default > 255 || m->agg_default < 0 || m->agg_default > 255)
    return TN_EINVAL;
  return TN_OK;
}
}  // namespace

int tn_reproduce(const tn_population* pop, int32_t n_children, const int32_t* parents,
                 const float* U, const float* Z, const tn_mutation_params* params,
                 int32_t next_key, const tn_population_arrays* children, int32_t* next_key_out,
                 void* workspace, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->node_off) return TN_EUNSUPPORTED;
  if (n_children < 0 || !next_key_out || !children) return TN_EINVAL;
  rc = check_params(params);
  if (rc != TN_OK) return rc;
  if (n_children > 0) {
    if (!parents || !U || !Z || !workspace) return TN_EINVAL;
    const tn_population_arrays& o = *children;
    if (!o.node_key || !o.node_bias || !o.node_resp || !o.node_act || !o.node_agg ||
        !o.conn_in || !o.conn_out || !o.conn_w || !o.conn_en)
      return TN_EINVAL;
    if (pop->P == 0) return TN_EINVAL;  // children need parents
  }
  return launch_reproduce(*pop, n_children, parents, U, Z, *params, next_key, *children,
                          next_key_out, workspace, stream);
}

int tn_forward_recurrent(const tn_population* pop, const float* obs, int64_t obs_genome_stride,
                         int32_t B, int32_t T, float* out, int32_t* status, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (T < 0) return TN_EINVAL;
  rc = check_obs(pop, obs, obs_genome_stride, B);
  if (rc != TN_OK) return rc;
  if (pop->P == 0) return TN_OK;
  if (B > 0 && !out) return TN_EINVAL;
  size_t bytes = 0;
  rc = recurrent_lds_check(*pop, &bytes);
  if (rc != TN_OK) return rc;
  return launch_forward_recurrent(*pop, obs, obs_genome_stride, B, T, out, status, stream);
}

namespace {
bool arrays_ok(const tn_population_arrays* o) {
  return o && o->node_key && o->node_bias && o->node_resp && o->node_act && o->node_agg &&
         o->conn_in && o->conn_out && o->conn_w && o->conn_en;
}

bool finite_nonneg(float x) { return x >= 0.0f && x < 3.0e38f; }  // false for NaN / inf

int check_table(const tn_species_table* t) {
  if (!t || t->max_species < 1 || t->max_species > TN_NEAT_MAX_SPECIES) return TN_EINVAL;
  if (!arrays_ok(&t->reps) || !t->alive || !t->best || !t->last_improved || !t->size)
    return TN_EINVAL;
  return TN_OK;
}
}  // namespace

int tn_neat_init(int32_t P, int32_t n_in, int32_t n_out, int32_t N_max, int32_t C_max,
                 const float* Z, const tn_mutation_params* mutation,
                 const tn_population_arrays* out, const tn_species_table* table,
                 hipStream_t stream) {
  if (P < 0 || n_in < 0 || n_out < 1 || N_max < 1 || C_max < 1) return TN_EINVAL;
  if (N_max > TN_MAX_NODES || C_max > TN_MAX_CONNS) return TN_EUNSUPPORTED;
  if (n_in + n_out > N_max || (int64_t)n_in * n_out > C_max) return TN_ESHAPE;
  int rc = check_params(mutation);
  if (rc != TN_OK) return rc;
  if (P > 0 && (!Z || !arrays_ok(out))) return TN_EINVAL;
  if (table) {
    rc = check_table(table);
    if (rc != TN_OK) return rc;
  }
  return launch_neat_init(P, n_in, n_out, N_max, C_max, Z, *mutation, *out, table, stream);
}

int tn_neat_workspace_size(const tn_population* pop, int32_t max_species, size_t* bytes) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (!bytes || max_species < 1 || max_species > TN_NEAT_MAX_SPECIES) return TN_EINVAL;
  *bytes = neat_workspace_bytes(pop->P, max_species, pop->N_max, pop->C_max);
  return TN_OK;
}

int tn_neat_generation(const tn_population* pop, const float* fitness, int32_t generation,
                       const tn_neat_params* params, const tn_species_table* table,
                       const float* sel, const float* U, const float* Z, int32_t next_key,
                       const tn_population_arrays* children, int32_t* species_of,
                       int32_t* parents, int32_t* next_key_out, void* workspace,
                       hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  if (pop->node_off) return TN_EUNSUPPORTED;
  if (pop->P < 1 || !params) return TN_EINVAL;
  const tn_neat_params& m = *params;
  if (!finite_nonneg(m.compatibility_threshold) || !finite_nonneg(m.compatibility_disjoint) ||
      !finite_nonneg(m.compatibility_homologous) || m.max_species < 1 ||
      m.max_species > TN_NEAT_MAX_SPECIES || m.species_elitism < 1 || m.max_stagnation < 1 ||
      m.genome_elitism < 0 || !(m.survival_threshold > 0.0f && m.survival_threshold <= 1.0f) ||
      !(m.spawn_number_change_rate >= 0.0f && m.spawn_number_change_rate <= 1.0f))
    return TN_EINVAL;
  rc = check_params(&m.mutation);
  if (rc != TN_OK) return rc;
  rc = check_table(table);
  if (rc != TN_OK) return rc;
  if (table->max_species != m.max_species) return TN_ESHAPE;
  if (!fitness || !sel || !U || !Z || !arrays_ok(children) || !next_key_out || !workspace)
    return TN_EINVAL;
  return launch_neat_generation(*pop, fitness, generation, m, *table, sel, U, Z, next_key,
                                *children, species_of, parents, next_key_out, workspace, stream);
}

int tn_cppn_query(const tn_population* pop, const tn_transformed* tr, const tn_substrate* sub,
                  uint16_t* w1t, uint16_t* w2t, float* raw1, float* raw2, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  if (pop->n_in != 5 || pop->n_out != 1) return TN_ESHAPE;
  if (pop->P == 0) return TN_OK;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!w1t || !w2t) return TN_EINVAL;
  return launch_cppn_query(*pop, *tr, *sub, w1t, w2t, raw1, raw2, stream);
}

int tn_substrate_forward(const tn_substrate* sub, int32_t P, const uint16_t* w1t,
                         const uint16_t* w2t, const uint16_t* x, int64_t x_genome_stride,
                         int32_t B, float* h, float* y, hipStream_t stream) {
  int rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  if (P < 0 || B < 0 || x_genome_stride < 0) return TN_EINVAL;
  const int64_t S = (int64_t)sub->grid * sub->grid;
  if (x_genome_stride > 0 && x_genome_stride < (int64_t)B * S) return TN_ESHAPE;
  if (P == 0 || B == 0) return TN_OK;
  if (!w1t || !w2t || !x || !h || !y) return TN_EINVAL;
  return launch_substrate_forward(*sub, P, w1t, w2t, x, x_genome_stride, B, h, y, stream);
}

int tn_substrate_workspace_size(const tn_substrate* sub, int32_t P, int32_t B,
                                int64_t x_genome_stride, size_t* bytes) {
  if (!bytes) return TN_EINVAL;
  int rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  if (P < 0 || B < 0 || x_genome_stride < 0) return TN_EINVAL;
  *bytes = substrate_workspace_bytes(*sub, P, B, x_genome_stride);
  return TN_OK;
}

int tn_substrate_backward(const tn_substrate* sub, int32_t P, const uint16_t* w2t,
                          const uint16_t* x, int64_t x_genome_stride, int32_t B, const float* h,
                          const float* dy, void* workspace, float* dw1t, float* dw2t,
                          hipStream_t stream) {
  int rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  if (P < 0 || B < 0 || x_genome_stride < 0) return TN_EINVAL;
  if (sub->n_out > 32 || (int64_t)B * sub->n_out > 16384) return TN_EUNSUPPORTED;
  const int64_t S = (int64_t)sub->grid * sub->grid;
  if (x_genome_stride > 0 && x_genome_stride < (int64_t)B * S) return TN_ESHAPE;
  if (P == 0) return TN_OK;
  if (!w2t || !x || !h || !dy || !workspace || !dw1t || !dw2t) return TN_EINVAL;
  return launch_substrate_backward(*sub, P, w2t, x, x_genome_stride, B, h, dy, workspace, dw1t,
                                   dw2t, stream);
}

int tn_cppn_backward_workspace_size(const tn_population* pop, const tn_substrate* sub,
                                    size_t* bytes) {
  if (!bytes) return TN_EINVAL;
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  *bytes = cppn_backward_workspace_bytes(*pop, *sub);
  return TN_OK;
}

int tn_cppn_backward(const tn_population* pop, const tn_transformed* tr, const tn_substrate* sub,
                     const float* dw1t, const float* dw2t, void* workspace, float* dW,
                     float* db, hipStream_t stream) {
  int rc = check_population(pop);
  if (rc != TN_OK) return rc;
  rc = check_substrate(sub);
  if (rc != TN_OK) return rc;
  if (pop->n_in != 5 || pop->n_out != 1) return TN_ESHAPE;
  if (pop->P == 0) return TN_OK;
  rc = check_transformed(tr);
  if (rc != TN_OK) return rc;
  if (!dw1t || !dw2t || !workspace || !dW || !db) return TN_EINVAL;
  return launch_cppn_backward(*pop, *tr, *sub, dw1t, dw2t, workspace, dW, db, stream);
}

}  // extern "C"
