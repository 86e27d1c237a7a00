/*
 * tensorneat_hip.h - C ABI of the MI355X (gfx950) tensorized NEAT population
 * evaluation library (libtnhip.so).
 *
 * What it computes follows TensorNEAT (arXiv 2504.08339):
 *   - the tensorized encoding of a population (Section 3.1): every genome is a
 *     node tensor N-hat and a connection tensor C-hat padded to fixed row
 *     capacities and stacked into P_N, P_C;
 *   - tensorized network inference (Section 3.3), split into the
 *     transformation (topological order + expanded connections, done once per
 *     network) and the calculation (node values in topological order);
 *   - the compatibility distance used to divide the population into species
 *     (Section 2.1, Algorithm 1; coefficients in Appendix A).
 *
 * Conventions for every call
 *   - All array pointers are DEVICE pointers unless stated otherwise, row-major,
 *     allocated and owned by the caller. The library never frees caller memory.
 *   - Every call that takes a hipStream_t is asynchronous on that stream and
 *     never synchronises the device unless its description says so.
 *   - Arguments are validated on the host before anything is launched; a bad
 *     argument returns an error status and launches nothing. A launch or
 *     runtime error observed right after launching returns TN_EHIP.
 *   - Problems in the DATA (a cycle, a dangling key, ...) never fail a call:
 *     they set bits in the per-genome status word (enum tn_genome_status), and
 *     that genome's outputs, losses and gradients are NaN.
 */
#ifndef TENSORNEAT_HIP_H
#define TENSORNEAT_HIP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */

typedef enum tn_status {
    TN_OK = 0,
    TN_EINVAL = 1,        /* null pointer where one is required, negative size     */
    TN_ESHAPE = 2,        /* inconsistent sizes (e.g. too few rows for P x N_max)   */
    TN_EUNSUPPORTED = 3,  /* above a compiled limit (TN_MAX_NODES, TN_MAX_CONNS, ...) */
    TN_EHIP = 4,          /* HIP launch / runtime error                              */
    TN_ENOMEM = 5         /* a library-owned allocation failed                       */
} tn_status;

/* Human-readable name of a tn_status (static string; never NULL). */
const char* tn_status_string(int status);

/* Library version as 10000*major + 100*minor + patch. */
int tn_version(void);

/* Text of the last HIP error this thread's calls returned TN_EHIP for ("" if
 * none). Static string; never NULL. */
const char* tn_last_error(void);

/* Compiled limits of the per-genome row capacities handled by one call. */
#define TN_MAX_NODES 1024
#define TN_MAX_CONNS 4096
#define TN_MAX_IO    1024

/* ------------------------------------------------------------- encodings */

/* Node activation codes (node attribute f_act, Section 3.1). Definitions:
 * identity z; sigmoid 1/(1+e^-z); tanh; relu max(0,z); sin; gaussian e^(-z^2);
 * abs |z|. */
enum tn_act {
    TN_ACT_IDENTITY = 0, TN_ACT_SIGMOID = 1, TN_ACT_TANH = 2, TN_ACT_RELU = 3,
    TN_ACT_SIN = 4, TN_ACT_GAUSSIAN = 5, TN_ACT_ABS = 6
};

/* Node aggregation codes (node attribute f_agg, Section 3.1). Over no terms
 * every aggregation gives 0; maxabs keeps the sign of the largest-magnitude term. */
enum tn_agg {
    TN_AGG_SUM = 0, TN_AGG_PRODUCT = 1, TN_AGG_MAX = 2, TN_AGG_MIN = 3,
    TN_AGG_MEAN = 4, TN_AGG_MAXABS = 5
};

/* Per-genome status bits written by tn_transform. */
enum tn_genome_status {
    TN_CYCLE = 1,        /* a cycle among enabled connections (feedforward only, Section 3.3);
                            looked for only when no other bit is set                       */
    TN_DANGLING = 2,     /* an enabled connection names a key no node row holds            */
    TN_DUP_CONN = 4,     /* two valid connection rows share (in-key, out-key)             */
    TN_DUP_NODE = 8,     /* two valid node rows share a key                                */
    TN_INPUT_DST = 16,   /* an enabled connection ends at an input key                     */
    TN_MISSING_IO = 32,  /* an input or output key has no node row                         */
    TN_OVERSIZE = 64,    /* ragged genome with more rows than N_max / C_max (reported alone) */
    TN_BAD_ATTR = 128    /* a node row with an activation / aggregation code out of range  */
};

/* --------------------------------------------------------- the population */

/*
 * A population in structure-of-arrays form (Section 3.1: P_N and P_C).
 *
 * Node row:       key (int32), bias (f32), response (f32), act (u8), agg (u8)
 * Connection row: in-key (int32), out-key (int32), weight (f32), enabled (u8)
 *
 * A node row with a negative key, or a connection row with a negative in- or
 * out-key, is an empty row (the paper's NaN padding row); empty rows may sit
 * anywhere. Keys are historical markers: inputs are keys 0..n_in-1 and
 * outputs n_in..n_in+n_out-1 (Appendix B, genome interface); hidden keys are
 * any other non-negative int32. Connection endpoints are keys, not rows.
 *
 * Layout
 *   padded (node_off == NULL): genome g's node rows are [g*N_max, (g+1)*N_max),
 *     its connection rows [g*C_max, (g+1)*C_max).
 *   ragged (node_off != NULL): genome g's node rows are [node_off[g],
 *     node_off[g+1]) and connection rows [conn_off[g], conn_off[g+1]); both
 *     offset arrays are device int64 [P+1] starting at 0. N_max / C_max are
 *     then the largest row counts the call must handle (they size on-chip
 *     buffers); a genome above them gets TN_OVERSIZE. total_nodes /
 *     total_conns (host values) give the array lengths: node_off[P] and
 *     conn_off[P].
 */
typedef struct tn_population {
    int32_t P;            /* number of genomes, >= 0                               */
    int32_t n_in;         /* I, >= 0                                               */
    int32_t n_out;        /* O, >= 1                                               */
    int32_t N_max;        /* node row capacity, 1..TN_MAX_NODES                    */
    int32_t C_max;        /* connection row capacity, 1..TN_MAX_CONNS              */
    int64_t total_nodes;  /* ragged only: node_off[P]; ignored when padded         */
    int64_t total_conns;  /* ragged only: conn_off[P]; ignored when padded         */
    const int64_t* node_off;   /* NULL (padded) or device [P+1]                    */
    const int64_t* conn_off;   /* NULL (padded) or device [P+1]                    */
    const int32_t* node_key;
    const float*   node_bias;
    const float*   node_resp;
    const uint8_t* node_act;
    const uint8_t* node_agg;
    const int32_t* conn_in;
    const int32_t* conn_out;
    const float*   conn_w;
    const uint8_t* conn_en;
} tn_population;

/* Host-only check of a population descriptor (pointers and sizes; the device
 * data is not read). Returns TN_OK, TN_EINVAL, TN_ESHAPE or TN_EUNSUPPORTED. */
int tn_validate_population(const tn_population* pop);

/* ------------------------------------------------ the paper's float layout */

/*
 * The tensorized encoding as the paper writes it (Section 3.1): a node tensor
 * P_N [P][N_max][5] float32 with rows n = [k, bias, response, act, agg] and a
 * connection tensor P_C [P][C_max][4] float32 with rows c = [k_in, k_out, e, w]
 * (markings, then the enabled flag, then the attribute), both padded with
 * NaN rows. tn_pack_paper_layout converts them into the structure-of-arrays
 * form every other call reads (padded layout, [P][N_max] / [P][C_max]):
 *   - a row whose first column is NaN is a padding row, wherever it sits, and
 *     becomes an empty row (key -1 / markings -1, other fields 0);
 *   - keys and markings must be integers 0 <= k < 2^24 (exact in float32),
 *     act and agg integer codes 0..255 (codes outside tn_act / tn_agg are
 *     left for tn_transform's TN_BAD_ATTR), e exactly 0 or 1; bias, response
 *     and weight are copied bitwise.
 * A row that breaks these rules sets its genome's bits in pack_err and is
 * written as an empty row; the call then returns TN_EINVAL (the other rows
 * are still converted).
 *
 *   PN, PC    device float32 arrays as above (caller-owned, read only; PC must
 *             be 16-byte aligned)
 *   out       device destination arrays (caller-owned): node_* [P][N_max],
 *             conn_* [P][C_max]
 *   pack_err  device int32 [P] (caller-owned): tn_pack_error bits per genome
 * This call SYNCHRONISES `stream`: it reads pack_err back to decide its
 * return value. TN_EINVAL also for null pointers or negative sizes.
 */
typedef struct tn_population_arrays {
    int32_t* node_key;
    float*   node_bias;
    float*   node_resp;
    uint8_t* node_act;
    uint8_t* node_agg;
    int32_t* conn_in;
    int32_t* conn_out;
    float*   conn_w;
    uint8_t* conn_en;
} tn_population_arrays;

enum tn_pack_error {
    TN_PACK_NODE_KEY = 1,    /* node key not an integer in [0, 2^24)             */
    TN_PACK_NODE_CODE = 2,   /* act or agg not an integer code in [0, 255]        */
    TN_PACK_CONN_KEY = 4,    /* k_in or k_out not an integer in [0, 2^24)         */
    TN_PACK_CONN_FLAG = 8    /* enabled flag neither 0 nor 1                      */
};

int tn_pack_paper_layout(const float* PN, const float* PC, int32_t P, int32_t N_max,
                         int32_t C_max, const tn_population_arrays* out, int32_t* pack_err,
                         hipStream_t stream);

/* --------------------------------------------------- the transformation */

/*
 * Output of the transformation (Section 3.3), per genome, in the same node /
 * connection row blocks as the population ("node block" = the genome's node
 * rows, "conn block" = its connection rows), plus per-genome arrays.
 *
 * The topological order N_order is the level-synchronous one: round r emits,
 * in ascending node-row order, every node whose enabled in-edges all come from
 * nodes emitted in earlier rounds; r is the node's level. The expanded
 * connections C_exp are kept in compressed form: the enabled in-edges of the
 * node at topological position p, in ascending connection-row order, are
 * entries row_ptr[p] .. row_ptr[p+1]-1 of the genome's conn block.
 *
 *   status  [P]          tn_genome_status bits (0 = valid)
 *   n_valid [P]          number of node positions (0 for a flagged genome)
 *   order   node block   node row at position p; -1 for p >= n_valid
 *   level   node block   level of position p; -1 for p >= n_valid
 *   row_ptr node block + 1 per genome: genome g's entries start at g*(N_max+1)
 *                        (padded) or node_off[g]+g (ragged); n_valid+1 valid
 *                        entries, relative to the genome's conn block; the
 *                        rest repeat the last valid entry
 *   edge_src conn block  topological position of the edge's source node
 *   edge_row conn block  connection row of the edge
 *   edge_w  conn block   weight of the edge (copied bitwise)
 *                        (edge entries past the last valid one: -1, -1, 0)
 *   pos_bias node block  bias of the node at position p
 *   pos_resp node block  response of the node at position p
 *   pos_fn  node block   act | agg << 8, with bit 31 set for an input node
 *                        (whose value is the observation, bits 16..30 = input index)
 *   io_pos  [P][n_in+n_out] position of input key i (i < n_in) and of output key
 *                        n_in+j at index n_in+j
 *   pos_row node block   value row of position p in the level-parallel forward
 *                        pass's on-chip buffer: input k takes row k; level by
 *                        level every other position takes the lowest free row,
 *                        and rows of positions whose last consumer is in the
 *                        level are freed after it (outputs keep theirs; a row
 *                        freed in level L is reused from level L+1 on).
 *                        -1 for p >= n_valid
 *   n_rows  [P]          rows pos_row uses (<= n_valid; 0 for a flagged genome)
 *   prog_node node block x 4 int32: packed program of the position-by-position
 *                        forward pass: {row_ptr[p+1], node function word, bits
 *                        of bias, bits of response}; the function word is
 *                        act | agg << 8 | prog row << 16, or pos_fn for an input
 *                        (whose prog row is its input index). Prog rows are
 *                        freed right after the last consumer has read them (it
 *                        may take one for its own value), outputs keep theirs.
 *   prog_edge conn block x 2 int32: {prog row of the source, bits of the weight},
 *                        followed by 8 padding entries after the whole array
 *                        (2 * (conn_elems + 8) int32 in all: the register
 *                        engine reads edges in groups of 8 ahead and uses none
 *                        past a node's last; the library never writes them)
 *   prog_rows [P]        rows the packed program uses (the largest number of
 *                        values live at once; 0 for a flagged genome)
 *   prog_rec node block x 16 int32: the packed program again, one record per
 *                        non-input position in order (records past the last
 *                        are 0): word 0 = act | agg << 3 | prog row << 6 |
 *                        in-edge count << 17; word 1 bias bits; word 2
 *                        response bits; word 3 = index (in the conn block of
 *                        prog_edge) of the node's 7th in-edge; words 4..15 its
 *                        first 6 in-edges as {source prog row, weight bits},
 *                        unused slots {prog_rows, +0} (never read: a reader
 *                        takes only the in-edge count of slots)
 */
typedef struct tn_transformed {
    int32_t* status;
    int32_t* n_valid;
    int32_t* order;
    int32_t* level;
    int32_t* row_ptr;
    int32_t* edge_src;
    int32_t* edge_row;
    float*   edge_w;
    float*   pos_bias;
    float*   pos_resp;
    int32_t* pos_fn;
    int32_t* io_pos;
    int32_t* pos_row;
    int32_t* n_rows;
    int32_t* prog_node;
    int32_t* prog_edge;
    int32_t* prog_rows;
    int32_t* prog_rec;
} tn_transformed;

/* Element counts of the tn_transformed arrays for a population (host only):
 * node_elems (order, level, pos_*), rowptr_elems, conn_elems (edge_*),
 * genome_elems (status, n_valid) and io_elems (io_pos). */
typedef struct tn_transformed_elems {
    int64_t node_elems;
    int64_t rowptr_elems;
    int64_t conn_elems;
    int64_t genome_elems;
    int64_t io_elems;
} tn_transformed_elems;

int tn_transformed_size(const tn_population* pop, tn_transformed_elems* out);

/* Transformation of every genome (Section 3.3; BaseGenome.transform of
 * Appendix B, batched over the population). One workgroup per genome (one to
 * eight wavefronts, by the population's row capacities); a ragged population
 * of at least 2048 genomes takes one launch per size class. The largest class
 * runs on `stream`, the others on side streams that the library creates once
 * per device (default priority, non-blocking); they start after the work
 * already queued on `stream` and `stream` waits for them before anything
 * queued after this call, so the call is ordered on `stream` like a single
 * launch. Calls from several host threads are serialized while they queue
 * their launches. Under stream capture the classes are launched one after
 * another on `stream` (no side streams join the capture).
 * Fills every array of *tr; the results do not depend on the launch shape. */
int tn_transform(const tn_population* pop, const tn_transformed* tr, hipStream_t stream);

/* ------------------------------------------------------ the calculation */

/*
 * Forward pass of every genome over B observations (Section 3.3;
 * BaseGenome.forward of Appendix B, batched over population and batch):
 *   v[input i] = x[i];  for each other node k in topological order
 *   v[k] = act_k(bias_k + resp_k * agg_k(w_e * v[src_e] over its in-edges));
 *   y[j] = v[output key n_in + j].
 * The response multiplies the aggregate (with response 1 this is the paper's
 * f_n = f_act(f_agg + b)). Computed in float32; the sum aggregation
 * accumulates in ascending connection-row order with fused multiply-add.
 *
 *   obs   observation b of genome g, component i, at
 *         obs[g*obs_genome_stride + b*n_in + i]; obs_genome_stride = 0 shares
 *         one [B][n_in] batch across genomes.
 *   out   [P][B][n_out] float32.
 * B >= 0 (B = 0 launches nothing). tr must come from tn_transform on pop.
 */
int tn_forward(const tn_population* pop, const tn_transformed* tr,
               const float* obs, int64_t obs_genome_stride, int32_t B,
               float* out, hipStream_t stream);

/* How the forward pass is laid out on the chip. Two engines:
 *   TN_ENGINE_LDS  a workgroup of waves_per_genome wavefronts (1..16 at
 *                  obs_per_lane 1, else 1..8) evaluates
 *                  one genome on tiles of 64 * obs_per_lane observations
 *                  (obs_per_lane = 1, 2 or 4 consecutive ones per lane) with
 *                  `rows` value rows of the tile in LDS (0: N_max), splitting
 *                  each level of the topological order among its wavefronts;
 *                  genomes whose n_rows exceeds `rows` get NaN outputs.
 *   TN_ENGINE_REG  each wavefront evaluates one genome on tiles of 64
 *                  observations (obs_per_lane 0 or 1) walking the packed
 *                  program, with the values in a register file of `rows`
 *                  rows per tile: 32, 64, 96, 128, 160 or 200 (one tile per
 *                  wavefront), 100 (two consecutive tiles) or 50 (four); 0:
 *                  64. waves_per_genome (1..8) wavefronts share a workgroup;
 *                  genomes whose prog_rows exceeds `rows` get NaN outputs.
 *   TN_ENGINE_AUTO the library's choice for every genome (the other fields
 *                  are ignored): TN_ENGINE_REG for prog_rows <= 200 (rows
 *                  50, 100, 128, 160, 200 when B spans at least 4 tiles of
 *                  64; 100, 128, 160, 200 for 2 or 3 tiles; 32, 64, 96, 128,
 *                  160, 200 for one; each launch takes the genomes the
 *                  smaller files could not), TN_ENGINE_LDS with rows =
 *                  min(N_max, the LDS capacity, about 600 rows on MI355X) for
 *                  the rest; a genome needing more than that capacity gets
 *                  NaN outputs.
 * Outputs are bitwise identical across engines and tile shapes. */
enum tn_engine { TN_ENGINE_AUTO = 0, TN_ENGINE_LDS = 1, TN_ENGINE_REG = 2 };

typedef struct tn_tile {
    int32_t engine;
    int32_t obs_per_lane;
    int32_t waves_per_genome;
    int32_t rows;
} tn_tile;

/* tn_forward with an explicit layout (tile may be NULL: TN_ENGINE_AUTO). TN_EINVAL for
 * field values outside the ranges above. */
int tn_forward_tiled(const tn_population* pop, const tn_transformed* tr,
                     const float* obs, int64_t obs_genome_stride, int32_t B,
                     float* out, const tn_tile* tile, hipStream_t stream);

/*
 * Forward pass with a fused squared-error epilogue (fitness / loss):
 *   loss[g] = offset + scale * sum_{b,j} (y[g][b][j] - target[b][j])^2
 * with target[b][j] at target[g*target_genome_stride + b*n_out + j]
 * (stride 0 = shared targets). XOR fitness 4 - SSE is offset 4, scale -1; the
 * mean squared error is offset 0, scale 1/(B*n_out). out may be NULL (outputs
 * not stored). The per-genome sum is reduced in a fixed order (deterministic).
 */
int tn_forward_loss(const tn_population* pop, const tn_transformed* tr,
                    const float* obs, int64_t obs_genome_stride, int32_t B,
                    const float* target, int64_t target_genome_stride,
                    float scale, float offset, float* out, float* loss,
                    hipStream_t stream);

/*
 * Forward pass of RECURRENT networks (network type "recurrent" of Appendix A:
 * enabled connections may form cycles, including self-loops). The paper
 * details the calculation only for feedforward networks (Section 3.3); here a
 * recurrent network is evaluated by T synchronous sweeps:
 *   v_0[input i] = x[i], v_0[k] = 0 for every other node;
 *   sweep t = 1..T: v_t[k] = act_k(bias_k + resp_k * agg_k(w_e * v_{t-1}[src_e]))
 *     for every non-input node k over its enabled in-edges (ascending
 *     connection row), all from the previous sweep; inputs keep their values;
 *   y[j] = v_T[output key n_in + j]  (T = 0: all outputs 0).
 * Sum aggregation accumulates with fused multiply-add in ascending in-edge
 * order and z = fma(resp, aggregate, bias), as tn_forward does, so an acyclic
 * sum-aggregation genome gives tn_forward's bits once T exceeds its largest
 * topological level.
 *
 * obs, obs_genome_stride, B and out as in tn_forward; T >= 0 sweeps.
 * status (may be NULL): device int32 [P], the tn_genome_status bits of each
 * genome with TN_CYCLE never set (cycles are allowed); a genome with any bit
 * gets NaN outputs. The whole genome's values sit in LDS: TN_EUNSUPPORTED when
 * 2 * N_max * 64 floats plus its tables exceed one workgroup's LDS (N_max up
 * to about 280 at C_max 256 on MI355X).
 */
int tn_forward_recurrent(const tn_population* pop, const float* obs, int64_t obs_genome_stride,
                         int32_t B, int32_t T, float* out, int32_t* status, hipStream_t stream);

/* ------------------------------------------------------- batched plan */

/*
 * Batched forward pass of a population whose genomes differ widely in size
 * (the space-time trade-off of the padded encoding, Section 3.3; the
 * population-level parallelism of Sections 4.1 and 5.4). A plan sorts the genomes once
 * into length buckets by the value rows their forward pass needs:
 *   prog_rows <= each register-file size TN_ENGINE_AUTO uses for B (50,
 *                 100, 128, 160, 200 for B > 192)   TN_ENGINE_REG with that
 *                                                   file;
 *   larger, n_rows <= 256, <= the LDS capacity (about 600 rows on MI355X)
 *                                                   TN_ENGINE_LDS.
 * Flagged genomes join the first bucket (NaN outputs). Each bucket lists its
 * genomes longest first (enabled edges + nodes).
 *
 * tn_plan_create reads the transformed sizes back (it synchronises `stream`)
 * and allocates the plan's device lists, counters, streams and events; the
 * plan keeps copies of *pop and *tr (the structs, not the arrays): the caller
 * keeps those arrays alive and unchanged while the plan is used. tune_cache
 * (may be NULL) is a text file written by tn_plan_tune whose tile choices are
 * applied to matching buckets. TN_EUNSUPPORTED if a genome needs more rows
 * than the LDS engine holds; TN_ENOMEM / TN_EHIP on allocation failures.
 *
 * tn_plan_forward_buckets: one plain launch per bucket, in bucket order.
 * tn_plan_forward: one persistent kernel per bucket (its wavefronts or
 * workgroups take the next genome or tile from a device counter, longest
 * first) on independent branches of a hipGraph, with a zeroing kernel in
 * front; the graph is captured on the first call and again whenever obs, its
 * stride or out change, then replayed with one launch on `stream`. Calls on
 * one plan must not overlap (they share its counters).
 * Both write out [P][B][n_out] for observations laid out as in tn_forward
 * (obs_genome_stride 0 = shared), bitwise equal to tn_forward's outputs.
 *
 * tn_plan_tune times every tile candidate of every bucket in the persistent
 * form tn_plan_forward's graph runs (best of five launches after a warm-up;
 * register buckets: 1, 2, 4, 8 wavefronts per workgroup; LDS buckets: 1, 2, 4
 * observations per lane x 1, 2, 4, 8 wavefronts, and 16 at one observation
 * per lane), keeps the fastest, and (tune_cache != NULL) merges the choices
 * into the cache file. It writes `out` while timing and synchronises `stream`.
 */
typedef struct tn_plan tn_plan;

typedef struct tn_bucket_info {
    int32_t engine;       /* TN_ENGINE_REG or TN_ENGINE_LDS */
    int32_t rows_class;   /* REG: register-file rows per tile (bound of prog_rows); LDS: bound of n_rows */
    int32_t count;        /* genomes */
    int64_t edges;        /* enabled edges over the bucket */
    tn_tile tile;         /* current tile (rows: register rows / LDS rows) */
} tn_bucket_info;

int  tn_plan_create(const tn_population* pop, const tn_transformed* tr, int32_t B,
                    const char* tune_cache, tn_plan** plan, hipStream_t stream);
void tn_plan_destroy(tn_plan* plan);
int  tn_plan_num_buckets(const tn_plan* plan);
int  tn_plan_bucket(const tn_plan* plan, int32_t i, tn_bucket_info* info);
/* Sets bucket i's tile: obs_per_lane (REG: 1; LDS: 1, 2, 4), waves (REG: 1..8; LDS:
 * 1..16 at one observation per lane, else 1..8). */
int  tn_plan_set_tile(tn_plan* plan, int32_t i, int32_t obs_per_lane, int32_t waves);
int  tn_plan_forward(tn_plan* plan, const float* obs, int64_t obs_genome_stride, float* out,
                     hipStream_t stream);
int  tn_plan_forward_buckets(tn_plan* plan, const float* obs, int64_t obs_genome_stride,
                             float* out, hipStream_t stream);
int  tn_plan_tune(tn_plan* plan, const float* obs, int64_t obs_genome_stride, float* out,
                  const char* tune_cache, hipStream_t stream);
/* Bucket i alone on `stream`: its persistent kernel (persistent != 0, after a
 * zeroing kernel for its counter) or its plain launch; writes that bucket's
 * genomes of out. For timing buckets one by one. */
int  tn_plan_forward_bucket(tn_plan* plan, int32_t i, int32_t persistent, const float* obs,
                            int64_t obs_genome_stride, float* out, hipStream_t stream);

/* ---------------------------------------------------------- HyperNEAT */

/*
 * HyperNEAT on a grid substrate (the indirect encoding among the library's
 * algorithms, Section 4.4). A CPPN genome (5 inputs, 1 output) is queried for
 * every substrate connection s -> t at (x_s, y_s, x_t, y_t, 1) with the
 * forward rule above; |w| < threshold gives 0; the result is rounded to
 * bfloat16 (round to nearest even). Geometry: the input and the hidden layer
 * are grid x grid layers with node grid*r + c at (-1 + 2c/(grid-1),
 * -1 + 2r/(grid-1)); output j of n_out sits at (-1 + 2j/(n_out-1), 0) (0 for
 * n_out = 1). One CPPN gives both layers. The substrate has no biases:
 *   H = tanh(X W1),  Y = bf16(H) W2
 * with bfloat16 operands and float32 accumulation. S = grid*grid must be a
 * multiple of 64 and S * n_out <= 32768 (TN_EUNSUPPORTED otherwise).
 */
typedef struct tn_substrate {
    int32_t grid;
    int32_t n_out;
    float   threshold;
} tn_substrate;

/* Weights of every CPPN genome (pop->n_in must be 5, pop->n_out 1; tr from
 * tn_transform on pop; every genome's prog_rows <= 50, else its weights are
 * NaN, as are a flagged genome's). Outputs, bfloat16 bits, transposed so that
 * rows run along the source index:
 *   w1t [P][S][S]       w1t[g][t][s] = weight input s -> hidden t
 *   w2t [P][n_out][S]   w2t[g][j][s] = weight hidden s -> output j
 * raw1 / raw2 (NULL: not stored): the float32 CPPN values before the
 * threshold, in the same layouts. */
int tn_cppn_query(const tn_population* pop, const tn_transformed* tr, const tn_substrate* sub,
                  uint16_t* w1t, uint16_t* w2t, float* raw1, float* raw2, hipStream_t stream);

/* Substrate forward of P genomes: x [B][S] bfloat16 bits per genome at
 * x + g*x_genome_stride (0: shared); h [P][B][S] float32 (tanh of the fp32
 * accumulation); y [P][B][n_out] float32, summed in ascending hidden index. */
int tn_substrate_forward(const tn_substrate* sub, int32_t P, const uint16_t* w1t,
                         const uint16_t* w2t, const uint16_t* x, int64_t x_genome_stride,
                         int32_t B, float* h, float* y, hipStream_t stream);

/* Gradient of L = sum(dY * Y) through the substrate forward above, with
 * respect to the weights as the forward used them (bfloat16 values):
 *   dw2t [P][n_out][S]  dw2t[g][j][t] = sum_b H[b][t] dY[b][j]
 *   dw1t [P][S][S]      dw1t[g][t][s] = sum_b dZ[b][t] x[b][s],
 *                       dZ = (dY W2^T) (1 - H^2) rounded to bfloat16
 * dy [P][B][n_out] float32; h the forward's output; w2t, x as given to the
 * forward. float32 accumulation (dw2t in ascending b; dw1t on the matrix
 * cores). workspace: tn_substrate_workspace_size bytes of device memory
 * (caller-owned, contents irrelevant). n_out <= 32 and B * n_out <= 16384 here
 * (TN_EUNSUPPORTED otherwise). */
int tn_substrate_workspace_size(const tn_substrate* sub, int32_t P, int32_t B,
                                int64_t x_genome_stride, size_t* bytes);
int tn_substrate_backward(const tn_substrate* sub, int32_t P, const uint16_t* w2t,
                          const uint16_t* x, int64_t x_genome_stride, int32_t B, const float* h,
                          const float* dy, void* workspace, float* dw1t, float* dw2t,
                          hipStream_t stream);

/* Gradient with respect to the CPPN genomes' connection weights and node
 * biases of L = sum over every substrate connection of u * w, where w is the
 * weight tn_cppn_query produced and the upstream u is dw1t[g][t][s] (input s
 * -> hidden t) or dw2t[g][j][s] (hidden s -> output j) when the CPPN value
 * survived the threshold, 0 otherwise (with dw1t, dw2t from
 * tn_substrate_backward this is the gradient of the substrate loss through the
 * whole encoding). The threshold decision is this call's own float32 CPPN
 * value, the same one tn_cppn_query thresholds. dW shaped like
 * pop->conn_w and db like pop->node_bias; disabled, padding and input rows get
 * 0; genomes that are flagged, have more than 32 nodes or 64 enabled
 * connections, or use an aggregation other than sum or mean get NaN.
 * Per-query terms are accumulated in float32 per lane and reduced in a fixed
 * order (deterministic). workspace: tn_cppn_backward_workspace_size bytes. */
int tn_cppn_backward_workspace_size(const tn_population* pop, const tn_substrate* sub,
                                    size_t* bytes);
int tn_cppn_backward(const tn_population* pop, const tn_transformed* tr, const tn_substrate* sub,
                     const float* dw1t, const float* dw2t, void* workspace, float* dW,
                     float* db, hipStream_t stream);

/* ---------------------------------------------------------- gradients */

/*
 * Reverse-mode gradient of the forward pass above with respect to every
 * connection weight and node bias (gradient refinement of evolved weights;
 * the chain rule applied to the Section 3.3 node rule). For a node k with
 * z = bias + resp * agg(t_e), t_e = w_e * v[src_e], v = act(z):
 *   delta_k = dL/dv_k * act'(z_k);  dL/dbias_k = sum over the batch of delta_k;
 *   dL/dw_e = sum over the batch of delta_k * resp_k * d agg/d t_e * v_src,
 *   and dL/dv_src accumulates delta_k * resp_k * d agg/d t_e * w_e.
 * d agg / d t_e is 1 (sum), 1/n (mean), the product of the other terms
 * (product), and 1 at the first extreme term in row order, 0 elsewhere (max,
 * min, maxabs). act' at the kinks of relu and abs is 0.
 *
 *   dY   upstream gradient dL/dy: element (b, j) of genome g at
 *        dY[g*dY_genome_stride + b*n_out + j]
 *   dW   one float per connection row (the population's conn layout): the
 *        gradient for an enabled row, exactly 0 for disabled and empty rows
 *   db   one float per node row: the gradient for a non-input node, exactly 0
 *        for input and empty rows
 * The forward pass is recomputed inside the call (nothing is saved by
 * tn_forward). Batch sums run in a fixed order, so results are deterministic.
 * A flagged genome gets NaN in all its rows.
 * Limits: genomes with at most 48 positions, 64 enabled connections and sum or
 * mean aggregations take a register-file adjoint; the others take an LDS
 * adjoint holding N_max rows of 65 values and of 65 gradients. When that
 * exceeds the device's LDS (N_max above about 300 on MI355X) those other
 * genomes get NaN gradients (the call still returns TN_OK).
 */
int tn_backward(const tn_population* pop, const tn_transformed* tr,
                const float* obs, int64_t obs_genome_stride, int32_t B,
                const float* dY, int64_t dY_genome_stride,
                float* dW, float* db, hipStream_t stream);

/*
 * Forward pass, mean-squared-error loss and its gradient in one call:
 *   loss[g] = 1/(B*n_out) * sum_{b,j} (y[g][b][j] - target[b][j])^2
 * (target at target[g*target_genome_stride + b*n_out + j]), and dW / db as
 * tn_backward with dY = 2 (y - target) / (B*n_out). loss may be NULL.
 */
int tn_forward_backward_mse(const tn_population* pop, const tn_transformed* tr,
                            const float* obs, int64_t obs_genome_stride, int32_t B,
                            const float* target, int64_t target_genome_stride,
                            float* loss, float* dW, float* db, hipStream_t stream);

/* ---------------------------------------------------------- distance */

/*
 * Compatibility distance between every pair of genomes (Section 2.1,
 * Algorithm 1's species division; coefficients as in Appendix A). The
 * original NEAT form over connection genes:
 *   delta = c1 * E / N + c2 * D / N + c3 * Wbar
 * Genes are all valid connection rows (enabled or not) identified by the
 * marking (in-key, out-key), ordered lexicographically. Matching genes share a
 * marking; excess genes E are non-matching genes beyond the smaller of the two
 * genomes' largest markings (all genes of the other genome when one has none);
 * disjoint D are the other non-matching genes; Wbar is the mean |w1 - w2| over
 * matching genes (0 if none); N is the larger gene count; two empty genomes are
 * at distance 0. A genome with a repeated marking gets NaN distances and
 * counts of -1.
 *
 *   workspace  device buffer of tn_distance_workspace_size() bytes
 *   dist       [P][P] float32
 *   excess, disjoint  [P][P] int32, may be NULL (both or neither)
 */
int tn_distance_workspace_size(const tn_population* pop, size_t* bytes);

int tn_distance(const tn_population* pop, float c1, float c2, float c3,
                void* workspace, float* dist, int32_t* excess, int32_t* disjoint,
                hipStream_t stream);

/*
 * tn_distance without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, results (bit for bit) and kernels as
 * tn_distance, except that the workspace is a fixed device array inside the
 * library, TN_DISTANCE_NOALLOC_SCRATCH_BYTES large on every device the
 * library runs on (held until the process ends). The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *
 * Limit: a population whose workspace (tn_distance_workspace_size) exceeds
 * TN_DISTANCE_NOALLOC_SCRATCH_BYTES returns TN_EUNSUPPORTED and launches
 * nothing (16 MiB hold, e.g., 4096 genomes at C_max 256 or 1000 at C_max
 * 1024).
 *
 * Every call on one device shares that device's array: calls that overlap on
 * one device (on two streams, or from two host threads without ordering)
 * race and their results are undefined. Calls ordered on one stream are safe;
 * each call rewrites every entry it later reads, so nothing carries over
 * from the previous call.
 */
#define TN_DISTANCE_NOALLOC_SCRATCH_BYTES (16u << 20)

int tn_distance_noalloc(const tn_population* pop, float c1, float c2, float c3,
                        float* dist, int32_t* excess, int32_t* disjoint,
                        hipStream_t stream);

/*
 * Node-inclusive compatibility distance with the coefficient pair the paper
 * lists for its own speciation (Appendix A: compatibility_disjoint c_d and
 * compatibility_homologous c_h; Section 5.2 states that this distance is not
 * NEAT-Python's, and the paper prints no formula). Reading implemented here,
 * over node genes and connection genes alike:
 *   delta = delta_nodes + delta_conns
 *   delta_X = (c_d * D_X + c_h * H_X) / max(|X1|, |X2|)   (0 if both are empty)
 * Node genes are the valid non-input node rows, identified by key; connection
 * genes are the valid connection rows, enabled or not, identified by the
 * marking (in-key, out-key). D_X counts the genes only one of the two genomes
 * holds. H_X sums over the genes both hold, in ascending key / marking order,
 *   |bias1 - bias2| + |resp1 - resp2| + [act1 != act2] + [agg1 != agg2]  (nodes)
 *   |w1 - w2| + [enabled1 != enabled2]                                    (connections)
 * in float32. The matrix is symmetric bit for bit and its diagonal is 0. A
 * genome with a repeated node key or marking, or a ragged genome above
 * N_max / C_max, has no gene set: its distances are NaN and its counts -1.
 *
 *   workspace  device buffer of tn_distance_nodes_workspace_size() bytes
 *   dist       [P][P] float32
 *   d_nodes, d_conns  [P][P] int32 (D_nodes, D_conns), may be NULL (both or neither)
 * P <= 65535 (TN_EUNSUPPORTED above).
 */
int tn_distance_nodes_workspace_size(const tn_population* pop, size_t* bytes);

int tn_distance_nodes(const tn_population* pop, float c_disjoint, float c_homologous,
                      void* workspace, float* dist, int32_t* d_nodes, int32_t* d_conns,
                      hipStream_t stream);

/* ------------------------------------------------------- reproduction */

/*
 * Crossover and mutation of a padded population as the paper's tensorized row
 * operations (Section 3.2: a node or connection is added in the first empty
 * row, removed by emptying its row, and its attributes are changed in place;
 * the hyperparameters are those of Appendix A, defaults in Appendix C). The
 * random draws are inputs: the children are a pure function of the parents
 * and the draws. Per child c, with parents a = parents[c][0] (the fitter one)
 * and b = parents[c][1]:
 *
 *  1. Crossover (NEAT's alignment by historical marking, Section 2.1): the
 *     child takes a's rows in a's positions. A node row of a whose key b also
 *     holds, and a connection row whose marking (in-key, out-key) b also
 *     holds, takes b's attributes (bias, response, act, agg; weight, enabled)
 *     when its coin is below 1/2 (b's first row with that key / marking).
 *     Genes only b holds are not inherited.
 *  2. Add node (draw below node_add): an enabled connection x -> y is picked
 *     and disabled; a new node takes the first empty node row with the key the
 *     call's innovation table gives (x, y), bias and response drawn from their
 *     initial distributions, act_default / agg_default; x -> new (weight 1) and
 *     new -> y (the old weight), enabled, take the first two empty connection
 *     rows. Skipped when no enabled connection, node row or two connection
 *     rows are free.
 *  3. Delete node (node_delete): a hidden node row is emptied with every
 *     connection row naming its key.
 *  4. Add connection (conn_add): a source among the input and hidden node rows
 *     and a destination among the hidden and output node rows are picked; the
 *     connection takes the first empty row, enabled, weight from its initial
 *     distribution, unless source = destination, the marking is present
 *     (enabled or not), no row is free, or (allow_cycles = 0) the destination
 *     reaches the source over valid connections.
 *  5. Delete connection (conn_delete): a valid connection row is emptied.
 *  6. Attributes of every valid non-input node row and valid connection row:
 *     a float attribute v with uniform u and normal z becomes v + power*z when
 *     u < mutate_rate, init_mean + init_std*z when u < mutate_rate +
 *     replace_rate, else stays; an act (agg) code is replaced, when its draw
 *     is below act_replace_rate (agg_replace_rate), by option
 *     floor(u2 * n_options) of the ascending option list.
 * "Picked" = candidate rows in ascending row order, index floor(u * n) (the
 * product rounded to float32), at most n - 1. Every float update rounds each
 * product and sum to float32 on its own (no fused multiply-add).
 *
 * Draws per child (tn_reproduce_draws gives the counts): uniforms U [n][nU]
 *   U[0..8]  add node: decision, pick; delete node: decision, pick; add
 *            connection: decision, source pick, destination pick; delete
 *            connection: decision, pick (U[9..15] unused)
 *   U[16 + r]                  crossover coin of node row r
 *   U[16 + N_max + r]          crossover coin of connection row r
 *   U[16 + N_max + C_max + 6r + k]  node row r: bias, response, act decision,
 *                              act pick, agg decision, agg pick
 *   U[16 + 7 N_max + C_max + r]     connection row r weight
 * normals Z [n][nZ]: Z[0] new node bias, Z[1] new node response, Z[2] new
 *   connection weight, Z[4 + 2r + k] node row r bias (k = 0) / response (1),
 *   Z[4 + 2 N_max + r] connection row r weight.
 *
 * Innovation table of one call: the distinct split markings among the
 * children get keys next_key + their rank in lexicographic order (one split
 * done by several children gives them one key); next_key must exceed every key
 * in the parents and next_key + n must stay below 2^31 (neither is checked).
 * *next_key_out (device int32) receives the next unused key.
 *
 *   pop        padded parent population (ragged: TN_EUNSUPPORTED)
 *   parents    device int32 [n][2]. A first parent outside [0, P) gives an
 *              all-empty child; a second parent outside [0, P) (e.g. -1) makes
 *              the child an unchanged copy of the first (an elite).
 *   U, Z       device float32 as above
 *   children   device arrays [n][N_max] / [n][C_max] (same capacities as pop);
 *              must not overlap the parents' arrays
 *   workspace  tn_reproduce_workspace_size(n) bytes of device memory
 * TN_EINVAL for null pointers, n < 0, probabilities outside [0, 1], an option
 * list that is empty, longer than 8 or not strictly ascending, or a default
 * code above 255; TN_EUNSUPPORTED when N_max / C_max exceed what one
 * workgroup's LDS holds.
 */
typedef struct tn_mutation_params {
    float node_add, node_delete, conn_add, conn_delete;
    float bias_init_mean, bias_init_std, bias_mutate_power, bias_mutate_rate, bias_replace_rate;
    float resp_init_mean, resp_init_std, resp_mutate_power, resp_mutate_rate, resp_replace_rate;
    float weight_init_mean, weight_init_std, weight_mutate_power, weight_mutate_rate,
          weight_replace_rate;
    float act_replace_rate, agg_replace_rate;
    int32_t act_default, agg_default;
    int32_t n_act_options, n_agg_options;
    uint8_t act_options[8];   /* ascending activation codes */
    uint8_t agg_options[8];   /* ascending aggregation codes */
    int32_t allow_cycles;     /* 0: feedforward genomes (cycle check on add connection) */
} tn_mutation_params;

/* Draw counts per child: *n_uniform = 16 + 7 N_max + 2 C_max,
 * *n_normal = 4 + 2 N_max + C_max. Host only. */
int tn_reproduce_draws(int32_t N_max, int32_t C_max, int32_t* n_uniform, int32_t* n_normal);

int tn_reproduce_workspace_size(int32_t n_children, size_t* bytes);

int tn_reproduce(const tn_population* pop, int32_t n_children, const int32_t* parents,
                 const float* U, const float* Z, const tn_mutation_params* params,
                 int32_t next_key, const tn_population_arrays* children, int32_t* next_key_out,
                 void* workspace, hipStream_t stream);

/* ------------------------------------------------------- NEAT generation */

/*
 * One generation of NEAT on a padded population (Algorithm 1's loop body:
 * divide the population into species by the distances between networks,
 * determine each species' number of new networks from the fitness, generate
 * them by crossover and mutation), with the hyperparameters of Appendix A.
 * The paper names these steps but not their rules; implemented here:
 *
 *  1. Speciation by the node-inclusive distance of tn_distance_nodes (c_d =
 *     compatibility_disjoint, c_h = compatibility_homologous), evaluated in
 *     float32 in ascending key order: every genome joins the alive species
 *     whose representative is nearest if below compatibility_threshold (ties:
 *     lowest slot); the others, in genome order, join the nearest species
 *     founded earlier in this call if below the threshold, else found one in
 *     the lowest free slot; with no free slot left, they join the nearest
 *     alive species whatever the distance (NaN counts as infinite).
 *  2. Species fitness = largest member fitness; it improves when above the
 *     slot's best. Stagnant (no improvement for max_stagnation generations)
 *     species get no children, except the species_elitism species of largest
 *     fitness.
 *  3. Children of each surviving species (float32, slot order): af = (mean
 *     member fitness - lo) / max(hi - lo, 1) over surviving members' range;
 *     target = P af / sum af; spawn = size + (target - size) *
 *     spawn_number_change_rate (size = last generation's children, 0 for a new
 *     species); share = spawn P / sum spawn; counts = floor(share), the rest
 *     one each by largest remainder (ties: lowest slot); the counts sum to P.
 *  4. Parents, children laid out by slot then rank: members ranked by fitness
 *     (largest first, ties lower index); the first min(genome_elitism, count,
 *     members) children copy ranks 0.. unchanged; each other child c takes
 *     ranks floor(sel[c][k] * m) (k = 0, 1) among the m = max(1,
 *     ceil(survival_threshold * members)) best, the fitter first.
 *  5. Children by tn_reproduce with U, Z, next_key (next_key_out as there).
 *  6. The table: surviving species with children keep their slot, rank-0
 *     member as representative, their count as size; the other slots are freed.
 *
 *   pop          padded population (ragged: TN_EUNSUPPORTED), P >= 1
 *   fitness      device float32 [P], finite (non-finite values give
 *                unspecified but in-range species and counts)
 *   generation   the generation index (stagnation clock)
 *   table        device species table (tn_species_table), read and updated
 *   sel          device float32 [P][2] selection uniforms in [0, 1)
 *   U, Z         reproduction draws as tn_reproduce
 *   children     device [P][N_max] / [P][C_max] arrays (not overlapping pop)
 *   species_of   device int32 [P] or NULL: the slot each genome joined
 *   parents      device int32 [P][2] or NULL: the parent pairs used
 *   workspace    tn_neat_workspace_size bytes
 * TN_EINVAL for bad parameters (max_species outside 1..TN_NEAT_MAX_SPECIES,
 * species_elitism < 1, max_stagnation < 1, genome_elitism < 0,
 * survival_threshold outside (0, 1], spawn rate outside [0, 1], a negative or
 * non-finite threshold or coefficient, mutation parameters as tn_reproduce).
 */
#define TN_NEAT_MAX_SPECIES 64

typedef struct tn_neat_params {
    float   compatibility_threshold;
    float   compatibility_disjoint;
    float   compatibility_homologous;
    int32_t max_species;
    int32_t species_elitism;
    int32_t max_stagnation;
    int32_t genome_elitism;
    float   survival_threshold;
    float   spawn_number_change_rate;
    tn_mutation_params mutation;
} tn_neat_params;

/* Species table, device arrays owned by the caller: max_species slots. */
typedef struct tn_species_table {
    int32_t max_species;
    tn_population_arrays reps;   /* representatives, [max_species][N_max] / [max_species][C_max] */
    int32_t* alive;              /* [max_species] 1 for a slot in use                       */
    float*   best;               /* [max_species] best species fitness so far               */
    int32_t* last_improved;      /* [max_species] generation of the last improvement        */
    int32_t* size;               /* [max_species] children given in the last generation     */
} tn_species_table;

/* The initial population (Algorithm 1's first step): genome g holds the
 * input and output nodes (keys 0 .. n_in + n_out - 1) in its first node rows and
 * every input -> output connection, enabled, in row i * n_out + o; node bias
 * and response and connection weights are init_mean + init_std * z with the
 * normals Z [P][n_normal] in tn_reproduce's layout (Z[4 + 2r + k] for node row
 * r, Z[4 + 2 N_max + r] for connection row r); act / agg the defaults. The
 * other rows are empty. table (may be NULL) is cleared: no slot alive.
 * Needs n_in + n_out <= N_max and n_in * n_out <= C_max. */
int tn_neat_init(int32_t P, int32_t n_in, int32_t n_out, int32_t N_max, int32_t C_max,
                 const float* Z, const tn_mutation_params* mutation,
                 const tn_population_arrays* out, const tn_species_table* table,
                 hipStream_t stream);

int tn_neat_workspace_size(const tn_population* pop, int32_t max_species, size_t* bytes);

int tn_neat_generation(const tn_population* pop, const float* fitness, int32_t generation,
                       const tn_neat_params* params, const tn_species_table* table,
                       const float* sel, const float* U, const float* Z, int32_t next_key,
                       const tn_population_arrays* children, int32_t* species_of,
                       int32_t* parents, int32_t* next_key_out, void* workspace,
                       hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TENSORNEAT_HIP_H */
