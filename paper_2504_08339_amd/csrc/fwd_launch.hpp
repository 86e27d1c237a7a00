// Host-side launchers of the forward kernels, shared by the C entry points and
// the batched plan.
#pragma once

#include "tn_internal.hpp"

namespace tn {

// Where a launch's genomes come from.
struct FwdWork {
  const int32_t* genomes = nullptr;  // device list of genome indices (nullptr: all P, in order)
  int n_genomes = 0;                 // list length
  int32_t* queue = nullptr;          // persistent form: device counters, 0 at launch (8 for the
                                     // register engine: one per XCD share; 1 for the LDS engine)
  int grid = 0;                      // persistent form: workgroups
};

// Register engine (forward_reg.hip).
struct RegTile {
  int waves = 4;            // wavefronts per workgroup (1..8)
  int rf = 64;              // rows per tile of the register file (32, 64, 96, 128, 160,
                            // 200: one tile of 64 observations per wavefront; 100: two;
                            // 50: four)
  int rows_lo = -1;         // genomes with prog_rows <= rows_lo are skipped
  bool skip_above = false;  // genomes with prog_rows > rf are skipped (else NaN)
};

// Level-parallel LDS engine (forward.hip).
// Wavefronts per workgroup it allows: 16 at one observation per lane (the
// kernel then fits 128 registers, four wavefronts per SIMD), else 8.
constexpr int lds_max_waves(int K) { return K <= 1 ? 16 : 8; }
struct LdsTile {
  int K = 1;          // observations per lane (1, 2, 4)
  int waves = 4;      // wavefronts per workgroup (1..lds_max_waves(K))
  int rows = 0;       // value rows per tile (0: N_max)
  int skip_le = -1;   // genomes with prog_rows <= skip_le are skipped
};

// Register-file sizes (rows per tile) the automatic engine choice and plans
// use for B observations per genome, smallest first: files that hold several
// tiles per wavefront when B spans that many tiles.
inline int reg_classes(int B, int (&cls)[6]) {
  const int tiles = (B + 63) / 64;
  int n = 0;
  if (tiles >= 4) {
    for (int r : {50, 100, 128, 160, 200}) cls[n++] = r;
  } else if (tiles >= 2) {
    for (int r : {100, 128, 160, 200}) cls[n++] = r;
  } else {
    for (int r : {32, 64, 96, 128, 160, 200}) cls[n++] = r;
  }
  return n;
}
constexpr int kRegRowsMax = 200;  // largest register file (rows per tile)

int launch_forward_reg(const tn_population& p, const tn_transformed& t, const float* obs,
                       int64_t obs_stride, int B, float* out, const RegTile& tile,
                       const FwdWork& work, hipStream_t stream);
// Forward pass with the squared-error epilogue on the register file of rf rows
// (one workgroup per genome; genomes outside (rows_lo, rf] skipped when
// skip_above).
int launch_forward_loss_reg(const tn_population& p, const tn_transformed& t, const float* obs,
                            int64_t obs_stride, int B, const float* target,
                            int64_t target_stride, float scale, float offset, float* out,
                            float* loss, int waves, int rf, int rows_lo, bool skip_above,
                            hipStream_t stream);
// Resident workgroups (whole device) of the persistent register kernel of a
// register-file size.
int reg_queue_grid(int variant, int waves, int n_in);

int launch_forward(const tn_population& p, const tn_transformed& t, const float* obs,
                   int64_t obs_stride, int B, float* out, const LdsTile& tile,
                   const FwdWork& work, hipStream_t stream);
int launch_forward_loss(const tn_population& p, const tn_transformed& t, const float* obs,
                        int64_t obs_stride, int B, const float* target, int64_t target_stride,
                        float scale, float offset, float* out, float* loss, int skip_le,
                        hipStream_t stream);
// Largest row count the LDS engine holds at one observation per lane.
int lds_rows_cap(const tn_population& p);
// LDS bytes of one workgroup of the LDS engine (0 if the tile does not fit).
size_t lds_tile_bytes(const tn_population& p, int K, int rows);
// Resident workgroups (whole device) of the persistent LDS kernel.
int lds_queue_grid(const tn_population& p, int K, int waves, int rows);

}  // namespace tn
