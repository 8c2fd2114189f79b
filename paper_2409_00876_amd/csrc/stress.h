// Stress kernels (sampled path stress, exact path stress, differentiable loss)
// and the utility kernels of stress_kernels.hip: launch arguments and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pgsgd {

constexpr uint32_t kStreamSpsSlot = 6;  // Philox stream of the window-major sampled path stress slots
constexpr uint32_t kStreamLossSlot = 7; // Philox stream of the window-major loss slots

struct StressLaunch {
  const StepRec* rec;
  const float* coords;
  const float2* work;      // interleaved copy of coords (sampled path stress only)
  const uint32_t* inv;     // renumbered graph: caller id of every device node id (else NULL)
  const float2* work2;     // a second layout's interleaved copy: the SPS passes evaluate it on the same pairs
  const uint64_t* path_off;
  const uint32_t* zipf;
  const uint16_t* guide;
  uint64_t n_nodes;
  uint64_t S;
  uint64_t count;          // steps (SPS) or pairs (loss)
  uint32_t m;              // SPS pairs per step
  uint32_t n_paths;
  uint32_t path_slots;
  uint32_t path_top;
  uint32_t W;
  uint32_t word2;          // counter word 2
  uint32_t c3;
  uint32_t k0, k1;
  // pass 1 of the sampled path stress, when out_count is set: pairs with stress
  // above out_threshold are appended (i, j, e_i | e_j << 1, stress; the first
  // out_max kept) and counted in *out_count
  uint64_t* out_count;
  uint64_t out_max;
  double out_threshold;
  uint64_t* out_i;
  uint64_t* out_j;
  uint8_t* out_e;
  double* out_s;
};

// SPS: pass 1 writes per-block (sum, n_valid, n_skipped); pass 2 per-block sum
// of squared deviations from mean_dev.  Final reductions write to out.
constexpr uint32_t kStressBlocks = 2048;
constexpr uint32_t kStressThreads = 256;
hipError_t launch_sps_pass(const StressLaunch& P, int pass, int mode, const double* mean_dev, double* part_f,
                           uint64_t* part_n, uint64_t* part_skip, hipStream_t s);
// out_f[0] = sum of part_f; out_n[0..1] = sums of part_n / part_skip;
// if mean_out: mean_out[0] = out_f[0] / out_n[0].
hipError_t launch_reduce_parts(const double* part_f, const uint64_t* part_n, const uint64_t* part_skip,
                               uint32_t n_parts, double* out_f, uint64_t* out_n, double* mean_out,
                               float* loss_out, uint64_t* n_valid_out, hipStream_t s);
// Sampled path stress in window-major order: segments (the windows of
// 2^win_shift steps cut at path boundaries, in step order) get the counts of
// the plain pair draws that fall in them; each segment's slots draw their pair
// inside it.  Runs: XCD x takes the segments [sbeg[x], sbeg[x + 1]).
struct SpsWinLaunch {
  StressLaunch P;             // rec, work, path_off, S, m, path table, c3 of the plain pair draws, key
  uint32_t slot_c3;           // Philox word 3 of the slot draws
  uint32_t win_shift;
  uint32_t n_seg;
  uint32_t xstride;           // row length of xitem
  uint32_t count_blocks;
  const uint64_t* seg_start;  // [n_seg + 1], seg_start[n_seg] = S
  const uint32_t* seg_path;   // [n_seg]
  const uint32_t* wseg;       // [n_win + 1] first segment of every window
  uint32_t* count;            // [n_seg] histogram (zeroed again by the scan)
  uint64_t* seg_off;          // [n_seg + 1] first slot of every segment
  const uint32_t* sbeg;       // [kXcds + 1] first segment of every run
  uint64_t* xitem;            // [kXcds][xstride] prefix of 64-slot items over the segments of each run
  uint64_t* queue;            // [2][kXcds][16] item counters of the two passes (zeroed by the scan)
  uint64_t loss_pairs;        // the loss's window-major pairs (reading R22): the number of plain pairs; 0 = SPS
};
hipError_t launch_sps_win_count_scan(const SpsWinLaunch& W, hipStream_t s);
// grid: blocks a multiple of kXcds
hipError_t launch_sps_win_pass(const SpsWinLaunch& W, int pass, const double* mean_dev, double* part_f,
                               uint64_t* part_n, uint64_t* part_skip, uint32_t blocks, hipStream_t s);
// The loss (reading R22) over the segments' slots counted with loss_pairs:
// forward per-block sums (grid: blocks a multiple of kXcds), and the adjoint
// added into the planar gradient.
hipError_t launch_loss_win_fwd(const SpsWinLaunch& W, double* part_f, uint64_t* part_n, uint32_t blocks,
                               hipStream_t s);
hipError_t launch_loss_win_bwd(const SpsWinLaunch& W, const float* grad_out, const uint64_t* n_valid, float* grad,
                               uint32_t blocks, hipStream_t s);
// The loss adjoint by tiles: block b takes tiles from *queue (zero at
// launch); tile t covers the segments seg[off[t] .. off[t + 1]) (at most
// kTileMaxSeg) and accumulates the gradient of device node ids [base[t],
// base[t] + 2 * kTileNodes) in LDS, flushed with one atomic add per touched
// entry; other endpoints are added directly.  The pairs are the window-major
// loss pairs of W, the same slots as launch_loss_win_bwd.
constexpr uint32_t kTileNodes = 2048;
constexpr uint32_t kTileMaxSeg = 256;
constexpr uint32_t kTileThreads = 512;
struct TileLaunch {
  const uint32_t* seg;
  const uint32_t* off;
  const uint32_t* base;
  uint32_t n_tiles;
  uint32_t* queue;
};
hipError_t launch_loss_tile_bwd(const SpsWinLaunch& W, const TileLaunch& T, const float* grad_out,
                                const uint64_t* n_valid, float* grad, uint32_t blocks, hipStream_t s);
// The forward pass over the same tiles: per-block sums into part_f / part_n[0 .. blocks).
hipError_t launch_loss_tile_fwd(const SpsWinLaunch& W, const TileLaunch& T, double* part_f, uint64_t* part_n,
                                uint32_t blocks, hipStream_t s);
size_t loss_tile_lds_bytes(uint32_t W, bool grad);  // dynamic LDS of k_loss_tile
constexpr size_t kTileStaticLds = 9 * 1024;   // static LDS of k_loss_tile (a tile's segment table), rounded up
// out[g] = the lowest device node id over the steps [start[g], start[g + 1])
hipError_t launch_segment_min_node(const StepRec* rec, const uint64_t* start, uint32_t nseg, uint32_t* out,
                                   hipStream_t s);
hipError_t launch_path_stress_exact(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s);
hipError_t launch_stress_fwd(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s);
hipError_t launch_stress_bwd(const StressLaunch& P, const float* grad_out, const uint64_t* n_valid, float* grad,
                             hipStream_t s);
hipError_t launch_init_coords(const StepRec* rec, const uint64_t* first_step, uint64_t n_nodes, const uint32_t* inv,
                              uint32_t k0, uint32_t k1, uint32_t c3, float jitter, float* coords, hipStream_t s);
hipError_t launch_first_visit(const StepRec* rec, uint64_t S, uint64_t n_nodes, uint64_t* first_step,
                              hipStream_t s);
hipError_t launch_adam(float* x, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);

}  // namespace pgsgd
