// Internal interface between the C-ABI host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgsgd {

struct StepRec;

// Arguments of one plain layout launch (one iteration of one graph).
struct LayoutLaunch {
  const StepRec* rec;
  float2* work;            // interleaved coordinates: [n_nodes][2 endpoints](x, y)
  const uint64_t* path_off;
  const uint32_t* zipf;
  const uint16_t* guide;
  uint64_t n_nodes;
  uint64_t S;
  uint64_t n_terms;
  uint64_t n_groups;
  uint64_t wave_stride;    // waves in the grid
  uint32_t n_paths;
  uint32_t path_slots;     // LDS entries for offsets: 2 * path_top
  uint32_t path_top;       // largest power of two <= n_paths
  uint32_t W;
  uint32_t iter;
  uint32_t cool_all;
  uint32_t c3;             // stream << 24 | graph_id
  uint32_t k0, k1;         // Philox key
  float eta;
  uint32_t drf;            // data reuse: updates per sampled term (1 = off)
  // term range [t_begin, t_end) of this launch, as 64-term groups [g_begin, g_end)
  uint64_t t_begin, t_end;
  uint64_t g_begin, g_end;
  // parity hook: when trace_f is set the terms are recorded (index t - t_begin)
  // instead of applied
  uint64_t* trace_i;
  uint64_t* trace_j;
  uint8_t* trace_f;
  uint8_t* trace_o;        // data reuse: offsets o_1..o_{drf-1} per group
};

// Binned processing of one iteration (binned_kernels.hip): terms are binned by
// the window of 2^win_shift consecutive steps holding their step i and the
// windows are processed XCD by XCD.
constexpr uint32_t kXcds = 8;                 // gfx950: 8 XCDs, blocks dispatched round-robin
constexpr uint32_t kMaxBinWindows = 8192;     // LDS histogram of 32 KB
constexpr uint64_t kBinChunk = 1ull << 30;    // terms per binning pass (4-byte offsets, bit 31 = coin)

struct BinLaunch {
  LayoutLaunch L;          // sampling parameters, coordinates, trace pointers
  uint64_t c0, c1;         // term chunk [c0, c1), c0 a multiple of 64
  uint32_t n_win;          // ceil(S / 2^win_shift)
  uint32_t win_shift;
  uint32_t count_blocks;   // grid of the count and scatter kernels
  uint32_t xstride;        // row length of xitem
  uint16_t* tag;           // [chunk] window | coin << 15
  uint32_t* entries;       // [chunk] term offset | coin << 31, window-contiguous
  uint32_t* wcount;        // [n_win] histogram (zero between chunks)
  uint32_t* woff;          // [n_win + 1] window offsets
  uint32_t* cursor;        // [n_win] scatter cursors
  uint32_t* xitem;         // [kXcds][xstride] prefix of 64-term items over the windows of each XCD
};

// Stress kernels (sampled path stress, differentiable loss).
struct StressLaunch {
  const StepRec* rec;
  const float* coords;
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
};

size_t layout_lds_bytes(uint32_t path_slots, uint32_t W);
hipError_t launch_layout_iter(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
hipError_t launch_layout_reuse(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
hipError_t launch_apply_terms(const StepRec* rec, float2* work, float eta, const uint64_t* i, const uint64_t* j,
                              const uint8_t* f, uint64_t count, hipStream_t s);
// boundary layout [2][n][2] <-> interleaved working copy [n][2](x, y)
hipError_t launch_to_work(const float* coords, float2* work, uint64_t n_nodes, hipStream_t s);
hipError_t launch_from_work(const float2* work, float* coords, uint64_t n_nodes, hipStream_t s);
const void* layout_iter_kernel();
hipError_t launch_bin_count_scan_scatter(const BinLaunch& B, hipStream_t s);
hipError_t launch_bin_layout(const BinLaunch& B, uint32_t blocks, hipStream_t s);
const void* bin_layout_kernel();

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
hipError_t launch_path_stress_exact(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s);
hipError_t launch_stress_fwd(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s);
hipError_t launch_stress_bwd(const StressLaunch& P, const float* grad_out, const uint64_t* n_valid, float* grad,
                             hipStream_t s);
hipError_t launch_init_coords(const StepRec* rec, const uint64_t* first_step, uint64_t n_nodes, uint32_t k0,
                              uint32_t k1, uint32_t c3, float jitter, float* coords, hipStream_t s);
hipError_t launch_first_visit(const StepRec* rec, uint64_t S, uint64_t n_nodes, uint64_t* first_step,
                              hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_adam(float* x, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);

}  // namespace pgsgd
