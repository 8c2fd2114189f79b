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
// fill kernel (stress_kernels.hip): p[0..n) = v, also inside captured HIP graphs
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);

}  // namespace pgsgd
