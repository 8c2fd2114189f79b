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
  // parity hook: when apply_mask is set (trace_f unset) only the terms t of
  // [t_begin, t_end) with apply_mask[t - t_begin] != 0 are applied
  const uint8_t* apply_mask;
};

// gfx950: 8 XCDs; blocks are dispatched to them round-robin (block b on XCD b mod 8).
constexpr uint32_t kXcds = 8;

size_t layout_lds_bytes(uint32_t path_slots, uint32_t W);
hipError_t launch_layout_iter(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
hipError_t launch_layout_reuse(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
hipError_t launch_apply_terms(const StepRec* rec, float2* work, float eta, const uint64_t* i, const uint64_t* j,
                              const uint8_t* f, uint64_t count, hipStream_t s);
// boundary layout [2][n][2] (caller's node ids) <-> interleaved working copy
// [n][2](x, y) (device node ids); inv[m] = caller id of device node m, or
// NULL when the two orders are the same
hipError_t launch_to_work(const float* coords, float2* work, uint64_t n_nodes, const uint32_t* inv, hipStream_t s);
hipError_t launch_from_work(const float2* work, float* coords, uint64_t n_nodes, const uint32_t* inv, hipStream_t s);
const void* layout_iter_kernel();
// Error reporting shared by the host files (capi.hip): set_error stores the
// calling thread's pgsgd_last_error() message and returns `code`;
// clear_error empties it and returns PGSGD_OK.
int32_t set_error(int32_t code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int32_t clear_error();
// fill kernel (stress_kernels.hip): p[0..n) = v, also inside captured HIP graphs
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);

}  // namespace pgsgd
