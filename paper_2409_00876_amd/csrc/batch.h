// Batched form: the structures shared by the host runtime and k_layout_batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pgsgd {

// Per-graph header of the batched launch.
struct BatchGraph {
  const StepRec* rec;
  float2* work;            // interleaved coordinates of this graph
  uint64_t n_nodes;
  uint64_t S;
  uint64_t n_terms;
  uint64_t n_groups_run;   // groups processed (all, except in tuning runs)
  uint64_t n_items;        // ceil(n_groups_run / groups_per_item)
  uint32_t path_base;      // index of this graph's offsets in the path blob
  uint32_t path_top;
  uint32_t c3;
  float eta;               // filled per iteration from eta_all
  // parity hook: when trace_f is set the terms are recorded (index t) instead
  // of applied
  uint64_t* trace_i;
  uint64_t* trace_j;
  uint8_t* trace_f;
};

struct BatchLaunch {
  const BatchGraph* graphs;
  const uint64_t* seg_off;     // phases * n_graphs + 1 segment prefix (segment = phase * n + graph)
  const uint64_t* path_blob;   // padded offsets of all graphs
  const float* eta_all;        // [n_graphs][n_iters]
  const uint32_t* zipf;
  const uint16_t* guide;
  uint64_t wave_stride;
  uint64_t groups_per_item;
  uint32_t n_graphs;
  uint32_t path_slots_total;
  uint32_t W;
  uint32_t n_iters;
  uint32_t iter;
  uint32_t cool_all;
  uint32_t k0, k1;
  uint32_t phases;             // work-item phases (see batch_kernels.hip)
};

constexpr uint32_t kMaxBranches = 16;  // windowed batches: concurrent branches of the HIP graph
constexpr uint32_t kAutoBranches = 4;

size_t batch_lds_bytes(uint32_t n_graphs, uint32_t phases, uint32_t path_slots_total, uint32_t W);
hipError_t launch_layout_batch(const BatchLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
const void* layout_batch_kernel();

}  // namespace pgsgd
