// Batched form of the PG-SGD layout for gfx950: one persistent launch per
// iteration covers the terms of many graphs.
//
// A work item is a run of groups_per_item consecutive 64-term groups of one
// graph; wave w takes items w, w + waves, ...  Items are ordered in `phases`
// phases: phase r holds, graph after graph, the r-th 1/phases share of every
// graph's items.  With one phase the graphs are processed one after another
// (the coordinates of the graph in progress stay in the 256 MB Infinity Cache,
// which on MI355X makes this the fastest order); more phases spread the
// concurrent updates over several graphs.  The segment (phase, graph) of an
// item is found by binary search over the segment prefix in LDS, next to the
// per-graph headers and path offsets.  The sampled terms do not depend on the
// tune (bit-exact with the plain kernel for the same graph_id).
#include "batch.h"
#include "device.h"

namespace pgsgd {

__global__ __launch_bounds__(1024) void k_layout_batch(BatchLaunch P) {
  extern __shared__ __align__(16) char lds[];
  const uint32_t n_seg = P.phases * P.n_graphs;
  BatchGraph* hdr = reinterpret_cast<BatchGraph*>(lds);
  uint64_t* seg_off = reinterpret_cast<uint64_t*>(lds + sizeof(BatchGraph) * P.n_graphs);
  uint64_t* off = seg_off + (n_seg + 1);
  uint32_t* zipf = reinterpret_cast<uint32_t*>(off + P.path_slots_total);
  uint16_t* guide = reinterpret_cast<uint16_t*>(zipf + (P.W + 1));

  for (uint32_t k = threadIdx.x; k < P.n_graphs; k += blockDim.x) {
    BatchGraph h = P.graphs[k];
    h.eta = P.eta_all[(size_t)k * P.n_iters + P.iter];
    hdr[k] = h;
  }
  for (uint32_t k = threadIdx.x; k <= n_seg; k += blockDim.x) seg_off[k] = P.seg_off[k];
  for (uint32_t k = threadIdx.x; k < P.path_slots_total; k += blockDim.x) off[k] = P.path_blob[k];
  for (uint32_t k = threadIdx.x; k <= P.W; k += blockDim.x) zipf[k] = P.zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) guide[k] = P.guide[k];
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = (uint64_t)blockIdx.x * (blockDim.x >> 6) + uniform_u32(threadIdx.x >> 6);
  const uint64_t n_items = seg_off[n_seg];
  for (uint64_t it = wave0; it < n_items; it += P.wave_stride) {
    // segment of this item: largest s with seg_off[s] <= it
    uint32_t lo = 0, hi = n_seg - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (seg_off[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t seg = uniform_u32(lo);
    const uint32_t gk = seg % P.n_graphs;
    const uint32_t phase = seg / P.n_graphs;
    const BatchGraph& H = hdr[gk];
    LdsView L;
    L.off = off + H.path_base;
    L.zipf = zipf;
    L.guide = guide;
    float2* __restrict__ W = H.work;
    const uint64_t local = (phase * H.n_items) / P.phases + (it - seg_off[seg]);
    const uint64_t g0 = local * P.groups_per_item;
    const uint64_t g1 = min(g0 + P.groups_per_item, H.n_groups_run);
    for (uint64_t g = g0; g < g1; ++g) {
      const uint64_t t = g * 64 + lane;
      const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), P.iter, H.c3, P.k0, P.k1);
      const uint32_t lead = uniform_u32(r.r3);
      const bool cooling = P.cool_all || ((lead >> 3) & 1u);
      if (t >= H.n_terms) continue;
      Term T = sample_term(r, cooling, H.S, L, H.path_top, P.W);
      if (H.trace_f) {  // parity hook: record the term instead of applying it
        if (!(T.flags & 8u)) {
          uint64_t a, b;
          float d;
          if (!resolve_term(H.rec, T, a, b, d)) T.flags |= 8u;
        }
        H.trace_i[t] = T.i;
        H.trace_j[t] = T.j;
        H.trace_f[t] = (uint8_t)T.flags;
        continue;
      }
      if (T.flags & 8u) continue;
      uint64_t a, b;
      float d;
      if (!resolve_term(H.rec, T, a, b, d)) continue;
      apply_update(W, a, b, d, H.eta);
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t batch_lds_bytes(uint32_t n_graphs, uint32_t phases, uint32_t path_slots_total, uint32_t W) {
  return sizeof(BatchGraph) * n_graphs + (size_t)(phases * n_graphs + 1) * 8 + (size_t)path_slots_total * 8 +
         (size_t)(W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
}

hipError_t launch_layout_batch(const BatchLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(k_layout_batch, dim3(blocks), dim3(threads),
                     batch_lds_bytes(P.n_graphs, P.phases, P.path_slots_total, P.W), s, P);
  return hipGetLastError();
}

const void* layout_batch_kernel() { return reinterpret_cast<const void*>(&k_layout_batch); }

}  // namespace pgsgd
