// PG-SGD layout kernels for gfx950: one launch per iteration of Alg. 1.
//
//   k_layout_iter   all terms of one iteration, fused: draw, sample, gather,
//                   update, scatter (the hot path); with trace pointers set it
//                   records the sampled terms instead (parity checks)
//   k_apply_terms   the update alone on given terms
//   k_layout_batch  the persistent multi-graph form of k_layout_iter
//
// Work mapping: a wavefront owns aligned groups of 64 consecutive terms, lane
// l doing term 64g+l.  The cooling coin of a group is bit 3 of word 3 of its
// first term's draw, read from lane 0 with readfirstlane, so the cooling branch
// is wave-uniform by construction (the paper's warp merging, here part of the
// sampling definition rather than a scheduling trick).
#include "device.h"
#include "internal.h"

namespace pgsgd {

// LDS image shared by the layout kernels: padded path offsets, then the
// power-law table C[0..W], then its guide (kGuideSize+1 entries).
struct LdsView {
  uint64_t* off;
  uint32_t* zipf;
  uint16_t* guide;
};

__device__ __forceinline__ LdsView lds_view(char* base, uint32_t path_slots, uint32_t W) {
  LdsView v;
  v.off = reinterpret_cast<uint64_t*>(base);
  v.zipf = reinterpret_cast<uint32_t*>(base + (size_t)path_slots * 8);
  v.guide = reinterpret_cast<uint16_t*>(base + (size_t)path_slots * 8 + (size_t)(W + 1) * 4);
  return v;
}

__device__ __forceinline__ void lds_fill(const LdsView& v, const uint64_t* __restrict__ path_off, uint32_t n_paths,
                                         uint32_t path_slots, const uint32_t* __restrict__ zipf,
                                         const uint16_t* __restrict__ guide, uint32_t W) {
  for (uint32_t k = threadIdx.x; k < path_slots; k += blockDim.x) v.off[k] = k <= n_paths ? path_off[k] : ~0ull;
  for (uint32_t k = threadIdx.x; k <= W; k += blockDim.x) v.zipf[k] = zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) v.guide[k] = guide[k];
}

// Sampling of term t (all integer): step, path, partner, flags.
__device__ __forceinline__ Term sample_term(const Rand4& r, bool cooling, uint64_t S, const LdsView& L,
                                            uint32_t path_top, uint32_t W) {
  Term T;
  T.i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), S);
  const uint32_t p = find_path(L.off, path_top, T.i);
  const uint64_t start = L.off[p];
  const uint64_t len = L.off[p + 1] - start;
  bool ok = true;
  if (cooling) {
    ok = partner_power_law(T.i, start, len, r.r2, r.r3, L.zipf, L.guide, W, T.j);
  } else {
    T.j = start + mulhi32(r.r2, (uint32_t)len);
  }
  T.flags = (r.r3 & 3u) | ((cooling ? 1u : 0u) << 2) | ((ok ? 0u : 1u) << 3);
  return T;
}

__global__ __launch_bounds__(256) void k_layout_iter(LayoutLaunch P) {
  extern __shared__ __align__(16) char lds[];
  const LdsView L = lds_view(lds, P.path_slots, P.W);
  lds_fill(L, P.path_off, P.n_paths, P.path_slots, P.zipf, P.guide, P.W);
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = (uint64_t)blockIdx.x * (blockDim.x >> 6) + uniform_u32(threadIdx.x >> 6);
  float2* __restrict__ W = P.work;
  for (uint64_t g = P.g_begin + wave0; g < P.g_end; g += P.wave_stride) {
    const uint64_t t = g * 64 + lane;
    const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), P.iter, P.c3, P.k0, P.k1);
    const uint32_t lead = uniform_u32(r.r3);
    const bool cooling = P.cool_all || ((lead >> 3) & 1u);
    if (t < P.t_begin || t >= P.t_end) continue;
    Term T = sample_term(r, cooling, P.S, L, P.path_top, P.W);
    if (P.trace_f) {  // parity hook: record the term instead of applying it
      if (!(T.flags & 8u)) {
        uint64_t a, b;
        float d;
        if (!resolve_term(P.rec, T, a, b, d)) T.flags |= 8u;
      }
      const uint64_t k = t - P.t_begin;
      P.trace_i[k] = T.i;
      P.trace_j[k] = T.j;
      P.trace_f[k] = (uint8_t)T.flags;
      continue;
    }
    if (T.flags & 8u) continue;
    uint64_t a, b;
    float d;
    if (!resolve_term(P.rec, T, a, b, d)) continue;
    apply_update(W, a, b, d, P.eta);
  }
}

// ---------------------------------------------------------------------------
// Data-reuse variant: a group of 64 terms shares a path; after the primary
// updates, rounds k = 1..drf-1 pair lane l's i-endpoint with lane
// (l + o_k) mod 64's j-endpoint from registers (ds_bpermute shuffles); the
// displacement of the j-endpoint is shuffled back to its owner lane.  Every
// endpoint is stored once, after the last round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 shfl_f2(float2 v, int src) {
  return make_float2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

__global__ __launch_bounds__(256) void k_layout_reuse(LayoutLaunch P) {
  extern __shared__ __align__(16) char lds[];
  const LdsView L = lds_view(lds, P.path_slots, P.W);
  lds_fill(L, P.path_off, P.n_paths, P.path_slots, P.zipf, P.guide, P.W);
  __syncthreads();

  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = (uint64_t)blockIdx.x * (blockDim.x >> 6) + uniform_u32(threadIdx.x >> 6);
  float2* __restrict__ Wc = P.work;
  const uint32_t reuse_c3 = (4u << 24) | (P.c3 & 0xFFFFFFu);
  for (uint64_t g = P.g_begin + wave0; g < P.g_end; g += P.wave_stride) {
    const uint64_t t = g * 64 + lane;
    const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), P.iter, P.c3, P.k0, P.k1);
    // the group's path: the path of the global step drawn by its first term
    const uint32_t lead0 = uniform_u32(r.r0), lead1 = uniform_u32(r.r1), lead3 = uniform_u32(r.r3);
    const bool cooling = P.cool_all || ((lead3 >> 3) & 1u);
    const uint64_t istar = mulhi64((uint64_t)lead0 | ((uint64_t)lead1 << 32), P.S);
    const uint32_t p = uniform_u32(find_path(L.off, P.path_top, istar));
    const uint64_t start = L.off[p], len = L.off[p + 1] - start;
    const bool in_range = t >= P.t_begin && t < P.t_end;
    Term T;
    T.i = start + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), len);
    bool ok = true;
    if (cooling) ok = partner_power_law(T.i, start, len, r.r2, r.r3, L.zipf, L.guide, P.W, T.j);
    else T.j = start + mulhi32(r.r2, (uint32_t)len);
    T.flags = (r.r3 & 3u) | ((cooling ? 1u : 0u) << 2) | ((ok ? 0u : 1u) << 3);
    // records, slots and endpoint path coordinates of this lane's term
    uint64_t a = 0, b = 0;
    int64_t pa = 0, pb = 0;
    bool valid = in_range && ok;
    if (valid) {
      const StepRec si = load_rec(P.rec, T.i);
      const StepRec sj = load_rec(P.rec, T.j);
      const uint32_t ei = T.flags & 1u, ej = (T.flags >> 1) & 1u;
      a = 2ull * (si.node_rev & kNodeMask) + ei;
      b = 2ull * (sj.node_rev & kNodeMask) + ej;
      pa = endpoint_pos(si, ei);
      pb = endpoint_pos(sj, ej);
      if (a == b || pa == pb) valid = false;
    }
    if (P.trace_f) {  // parity hook: record the group's terms and reuse offsets
      if (in_range) {
        const uint64_t k = t - P.t_begin;
        P.trace_i[k] = T.i;
        P.trace_j[k] = T.j;
        P.trace_f[k] = (uint8_t)(T.flags | (in_range && ok && !valid ? 8u : 0u));
      }
      if (lane == 0 && P.trace_o && P.drf > 1) {  // offsets of every group of the launch
        const Rand4 ro = philox10((uint32_t)g, (uint32_t)(g >> 32), P.iter, reuse_c3, P.k0, P.k1);
        const uint32_t w[4] = {ro.r0, ro.r1, ro.r2, ro.r3};
        for (uint32_t k = 1; k < P.drf; ++k)
          P.trace_o[(g - P.g_begin) * (P.drf - 1) + k - 1] =
              (uint8_t)(1 + ((w[(k - 1) >> 2] >> (8 * ((k - 1) & 3))) & 0xFFu) % 63);
      }
      continue;
    }
    float2 A = make_float2(0.0f, 0.0f), B = make_float2(0.0f, 0.0f);
    if (valid) {
      A = Wc[a];
      B = Wc[b];
      const float d = (float)(pa < pb ? pb - pa : pa - pb);
      const float dx = A.x - B.x, dy = A.y - B.y;
      const float mag = sqrtf(dx * dx + dy * dy);
      if (mag != 0.0f) {
        const float mu = fminf(P.eta / (d * d), 1.0f);
        const float rr = mu * (mag - d) / (2.0f * mag);
        A = make_float2(A.x - rr * dx, A.y - rr * dy);
        B = make_float2(B.x + rr * dx, B.y + rr * dy);
      }
    }
    if (P.drf > 1) {
      const Rand4 ro = philox10((uint32_t)g, (uint32_t)(g >> 32), P.iter, reuse_c3, P.k0, P.k1);
      const uint32_t w[4] = {ro.r0, ro.r1, ro.r2, ro.r3};
      for (uint32_t k = 1; k < P.drf; ++k) {
        const uint32_t o = 1 + ((w[(k - 1) >> 2] >> (8 * ((k - 1) & 3))) & 0xFFu) % 63;
        const int src = (int)((lane + o) & 63u);       // the j-endpoint this lane pairs with
        const int dst = (int)((lane + 64u - o) & 63u);  // the lane pairing with this lane's j-endpoint
        const uint32_t vm = __shfl((uint32_t)valid, src, 64);
        const uint64_t bm = __shfl(b, src, 64);
        const int64_t pbm = __shfl(pb, src, 64);
        const float2 Bm = shfl_f2(B, src);
        float2 disp = make_float2(0.0f, 0.0f);
        if (valid && vm && a != bm && pa != pbm) {
          const float d = (float)(pa < pbm ? pbm - pa : pa - pbm);
          const float dx = A.x - Bm.x, dy = A.y - Bm.y;
          const float mag = sqrtf(dx * dx + dy * dy);
          if (mag != 0.0f) {
            const float mu = fminf(P.eta / (d * d), 1.0f);
            const float rr = mu * (mag - d) / (2.0f * mag);
            A = make_float2(A.x - rr * dx, A.y - rr * dy);
            disp = make_float2(rr * dx, rr * dy);
          }
        }
        const float2 back = shfl_f2(disp, dst);
        B = make_float2(B.x + back.x, B.y + back.y);
      }
    }
    if (valid) {
      Wc[a] = A;
      Wc[b] = B;
    }
  }
}

__global__ __launch_bounds__(256) void k_apply_terms(const StepRec* __restrict__ rec, float2* __restrict__ work,
                                                     float eta, const uint64_t* __restrict__ ti,
                                                     const uint64_t* __restrict__ tj,
                                                     const uint8_t* __restrict__ tf, uint64_t count) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  Term T;
  T.i = ti[k];
  T.j = tj[k];
  T.flags = tf[k];
  if (T.flags & 8u) return;
  uint64_t a, b;
  float d;
  if (!resolve_term(rec, T, a, b, d)) return;
  apply_update(work, a, b, d, eta);
}

// Boundary layout [2][n][2] (X plane, Y plane) <-> working copy W[2n+e] = (x, y).
__global__ __launch_bounds__(256) void k_to_work(const float* __restrict__ coords, float2* __restrict__ work,
                                                 uint64_t n2) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2; k += stride)
    work[k] = make_float2(coords[k], coords[n2 + k]);
}

__global__ __launch_bounds__(256) void k_from_work(const float2* __restrict__ work, float* __restrict__ coords,
                                                   uint64_t n2) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2; k += stride) {
    const float2 v = work[k];
    coords[k] = v.x;
    coords[n2 + k] = v.y;
  }
}

// ---------------------------------------------------------------------------
// Batched form: one persistent launch per iteration over all graphs.  A work
// item is a run of groups_per_item consecutive 64-term groups of one graph;
// wave w takes items w, w + waves, ...  Items are ordered by phase (see
// kBatchPhases), and the segment (phase, graph) of an item is found by binary
// search over the segment prefix in LDS, next to the per-graph headers and
// path offsets.
// ---------------------------------------------------------------------------
__global__ void k_layout_batch(BatchLaunch P) {
  extern __shared__ __align__(16) char lds[];
  const uint32_t n_seg = kBatchPhases * P.n_graphs;
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
    const uint64_t local = (phase * H.n_items) / kBatchPhases + (it - seg_off[seg]);
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
size_t layout_lds_bytes(uint32_t path_slots, uint32_t W) {
  return (size_t)path_slots * 8 + (size_t)(W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
}

hipError_t launch_layout_iter(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(k_layout_iter, dim3(blocks), dim3(threads), layout_lds_bytes(P.path_slots, P.W), s, P);
  return hipGetLastError();
}

hipError_t launch_layout_reuse(const LayoutLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(k_layout_reuse, dim3(blocks), dim3(threads), layout_lds_bytes(P.path_slots, P.W), s, P);
  return hipGetLastError();
}

hipError_t launch_apply_terms(const StepRec* rec, float2* work, float eta, const uint64_t* i, const uint64_t* j,
                              const uint8_t* f, uint64_t count, hipStream_t s) {
  const uint64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_apply_terms, dim3((uint32_t)blocks), dim3(256), 0, s, rec, work, eta, i, j, f, count);
  return hipGetLastError();
}

static uint32_t elementwise_grid(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (uint32_t)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

hipError_t launch_to_work(const float* coords, float2* work, uint64_t n_nodes, hipStream_t s) {
  hipLaunchKernelGGL(k_to_work, dim3(elementwise_grid(2 * n_nodes)), dim3(256), 0, s, coords, work, 2 * n_nodes);
  return hipGetLastError();
}

hipError_t launch_from_work(const float2* work, float* coords, uint64_t n_nodes, hipStream_t s) {
  hipLaunchKernelGGL(k_from_work, dim3(elementwise_grid(2 * n_nodes)), dim3(256), 0, s, work, coords, 2 * n_nodes);
  return hipGetLastError();
}

size_t batch_lds_bytes(uint32_t n_graphs, uint32_t path_slots_total, uint32_t W) {
  return sizeof(BatchGraph) * n_graphs + (size_t)(kBatchPhases * n_graphs + 1) * 8 + (size_t)path_slots_total * 8 +
         (size_t)(W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
}

hipError_t launch_layout_batch(const BatchLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(k_layout_batch, dim3(blocks), dim3(threads),
                     batch_lds_bytes(P.n_graphs, P.path_slots_total, P.W), s, P);
  return hipGetLastError();
}

const void* layout_iter_kernel() { return reinterpret_cast<const void*>(&k_layout_iter); }
const void* layout_batch_kernel() { return reinterpret_cast<const void*>(&k_layout_batch); }

}  // namespace pgsgd
