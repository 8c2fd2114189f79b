// PG-SGD layout kernels for gfx950: one launch per iteration of Alg. 1.
//
//   k_layout_iter   all terms of one iteration, fused: draw, sample, gather,
//                   update, scatter (the hot path); with trace pointers set it
//                   records the sampled terms instead (parity checks)
//   k_apply_terms   the update alone on given terms (grid-stride)
//   k_layout_reuse  the data-reuse variant (shared group path, reuse rounds in registers)
//
// Work mapping: a wavefront owns aligned groups of 64 consecutive terms, lane
// l doing term 64g+l.  The cooling coin of a group is bit 3 of word 3 of its
// first term's draw, read from lane 0 with readfirstlane, so the cooling branch
// is wave-uniform by construction (the paper's warp merging, here part of the
// sampling definition rather than a scheduling trick).
#include "device.h"
#include "internal.h"

namespace pgsgd {

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
    if (P.apply_mask && !P.apply_mask[t - P.t_begin]) continue;  // parity hook: a chosen subset
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
      float2 m;
      if (clamped_step(A, B, d, P.eta, m)) {
        A = make_float2(A.x - m.x, A.y - m.y);
        B = make_float2(B.x + m.x, B.y + m.y);
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
          if (clamped_step(A, Bm, d, P.eta, disp)) A = make_float2(A.x - disp.x, A.y - disp.y);
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
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    Term T;
    T.i = ti[k];
    T.j = tj[k];
    T.flags = tf[k];
    if (T.flags & 8u) continue;
    uint64_t a, b;
    float d;
    if (!resolve_term(rec, T, a, b, d)) continue;
    apply_update(work, a, b, d, eta);
  }
}

// Boundary layout [2][n][2] (X plane, Y plane) <-> working copy W[2n+e] = (x, y).
// Working copy <-> boundary layout.  Thread k handles endpoint k = 2m + e of
// device node m; with a renumbered graph its caller id is inv[m].
__global__ __launch_bounds__(256) void k_to_work(const float* __restrict__ coords, float2* __restrict__ work,
                                                 uint64_t n2, const uint32_t* __restrict__ inv) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2; k += stride) {
    const uint64_t c = inv ? 2ull * inv[k >> 1] + (k & 1) : k;
    work[k] = make_float2(coords[c], coords[n2 + c]);
  }
}

__global__ __launch_bounds__(256) void k_from_work(const float2* __restrict__ work, float* __restrict__ coords,
                                                   uint64_t n2, const uint32_t* __restrict__ inv) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n2; k += stride) {
    const float2 v = work[k];
    const uint64_t c = inv ? 2ull * inv[k >> 1] + (k & 1) : k;
    coords[c] = v.x;
    coords[n2 + c] = v.y;
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

static uint32_t elementwise_grid(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (uint32_t)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

hipError_t launch_apply_terms(const StepRec* rec, float2* work, float eta, const uint64_t* i, const uint64_t* j,
                              const uint8_t* f, uint64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_terms, dim3(elementwise_grid(count)), dim3(256), 0, s, rec, work, eta, i, j, f, count);
  return hipGetLastError();
}

hipError_t launch_to_work(const float* coords, float2* work, uint64_t n_nodes, const uint32_t* inv, hipStream_t s) {
  hipLaunchKernelGGL(k_to_work, dim3(elementwise_grid(2 * n_nodes)), dim3(256), 0, s, coords, work, 2 * n_nodes,
                     inv);
  return hipGetLastError();
}

hipError_t launch_from_work(const float2* work, float* coords, uint64_t n_nodes, const uint32_t* inv,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_from_work, dim3(elementwise_grid(2 * n_nodes)), dim3(256), 0, s, work, coords, 2 * n_nodes,
                     inv);
  return hipGetLastError();
}

const void* layout_iter_kernel() { return reinterpret_cast<const void*>(&k_layout_iter); }

}  // namespace pgsgd
