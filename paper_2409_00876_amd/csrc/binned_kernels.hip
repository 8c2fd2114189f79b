// Binned (locality-ordered) processing of one PG-SGD iteration for gfx950.
//
// The terms of an iteration are independent draws, and Hogwild execution
// already runs them in an arbitrary interleaving, so any processing order is a
// valid schedule of the same term multiset.  These kernels choose an order with
// cache locality: terms are binned by the window of 2^win_shift consecutive
// path steps their step i falls in, and each XCD walks its own windows in turn
// (windows w = x, x + 8, ... on XCD x), so while a window is processed its step
// records and the coordinates of the nodes those steps visit stay in that XCD's
// L2.  Per chunk of at most 2^30 terms:
//   k_bin_count    draw, step i, window; a 2-byte tag (window | coin << 15) per
//                  term and a window histogram
//   k_bin_scan     window offsets, per-XCD item prefixes; clears the histogram
//   k_bin_scatter  4-byte term offsets (| coin << 31) into window-contiguous lists
//   k_bin_layout   the terms of each window: sample, gather, update (as
//                  k_layout_iter, with the cooling coin carried per term)
#include "device.h"
#include "internal.h"

namespace pgsgd {

// Same sampling as k_layout_iter (layout_kernels.hip) but per lane cooling.
__device__ __forceinline__ void bin_sample(const Rand4& r, bool cooling, uint64_t S, const uint64_t* off,
                                           uint32_t path_top, const uint32_t* zipf, const uint16_t* guide,
                                           uint32_t W, uint64_t& i, uint64_t& j, uint32_t& flags) {
  i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), S);
  const uint32_t p = find_path(off, path_top, i);
  const uint64_t start = off[p];
  const uint64_t len = off[p + 1] - start;
  bool ok = true;
  if (cooling) ok = partner_power_law(i, start, len, r.r2, r.r3, zipf, guide, W, j);
  else j = start + mulhi32(r.r2, (uint32_t)len);
  flags = (r.r3 & 3u) | ((cooling ? 1u : 0u) << 2) | ((ok ? 0u : 1u) << 3);
}

__global__ __launch_bounds__(1024) void k_bin_count(BinLaunch B) {
  extern __shared__ __align__(16) char lds[];
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds);
  for (uint32_t k = threadIdx.x; k < B.n_win; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const LayoutLaunch& L = B.L;
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t wave0 = (uint64_t)blockIdx.x * (blockDim.x >> 6) + uniform_u32(threadIdx.x >> 6);
  const uint64_t stride = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t g0 = B.c0 >> 6, g1 = (B.c1 + 63) >> 6;
  for (uint64_t g = g0 + wave0; g < g1; g += stride) {
    const uint64_t t = g * 64 + lane;
    const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), L.iter, L.c3, L.k0, L.k1);
    const uint32_t lead = uniform_u32(r.r3);
    const uint32_t coin = (L.cool_all || ((lead >> 3) & 1u)) ? 1u : 0u;
    if (t >= B.c1) continue;
    const uint64_t i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), L.S);
    const uint32_t w = (uint32_t)(i >> B.win_shift);
    B.tag[t - B.c0] = (uint16_t)(w | (coin << 15));
    atomicAdd(&hist[w], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < B.n_win; k += blockDim.x)
    if (hist[k]) atomicAdd(&B.wcount[k], hist[k]);
}

// One block.  woff = exclusive prefix of wcount; cursor = woff; per XCD x the
// prefix of ceil(count/64) over its windows x, x+8, ...; then wcount = 0.
__global__ __launch_bounds__(1024) void k_bin_scan(BinLaunch B) {
  __shared__ uint32_t part[1024];
  const uint32_t n = B.n_win;
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t k0 = threadIdx.x * per;
  const uint32_t k1 = min(n, k0 + per);
  uint32_t s = 0;
  for (uint32_t k = k0; k < k1; ++k) s += B.wcount[k];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (uint32_t k = 0; k < blockDim.x; ++k) {
      const uint32_t v = part[k];
      part[k] = acc;
      acc += v;
    }
    B.woff[n] = acc;
  }
  __syncthreads();
  uint32_t acc = part[threadIdx.x];
  for (uint32_t k = k0; k < k1; ++k) {
    B.woff[k] = acc;
    B.cursor[k] = acc;
    acc += B.wcount[k];
  }
  __syncthreads();
  if (threadIdx.x < kXcds) {
    const uint32_t x = threadIdx.x;
    uint32_t items = 0, q = 0;
    for (uint32_t w = x; w < n; w += kXcds, ++q) {
      B.xitem[x * B.xstride + q] = items;
      items += (B.wcount[w] + 63) >> 6;
    }
    B.xitem[x * B.xstride + q] = items;
  }
  __syncthreads();
  for (uint32_t k = k0; k < k1; ++k) B.wcount[k] = 0;
}

__global__ __launch_bounds__(1024) void k_bin_scatter(BinLaunch B) {
  extern __shared__ __align__(16) char lds[];
  uint32_t* slot = reinterpret_cast<uint32_t*>(lds);
  for (uint32_t k = threadIdx.x; k < B.n_win; k += blockDim.x) slot[k] = 0;
  __syncthreads();
  const uint64_t n = B.c1 - B.c0;
  const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t r0 = min(n, (uint64_t)blockIdx.x * per);
  const uint64_t r1 = min(n, r0 + per);
  for (uint64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) atomicAdd(&slot[B.tag[k] & 0x7FFFu], 1u);
  __syncthreads();
  for (uint32_t w = threadIdx.x; w < B.n_win; w += blockDim.x)
    if (slot[w]) slot[w] = atomicAdd(&B.cursor[w], slot[w]);
  __syncthreads();
  for (uint64_t k = r0 + threadIdx.x; k < r1; k += blockDim.x) {
    const uint32_t tg = B.tag[k];
    const uint32_t pos = atomicAdd(&slot[tg & 0x7FFFu], 1u);
    B.entries[pos] = (uint32_t)k | ((uint32_t)(tg >> 15) << 31);
  }
}

__global__ __launch_bounds__(256) void k_bin_layout(BinLaunch B) {
  extern __shared__ __align__(16) char lds[];
  const LayoutLaunch& L = B.L;
  uint64_t* off = reinterpret_cast<uint64_t*>(lds);
  uint32_t* zipf = reinterpret_cast<uint32_t*>(lds + (size_t)L.path_slots * 8);
  uint16_t* guide = reinterpret_cast<uint16_t*>(lds + (size_t)L.path_slots * 8 + (size_t)(L.W + 1) * 4);
  for (uint32_t k = threadIdx.x; k < L.path_slots; k += blockDim.x) off[k] = k <= L.n_paths ? L.path_off[k] : ~0ull;
  for (uint32_t k = threadIdx.x; k <= L.W; k += blockDim.x) zipf[k] = L.zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) guide[k] = L.guide[k];
  __syncthreads();

  // blocks are dispatched to the XCDs round-robin: block b runs on XCD b % 8
  const uint32_t x = blockIdx.x % kXcds;
  const uint32_t waves_per_block = blockDim.x >> 6;
  const uint64_t m0 = (uint64_t)(blockIdx.x / kXcds) * waves_per_block + uniform_u32(threadIdx.x >> 6);
  const uint64_t mstride = (uint64_t)(gridDim.x / kXcds) * waves_per_block;
  const uint32_t* __restrict__ xi = B.xitem + (size_t)x * B.xstride;
  if (x >= B.n_win) return;  // fewer windows than XCDs
  const uint32_t nq = (B.n_win - x + kXcds - 1) / kXcds;  // windows of this XCD, >= 1
  const uint32_t n_items = xi[nq];
  const uint32_t lane = threadIdx.x & 63u;
  float2* __restrict__ Wc = L.work;
  for (uint64_t m = m0; m < n_items; m += mstride) {
    // window of this item: largest q with xi[q] <= m (wave-uniform search)
    uint32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (xi[mid] <= m) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t q = uniform_u32(lo);
    const uint32_t w = x + q * kXcds;
    const uint32_t idx = (uint32_t)(m - xi[q]) * 64u + lane;
    const uint32_t wbeg = B.woff[w], wend = B.woff[w + 1];
    if (wbeg + idx >= wend) continue;
    const uint32_t e = B.entries[wbeg + idx];
    const uint64_t t = B.c0 + (e & 0x7FFFFFFFu);
    const bool cooling = (e >> 31) != 0;
    const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), L.iter, L.c3, L.k0, L.k1);
    Term T;
    bin_sample(r, cooling, L.S, off, L.path_top, zipf, guide, L.W, T.i, T.j, T.flags);
    if (L.trace_f) {  // parity hook: record terms of [t_begin, t_end) instead of applying them
      if (t < L.t_begin || t >= L.t_end) continue;
      if (!(T.flags & 8u)) {
        uint64_t a, b;
        float d;
        if (!resolve_term(L.rec, T, a, b, d)) T.flags |= 8u;
      }
      const uint64_t k = t - L.t_begin;
      L.trace_i[k] = T.i;
      L.trace_j[k] = T.j;
      L.trace_f[k] = (uint8_t)T.flags;
      continue;
    }
    if (T.flags & 8u) continue;
    uint64_t a, b;
    float d;
    if (!resolve_term(L.rec, T, a, b, d)) continue;
    apply_update(Wc, a, b, d, L.eta);
  }
}

hipError_t launch_bin_count_scan_scatter(const BinLaunch& B, hipStream_t s) {
  const size_t hist_lds = (size_t)B.n_win * 4;
  hipLaunchKernelGGL(k_bin_count, dim3(B.count_blocks), dim3(1024), hist_lds, s, B);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, B);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_bin_scatter, dim3(B.count_blocks), dim3(1024), hist_lds, s, B);
  return hipGetLastError();
}

hipError_t launch_bin_layout(const BinLaunch& B, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_layout, dim3(blocks), dim3(256), layout_lds_bytes(B.L.path_slots, B.L.W), s, B);
  return hipGetLastError();
}

const void* bin_layout_kernel() { return reinterpret_cast<const void*>(&k_bin_layout); }

}  // namespace pgsgd
