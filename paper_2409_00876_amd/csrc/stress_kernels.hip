// Stress kernels for gfx950: the sampled path stress of Eq. 2 (two passes for
// the CI95), the differentiable loss and its adjoint, the initial layout and a
// fused Adam step.
//
// Stress terms are evaluated in FP64 from the float32 coordinates with FMA
// contraction off, so each term is the exactly rounded value of
// ((|v_i - v_j| - d)/d)^2; block partials are FP64 and reduced in a fixed
// order, so results are deterministic for a given launch shape.
#include "device.h"
#include "internal.h"
#include "stress.h"

namespace pgsgd {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums over the block; the result is valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch) {
  v = wave_sum(v);
  const uint32_t w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63u) == 0) scratch[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (uint32_t k = 0; k < nw; ++k) r += scratch[k];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void fill_offsets(uint64_t* off, const StressLaunch& P) {
  for (uint32_t k = threadIdx.x; k < P.path_slots; k += blockDim.x) off[k] = k <= P.n_paths ? P.path_off[k] : ~0ull;
}

// Stress of one pair of slots in FP64.  Returns false when d == 0.
__device__ __forceinline__ bool pair_terms(const StepRec* __restrict__ rec, uint64_t i, uint64_t j, uint32_t ei,
                                           uint32_t ej, uint64_t& a, uint64_t& b, double& d) {
  const StepRec si = load_rec(rec, i);
  const StepRec sj = load_rec(rec, j);
  const int64_t dd = endpoint_pos(si, ei) - endpoint_pos(sj, ej);
  a = 2ull * (si.node_rev & kNodeMask) + ei;
  b = 2ull * (sj.node_rev & kNodeMask) + ej;
  d = (double)(dd < 0 ? -dd : dd);
  return dd != 0;
}

// ((|v_a - v_b| - d)/d)^2 in FP64 from the two endpoints' float32 coordinates.
__device__ __forceinline__ double stress_xy(float xa, float ya, float xb, float yb, double d) {
#pragma clang fp contract(off)
  const double dx = (double)xa - (double)xb;
  const double dy = (double)ya - (double)yb;
  const double mag = sqrt(dx * dx + dy * dy);
  const double e = (mag - d) / d;
  return e * e;
}

// v_a - v_b from the interleaved copy in FP64; returns |v_a - v_b|.
__device__ __forceinline__ double delta_work(const float2* __restrict__ W, uint64_t a, uint64_t b, double& dx,
                                             double& dy) {
#pragma clang fp contract(off)
  const float2 va = W[a], vb = W[b];
  dx = (double)va.x - (double)vb.x;
  dy = (double)va.y - (double)vb.y;
  return sqrt(dx * dx + dy * dy);
}

// The stress of endpoints a and b of the interleaved copy (W[e] = (x, y) of endpoint e).
__device__ __forceinline__ double stress_work(const float2* __restrict__ W, uint64_t a, uint64_t b, double d) {
  const float2 va = W[a], vb = W[b];
  return stress_xy(va.x, va.y, vb.x, vb.y, d);
}

// Pass 1 with outlier collection: a pair whose stress exceeds the threshold is
// appended (slot from one atomic; the first out_max are kept).
__device__ __forceinline__ void keep_outlier(const StressLaunch& P, uint64_t i, uint64_t j, uint32_t e, double st) {
  if (!P.out_count || !(st > P.out_threshold)) return;
  const unsigned long long k = atomicAdd(reinterpret_cast<unsigned long long*>(P.out_count), 1ull);
  if (k < P.out_max) {
    P.out_i[k] = i;
    P.out_j[k] = j;
    P.out_e[k] = (uint8_t)e;
    P.out_s[k] = st;
  }
}

// A second layout (P.work2) on the same pair: pass 1 sums its stress into acc2;
// pass 2 (mean_dev = mean_a, mean_b, R) sums (s_b - mean_b)^2 into acc2 and
// (s_a - R s_b)^2 into acc3.
__device__ __forceinline__ void paired_terms(const StressLaunch& P, int pass, const double* mean_dev, uint64_t a,
                                             uint64_t b, double d, double st, double& acc2, double& acc3) {
#pragma clang fp contract(off)
  const double sb = stress_work(P.work2, a, b, d);
  if (pass == 1) {
    acc2 += sb;
  } else {
    acc2 += (sb - mean_dev[1]) * (sb - mean_dev[1]);
    acc3 += (st - mean_dev[2] * sb) * (st - mean_dev[2] * sb);
  }
}

// Per-block partial sums: part_f[blockIdx.x] = acc, and for a paired
// evaluation part_f[gridDim.x + blockIdx.x] = acc2, part_f[2 gridDim.x + blockIdx.x] = acc3.
__device__ __forceinline__ void write_parts(const StressLaunch& P, double acc, double acc2, double acc3, uint64_t nv,
                                            uint64_t ns, double* red_f, uint64_t* red_n, double* part_f,
                                            uint64_t* part_n, uint64_t* part_skip) {
  acc = block_sum(acc, red_f);
  if (P.work2) {
    acc2 = block_sum(acc2, red_f);
    acc3 = block_sum(acc3, red_f);
  }
  nv = block_sum(nv, red_n);
  ns = block_sum(ns, red_n);
  if (threadIdx.x == 0) {
    part_f[blockIdx.x] = acc;
    if (P.work2) {
      part_f[gridDim.x + blockIdx.x] = acc2;
      part_f[2 * gridDim.x + blockIdx.x] = acc3;
    }
    if (part_n) part_n[blockIdx.x] = nv;
    if (part_skip) part_skip[blockIdx.x] = ns;
  }
}

// ---------------------------------------------------------------------------
// Sampled path stress: thread-strided over steps s; step s owns pairs
// q = m*s .. m*s+m-1, which all belong to the path of s.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fill_loss_lds(char* lds, const StressLaunch& P, uint64_t*& off, uint32_t*& zipf,
                                              uint16_t*& guide);

// mode 0: uniform partner in the path (Eq. 2); mode 1: the power-law partner
// of the layout's cooling phase (same draw words; no partner in a single-step
// path: the pair is skipped).
__global__ __launch_bounds__(256) void k_sps(StressLaunch P, int pass, int mode, const double* __restrict__ mean_dev,
                                             double* __restrict__ part_f, uint64_t* __restrict__ part_n,
                                             uint64_t* __restrict__ part_skip) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* off;
  uint32_t* zipf;
  uint16_t* guide;
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  if (mode == 1) {
    fill_loss_lds(lds, P, off, zipf, guide);
  } else {
    off = reinterpret_cast<uint64_t*>(lds);
    zipf = nullptr;
    guide = nullptr;
    fill_offsets(off, P);
  }
  __syncthreads();
  const double mean = pass == 2 ? mean_dev[0] : 0.0;
  double acc = 0.0, acc2 = 0.0, acc3 = 0.0;
  uint64_t nv = 0, ns = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < P.S; s += stride) {
    const uint32_t p = find_path(off, P.path_top, s);
    const uint64_t start = off[p], len = off[p + 1] - start;
    for (uint32_t k = 0; k < P.m; ++k) {
      const uint64_t q = (uint64_t)P.m * s + k;
      const Rand4 r = philox10((uint32_t)q, (uint32_t)(q >> 32), 0u, P.c3, P.k0, P.k1);
      const uint64_t i = start + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), len);
      uint64_t j;
      if (mode == 1) {
        if (!partner_power_law(i, start, len, r.r2, r.r3, zipf, guide, P.W, j)) {
          ++ns;
          continue;
        }
      } else {
        j = start + mulhi32(r.r2, (uint32_t)len);
      }
      uint64_t a, b;
      double d;
      if (!pair_terms(P.rec, i, j, r.r3 & 1u, (r.r3 >> 1) & 1u, a, b, d)) {
        ++ns;
        continue;
      }
      const double st = stress_work(P.work, a, b, d);
      if (pass == 1) {
        acc += st;
        ++nv;
        keep_outlier(P, i, j, r.r3 & 3u, st);
      } else {
#pragma clang fp contract(off)
        acc += (st - mean) * (st - mean);
      }
      if (P.work2) paired_terms(P, pass, mean_dev, a, b, d, st, acc2, acc3);
    }
  }
  write_parts(P, acc, acc2, acc3, nv, ns, red_f, red_n, part_f, part_n, part_skip);
}

// ---------------------------------------------------------------------------
// Sampled path stress in window-major order.  The pairs of Eq. 2 keep their
// law (path p receives m|p| pairs, i and j independent and uniform in p) and
// are listed segment by segment: segment g (a window of 2^win_shift steps cut
// at path boundaries) receives the number n_g of the plain pair draws whose
// step i falls in it, and slot u (numbered consecutively over the segments)
// draws i uniformly in its segment and j uniformly in its path from the slot
// stream at counter u.  XCD x (blocks b with b mod 8 = x) walks the segments
// of run x with all its waves, 64 slots per wave and item, so the i side of
// the pairs (records and coordinates of one window) stays in the XCD's L2 and
// only the j side reaches into the rest of the path.  The waves take their
// items from one counter per run, so they all stay near the same window (a
// static share per wave drifts apart over thousands of items); the FP64
// block sums then depend on which wave took which item, so a result is
// reproducible up to the rounding of that sum order.
// ---------------------------------------------------------------------------
namespace {

constexpr uint64_t kSpsGrab = 4;  // items a wave takes from its run's counter at once

// loads at wave-uniform addresses through the constant address space (scalar loads)
template <typename T>
__device__ __forceinline__ T uload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  return ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32) | uniform_u32((uint32_t)v);
}

}  // namespace

// The segment histogram: step s owns the plain pairs q = m*s .. m*s+m-1 (all
// of the path of s); each draws its i as k_sps does and counts its segment.
// With loss_pairs set, the loss's plain pairs q < loss_pairs are counted
// instead.
__global__ __launch_bounds__(1024) void k_sps_win_count(SpsWinLaunch W) {
  extern __shared__ __align__(16) char lds[];
  const StressLaunch& P = W.P;
  uint64_t* off = reinterpret_cast<uint64_t*>(lds);
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds + (size_t)P.path_slots * 8);
  fill_offsets(off, P);
  for (uint32_t k = threadIdx.x; k < W.n_seg; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  // the loss's pairs (reading R22): pair q < loss_pairs draws i uniformly over all steps
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < W.loss_pairs; q += stride) {
    const Rand4 r = philox10((uint32_t)q, (uint32_t)(q >> 32), P.word2, P.c3, P.k0, P.k1);
    const uint64_t i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), P.S);
    const uint32_t w = (uint32_t)(i >> W.win_shift);
    uint32_t lo = W.wseg[w], hi = W.wseg[w + 1];
    while (hi - lo > 1) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (W.seg_start[mid] <= i) lo = mid;
      else hi = mid;
    }
    atomicAdd(&hist[lo], 1u);
  }
  const uint64_t sps_steps = W.loss_pairs ? 0 : P.S;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < sps_steps; s += stride) {
    const uint32_t p = find_path(off, P.path_top, s);
    const uint64_t start = off[p], len = off[p + 1] - start;
    for (uint32_t k = 0; k < P.m; ++k) {
      const uint64_t q = (uint64_t)P.m * s + k;
      const Rand4 r = philox10((uint32_t)q, (uint32_t)(q >> 32), 0u, P.c3, P.k0, P.k1);
      const uint64_t i = start + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), len);
      const uint32_t w = (uint32_t)(i >> W.win_shift);
      uint32_t lo = W.wseg[w], hi = W.wseg[w + 1];  // the segments of window w: the last with start <= i
      while (hi - lo > 1) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (W.seg_start[mid] <= i) lo = mid;
        else hi = mid;
      }
      atomicAdd(&hist[lo], 1u);
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < W.n_seg; k += blockDim.x)
    if (hist[k]) atomicAdd(&W.count[k], hist[k]);
}

// One block of 1024 threads: seg_off = exclusive prefix of the counts, the
// per-run item prefixes and zeroed item counters, then the histogram back to
// zero.  Each thread owns a contiguous chunk; every stage is a chunk pass and
// a block scan.
// One block.  The histogram is read into LDS with coalesced loads (and
// cleared for the next use), so the chunk passes below read LDS, not memory.
__global__ __launch_bounds__(1024) void k_sps_win_scan(SpsWinLaunch W) {
  extern __shared__ __align__(16) char lds[];
  __shared__ uint64_t lds16[16];
  uint32_t* cnt = reinterpret_cast<uint32_t*>(lds);
  const uint32_t n = W.n_seg;
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
    cnt[k] = W.count[k];
    W.count[k] = 0;
  }
  __syncthreads();
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t k0 = min(n, threadIdx.x * per);
  const uint32_t k1 = min(n, k0 + per);
  uint64_t s = 0;
  for (uint32_t k = k0; k < k1; ++k) s += cnt[k];
  uint64_t total;
  uint64_t acc = block_exclusive_scan(s, lds16, &total);
  for (uint32_t k = k0; k < k1; ++k) {
    W.seg_off[k] = acc;
    acc += cnt[k];
  }
  if (threadIdx.x == 0) W.seg_off[n] = total;
  for (uint32_t run = 0; run < kXcds; ++run) {  // run x: segments [sbeg[x], sbeg[x + 1])
    const uint32_t b = W.sbeg[run], e = W.sbeg[run + 1], nq = e - b;
    const uint32_t rper = (nq + blockDim.x - 1) / blockDim.x;
    const uint32_t q0 = min(nq, threadIdx.x * rper), q1 = min(nq, q0 + rper);
    uint64_t items = 0;
    for (uint32_t q = q0; q < q1; ++q) items += (cnt[b + q] + 63) >> 6;
    uint64_t run_total;
    uint64_t pre = block_exclusive_scan(items, lds16, &run_total);
    uint64_t* xi = W.xitem + (size_t)run * W.xstride;
    for (uint32_t q = q0; q < q1; ++q) {
      xi[q] = pre;
      pre += (cnt[b + q] + 63) >> 6;
    }
    if (threadIdx.x == 0) xi[nq] = run_total;
  }
  if (threadIdx.x < 2 * kXcds) W.queue[(size_t)threadIdx.x * 16] = 0;
}

// One pass: the waves of XCD x take the items of run x from its counter,
// kSpsGrab at a time; every wave leaves once the counter has passed the run's
// last item.
__global__ __launch_bounds__(256) void k_sps_win(SpsWinLaunch W, int pass, const double* __restrict__ mean_dev,
                                                 double* __restrict__ part_f, uint64_t* __restrict__ part_n,
                                                 uint64_t* __restrict__ part_skip) {
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  const StressLaunch& P = W.P;
  const double mean = pass == 2 ? mean_dev[0] : 0.0;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t x = blockIdx.x % kXcds;
  const uint32_t gb = uload(W.sbeg + x);
  const uint32_t nq = uload(W.sbeg + x + 1) - gb;
  const uint64_t* __restrict__ xi = W.xitem + (size_t)x * W.xstride;
  const uint64_t n_items = uniform_u64(uload(xi + nq));
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(W.queue + ((size_t)(pass - 1) * kXcds + x) * 16);
  double acc = 0.0, acc2 = 0.0, acc3 = 0.0;
  uint64_t nv = 0, ns = 0;
  uint32_t q = 0;
  for (uint64_t m = 0, m_end = 0;; ++m) {
    if (m >= m_end) {
      uint64_t base = 0;
      if (lane == 0) base = atomicAdd(ctr, (unsigned long long)kSpsGrab);
      m = uniform_u64(base);
      if (m >= n_items) break;
      m_end = min(m + kSpsGrab, n_items);
    }
    while (q + 1 < nq && uniform_u64(uload(xi + q + 1)) <= m) q = uniform_u32(q + 1);
    const uint32_t g = gb + q;
    const uint64_t u0 = uniform_u64(uload(W.seg_off + g)) + (m - uniform_u64(uload(xi + q))) * 64;
    const uint64_t u_end = uniform_u64(uload(W.seg_off + g + 1));
    const uint64_t sst = uniform_u64(uload(W.seg_start + g));
    const uint64_t slen = uniform_u64(uload(W.seg_start + g + 1)) - sst;
    const uint32_t p = uniform_u32(uload(W.seg_path + g));
    const uint64_t pst = uniform_u64(uload(P.path_off + p));
    const uint64_t plen = uniform_u64(uload(P.path_off + p + 1)) - pst;
    const uint64_t u = u0 + lane;
    if (u < u_end) {
      const Rand4 r = philox10((uint32_t)u, (uint32_t)(u >> 32), 0u, W.slot_c3, P.k0, P.k1);
      const uint64_t i = sst + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), slen);
      const uint64_t j = pst + mulhi32(r.r2, (uint32_t)plen);
      uint64_t a, b;
      double d;
      if (!pair_terms(P.rec, i, j, r.r3 & 1u, (r.r3 >> 1) & 1u, a, b, d)) {
        ++ns;
      } else {
        const double st = stress_work(P.work, a, b, d);
        if (pass == 1) {
          acc += st;
          ++nv;
          keep_outlier(P, i, j, r.r3 & 3u, st);
        } else {
#pragma clang fp contract(off)
          acc += (st - mean) * (st - mean);
        }
        if (P.work2) paired_terms(P, pass, mean_dev, a, b, d, st, acc2, acc3);
      }
    }
  }
  write_parts(P, acc, acc2, acc3, nv, ns, red_f, red_n, part_f, part_n, part_skip);
}

// ---------------------------------------------------------------------------
// Path stress, Eq. 1: for every path and every step pair i < j of it, the mean
// of the stress over the endpoint combinations with d > 0; averaged over all
// pairs.  Thread-strided over rows i; a row visits j = i+1 .. end of the path.
// O(sum |p|^2) work: for small graphs and for validating the sampled metric.
// part_f: per-block sum of the pair means; part_n: per-block pair count.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_path_stress_exact(StressLaunch P, double* __restrict__ part_f,
                                                           uint64_t* __restrict__ part_n) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* off = reinterpret_cast<uint64_t*>(lds);
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  fill_offsets(off, P);
  __syncthreads();
  // both endpoints of a node are 16 contiguous bytes of the interleaved copy
  const float4* __restrict__ W4 = reinterpret_cast<const float4*>(P.work);
  double acc = 0.0;
  uint64_t np = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.S; i += stride) {
    const uint32_t p = find_path(off, P.path_top, i);
    const uint64_t end = off[p + 1];
    const StepRec si = load_rec(P.rec, i);
    const float4 ci = W4[si.node_rev & kNodeMask];
    for (uint64_t j = i + 1; j < end; ++j) {
      const StepRec sj = load_rec(P.rec, j);
      const float4 cj = W4[sj.node_rev & kNodeMask];
      double sum = 0.0;
      uint32_t nv = 0;
      for (uint32_t e = 0; e < 4; ++e) {
        const uint32_t ei = e & 1u, ej = e >> 1;
        const int64_t dd = endpoint_pos(si, ei) - endpoint_pos(sj, ej);
        if (dd == 0) continue;
        sum += stress_xy(ei ? ci.z : ci.x, ei ? ci.w : ci.y, ej ? cj.z : cj.x, ej ? cj.w : cj.y,
                         (double)(dd < 0 ? -dd : dd));
        ++nv;
      }
      if (nv) {
#pragma clang fp contract(off)
        acc += sum / (double)nv;
        ++np;
      }
    }
  }
  acc = block_sum(acc, red_f);
  np = block_sum(np, red_n);
  if (threadIdx.x == 0) {
    part_f[blockIdx.x] = acc;
    part_n[blockIdx.x] = np;
  }
}

// One block sums the partials in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_parts(const double* __restrict__ part_f,
                                                       const uint64_t* __restrict__ part_n,
                                                       const uint64_t* __restrict__ part_skip, uint32_t n_parts,
                                                       double* out_f, uint64_t* out_n, double* mean_out,
                                                       float* loss_out, uint64_t* n_valid_out) {
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  double f = 0.0;
  uint64_t n = 0, sk = 0;
  for (uint32_t k = threadIdx.x; k < n_parts; k += blockDim.x) {
    f += part_f[k];
    if (part_n) n += part_n[k];
    if (part_skip) sk += part_skip[k];
  }
  f = block_sum(f, red_f);
  n = block_sum(n, red_n);
  sk = block_sum(sk, red_n);
  if (threadIdx.x == 0) {
    if (out_f) out_f[0] = f;
    if (out_n) {
      if (part_n) out_n[0] = n;
      if (part_skip) out_n[1] = sk;
    }
    if (mean_out) mean_out[0] = n ? f / (double)n : 0.0;
    if (loss_out) loss_out[0] = n ? (float)(f / (double)n) : 0.0f;
    if (n_valid_out) n_valid_out[0] = n;
  }
}

// ---------------------------------------------------------------------------
// Differentiable loss: pairs q in [0, count) from the power-law sampler.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool loss_pair(const StressLaunch& P, const uint64_t* off, const uint32_t* zipf,
                                          const uint16_t* guide, uint64_t q, uint64_t& a, uint64_t& b, double& d) {
  const Rand4 r = philox10((uint32_t)q, (uint32_t)(q >> 32), P.word2, P.c3, P.k0, P.k1);
  const uint64_t i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), P.S);
  const uint32_t p = find_path(off, P.path_top, i);
  const uint64_t start = off[p], len = off[p + 1] - start;
  uint64_t j;
  if (!partner_power_law(i, start, len, r.r2, r.r3, zipf, guide, P.W, j)) return false;
  if (!pair_terms(P.rec, i, j, r.r3 & 1u, (r.r3 >> 1) & 1u, a, b, d)) return false;
  return a != b;
}

__device__ __forceinline__ void fill_loss_lds(char* lds, const StressLaunch& P, uint64_t*& off, uint32_t*& zipf,
                                              uint16_t*& guide) {
  off = reinterpret_cast<uint64_t*>(lds);
  zipf = reinterpret_cast<uint32_t*>(lds + (size_t)P.path_slots * 8);
  guide = reinterpret_cast<uint16_t*>(lds + (size_t)P.path_slots * 8 + (size_t)(P.W + 1) * 4);
  fill_offsets(off, P);
  for (uint32_t k = threadIdx.x; k <= P.W; k += blockDim.x) zipf[k] = P.zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) guide[k] = P.guide[k];
}

__global__ __launch_bounds__(256) void k_stress_fwd(StressLaunch P, double* __restrict__ part_f,
                                                    uint64_t* __restrict__ part_n) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  uint64_t* off;
  uint32_t* zipf;
  uint16_t* guide;
  fill_loss_lds(lds, P, off, zipf, guide);
  __syncthreads();
  double acc = 0.0;
  uint64_t nv = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P.count; q += stride) {
    uint64_t a, b;
    double d;
    if (!loss_pair(P, off, zipf, guide, q, a, b, d)) continue;
    acc += stress_work(P.work, a, b, d);
    ++nv;
  }
  acc = block_sum(acc, red_f);
  nv = block_sum(nv, red_n);
  if (threadIdx.x == 0) {
    part_f[blockIdx.x] = acc;
    part_n[blockIdx.x] = nv;
  }
}

// The adjoint, scattered with float32 atomics into the planar gradient
// (atomics are served per 4-byte word, so an interleaved scratch would not
// make them cheaper); the coordinates come from the interleaved copy.
__global__ __launch_bounds__(256) void k_stress_bwd(StressLaunch P, const float* __restrict__ grad_out,
                                                    const uint64_t* __restrict__ n_valid,
                                                    float* __restrict__ grad) {
  extern __shared__ __align__(16) char lds[];
  uint64_t* off;
  uint32_t* zipf;
  uint16_t* guide;
  fill_loss_lds(lds, P, off, zipf, guide);
  __syncthreads();
  const uint64_t n = n_valid[0];
  if (n == 0) return;
  const double scale = (double)grad_out[0] * 2.0 / (double)n;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < P.count; q += stride) {
    uint64_t a, b;
    double d;
    if (!loss_pair(P, off, zipf, guide, q, a, b, d)) continue;
    double dx, dy;
    const double mag = delta_work(P.work, a, b, dx, dy);
    if (mag == 0.0) continue;
    const double c = scale * (mag - d) / (d * d) / mag;
    const float gx = (float)(c * dx), gy = (float)(c * dy);
    float* __restrict__ GX = grad;
    float* __restrict__ GY = grad + 2ull * P.n_nodes;
    if (P.inv) {  // the gradient is in the caller's node order
      a = 2ull * P.inv[a >> 1] + (a & 1);
      b = 2ull * P.inv[b >> 1] + (b & 1);
    }
    unsafeAtomicAdd(&GX[a], gx);
    unsafeAtomicAdd(&GY[a], gy);
    unsafeAtomicAdd(&GX[b], -gx);
    unsafeAtomicAdd(&GY[b], -gy);
  }
}

// ---------------------------------------------------------------------------
// The loss over its window-major pairs (reading R22): the waves of XCD x take
// the items (64 slots of one segment) of run x from the counter of row
// `kGrad` of the queue; slot u draws Philox stream 7 (W.slot_c3) at counter u
// with word 2 = the optimiser step: i uniform in the segment, j its power-law
// partner, endpoint coins.  A segment's steps, their partners (at most W steps
// away) and the coordinates and gradient entries of the nodes they visit stay
// in the XCD's L2 while the XCD works on it.  Forward: per-block sums of the
// stress and the valid-pair count; adjoint: as k_stress_bwd.
// ---------------------------------------------------------------------------
template <bool kGrad>
__global__ __launch_bounds__(256) void k_loss_win(SpsWinLaunch W, const float* __restrict__ grad_out,
                                                  const uint64_t* __restrict__ n_valid, float* __restrict__ grad,
                                                  double* __restrict__ part_f, uint64_t* __restrict__ part_n) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  const StressLaunch& P = W.P;
  uint32_t* zipf = reinterpret_cast<uint32_t*>(lds);
  uint16_t* guide = reinterpret_cast<uint16_t*>(lds + (size_t)(P.W + 1) * 4);
  for (uint32_t k = threadIdx.x; k <= P.W; k += blockDim.x) zipf[k] = P.zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) guide[k] = P.guide[k];
  __syncthreads();
  double scale = 0.0;
  if (kGrad) {
    const uint64_t n = n_valid[0];
    if (n == 0) return;
    scale = (double)grad_out[0] * 2.0 / (double)n;
  }
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t x = blockIdx.x % kXcds;
  const uint32_t gb = uload(W.sbeg + x);
  const uint32_t nq = uload(W.sbeg + x + 1) - gb;
  const uint64_t* __restrict__ xi = W.xitem + (size_t)x * W.xstride;
  const uint64_t n_items = uniform_u64(uload(xi + nq));
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(W.queue + ((size_t)(kGrad ? 1 : 0) * kXcds + x) * 16);
  float* __restrict__ GX = grad;
  float* __restrict__ GY = grad + 2ull * P.n_nodes;
  double acc = 0.0;
  uint64_t nv = 0;
  uint32_t q = 0;
  for (uint64_t m = 0, m_end = 0;; ++m) {
    if (m >= m_end) {
      uint64_t base = 0;
      if (lane == 0) base = atomicAdd(ctr, (unsigned long long)kSpsGrab);
      m = uniform_u64(base);
      if (m >= n_items) break;
      m_end = min(m + kSpsGrab, n_items);
    }
    while (q + 1 < nq && uniform_u64(uload(xi + q + 1)) <= m) q = uniform_u32(q + 1);
    const uint32_t g = gb + q;
    const uint64_t u0 = uniform_u64(uload(W.seg_off + g)) + (m - uniform_u64(uload(xi + q))) * 64;
    const uint64_t u_end = uniform_u64(uload(W.seg_off + g + 1));
    const uint64_t sst = uniform_u64(uload(W.seg_start + g));
    const uint64_t slen = uniform_u64(uload(W.seg_start + g + 1)) - sst;
    const uint32_t p = uniform_u32(uload(W.seg_path + g));
    const uint64_t pst = uniform_u64(uload(P.path_off + p));
    const uint64_t plen = uniform_u64(uload(P.path_off + p + 1)) - pst;
    const uint64_t u = u0 + lane;
    if (u >= u_end) continue;
    const Rand4 r = philox10((uint32_t)u, (uint32_t)(u >> 32), P.word2, W.slot_c3, P.k0, P.k1);
    const uint64_t i = sst + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), slen);
    uint64_t j, a, b;
    double d;
    if (!partner_power_law(i, pst, plen, r.r2, r.r3, zipf, guide, P.W, j)) continue;
    if (!pair_terms(P.rec, i, j, r.r3 & 1u, (r.r3 >> 1) & 1u, a, b, d) || a == b) continue;
    if (!kGrad) {
      acc += stress_work(P.work, a, b, d);
      ++nv;
    } else {
      double dx, dy;
      const double mag = delta_work(P.work, a, b, dx, dy);
      if (mag == 0.0) continue;
      const double c = scale * (mag - d) / (d * d) / mag;
      const float gx = (float)(c * dx), gy = (float)(c * dy);
      if (P.inv) {  // the gradient is in the caller's node order
        a = 2ull * P.inv[a >> 1] + (a & 1);
        b = 2ull * P.inv[b >> 1] + (b & 1);
      }
      unsafeAtomicAdd(&GX[a], gx);
      unsafeAtomicAdd(&GY[a], gy);
      unsafeAtomicAdd(&GX[b], -gx);
      unsafeAtomicAdd(&GY[b], -gy);
    }
  }
  if (!kGrad) {
    acc = block_sum(acc, red_f);
    nv = block_sum(nv, red_n);
    if (threadIdx.x == 0) {
      part_f[blockIdx.x] = acc;
      part_n[blockIdx.x] = nv;
    }
  }
}

// ---------------------------------------------------------------------------
// The loss adjoint by tiles.  The ~30 paths through a node each add to its
// gradient, from their own segments; a tile gathers the segments of all paths
// whose steps start in one range of device node ids (the ids follow the
// paths), so most of a tile's adjoint lands in an LDS image of that range and
// reaches memory once per touched entry instead of once per pair.
// ---------------------------------------------------------------------------
size_t loss_tile_lds_bytes(uint32_t W, bool grad) {
  const size_t head = ((size_t)(W + 1) * 4 + (size_t)(kGuideSize + 1) * 2 + 15) & ~(size_t)15;
  return head + (grad ? (size_t)4 * kTileNodes * sizeof(float2) : 0);
}

// kGrad = false: the forward pass over the same tiles (per-block sums of the
// stress and the valid-pair count; the tile order keeps a block's coordinate
// reads within one range of node ids).
template <bool kGrad>
__global__ __launch_bounds__(kTileThreads) void k_loss_tile(SpsWinLaunch W, TileLaunch T,
                                                           const float* __restrict__ grad_out,
                                                           const uint64_t* __restrict__ n_valid,
                                                           float* __restrict__ grad, double* __restrict__ part_f,
                                                           uint64_t* __restrict__ part_n) {
  __shared__ double red_f[16];
  __shared__ uint64_t red_n[16];
  extern __shared__ __align__(16) char lds[];
  __shared__ uint64_t s_flat[kTileMaxSeg + 1];  // slot prefix over the tile's segments
  __shared__ uint64_t s_slot[kTileMaxSeg];      // first slot of each segment
  __shared__ uint64_t s_start[kTileMaxSeg];     // first step of each segment
  __shared__ uint32_t s_len[kTileMaxSeg];       // steps of each segment
  __shared__ uint32_t s_path[kTileMaxSeg];
  __shared__ uint32_t s_tile;
  const StressLaunch& P = W.P;
  uint32_t* zipf = reinterpret_cast<uint32_t*>(lds);
  uint16_t* guide = reinterpret_cast<uint16_t*>(lds + (size_t)(P.W + 1) * 4);
  float2* acc = reinterpret_cast<float2*>(
      lds + (((size_t)(P.W + 1) * 4 + (size_t)(kGuideSize + 1) * 2 + 15) & ~(size_t)15));
  constexpr uint32_t kAcc = 4 * kTileNodes;  // entries: 2 * kTileNodes nodes x 2 endpoints
  for (uint32_t k = threadIdx.x; k <= P.W; k += blockDim.x) zipf[k] = P.zipf[k];
  for (uint32_t k = threadIdx.x; k <= kGuideSize; k += blockDim.x) guide[k] = P.guide[k];
  double scale = 0.0;
  if (kGrad) {
    const uint64_t n = n_valid[0];
    if (n == 0) return;  // uniform over the grid: no block waits at a barrier below
    scale = (double)grad_out[0] * 2.0 / (double)n;
  }
  double sum = 0.0;
  uint64_t nv = 0;
  float* __restrict__ GX = grad;
  float* __restrict__ GY = grad + 2ull * P.n_nodes;
  auto global_add = [&](uint64_t a, float gx, float gy) {
    if (P.inv) a = 2ull * P.inv[a >> 1] + (a & 1);  // the gradient is in the caller's node order
    unsafeAtomicAdd(&GX[a], gx);
    unsafeAtomicAdd(&GY[a], gy);
  };
  for (;;) {
    __syncthreads();  // the previous tile's flush (and the tables above) are done
    if (threadIdx.x == 0) s_tile = atomicAdd(T.queue, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    if (t >= T.n_tiles) break;
    const uint64_t base = T.base[t];
    const uint32_t k0 = T.off[t];
    const uint32_t nk = T.off[t + 1] - k0;
    if (kGrad)
      for (uint32_t e = threadIdx.x; e < kAcc; e += blockDim.x) acc[e] = make_float2(0.0f, 0.0f);
    for (uint32_t k = threadIdx.x; k < nk; k += blockDim.x) {
      const uint32_t g = T.seg[k0 + k];
      s_slot[k] = W.seg_off[g];
      s_flat[k + 1] = W.seg_off[g + 1] - W.seg_off[g];
      s_start[k] = W.seg_start[g];
      s_len[k] = (uint32_t)(W.seg_start[g + 1] - W.seg_start[g]);
      s_path[k] = W.seg_path[g];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_flat[0] = 0;
      for (uint32_t k = 0; k < nk; ++k) s_flat[k + 1] += s_flat[k];
    }
    __syncthreads();
    const uint64_t total = s_flat[nk];
    for (uint64_t f = threadIdx.x; f < total; f += blockDim.x) {
      uint32_t lo = 0, hi = nk;  // the segment k with s_flat[k] <= f < s_flat[k + 1]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_flat[mid] <= f) lo = mid;
        else hi = mid;
      }
      const uint64_t u = s_slot[lo] + (f - s_flat[lo]);
      const uint32_t p = s_path[lo];
      const uint64_t pst = P.path_off[p];
      const uint64_t plen = P.path_off[p + 1] - pst;
      const Rand4 r = philox10((uint32_t)u, (uint32_t)(u >> 32), P.word2, W.slot_c3, P.k0, P.k1);
      const uint64_t i = s_start[lo] + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), s_len[lo]);
      uint64_t j, a, b;
      double d;
      if (!partner_power_law(i, pst, plen, r.r2, r.r3, zipf, guide, P.W, j)) continue;
      if (!pair_terms(P.rec, i, j, r.r3 & 1u, (r.r3 >> 1) & 1u, a, b, d) || a == b) continue;
      if (!kGrad) {
        sum += stress_work(P.work, a, b, d);
        ++nv;
        continue;
      }
      double dx, dy;
      const double mag = delta_work(P.work, a, b, dx, dy);
      if (mag == 0.0) continue;
      const double c = scale * (mag - d) / (d * d) / mag;
      const float gx = (float)(c * dx), gy = (float)(c * dy);
      const uint64_t oa = (a >> 1) - base, ob = (b >> 1) - base;  // wraps to huge below the base
      if (oa < 2ull * kTileNodes) {
        atomicAdd(&acc[(oa << 1) | (a & 1)].x, gx);
        atomicAdd(&acc[(oa << 1) | (a & 1)].y, gy);
      } else {
        global_add(a, gx, gy);
      }
      if (ob < 2ull * kTileNodes) {
        atomicAdd(&acc[(ob << 1) | (b & 1)].x, -gx);
        atomicAdd(&acc[(ob << 1) | (b & 1)].y, -gy);
      } else {
        global_add(b, -gx, -gy);
      }
    }
    if (kGrad) {
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < kAcc; e += blockDim.x) {
        const float2 v = acc[e];
        const uint64_t node = base + (e >> 1);
        if ((v.x != 0.0f || v.y != 0.0f) && node < P.n_nodes) global_add(2ull * node + (e & 1), v.x, v.y);
      }
    }
  }
  if (!kGrad) {
    sum = block_sum(sum, red_f);
    nv = block_sum(nv, red_n);
    if (threadIdx.x == 0) {
      part_f[blockIdx.x] = sum;
      part_n[blockIdx.x] = nv;
    }
  }
}

__global__ __launch_bounds__(256) void k_segment_min_node(const StepRec* __restrict__ rec,
                                                          const uint64_t* __restrict__ start, uint32_t nseg,
                                                          uint32_t* __restrict__ out) {
  const uint32_t g = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);  // one wave per segment
  if (g >= nseg) return;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t m = 0xFFFFFFFFu;
  for (uint64_t k = start[g] + lane; k < start[g + 1]; k += 64) m = min(m, rec[k].node_rev & kNodeMask);
  for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o, 64));
  if (lane == 0) out[g] = m;
}

// ---------------------------------------------------------------------------
// Initial layout and first visits
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

__global__ __launch_bounds__(256) void k_first_visit(const StepRec* __restrict__ rec, uint64_t S,
                                                     uint64_t* __restrict__ first) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += stride) {
    const uint32_t node = rec[s].node_rev & kNodeMask;
    atomicMin(reinterpret_cast<unsigned long long*>(&first[node]), (unsigned long long)s);
  }
}

// Thread k handles endpoint k = 2m + e of device node m (caller id inv[m] on a
// renumbered graph); the jitter draw is keyed by the caller's endpoint index.
__global__ __launch_bounds__(256) void k_init_coords(const StepRec* __restrict__ rec,
                                                     const uint64_t* __restrict__ first, uint64_t n_nodes,
                                                     const uint32_t* __restrict__ inv, uint32_t k0, uint32_t k1,
                                                     uint32_t c3, float jitter, float* __restrict__ coords) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  float* __restrict__ X = coords;
  float* __restrict__ Y = coords + 2 * n_nodes;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 2 * n_nodes; k += stride) {
    const uint64_t s = first[k >> 1];
    const uint64_t c = inv ? 2ull * inv[k >> 1] + (k & 1) : k;
    float x = 0.0f;
    if (s != ~0ull) {
      const StepRec r = load_rec(rec, s);
      x = (float)(r.pos + (int64_t)r.len * (int64_t)(k & 1));
    }
    X[c] = x;
    const Rand4 rn = philox10((uint32_t)c, (uint32_t)(c >> 32), 0u, c3, k0, k1);
    const float u = (float)(rn.r0 >> 8) * (1.0f / 16777216.0f);
    Y[c] = jitter * (u - 0.5f);
  }
}

// ---------------------------------------------------------------------------
// Adam (Kingma and Ba, 2015); c1 = 1 - beta1^t, c2 = 1 - beta2^t.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ x, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, uint64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    x[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static size_t loss_lds_bytes(const StressLaunch& P) {
  return (size_t)P.path_slots * 8 + (size_t)(P.W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
}

static uint32_t grid_for(uint64_t n, uint32_t cap) {
  const uint64_t b = (n + 255) / 256;
  return (uint32_t)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t launch_sps_pass(const StressLaunch& P, int pass, int mode, const double* mean_dev, double* part_f,
                           uint64_t* part_n, uint64_t* part_skip, hipStream_t s) {
  const size_t lds = mode == 1 ? loss_lds_bytes(P) : (size_t)P.path_slots * 8;
  hipLaunchKernelGGL(k_sps, dim3(kStressBlocks), dim3(kStressThreads), lds, s, P, pass, mode, mean_dev, part_f,
                     part_n, part_skip);
  return hipGetLastError();
}

hipError_t launch_sps_win_count_scan(const SpsWinLaunch& W, hipStream_t s) {
  const size_t lds = (size_t)W.P.path_slots * 8 + (size_t)W.n_seg * 4;
  hipLaunchKernelGGL(k_sps_win_count, dim3(W.count_blocks), dim3(1024), lds, s, W);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_sps_win_scan, dim3(1), dim3(1024), (size_t)W.n_seg * 4, s, W);
  return hipGetLastError();
}

hipError_t launch_sps_win_pass(const SpsWinLaunch& W, int pass, const double* mean_dev, double* part_f,
                               uint64_t* part_n, uint64_t* part_skip, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_sps_win, dim3(blocks), dim3(kStressThreads), 0, s, W, pass, mean_dev, part_f, part_n,
                     part_skip);
  return hipGetLastError();
}

hipError_t launch_path_stress_exact(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s) {
  hipLaunchKernelGGL(k_path_stress_exact, dim3(kStressBlocks), dim3(kStressThreads), (size_t)P.path_slots * 8, s, P,
                     part_f, part_n);
  return hipGetLastError();
}

hipError_t launch_reduce_parts(const double* part_f, const uint64_t* part_n, const uint64_t* part_skip,
                               uint32_t n_parts, double* out_f, uint64_t* out_n, double* mean_out,
                               float* loss_out, uint64_t* n_valid_out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(1024), 0, s, part_f, part_n, part_skip, n_parts, out_f, out_n,
                     mean_out, loss_out, n_valid_out);
  return hipGetLastError();
}

hipError_t launch_stress_fwd(const StressLaunch& P, double* part_f, uint64_t* part_n, hipStream_t s) {
  hipLaunchKernelGGL(k_stress_fwd, dim3(kStressBlocks), dim3(kStressThreads), loss_lds_bytes(P), s, P, part_f,
                     part_n);
  return hipGetLastError();
}

hipError_t launch_stress_bwd(const StressLaunch& P, const float* grad_out, const uint64_t* n_valid, float* grad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_stress_bwd, dim3(kStressBlocks), dim3(kStressThreads), loss_lds_bytes(P), s, P, grad_out,
                     n_valid, grad);
  return hipGetLastError();
}

hipError_t launch_loss_win_fwd(const SpsWinLaunch& W, double* part_f, uint64_t* part_n, uint32_t blocks,
                               hipStream_t s) {
  const size_t lds = (size_t)(W.P.W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
  hipLaunchKernelGGL(k_loss_win<false>, dim3(blocks), dim3(kStressThreads), lds, s, W, nullptr, nullptr, nullptr,
                     part_f, part_n);
  return hipGetLastError();
}

hipError_t launch_loss_win_bwd(const SpsWinLaunch& W, const float* grad_out, const uint64_t* n_valid, float* grad,
                               uint32_t blocks, hipStream_t s) {
  const size_t lds = (size_t)(W.P.W + 1) * 4 + (size_t)(kGuideSize + 1) * 2;
  hipLaunchKernelGGL(k_loss_win<true>, dim3(blocks), dim3(kStressThreads), lds, s, W, grad_out, n_valid, grad,
                     nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_loss_tile_bwd(const SpsWinLaunch& W, const TileLaunch& T, const float* grad_out,
                                const uint64_t* n_valid, float* grad, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_tile<true>, dim3(blocks), dim3(kTileThreads), loss_tile_lds_bytes(W.P.W, true), s, W,
                     T, grad_out, n_valid, grad, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_loss_tile_fwd(const SpsWinLaunch& W, const TileLaunch& T, double* part_f, uint64_t* part_n,
                                uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_loss_tile<false>, dim3(blocks), dim3(kTileThreads), loss_tile_lds_bytes(W.P.W, false), s,
                     W, T, nullptr, nullptr, nullptr, part_f, part_n);
  return hipGetLastError();
}

hipError_t launch_segment_min_node(const StepRec* rec, const uint64_t* start, uint32_t nseg, uint32_t* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_segment_min_node, dim3((nseg + 3) / 4), dim3(256), 0, s, rec, start, nseg, out);
  return hipGetLastError();
}

hipError_t launch_first_visit(const StepRec* rec, uint64_t S, uint64_t n_nodes, uint64_t* first_step,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n_nodes, 4096)), dim3(256), 0, s, first_step, n_nodes, ~0ull);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 0) return e;
  hipLaunchKernelGGL(k_first_visit, dim3(grid_for(S, 8192)), dim3(256), 0, s, rec, S, first_step);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_init_coords(const StepRec* rec, const uint64_t* first_step, uint64_t n_nodes, const uint32_t* inv,
                              uint32_t k0, uint32_t k1, uint32_t c3, float jitter, float* coords, hipStream_t s) {
  hipLaunchKernelGGL(k_init_coords, dim3(grid_for(2 * n_nodes, 8192)), dim3(256), 0, s, rec, first_step, n_nodes,
                     inv, k0, k1, c3, jitter, coords);
  return hipGetLastError();
}

hipError_t launch_adam(float* x, const float* g, float* m, float* v, uint64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n, 8192)), dim3(256), 0, s, x, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace pgsgd
