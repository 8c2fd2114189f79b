// Window-major schedule of one PG-SGD iteration for gfx950.
//
// The steps are cut into windows of 2^win_shift consecutive global steps.  An
// iteration of T terms is enumerated window by window:
//   1. counts: n_w = the number of the iteration's plain step draws (term t:
//      i_t = floor(u64(t) * S / 2^64), the same draw as the plain schedule)
//      that fall in window w, so (n_w) is exactly multinomial(T, |w| / S);
//   2. slot k of window w (global slot s = sum_{v<w} n_v + k) draws its step
//      uniformly inside the window from Philox stream 5 at counter s, and its
//      partner, endpoint coins and cooling exactly as a plain term does; the
//      cooling coin belongs to aligned groups of 64 slots of a window.
// A multinomial number of uniform draws per window is an i.i.d. uniform draw
// over all steps, so an iteration samples the same distribution of terms as
// Alg. 1; only the processing order differs (Hogwild leaves it free).
//
// Every path is cut into 8 * streams equal pieces and the windows are grouped
// into runs by the piece they start in (run sigma: piece sigma of path 0, then
// of path 1, ...).  XCD x (blocks b with b mod 8 = x) works on its `streams`
// runs at the same time, each run window after window.  So a window's step
// records and the coordinates of the nodes its steps visit (close ids in a
// locality-ordered graph) stay in the XCD's 4 MB L2, cooling partners (within W
// steps) fall into the same window, uniform partners stay inside the one or
// two paths in progress (few address translation misses), and the concurrent
// updates are spread over 8 * streams far-apart stretches of the graph (few
// lost Hogwild updates).
//   k_local_count  plain draw i_t, window histogram (LDS, then global)
//   k_local_scan   window offsets, per-run group prefixes; clears the histogram
//   k_layout_local slot draw, sample, gather, update
#include "device.h"
#include "local.h"

namespace pgsgd {

// Loads of the read-only run metadata at wave-uniform addresses: through the
// constant address space, so they become scalar loads (scalar cache) instead
// of vector loads with a full memory round trip each.
template <typename T>
__device__ __forceinline__ T uload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)(p);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  return ((uint64_t)uniform_u32((uint32_t)(v >> 32)) << 32) | uniform_u32((uint32_t)v);
}

__global__ __launch_bounds__(1024) void k_local_count(LocalLaunch P) {
  extern __shared__ __align__(16) char lds[];
  uint32_t* hist = reinterpret_cast<uint32_t*>(lds);
  for (uint32_t k = threadIdx.x; k < P.n_win; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const LayoutLaunch& L = P.L;
  const uint64_t lane_stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < L.n_terms; t += lane_stride) {
    const Rand4 r = philox10((uint32_t)t, (uint32_t)(t >> 32), L.iter, L.c3, L.k0, L.k1);
    const uint64_t i = mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), L.S);
    atomicAdd(&hist[(uint32_t)(i >> P.win_shift)], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < P.n_win; k += blockDim.x)
    if (hist[k]) atomicAdd(&P.wcount[k], hist[k]);
}

// One block of 1024 threads.  woff = exclusive prefix of wcount (window-id
// order); per run the prefix of ceil(n_w / 64) over its windows (run order);
// then wcount = 0.  Each thread owns a contiguous chunk of windows; every
// stage is a chunk pass plus a block scan, so no thread walks a long chain of
// dependent loads.
__global__ __launch_bounds__(1024) void k_local_scan(LocalLaunch P) {
  __shared__ uint64_t lds16[16];
  const uint32_t n = P.n_win;
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t k0 = min(n, threadIdx.x * per);
  const uint32_t k1 = min(n, k0 + per);
  uint64_t s = 0;
  for (uint32_t k = k0; k < k1; ++k) s += P.wcount[k];
  uint64_t total;
  uint64_t acc = block_exclusive_scan(s, lds16, &total);
  for (uint32_t k = k0; k < k1; ++k) {
    P.woff[k] = acc;
    acc += P.wcount[k];
  }
  if (threadIdx.x == 0) P.woff[n] = total;
  // per run: the threads split the run's windows (in run order) into chunks
  const uint32_t runs = kXcds * P.streams;
  for (uint32_t run = 0; run < runs; ++run) {
    const uint32_t b = P.sbeg[run], e = P.sbeg[run + 1], nq = e - b;
    const uint32_t rper = (nq + blockDim.x - 1) / blockDim.x;
    const uint32_t q0 = min(nq, threadIdx.x * rper), q1 = min(nq, q0 + rper);
    uint64_t items = 0;
    for (uint32_t q = q0; q < q1; ++q) items += (P.wcount[P.worder[b + q]] + 63) >> 6;
    uint64_t run_total;
    uint64_t pre = block_exclusive_scan(items, lds16, &run_total);
    uint64_t* xi = P.xitem + (size_t)run * P.xstride;
    for (uint32_t q = q0; q < q1; ++q) {
      xi[q] = pre;
      pre += (P.wcount[P.worder[b + q]] + 63) >> 6;
    }
    if (threadIdx.x == 0) xi[nq] = run_total;
  }
  __syncthreads();
  for (uint32_t k = k0; k < k1; ++k) P.wcount[k] = 0;
}

// The update of apply_update with the loads ordered for a window-local i
// endpoint a and a partner b that may lie anywhere in the path (uniform
// partners): b is read first and a only once b has arrived, so the span in
// which a concurrent update of a (a node of the active window, where the
// in-flight terms concentrate) can be lost is one L2 round trip instead of a
// far memory access.  The empty asm makes the address of a depend on the
// loaded b (no instruction is emitted).  The step is clamped_step's.
__device__ __forceinline__ void apply_update_far_first(float2* __restrict__ W, uint64_t a, uint64_t b, float d,
                                                       float eta) {
  const float2 pb = W[b];
  uint32_t lo = (uint32_t)a;
  asm volatile("" : "+v"(lo) : "v"(pb.x), "v"(pb.y));
  a = (a & ~0xFFFFFFFFull) | lo;
  const float2 pa = W[a];
  float2 m;
  if (!clamped_step(pa, pb, d, eta, m)) return;
  W[a] = make_float2(pa.x - m.x, pa.y - m.y);
  W[b] = make_float2(pb.x + m.x, pb.y + m.y);
}

// The 64 slots of item m of a run (windows worder[wb], worder[wb + 1], ...);
// q is the calling wave's window cursor in the run (items only grow).
__device__ __forceinline__ void local_item(const LocalLaunch& P, const LdsView& V, uint32_t wb, uint32_t nq,
                                           const uint64_t* __restrict__ xi, uint64_t m, uint32_t& q) {
  const LayoutLaunch& L = P.L;
  const uint32_t lane = threadIdx.x & 63u;
  while (q + 1 < nq && uniform_u64(uload(xi + q + 1)) <= m) q = uniform_u32(q + 1);
  const uint32_t w = uniform_u32(uload(P.worder + wb + q));
  const uint64_t wbeg = uniform_u64(uload(P.woff + w));
  const uint64_t nw = uniform_u64(uload(P.woff + w + 1)) - wbeg;
  const uint64_t k = (m - uniform_u64(uload(xi + q))) * 64 + lane;
  const uint64_t s = wbeg + k;  // global slot
  const uint32_t slot_c3 = (kStreamWindow << 24) | (L.c3 & 0xFFFFFFu);
  const Rand4 r = philox10((uint32_t)s, (uint32_t)(s >> 32), L.iter, slot_c3, L.k0, L.k1);
  const uint32_t lead = uniform_u32(r.r3);  // lane 0: slot 64 * group, always inside the window
  const bool cooling = L.cool_all || ((lead >> 3) & 1u);
  if (k >= nw) return;
  const uint64_t wstart = (uint64_t)w << P.win_shift;
  const uint64_t wlen = min((uint64_t)1 << P.win_shift, L.S - wstart);
  Term T;
  T.i = wstart + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), wlen);
  // the path of a window inside one path is known; a window across paths searches
  const uint32_t wp = uniform_u32(uload(P.wpath + w));
  const uint32_t p = (wp >> 31) ? find_path(V.off, L.path_top, T.i) : wp;
  const uint64_t start = V.off[p];
  const uint64_t len = V.off[p + 1] - start;
  bool ok = true;
  if (cooling) ok = partner_power_law(T.i, start, len, r.r2, r.r3, V.zipf, V.guide, L.W, T.j);
  else T.j = start + mulhi32(r.r2, (uint32_t)len);
  T.flags = (r.r3 & 3u) | ((cooling ? 1u : 0u) << 2) | ((ok ? 0u : 1u) << 3);
  if (L.trace_f) {  // parity hook: record the slots of [t_begin, t_end) instead of applying them
    if (s < L.t_begin || s >= L.t_end) return;
    if (!(T.flags & 8u)) {
      uint64_t a, b;
      float d;
      if (!resolve_term(L.rec, T, a, b, d)) T.flags |= 8u;
    }
    const uint64_t o = s - L.t_begin;
    L.trace_i[o] = T.i;
    L.trace_j[o] = T.j;
    L.trace_f[o] = (uint8_t)T.flags;
    return;
  }
  if (T.flags & 8u) return;
  // parity hook: only a chosen subset of the slots of [t_begin, t_end)
  if (L.apply_mask && (s < L.t_begin || s >= L.t_end || !L.apply_mask[s - L.t_begin])) return;
  uint64_t a, b;
  float d;
  if (!resolve_term(L.rec, T, a, b, d)) return;
  if (cooling) apply_update(L.work, a, b, d, L.eta);  // both endpoints in or next to the window
  else apply_update_far_first(L.work, a, b, d, L.eta);
}

// The draws of item m of a run in an all-cooling iteration (no loads beyond
// the run's metadata, read at wave-uniform addresses, and the LDS tables):
// the lane's term, or flags bit 3 when the lane has no slot or no partner;
// slot = the lane's global slot, ~0 when it has none.
__device__ __forceinline__ Term cooling_draw(const LocalLaunch& P, const LdsView& V, uint32_t wb, uint32_t nq,
                                             const uint64_t* __restrict__ xi, uint64_t m, uint32_t& q,
                                             uint64_t& slot) {
  const LayoutLaunch& L = P.L;
  const uint32_t lane = threadIdx.x & 63u;
  while (q + 1 < nq && uniform_u64(uload(xi + q + 1)) <= m) q = uniform_u32(q + 1);
  const uint32_t w = uniform_u32(uload(P.worder + wb + q));
  const uint64_t wbeg = uniform_u64(uload(P.woff + w));
  const uint64_t nw = uniform_u64(uload(P.woff + w + 1)) - wbeg;
  const uint64_t k = (m - uniform_u64(uload(xi + q))) * 64 + lane;
  const uint64_t s = wbeg + k;
  const uint32_t slot_c3 = (kStreamWindow << 24) | (L.c3 & 0xFFFFFFu);
  const Rand4 r = philox10((uint32_t)s, (uint32_t)(s >> 32), L.iter, slot_c3, L.k0, L.k1);
  Term T;
  T.j = 0;
  slot = ~0ull;
  if (k >= nw) {
    T.i = 0;
    T.flags = 8u;
    return T;
  }
  slot = s;
  const uint64_t wstart = (uint64_t)w << P.win_shift;
  const uint64_t wlen = min((uint64_t)1 << P.win_shift, L.S - wstart);
  T.i = wstart + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), wlen);
  const uint32_t wp = uniform_u32(uload(P.wpath + w));
  const uint32_t p = (wp >> 31) ? find_path(V.off, L.path_top, T.i) : wp;
  const uint64_t start = V.off[p];
  const uint64_t len = V.off[p + 1] - start;
  const bool ok = partner_power_law(T.i, start, len, r.r2, r.r3, V.zipf, V.guide, L.W, T.j);
  T.flags = (r.r3 & 3u) | 4u | ((ok ? 0u : 1u) << 3);
  return T;
}

// A run of an all-cooling iteration, two items deep: the step records of
// item m are requested, then item m + 1 is drawn (Philox, path, power-law
// partner: arithmetic and LDS only) while they arrive, then item m is updated.
// Only the draw runs ahead; the coordinates of item m are read and written as
// in local_item, so no more updates are in flight.  The slots and their terms
// are those of local_item; with the recording hook set (trace_f) the terms of
// the slots [t_begin, t_end) are recorded instead of applied, as local_item
// records them.
__device__ __forceinline__ void local_run_cooling(const LocalLaunch& P, const LdsView& V, uint32_t wb, uint32_t nq,
                                                  const uint64_t* __restrict__ xi_in, uint64_t n_items,
                                                  unsigned long long* ctr) {
  const LayoutLaunch& L = P.L;
  const uint32_t lane = threadIdx.x & 63u;
  // the run's prefix row at a wave-uniform address: its reads are scalar loads, which the
  // vector-memory waits for the records below do not include
  const uint64_t* __restrict__ xi = reinterpret_cast<const uint64_t*>(uniform_u64(reinterpret_cast<uint64_t>(xi_in)));
  auto grab = [&](uint64_t& m, uint64_t& m_end) -> bool {
    uint64_t base = 0;
    if (lane == 0) base = atomicAdd(ctr, (unsigned long long)P.grab);
    m = ((uint64_t)uniform_u32((uint32_t)(base >> 32)) << 32) | uniform_u32((uint32_t)base);
    if (m >= n_items) return false;
    m_end = min(m + P.grab, n_items);
    return true;
  };
  uint32_t q = 0;
  uint64_t m = 0, m_end = 0;
  if (!grab(m, m_end)) return;
  uint64_t slot;
  if (L.trace_f) {  // parity hook: the drawn terms of the slots [t_begin, t_end), nothing applied
    for (;;) {
      Term T = cooling_draw(P, V, wb, nq, xi, m, q, slot);
      if (slot >= L.t_begin && slot < L.t_end) {
        if (!(T.flags & 8u)) {
          uint64_t a, b;
          float d;
          if (!resolve_term(L.rec, T, a, b, d)) T.flags |= 8u;
        }
        const uint64_t o = slot - L.t_begin;
        L.trace_i[o] = T.i;
        L.trace_j[o] = T.j;
        L.trace_f[o] = (uint8_t)T.flags;
      }
      if (++m >= m_end && !grab(m, m_end)) return;
    }
  }
  Term cur = cooling_draw(P, V, wb, nq, xi, m, q, slot);
  for (;;) {
    // the next item's index first: a grab waits for its atomic before this item's loads are issued
    uint64_t mn = m + 1, mn_end = m_end;
    const bool more = mn < m_end || grab(mn, mn_end);
    const bool live = !(cur.flags & 8u);
    StepRec si, sj;
    if (live) {
      si = load_rec(L.rec, cur.i);
      sj = load_rec(L.rec, cur.j);
    }
    Term nxt;
    nxt.flags = 8u;
    if (more) nxt = cooling_draw(P, V, wb, nq, xi, mn, q, slot);
    if (live) {
      const uint32_t ei = cur.flags & 1u, ej = (cur.flags >> 1) & 1u;
      const uint64_t a = 2ull * (si.node_rev & kNodeMask) + ei;
      const uint64_t b = 2ull * (sj.node_rev & kNodeMask) + ej;
      const int64_t dd = endpoint_pos(si, ei) - endpoint_pos(sj, ej);
      if (a != b && dd != 0) apply_update(L.work, a, b, (float)(dd < 0 ? -dd : dd), L.eta);
    }
    if (!more) break;
    cur = nxt;
    m = mn;
    m_end = mn_end;
  }
}

__device__ __forceinline__ float2 shfl_f2(float2 v, int src) {
  return make_float2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// The data-reuse variant on the window-major slots: the group of item m (64
// slots of one window) makes its primary updates in registers, then rounds k =
// 1..drf-1 pair lane l's i-endpoint with lane (l + o_k) mod 64's j-endpoint
// (both live, unskipped, steps on the same path) through cross-lane shuffles;
// the j-endpoint's move is shuffled back to its owner, and every endpoint is
// stored once at the end.  o_k from Philox stream 4 at counter (the group's
// first slot, iteration).  All lanes stay active up to the shuffles.
__device__ __forceinline__ void local_item_reuse(const LocalLaunch& P, const LdsView& V, uint32_t wb, uint32_t nq,
                                                 const uint64_t* __restrict__ xi, uint64_t m, uint32_t& q) {
  const LayoutLaunch& L = P.L;
  const uint32_t lane = threadIdx.x & 63u;
  while (q + 1 < nq && uniform_u64(uload(xi + q + 1)) <= m) q = uniform_u32(q + 1);
  const uint32_t w = uniform_u32(uload(P.worder + wb + q));
  const uint64_t wbeg = uniform_u64(uload(P.woff + w));
  const uint64_t nw = uniform_u64(uload(P.woff + w + 1)) - wbeg;
  const uint64_t k0 = (m - uniform_u64(uload(xi + q))) * 64;  // the group's first slot in the window
  const uint64_t k = k0 + lane;
  const uint64_t s = wbeg + k;
  const uint32_t slot_c3 = (kStreamWindow << 24) | (L.c3 & 0xFFFFFFu);
  const Rand4 r = philox10((uint32_t)s, (uint32_t)(s >> 32), L.iter, slot_c3, L.k0, L.k1);
  const uint32_t lead = uniform_u32(r.r3);
  const bool cooling = L.cool_all || ((lead >> 3) & 1u);
  const bool live = k < nw;
  const uint64_t wstart = (uint64_t)w << P.win_shift;
  const uint64_t wlen = min((uint64_t)1 << P.win_shift, L.S - wstart);
  Term T;
  T.i = wstart + mulhi64((uint64_t)r.r0 | ((uint64_t)r.r1 << 32), wlen);
  const uint32_t wp = uniform_u32(uload(P.wpath + w));
  const uint32_t p = (wp >> 31) ? find_path(V.off, L.path_top, T.i) : wp;
  const uint64_t start = V.off[p];
  const uint64_t len = V.off[p + 1] - start;
  bool ok = true;
  if (cooling) ok = partner_power_law(T.i, start, len, r.r2, r.r3, V.zipf, V.guide, L.W, T.j);
  else T.j = start + mulhi32(r.r2, (uint32_t)len);
  T.flags = (r.r3 & 3u) | ((cooling ? 1u : 0u) << 2) | ((ok ? 0u : 1u) << 3);
  bool valid = live && ok;
  uint64_t a = 0, b = 0;
  int64_t pa = 0, pb = 0;
  if (valid) {
    const StepRec si = load_rec(L.rec, T.i);
    const StepRec sj = load_rec(L.rec, T.j);
    const uint32_t ei = T.flags & 1u, ej = (T.flags >> 1) & 1u;
    a = 2ull * (si.node_rev & kNodeMask) + ei;
    b = 2ull * (sj.node_rev & kNodeMask) + ej;
    pa = endpoint_pos(si, ei);
    pb = endpoint_pos(sj, ej);
    if (a == b || pa == pb) valid = false;
  }
  const uint32_t reuse_c3 = (4u << 24) | (L.c3 & 0xFFFFFFu);
  const uint64_t s0 = wbeg + k0;
  const Rand4 ro = philox10((uint32_t)s0, (uint32_t)(s0 >> 32), L.iter, reuse_c3, L.k0, L.k1);
  const uint32_t ow[4] = {ro.r0, ro.r1, ro.r2, ro.r3};
  if (L.trace_f) {  // parity hook: record the slots (and their groups' offsets) of [t_begin, t_end)
    if (live && s >= L.t_begin && s < L.t_end) {
      const uint64_t o = s - L.t_begin;
      L.trace_i[o] = T.i;
      L.trace_j[o] = T.j;
      L.trace_f[o] = (uint8_t)(T.flags | (ok && !valid ? 8u : 0u));
      if (L.trace_o)
        for (uint32_t kk = 1; kk < L.drf; ++kk)
          L.trace_o[o * (L.drf - 1) + kk - 1] =
              (uint8_t)(1 + ((ow[(kk - 1) >> 2] >> (8 * ((kk - 1) & 3))) & 0xFFu) % 63);
    }
    return;
  }
  float2* __restrict__ Wc = L.work;
  float2 A = make_float2(0.0f, 0.0f), B = make_float2(0.0f, 0.0f);
  if (valid) {
    if (cooling) {
      A = Wc[a];
      B = Wc[b];
    } else {  // far-first: the uniform partner, then the window-local endpoint
      B = Wc[b];
      uint32_t lo = (uint32_t)a;
      asm volatile("" : "+v"(lo) : "v"(B.x), "v"(B.y));
      A = Wc[(a & ~0xFFFFFFFFull) | lo];
    }
    const float d = (float)(pa < pb ? pb - pa : pa - pb);
    float2 m;
    if (clamped_step(A, B, d, L.eta, m)) {
      A = make_float2(A.x - m.x, A.y - m.y);
      B = make_float2(B.x + m.x, B.y + m.y);
    }
  }
  for (uint32_t kk = 1; kk < L.drf; ++kk) {
    const uint32_t o = 1 + ((ow[(kk - 1) >> 2] >> (8 * ((kk - 1) & 3))) & 0xFFu) % 63;
    const int src = (int)((lane + o) & 63u);       // the j-endpoint this lane pairs with
    const int dst = (int)((lane + 64u - o) & 63u);  // the lane pairing with this lane's j-endpoint
    const uint32_t vm = __shfl((uint32_t)valid, src, 64);
    const uint32_t pm = __shfl(p, src, 64);
    const uint64_t bm = __shfl(b, src, 64);
    const int64_t pbm = __shfl(pb, src, 64);
    const float2 Bm = shfl_f2(B, src);
    float2 disp = make_float2(0.0f, 0.0f);
    if (valid && vm && pm == p && a != bm && pa != pbm) {
      const float d = (float)(pa < pbm ? pbm - pa : pa - pbm);
      if (clamped_step(A, Bm, d, L.eta, disp)) A = make_float2(A.x - disp.x, A.y - disp.y);
    }
    const float2 back = shfl_f2(disp, dst);
    B = make_float2(B.x + back.x, B.y + back.y);
  }
  if (valid) {
    Wc[a] = A;
    Wc[b] = B;
  }
}

__global__ __launch_bounds__(256) void k_layout_local(LocalLaunch P) {
  extern __shared__ __align__(16) char lds[];
  const LayoutLaunch& L = P.L;
  const LdsView V = lds_view(lds, L.path_slots, L.W);
  lds_fill(V, L.path_off, L.n_paths, L.path_slots, L.zipf, L.guide, L.W);
  __syncthreads();

  // blocks are dispatched to the XCDs round-robin: block b runs on XCD b % 8
  // and takes the runs of XCD share b % 8 (with fewer than 8 blocks, block b
  // takes the shares b, b + blocks, ...); wave v of a share starts on stream
  // v mod streams and, when that run is exhausted, helps the share's other
  // runs in turn
  const uint32_t nx = min(gridDim.x, kXcds);
  const uint32_t v = (blockIdx.x / nx) * (blockDim.x >> 6) + uniform_u32(threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t x = blockIdx.x % nx; x < kXcds; x += nx)
  for (uint32_t h = 0; h < P.streams; ++h) {
    const uint32_t run = x * P.streams + (v + h) % P.streams;
    const uint32_t wb = uniform_u32(uload(P.sbeg + run));
    const uint32_t nq = uniform_u32(uload(P.sbeg + run + 1)) - wb;
    const uint64_t* __restrict__ xi = P.xitem + (size_t)run * P.xstride;
    const uint64_t n_items = uniform_u64(uload(xi + nq));
    unsigned long long* ctr = reinterpret_cast<unsigned long long*>(P.queue + (size_t)run * 16);
    if (L.cool_all && L.drf <= 1 && !L.apply_mask) {
      local_run_cooling(P, V, wb, nq, xi, n_items, ctr);
      continue;
    }
    uint32_t q = 0;
    for (uint64_t m = 0, m_end = 0;; ++m) {
      if (m >= m_end) {
        uint64_t base = 0;
        if (lane == 0) base = atomicAdd(ctr, (unsigned long long)P.grab);
        m = ((uint64_t)uniform_u32((uint32_t)(base >> 32)) << 32) | uniform_u32((uint32_t)base);
        if (m >= n_items) break;
        m_end = min(m + P.grab, n_items);
      }
      if (L.drf > 1) local_item_reuse(P, V, wb, nq, xi, m, q);
      else local_item(P, V, wb, nq, xi, m, q);
    }
  }
}

hipError_t launch_local_count_scan(const LocalLaunch& P, hipStream_t s) {
  hipLaunchKernelGGL(k_local_count, dim3(P.count_blocks), dim3(1024), (size_t)P.n_win * 4, s, P);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_local_scan, dim3(1), dim3(1024), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_layout_local(const LocalLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s) {
  hipLaunchKernelGGL(k_layout_local, dim3(blocks), dim3(threads), layout_lds_bytes(P.L.path_slots, P.L.W), s, P);
  return hipGetLastError();
}

const void* layout_local_kernel() { return reinterpret_cast<const void*>(&k_layout_local); }

}  // namespace pgsgd
