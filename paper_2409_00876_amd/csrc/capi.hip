// Host runtime and C ABI of the PG-SGD layout library (see include/pgsgd.h).
//
// Responsibilities: graph validation (all on the host, before any device
// work), packing of path steps into 16-byte records and their chunked upload
// through pinned staging buffers, the learning-rate schedule and power-law
// table, launch shapes, the two-pass sampled path stress, the differentiable
// loss, and the batched form (HIP-graph capture and autotuning).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pgsgd.h"
#include "batch.h"
#include "device.h"
#include "internal.h"
#include "stress.h"
#include "local.h"

using namespace pgsgd;

namespace {

thread_local std::string g_last_error;

void set_message(const char* fmt, va_list ap) {
  char buf[512];
  vsnprintf(buf, sizeof(buf), fmt, ap);
  g_last_error = buf;
}

pgsgd_status fail(pgsgd_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  set_message(fmt, ap);
  va_end(ap);
  return code;
}

pgsgd_status ok() {
  g_last_error.clear();
  return PGSGD_OK;
}

}  // namespace

namespace pgsgd {

int32_t set_error(int32_t code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  set_message(fmt, ap);
  va_end(ap);
  return code;
}

int32_t clear_error() { return ok(); }

}  // namespace pgsgd

namespace {

#define HIP_TRY(expr)                                                                                    \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) {                                                                              \
      (void)hipGetLastError();                                                                           \
      return fail(e_ == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE, "%s failed: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                                      \
    }                                                                                                    \
  } while (0)

constexpr uint64_t kMaxSteps = 1ull << 40;
constexpr uint64_t kMaxTerms = 1ull << 48;
constexpr int64_t kMaxPathNt = (int64_t)1 << 62;
constexpr uint32_t kMaxPaths = 1u << 20;

uint32_t pow2_floor(uint32_t v) {
  uint32_t p = 1;
  while ((p << 1) != 0 && (p << 1) <= v) p <<= 1;
  return p;
}

// Power-law table of pgsgd_zipf_table plus its guide: guide[b] = smallest k in
// [1, W] with C[k] > b * 2^(32-kGuideBits), guide[kGuideSize] = W.
void build_zipf(double theta, uint32_t W, std::vector<uint32_t>& C, std::vector<uint16_t>& guide) {
  std::vector<double> F(W + 1);
  F[0] = 0.0;
  for (uint32_t k = 1; k <= W; ++k) F[k] = F[k - 1] + std::pow((double)k, -theta);
  C.assign(W + 1, 0);
  for (uint32_t k = 1; k <= W; ++k) C[k] = (uint32_t)std::floor(F[k] / F[W] * 4294967295.0);
  guide.assign(kGuideSize + 1, (uint16_t)W);
  uint32_t k = 1;
  for (uint32_t b = 0; b < kGuideSize; ++b) {
    const uint64_t lo = (uint64_t)b << (32 - kGuideBits);
    while (k < W && (uint64_t)C[k] <= lo) ++k;
    guide[b] = (uint16_t)k;
  }
  guide[kGuideSize] = (uint16_t)W;
}

void build_schedule(uint32_t n_iters, double eta_max, double eta_min, std::vector<float>& eta) {
  eta.assign(n_iters, 0.0f);
  if (n_iters == 0) return;
  if (n_iters == 1) {
    eta[0] = (float)eta_max;
    return;
  }
  const double lambda = std::log(eta_max / eta_min) / (double)(n_iters - 1);
  for (uint32_t t = 0; t < n_iters; ++t) eta[t] = (float)(eta_max * std::exp(-lambda * (double)t));
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Graph handle
// ---------------------------------------------------------------------------
// Window-major segment tables: the windows of 2^shift steps cut at path
// boundaries, in step order; run x (XCD x) holds the segments starting in the
// x-th eighth of the steps.
struct SegTables {
  uint32_t shift = 0, nseg = 0, xstride = 0;
  uint64_t* start = nullptr;   // [nseg + 1]
  uint32_t* path = nullptr;    // [nseg]
  uint32_t* wseg = nullptr;    // [n_win + 1] first segment of every window
  uint32_t* count = nullptr;   // [nseg] histogram
  uint64_t* off = nullptr;     // [nseg + 1] first slot of every segment
  uint32_t* sbeg = nullptr;    // [kXcds + 1]
  uint64_t* xitem = nullptr;   // [kXcds][xstride]
  uint64_t* queue = nullptr;   // [2][kXcds][16]
};

struct pgsgd_graph {
  int device = 0;
  uint32_t n_nodes = 0, n_paths = 0, path_top = 1, path_slots = 2, max_path_steps = 0;
  uint64_t S = 0;
  int64_t d_max = 0;
  int n_cu = 256;
  size_t lds_limit = 65536;
  std::vector<uint64_t> h_path_off;
  StepRec* d_rec = nullptr;
  uint64_t* d_path_off = nullptr;
  uint64_t* d_first = nullptr;
  float2* d_work = nullptr;     // interleaved working copy of the coordinates
  uint32_t* d_inv = nullptr;    // renumbered graphs: caller id of every device node id (else NULL)
  std::vector<uint32_t> h_perm; // renumbered graphs: device node id of every caller id (else empty)
  // power-law table cache
  double zipf_theta = -1.0;
  uint32_t zipf_W = 0;
  uint32_t* d_zipf = nullptr;
  uint16_t* d_guide = nullptr;
  // reduction scratch
  double* d_part_f = nullptr;
  uint64_t* d_part_n = nullptr;
  uint64_t* d_part_skip = nullptr;
  double* d_out_f = nullptr;    // [8]
  uint64_t* d_out_n = nullptr;  // [4]
  double* d_mean = nullptr;     // [4]
  float2* d_work2 = nullptr;    // a second layout's working copy (pgsgd_path_stress_compare, on first use)
  size_t device_bytes = 0;
  std::unordered_map<void*, size_t> alloc_bytes;  // size of every lazily allocated buffer
  int layout_blocks_per_cu = 0;  // occupancy of k_layout_iter, filled on first use
  // window-major scratch (allocated on first use)
  uint32_t loc_nwin = 0, loc_shift = 0, loc_xstride = 0, loc_streams = 0;
  // host copy of the window tables (order, run bounds, path of a window) for
  // h_loc_shift / h_loc_streams, built on first use
  uint32_t h_loc_shift = 0, h_loc_streams = 0, h_loc_xstride = 0;
  std::vector<uint32_t> h_lorder, h_lsbeg, h_lwpath;
  uint32_t* d_lcount = nullptr;
  uint64_t* d_loff = nullptr;
  uint64_t* d_lxitem = nullptr;
  uint64_t* d_lqueue = nullptr;
  uint32_t* d_lorder = nullptr;
  uint32_t* d_lsbeg = nullptr;
  uint32_t* d_lwpath = nullptr;
  // window-major segment tables of the sampled path stress (R21) and of the
  // loss (R22), and the loss adjoint's tiles (allocated on first use)
  SegTables sps, loss;
  uint32_t n_tiles = 0, tile_shift = 0;
  uint32_t* d_tile_seg = nullptr;
  uint32_t* d_tile_off = nullptr;
  uint32_t* d_tile_base = nullptr;
  uint32_t* d_tile_queue = nullptr;
  // the loss step whose segment offsets the loss tables hold (a backward after
  // the forward of the same step reuses them)
  struct {
    const void* tables = nullptr;
    uint64_t n_pairs = 0;
    uint32_t word2 = 0, c3 = 0, k0 = 0, k1 = 0;
  } loss_key;
  // second count/offset set and the counting stream: the counts of iteration
  // t + 1 are computed on count_stream while iteration t is laid out
  uint32_t* d_lcount2 = nullptr;
  uint64_t* d_loff2 = nullptr;
  uint64_t* d_lxitem2 = nullptr;
  uint64_t* d_lqueue2 = nullptr;
  hipStream_t count_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_count[2] = {nullptr, nullptr}, ev_layout[2] = {nullptr, nullptr};

  ~pgsgd_graph() {
    DeviceGuard g(device);
    (void)hipDeviceSynchronize();
    for (void* p : {(void*)d_rec, (void*)d_path_off, (void*)d_first, (void*)d_work, (void*)d_inv, (void*)d_zipf, (void*)d_guide, (void*)d_part_f,
                    (void*)d_part_n, (void*)d_part_skip, (void*)d_out_f, (void*)d_out_n, (void*)d_mean, (void*)d_work2, (void*)d_lcount, (void*)d_loff, (void*)d_lxitem, (void*)d_lqueue, (void*)d_lorder,
                    (void*)d_lsbeg, (void*)d_lwpath, (void*)d_lcount2, (void*)d_loff2, (void*)d_lxitem2,
                    (void*)d_lqueue2, (void*)d_tile_seg, (void*)d_tile_off, (void*)d_tile_base, (void*)d_tile_queue})
      if (p) (void)hipFree(p);
    for (SegTables* t : {&sps, &loss})
      for (void* p : {(void*)t->start, (void*)t->path, (void*)t->wseg, (void*)t->count, (void*)t->off,
                      (void*)t->sbeg, (void*)t->xitem, (void*)t->queue})
        if (p) (void)hipFree(p);
    for (hipEvent_t e : {ev_start, ev_count[0], ev_count[1], ev_layout[0], ev_layout[1]})
      if (e) (void)hipEventDestroy(e);
    if (count_stream) (void)hipStreamDestroy(count_stream);
  }
};

namespace {

// PGSGD_MAX_DEVICE_BYTES (decimal bytes; unset, 0 or not a number: no cap)
// bounds the device memory each graph handle may hold, so an out-of-memory
// path can be forced without exhausting the device.
uint64_t device_byte_cap() {
  const char* v = std::getenv("PGSGD_MAX_DEVICE_BYTES");
  if (!v || !*v) return 0;
  char* end = nullptr;
  const unsigned long long x = std::strtoull(v, &end, 10);
  return (end && *end == '\0') ? (uint64_t)x : 0;
}

template <typename T>
pgsgd_status dev_alloc(pgsgd_graph* g, T** p, size_t count) {
  size_t bytes = sizeof(T) * (count ? count : 1);
  const uint64_t cap = device_byte_cap();
  if (cap && g->device_bytes + bytes > cap) {
    *p = nullptr;
    return fail(PGSGD_ERR_OOM, "allocating %zu bytes would take the graph to %llu bytes, above "
                "PGSGD_MAX_DEVICE_BYTES = %llu", bytes, (unsigned long long)(g->device_bytes + bytes),
                (unsigned long long)cap);
  }
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE, "hipMalloc(%zu bytes) failed: %s",
                bytes, hipGetErrorString(e));
  }
  g->device_bytes += bytes;
  g->alloc_bytes[(void*)*p] = bytes;
  return PGSGD_OK;
}

// Frees a set of lazily allocated device buffers and nulls their pointers.
// The ensure_* functions below free their whole set when any allocation or
// copy fails, so a later call never finds a partly built set behind a
// non-null first pointer.
void free_set(pgsgd_graph* g, std::initializer_list<void**> set) {
  for (void** q : set)
    if (*q) {
      auto it = g->alloc_bytes.find(*q);
      if (it != g->alloc_bytes.end()) {
        g->device_bytes -= it->second;
        g->alloc_bytes.erase(it);
      }
      (void)hipFree(*q);
      *q = nullptr;
    }
}

// Ensures the graph holds the power-law table for (theta, W) on the device
// (its buffers are allocated with the graph, sized for the largest window).
pgsgd_status ensure_zipf(pgsgd_graph* g, double theta, uint32_t W, hipStream_t s) {
  if (g->d_zipf && g->zipf_theta == theta && g->zipf_W == W) return PGSGD_OK;
  std::vector<uint32_t> C;
  std::vector<uint16_t> guide;
  build_zipf(theta, W, C, guide);
  HIP_TRY(hipStreamSynchronize(s));  // earlier work on this stream may still read the old table
  HIP_TRY(hipMemcpy(g->d_zipf, C.data(), sizeof(uint32_t) * C.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->d_guide, guide.data(), sizeof(uint16_t) * guide.size(), hipMemcpyHostToDevice));
  g->zipf_theta = theta;
  g->zipf_W = W;
  return PGSGD_OK;
}

pgsgd_status check_params(const pgsgd_params* p) {
  if (!p) return fail(PGSGD_ERR_INVALID_ARG, "params is NULL");
  if (p->flags & ~(uint32_t)(PGSGD_FLAG_COUNT_AHEAD | PGSGD_FLAG_COUNT_IN_ORDER))
    return fail(PGSGD_ERR_INVALID_ARG, "unknown bits in params.flags");
  if ((p->flags & PGSGD_FLAG_COUNT_AHEAD) && (p->flags & PGSGD_FLAG_COUNT_IN_ORDER))
    return fail(PGSGD_ERR_INVALID_ARG, "params.flags: COUNT_AHEAD and COUNT_IN_ORDER exclude each other");
  if (p->reuse_factor > 16) return fail(PGSGD_ERR_INVALID_ARG, "reuse_factor must be at most 16");
  if (p->schedule > PGSGD_SCHEDULE_WINDOWED || p->schedule == 2)
    return fail(PGSGD_ERR_INVALID_ARG, "unknown schedule %u (2 is reserved)", p->schedule);
  if (p->zipf_window < 1 || p->zipf_window > 65535)
    return fail(PGSGD_ERR_INVALID_ARG, "zipf_window %u outside [1, 65535]", p->zipf_window);
  if (!(p->zipf_theta >= 0.0) || !std::isfinite(p->zipf_theta))
    return fail(PGSGD_ERR_INVALID_ARG, "zipf_theta must be finite and >= 0");
  if (p->graph_id >= (1u << 24)) return fail(PGSGD_ERR_INVALID_ARG, "graph_id must be < 2^24");
  if (p->terms_per_step == 0) return fail(PGSGD_ERR_INVALID_ARG, "terms_per_step must be >= 1");
  if (!(p->eta_min > 0.0) || !std::isfinite(p->eta_min)) return fail(PGSGD_ERR_INVALID_ARG, "eta_min must be > 0");
  if (!std::isfinite(p->eta_max)) return fail(PGSGD_ERR_INVALID_ARG, "eta_max must be finite");
  const uint32_t last = p->last_iter == 0 ? p->n_iters : p->last_iter;
  if (p->first_iter > last || last > p->n_iters)
    return fail(PGSGD_ERR_INVALID_ARG, "iteration range [%u, %u) invalid for n_iters %u", p->first_iter, last,
                p->n_iters);
  return PGSGD_OK;
}

double eta_max_of(const pgsgd_params* p, int64_t d_max) {
  if (p->eta_max > 0.0) return p->eta_max;
  const double d = (double)(d_max > 0 ? d_max : 1);
  return d * d;
}

LayoutLaunch make_layout_launch(const pgsgd_graph* g, const pgsgd_params* p) {
  LayoutLaunch L{};
  L.rec = g->d_rec;
  L.work = g->d_work;
  L.path_off = g->d_path_off;
  L.zipf = g->d_zipf;
  L.guide = g->d_guide;
  L.n_nodes = g->n_nodes;
  L.S = g->S;
  const uint64_t srf = p->step_reduction > 1 ? p->step_reduction : 1;
  L.n_terms = ((uint64_t)p->terms_per_step * g->S + srf - 1) / srf;
  L.n_groups = (L.n_terms + 63) / 64;
  L.drf = p->reuse_factor > 1 ? p->reuse_factor : 1;
  L.n_paths = g->n_paths;
  L.path_slots = g->path_slots;
  L.path_top = g->path_top;
  L.W = p->zipf_window;
  L.c3 = (kStreamLayout << 24) | p->graph_id;
  L.k0 = (uint32_t)p->seed;
  L.k1 = (uint32_t)(p->seed >> 32);
  return L;
}

StressLaunch make_stress_launch(const pgsgd_graph* g, const float* coords, uint32_t stream, uint32_t graph_id,
                                uint64_t seed) {
  StressLaunch P{};
  P.rec = g->d_rec;
  P.coords = coords;
  P.path_off = g->d_path_off;
  P.inv = g->d_inv;
  P.zipf = g->d_zipf;
  P.guide = g->d_guide;
  P.n_nodes = g->n_nodes;
  P.S = g->S;
  P.n_paths = g->n_paths;
  P.path_slots = g->path_slots;
  P.path_top = g->path_top;
  P.c3 = (stream << 24) | (graph_id & 0xFFFFFFu);
  P.k0 = (uint32_t)seed;
  P.k1 = (uint32_t)(seed >> 32);
  return P;
}

pgsgd_status layout_blocks_per_cu(pgsgd_graph* g, size_t lds, int* out) {
  if (g->layout_blocks_per_cu <= 0) {
    int nb = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, layout_iter_kernel(), 256, lds));
    g->layout_blocks_per_cu = nb > 0 ? nb : 1;
  }
  *out = g->layout_blocks_per_cu;
  return PGSGD_OK;
}

// Path-guided node order (the locality the windowed schedule relies on): a
// progressive linearization along the paths.  The first path's nodes come in
// path order; every later path inserts each node not placed yet right after
// the last node of that path that is already placed (at the front when there
// is none), so a node first met on another path sits next to its neighbours
// there; nodes that no path visits go last in id order.  perm[n] = new id of n.
void path_guided_order(uint32_t n_nodes, const uint32_t* /*node_len*/, uint32_t n_paths, const uint64_t* path_off,
                       const uint32_t* step_node, std::vector<uint32_t>& perm) {
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  std::vector<uint32_t> next(n_nodes, kNone);  // linked order of the placed nodes
  std::vector<uint8_t> placed(n_nodes, 0);
  uint32_t head = kNone;
  for (uint32_t p = 0; p < n_paths; ++p) {
    uint32_t anchor = kNone;
    for (uint64_t s = path_off[p]; s < path_off[p + 1]; ++s) {
      const uint32_t n = step_node[s] & kNodeMask;
      if (!placed[n]) {
        placed[n] = 1;
        if (anchor == kNone) {
          next[n] = head;
          head = n;
        } else {
          next[n] = next[anchor];
          next[anchor] = n;
        }
      }
      anchor = n;
    }
  }
  perm.assign(n_nodes, 0);
  uint32_t k = 0;
  for (uint32_t n = head; n != kNone; n = next[n]) perm[n] = k++;
  for (uint32_t n = 0; n < n_nodes; ++n)
    if (!placed[n]) perm[n] = k++;
}

// Fraction of consecutive steps of a path whose node ids (after perm, if
// given) differ by more than kRenumberGap: steps whose coordinates cannot
// share cache lines.
constexpr uint32_t kRenumberGap = 32;
constexpr double kRenumberMinFar = 0.2;  // AUTO renumbers only above this fraction ...
constexpr double kRenumberGain = 0.5;    // ... and when the path-guided order at least halves it
double far_step_fraction(uint32_t n_paths, const uint64_t* path_off, const uint32_t* step_node,
                         const uint32_t* perm) {
  uint64_t pairs = 0, far = 0;
  for (uint32_t p = 0; p < n_paths; ++p)
    for (uint64_t s = path_off[p] + 1; s < path_off[p + 1]; ++s) {
      uint32_t u = step_node[s - 1] & kNodeMask, v = step_node[s] & kNodeMask;
      if (perm) u = perm[u], v = perm[v];
      ++pairs;
      far += (u > v ? u - v : v - u) > kRenumberGap;
    }
  return pairs ? (double)far / (double)pairs : 0.0;
}

}  // namespace

extern "C" {

const char* pgsgd_last_error(void) { return g_last_error.c_str(); }
const char* pgsgd_version(void) { return "pgsgd-gfx950 0.1.0"; }

void pgsgd_params_default(pgsgd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_iters = 30;
  p->terms_per_step = 10;
  p->eta_max = 0.0;
  p->eta_min = 0.01;
  p->zipf_theta = 0.99;
  p->zipf_window = 1000;
  p->graph_id = 0;
  p->seed = 24301;
  p->first_iter = 0;
  p->last_iter = 0;
  p->max_inflight_waves = 0;
  p->flags = 0;
  p->schedule = PGSGD_SCHEDULE_AUTO;
  p->reuse_factor = 1;
  p->step_reduction = 1;
}

pgsgd_status pgsgd_schedule(const pgsgd_params* p, int64_t d_max, float* eta_out) {
  if (!p || !eta_out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (!(p->eta_min > 0.0)) return fail(PGSGD_ERR_INVALID_ARG, "eta_min must be > 0");
  std::vector<float> eta;
  build_schedule(p->n_iters, eta_max_of(p, d_max), p->eta_min, eta);
  std::copy(eta.begin(), eta.end(), eta_out);
  return ok();
}

pgsgd_status pgsgd_zipf_table(double theta, uint32_t W, uint32_t* C_out) {
  if (!C_out) return fail(PGSGD_ERR_INVALID_ARG, "C_out is NULL");
  if (W < 1 || W > 65535) return fail(PGSGD_ERR_INVALID_ARG, "W %u outside [1, 65535]", W);
  if (!(theta >= 0.0) || !std::isfinite(theta)) return fail(PGSGD_ERR_INVALID_ARG, "theta must be finite, >= 0");
  std::vector<uint32_t> C;
  std::vector<uint16_t> guide;
  build_zipf(theta, W, C, guide);
  std::copy(C.begin(), C.end(), C_out);
  return ok();
}

pgsgd_status pgsgd_graph_create(uint32_t n_nodes, const uint32_t* node_len, uint32_t n_paths,
                                const uint64_t* path_off, const uint32_t* step_node, const int64_t* step_pos,
                                int device, pgsgd_graph** out) {
  return pgsgd_graph_create_ex(n_nodes, node_len, n_paths, path_off, step_node, step_pos, device,
                               PGSGD_RENUMBER_AUTO, out);
}

pgsgd_status pgsgd_graph_create_ex(uint32_t n_nodes, const uint32_t* node_len, uint32_t n_paths,
                                   const uint64_t* path_off, const uint32_t* step_node, const int64_t* step_pos,
                                   int device, uint32_t renumber, pgsgd_graph** out) {
  if (!out) return fail(PGSGD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (renumber > PGSGD_RENUMBER_ALWAYS) return fail(PGSGD_ERR_INVALID_ARG, "unknown renumber mode %u", renumber);
  if (!node_len && n_nodes > 0) return fail(PGSGD_ERR_INVALID_ARG, "node_len is NULL");
  if (!path_off) return fail(PGSGD_ERR_INVALID_ARG, "path_offsets is NULL");
  if (n_paths == 0) return fail(PGSGD_ERR_INVALID_ARG, "n_paths must be >= 1");
  if (n_paths > kMaxPaths) return fail(PGSGD_ERR_RANGE, "n_paths %u exceeds %u", n_paths, kMaxPaths);
  if (n_nodes >= (1u << 31)) return fail(PGSGD_ERR_RANGE, "n_nodes must be < 2^31");
  // ---- validation: host only, before any device work ----
  for (uint32_t n = 0; n < n_nodes; ++n)
    if (node_len[n] == 0) return fail(PGSGD_ERR_INVALID_ARG, "node %u has length 0", n);
  if (path_off[0] != 0) return fail(PGSGD_ERR_INVALID_ARG, "path_offsets[0] must be 0");
  uint64_t max_len = 0;
  for (uint32_t p = 0; p < n_paths; ++p) {
    if (path_off[p + 1] < path_off[p])
      return fail(PGSGD_ERR_INVALID_ARG, "path_offsets not monotone at path %u", p);
    max_len = std::max(max_len, path_off[p + 1] - path_off[p]);
  }
  const uint64_t S = path_off[n_paths];
  if (S >= kMaxSteps) return fail(PGSGD_ERR_RANGE, "total steps %llu >= 2^40", (unsigned long long)S);
  if (max_len >= (1ull << 32)) return fail(PGSGD_ERR_RANGE, "a path has >= 2^32 steps");
  if (S > 0 && !step_node) return fail(PGSGD_ERR_INVALID_ARG, "step_node is NULL");
  if (S > 0 && n_nodes == 0) return fail(PGSGD_ERR_INVALID_ARG, "steps given but n_nodes = 0");
  int64_t d_max = 0;
  for (uint32_t p = 0; p < n_paths; ++p) {
    int64_t acc = 0;
    for (uint64_t s = path_off[p]; s < path_off[p + 1]; ++s) {
      const uint32_t n = step_node[s] & kNodeMask;
      if (n >= n_nodes)
        return fail(PGSGD_ERR_INVALID_ARG, "step %llu refers to node %u >= n_nodes %u", (unsigned long long)s, n,
                    n_nodes);
      if (step_pos && step_pos[s] != acc)
        return fail(PGSGD_ERR_INVALID_ARG, "step_pos[%llu] = %lld but the length prefix sum is %lld",
                    (unsigned long long)s, (long long)step_pos[s], (long long)acc);
      acc += node_len[n];
      if (acc >= kMaxPathNt) return fail(PGSGD_ERR_RANGE, "path %u is longer than 2^62 nt", p);
    }
    d_max = std::max(d_max, acc);
  }
  // node order on the device: the caller's, or the path-guided order when the
  // caller's ids are scattered along the paths
  std::vector<uint32_t> perm;
  if (renumber == PGSGD_RENUMBER_ALWAYS ||
      (renumber == PGSGD_RENUMBER_AUTO &&
       far_step_fraction(n_paths, path_off, step_node, nullptr) > kRenumberMinFar)) {
    path_guided_order(n_nodes, node_len, n_paths, path_off, step_node, perm);
    if (renumber == PGSGD_RENUMBER_AUTO &&
        !(far_step_fraction(n_paths, path_off, step_node, perm.data()) <
          kRenumberGain * far_step_fraction(n_paths, path_off, step_node, nullptr)))
      perm.clear();
  }
  // the buffers allocated below, checked against PGSGD_MAX_DEVICE_BYTES before any device work
  const uint64_t need = 16ull * std::max<uint64_t>(S, 1) + 8ull * (n_paths + 1) + 8ull * std::max(n_nodes, 1u) +
                        16ull * std::max(n_nodes, 1u) + 40ull * kStressBlocks + 8 * 8 + 4 * 8 + 4 * 8 + 4ull * 65536 +
                        2ull * (kGuideSize + 1) + (perm.empty() ? 0 : 4ull * n_nodes);
  const uint64_t cap = device_byte_cap();
  if (cap && need > cap)
    return fail(PGSGD_ERR_OOM, "the graph needs %llu bytes of device memory, above PGSGD_MAX_DEVICE_BYTES = %llu",
                (unsigned long long)need, (unsigned long long)cap);
  int n_dev = 0;
  hipError_t e = hipGetDeviceCount(&n_dev);
  if (e != hipSuccess || n_dev == 0) {
    (void)hipGetLastError();
    return fail(PGSGD_ERR_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  }
  if (device < 0 || device >= n_dev) return fail(PGSGD_ERR_INVALID_ARG, "device %d out of range", device);

  // ---- device work ----
  pgsgd_graph* g = new (std::nothrow) pgsgd_graph();
  if (!g) return fail(PGSGD_ERR_OOM, "host allocation failed");
  g->device = device;
  DeviceGuard guard(device);
  g->n_nodes = n_nodes;
  g->n_paths = n_paths;
  g->S = S;
  g->d_max = d_max;
  g->max_path_steps = (uint32_t)max_len;
  g->path_top = pow2_floor(n_paths);
  g->path_slots = 2 * g->path_top;
  g->h_path_off.assign(path_off, path_off + n_paths + 1);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    g->n_cu = prop.multiProcessorCount;
    g->lds_limit = prop.sharedMemPerBlock;
  }
  pgsgd_status st;
  auto bail = [&](pgsgd_status code) {
    delete g;
    return code;
  };
  if ((st = dev_alloc(g, &g->d_rec, S))) return bail(st);
  if ((st = dev_alloc(g, &g->d_path_off, n_paths + 1))) return bail(st);
  if ((st = dev_alloc(g, &g->d_first, n_nodes))) return bail(st);
  if ((st = dev_alloc(g, &g->d_work, 2ull * n_nodes))) return bail(st);
  if ((st = dev_alloc(g, &g->d_part_f, 3 * kStressBlocks))) return bail(st);
  if ((st = dev_alloc(g, &g->d_part_n, kStressBlocks))) return bail(st);
  if ((st = dev_alloc(g, &g->d_part_skip, kStressBlocks))) return bail(st);
  if ((st = dev_alloc(g, &g->d_out_f, 8))) return bail(st);
  if ((st = dev_alloc(g, &g->d_out_n, 4))) return bail(st);
  if ((st = dev_alloc(g, &g->d_mean, 4))) return bail(st);
  if ((st = dev_alloc(g, &g->d_zipf, 65536))) return bail(st);
  if ((st = dev_alloc(g, &g->d_guide, kGuideSize + 1))) return bail(st);
  if (!perm.empty() && (st = dev_alloc(g, &g->d_inv, n_nodes))) return bail(st);
  auto dev_err = [&](hipError_t err, const char* what) {
    (void)hipGetLastError();
    fail(err == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(err));
    delete g;
    return err == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE;
  };
  if ((e = hipMemcpy(g->d_path_off, path_off, sizeof(uint64_t) * (n_paths + 1), hipMemcpyHostToDevice)))
    return dev_err(e, "path offsets upload");
  if (!perm.empty()) {
    std::vector<uint32_t> inv(n_nodes);
    for (uint32_t n = 0; n < n_nodes; ++n) inv[perm[n]] = n;
    if ((e = hipMemcpy(g->d_inv, inv.data(), sizeof(uint32_t) * n_nodes, hipMemcpyHostToDevice)))
      return dev_err(e, "node order upload");
    g->h_perm.swap(perm);
  }

  // Pack and upload the step records through two pinned staging buffers.
  if (S > 0) {
    const uint64_t chunk = std::min<uint64_t>(S, 1ull << 22);  // 64 MiB of records per buffer
    StepRec* stage[2] = {nullptr, nullptr};
    hipEvent_t done[2];
    hipStream_t cs;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) return dev_err(e, "stream create");
    bool ok_all = true;
    for (int k = 0; k < 2 && ok_all; ++k) {
      if ((e = hipHostMalloc((void**)&stage[k], sizeof(StepRec) * chunk, hipHostMallocDefault))) ok_all = false;
      else if ((e = hipEventCreateWithFlags(&done[k], hipEventDisableTiming))) ok_all = false;
    }
    if (ok_all) {
      uint32_t p = 0;
      int64_t acc = 0;
      uint64_t next_path_start = path_off[1];
      int buf = 0;
      bool pending[2] = {false, false};
      for (uint64_t base = 0; base < S && ok_all; base += chunk) {
        const uint64_t n = std::min(chunk, S - base);
        if (pending[buf]) {
          if ((e = hipEventSynchronize(done[buf]))) { ok_all = false; break; }
        }
        StepRec* out_rec = stage[buf];
        for (uint64_t k = 0; k < n; ++k) {
          const uint64_t s = base + k;
          while (s >= next_path_start) {  // entering the next non-empty path
            ++p;
            acc = 0;
            next_path_start = path_off[p + 1];
          }
          const uint32_t v = step_node[s];
          const uint32_t len = node_len[v & kNodeMask];
          out_rec[k].pos = acc;
          out_rec[k].node_rev = g->h_perm.empty() ? v : (g->h_perm[v & kNodeMask] | (v & kRevBit));
          out_rec[k].len = len;
          acc += len;
        }
        if ((e = hipMemcpyAsync(g->d_rec + base, out_rec, sizeof(StepRec) * n, hipMemcpyHostToDevice, cs))) {
          ok_all = false;
          break;
        }
        if ((e = hipEventRecord(done[buf], cs))) { ok_all = false; break; }
        pending[buf] = true;
        buf ^= 1;
      }
      if (ok_all) e = hipStreamSynchronize(cs);
    }
    (void)hipStreamSynchronize(cs);
    for (int k = 0; k < 2; ++k) {
      if (stage[k]) (void)hipHostFree(stage[k]);
      (void)hipEventDestroy(done[k]);
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return dev_err(e, "step record upload");
  }
  if ((e = launch_first_visit(g->d_rec, S, n_nodes, g->d_first, nullptr))) return dev_err(e, "first-visit kernel");
  if ((e = hipDeviceSynchronize())) return dev_err(e, "graph upload");
  *out = g;
  return ok();
}

void pgsgd_graph_destroy(pgsgd_graph* g) { delete g; }

pgsgd_status pgsgd_graph_get_info(const pgsgd_graph* g, pgsgd_graph_info* out) {
  if (!g || !out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  out->n_steps = g->S;
  out->n_nodes = g->n_nodes;
  out->n_paths = g->n_paths;
  out->d_max = g->d_max;
  out->device_bytes = g->device_bytes;
  out->device = g->device;
  out->max_path_steps = g->max_path_steps;
  out->renumbered = g->h_perm.empty() ? 0u : 1u;
  return ok();
}

pgsgd_status pgsgd_graph_get_order(const pgsgd_graph* g, uint32_t* perm_out) {
  if (!g || !perm_out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  for (uint32_t n = 0; n < g->n_nodes; ++n) perm_out[n] = g->h_perm.empty() ? n : g->h_perm[n];
  return ok();
}

pgsgd_status pgsgd_path_order(uint32_t n_nodes, const uint32_t* node_len, uint32_t n_paths,
                              const uint64_t* path_off, const uint32_t* step_node, uint32_t* perm_out,
                              double* far_before, double* far_after) {
  if (!perm_out || (!node_len && n_nodes) || !path_off || (!step_node && path_off[n_paths]))
    return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  for (uint64_t s = 0; s < path_off[n_paths]; ++s)
    if ((step_node[s] & kNodeMask) >= n_nodes)
      return fail(PGSGD_ERR_INVALID_ARG, "step %llu refers to node %u >= n_nodes %u", (unsigned long long)s,
                  step_node[s] & kNodeMask, n_nodes);
  std::vector<uint32_t> perm;
  path_guided_order(n_nodes, node_len, n_paths, path_off, step_node, perm);
  std::copy(perm.begin(), perm.end(), perm_out);
  if (far_before) *far_before = far_step_fraction(n_paths, path_off, step_node, nullptr);
  if (far_after) *far_after = far_step_fraction(n_paths, path_off, step_node, perm.data());
  return ok();
}

pgsgd_status pgsgd_init_coords(pgsgd_graph* g, uint64_t seed, uint32_t graph_id, float jitter, float* coords,
                               void* stream) {
  if (!g || !coords) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (((uintptr_t)coords & 15u) != 0) return fail(PGSGD_ERR_INVALID_ARG, "coords must be 16-byte aligned");
  if (graph_id >= (1u << 24)) return fail(PGSGD_ERR_INVALID_ARG, "graph_id must be < 2^24");
  if (g->n_nodes == 0) return ok();
  DeviceGuard guard(g->device);
  HIP_TRY(launch_init_coords(g->d_rec, g->d_first, g->n_nodes, g->d_inv, (uint32_t)seed, (uint32_t)(seed >> 32),
                             (kStreamInit << 24) | graph_id, jitter, coords, (hipStream_t)stream));
  return ok();
}

}  // extern "C"

namespace {

// Launch shape of k_layout_iter: a full device of resident waves, capped by
// params.max_inflight_waves (automatic: see auto_inflight_waves) and by the
// number of 64-term groups.  Large grids use 4-wave blocks; small caps use
// one-wave blocks so the number of concurrent waves is exactly the cap.
// Automatic cap: about n_nodes / 32 terms in flight (n_nodes / 2048 waves), so
// a term shares an endpoint with another in-flight term with probability of
// about 3% (the Hogwild sparsity assumption).  Small graphs are sensitive to
// this: on a 2.6K-node graph one wave keeps the sampled path stress of the
// sequential loop, two waves raise it by about 12%.
uint64_t auto_inflight_waves(const pgsgd_graph* g) { return std::max<uint64_t>(1, g->n_nodes / 2048); }

pgsgd_status layout_grid(pgsgd_graph* g, const pgsgd_params* p, size_t lds, uint64_t n_groups, uint32_t* blocks,
                         uint32_t* threads) {
  int bpc = 1;
  pgsgd_status st = layout_blocks_per_cu(g, lds, &bpc);
  if (st) return st;
  uint64_t waves = (uint64_t)g->n_cu * bpc * 4;
  const uint64_t cap = p->max_inflight_waves ? p->max_inflight_waves : auto_inflight_waves(g);
  waves = std::min(waves, cap);
  waves = std::min(waves, std::max<uint64_t>(1, n_groups));
  if (waves >= 4ull * g->n_cu) {
    *threads = 256;
    *blocks = (uint32_t)((waves + 3) / 4);
  } else {
    *threads = 64;
    *blocks = (uint32_t)waves;
  }
  return PGSGD_OK;
}

pgsgd_status layout_prepare(pgsgd_graph* g, const pgsgd_params* p, hipStream_t s, size_t* lds) {
  *lds = layout_lds_bytes(g->path_slots, p->zipf_window);
  if (*lds > g->lds_limit)
    return fail(PGSGD_ERR_UNSUPPORTED, "LDS image of %zu bytes exceeds the %zu-byte block limit", *lds,
                g->lds_limit);
  return ensure_zipf(g, p->zipf_theta, p->zipf_window, s);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// AUTO selects WINDOWED: on MI355X the window-major order keeps a window's
// records and coordinates in the L2 and is about 3x faster than PLAIN at the
// same layout quality.
uint32_t resolve_schedule(const pgsgd_params* p) {
  return p->schedule != PGSGD_SCHEDULE_AUTO ? p->schedule : (uint32_t)PGSGD_SCHEDULE_WINDOWED;
}

// Host tables of the window-major schedule for `streams` runs per XCD:
// windows of 2^window_shift(S) steps, grouped into kXcds * streams runs by
// the piece of their path they lie in (built once, kept on the graph).
pgsgd_status local_host_tables(pgsgd_graph* g, uint32_t streams) {
  const uint32_t shift = window_shift(g->S);
  const uint32_t nwin = (uint32_t)((g->S + (1ull << shift) - 1) >> shift);
  if ((size_t)nwin * 4 > g->lds_limit)
    return fail(PGSGD_ERR_UNSUPPORTED, "the window histogram (%u windows) exceeds the %zu-byte LDS of a block", nwin,
                g->lds_limit);
  if (!g->h_lorder.empty() && g->h_loc_shift == shift && g->h_loc_streams == streams) return PGSGD_OK;
  const uint32_t runs = kXcds * streams;
  // run of a window: the piece of its path it starts in (each path cut into
  // `runs` equal pieces); windows keep their id order inside a run
  std::vector<uint32_t> order(nwin), sbeg(runs + 1, 0), run_of(nwin), wpath(nwin);
  uint32_t p = 0;
  for (uint32_t w = 0; w < nwin; ++w) {
    const uint64_t st0 = (uint64_t)w << shift;
    while (p + 1 < g->n_paths && g->h_path_off[p + 1] <= st0) ++p;
    const uint64_t b = g->h_path_off[p], len = g->h_path_off[p + 1] - b;
    const uint64_t st1 = std::min<uint64_t>(g->S, st0 + (1ull << shift));  // window [st0, st1)
    wpath[w] = st1 <= g->h_path_off[p + 1] ? p : (p | 0x80000000u);
    const uint64_t r = len ? ((st0 - b) * runs) / len : 0;
    run_of[w] = (uint32_t)std::min<uint64_t>(r, runs - 1);
    ++sbeg[run_of[w] + 1];
  }
  for (uint32_t r = 0; r < runs; ++r) sbeg[r + 1] += sbeg[r];
  std::vector<uint32_t> cur(sbeg.begin(), sbeg.end() - 1);
  for (uint32_t w = 0; w < nwin; ++w) order[cur[run_of[w]]++] = w;
  // a row of xitem holds the prefix over the windows of one run and its total
  uint32_t longest = 0;
  for (uint32_t r = 0; r < runs; ++r) longest = std::max(longest, sbeg[r + 1] - sbeg[r]);
  g->h_lorder.swap(order);
  g->h_lsbeg.swap(sbeg);
  g->h_lwpath.swap(wpath);
  g->h_loc_xstride = longest + 1;
  g->h_loc_shift = shift;
  g->h_loc_streams = streams;
  return PGSGD_OK;
}

// Window-major scratch of the graph: the host tables on the device plus two
// count/offset sets (allocated on first use).
pgsgd_status ensure_local(pgsgd_graph* g, uint32_t streams, hipStream_t s) {
  pgsgd_status st0 = local_host_tables(g, streams);
  if (st0) return st0;
  const uint32_t shift = g->h_loc_shift;
  const uint32_t nwin = (uint32_t)g->h_lwpath.size();
  if (g->d_lcount && g->loc_nwin == nwin && g->loc_shift == shift && g->loc_streams == streams) return PGSGD_OK;
  HIP_TRY(hipStreamSynchronize(s));
  const auto set = {(void**)&g->d_lcount, (void**)&g->d_loff, (void**)&g->d_lxitem, (void**)&g->d_lqueue,
                    (void**)&g->d_lorder, (void**)&g->d_lsbeg, (void**)&g->d_lwpath, (void**)&g->d_lcount2,
                    (void**)&g->d_loff2, (void**)&g->d_lxitem2, (void**)&g->d_lqueue2};
  free_set(g, set);
  g->loc_nwin = nwin;
  g->loc_shift = shift;
  g->loc_streams = streams;
  g->loc_xstride = g->h_loc_xstride;
  const uint32_t runs = kXcds * streams;
  const pgsgd_status st = [&]() -> pgsgd_status {
    pgsgd_status e;
    if ((e = dev_alloc(g, &g->d_lcount, nwin))) return e;
    if ((e = dev_alloc(g, &g->d_loff, nwin + 1))) return e;
    if ((e = dev_alloc(g, &g->d_lxitem, (size_t)runs * g->loc_xstride))) return e;
    if ((e = dev_alloc(g, &g->d_lqueue, (size_t)runs * 16))) return e;
    if ((e = dev_alloc(g, &g->d_lorder, nwin))) return e;
    if ((e = dev_alloc(g, &g->d_lsbeg, runs + 1))) return e;
    if ((e = dev_alloc(g, &g->d_lwpath, nwin))) return e;
    if ((e = dev_alloc(g, &g->d_lcount2, nwin))) return e;
    if ((e = dev_alloc(g, &g->d_loff2, nwin + 1))) return e;
    if ((e = dev_alloc(g, &g->d_lxitem2, (size_t)runs * g->loc_xstride))) return e;
    if ((e = dev_alloc(g, &g->d_lqueue2, (size_t)runs * 16))) return e;
    HIP_TRY(hipMemcpy(g->d_lorder, g->h_lorder.data(), sizeof(uint32_t) * nwin, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_lsbeg, g->h_lsbeg.data(), sizeof(uint32_t) * (runs + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_lwpath, g->h_lwpath.data(), sizeof(uint32_t) * nwin, hipMemcpyHostToDevice));
    HIP_TRY(launch_fill_u32(g->d_lcount, nwin, 0u, s));  // the histograms must start at zero
    HIP_TRY(launch_fill_u32(g->d_lcount2, nwin, 0u, s));
    return PGSGD_OK;
  }();
  if (st) free_set(g, set);
  return st;
}

// The counting stream and its events (created on first use).
// The stream is set last, so a failed creation leaves no half-made set behind it.
pgsgd_status ensure_count_stream(pgsgd_graph* g) {
  if (g->count_stream) return PGSGD_OK;
  for (hipEvent_t* e : {&g->ev_start, &g->ev_count[0], &g->ev_count[1], &g->ev_layout[0], &g->ev_layout[1]})
    if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
  hipStream_t st = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  g->count_stream = st;
  return PGSGD_OK;
}

// Segment tables for windows of 2^shift steps (built once per shift, kept on
// the graph).
pgsgd_status ensure_seg_tables(pgsgd_graph* g, SegTables& T, uint32_t shift, hipStream_t s) {
  if (T.start && T.shift == shift) return PGSGD_OK;
  HIP_TRY(hipStreamSynchronize(s));
  const auto set = {(void**)&T.start, (void**)&T.path, (void**)&T.wseg, (void**)&T.count, (void**)&T.off,
                    (void**)&T.sbeg, (void**)&T.xitem, (void**)&T.queue};
  free_set(g, set);
  const uint64_t nwin = (g->S + (1ull << shift) - 1) >> shift;
  std::vector<uint64_t> start;
  std::vector<uint32_t> path;
  for (uint32_t p = 0; p < g->n_paths; ++p)
    for (uint64_t a = g->h_path_off[p], b = g->h_path_off[p + 1]; a < b;) {
      const uint64_t e = std::min<uint64_t>(b, ((a >> shift) + 1) << shift);
      start.push_back(a);
      path.push_back(p);
      a = e;
    }
  start.push_back(g->S);
  const uint64_t nseg = path.size();
  if (nseg >= (1ull << 31)) return fail(PGSGD_ERR_UNSUPPORTED, "too many segments");
  std::vector<uint32_t> wseg(nwin + 1), sbeg(kXcds + 1);
  for (uint64_t w = 0, k = 0; w <= nwin; ++w) {  // first segment starting at or after the window's start
    while (k < nseg && start[k] < (w << shift)) ++k;
    wseg[w] = (uint32_t)(w == nwin ? nseg : k);
  }
  for (uint32_t x = 0, k = 0; x <= kXcds; ++x) {  // first segment starting at or after x * S / 8
    while (k < nseg && (unsigned __int128)start[k] * kXcds < (unsigned __int128)x * g->S) ++k;
    sbeg[x] = x == kXcds ? (uint32_t)nseg : k;
  }
  uint32_t longest = 0;
  for (uint32_t x = 0; x < kXcds; ++x) longest = std::max(longest, sbeg[x + 1] - sbeg[x]);
  T.shift = shift;
  T.nseg = (uint32_t)nseg;
  T.xstride = longest + 1;
  const pgsgd_status st = [&]() -> pgsgd_status {
    pgsgd_status e;
    if ((e = dev_alloc(g, &T.start, nseg + 1))) return e;
    if ((e = dev_alloc(g, &T.path, nseg))) return e;
    if ((e = dev_alloc(g, &T.wseg, nwin + 1))) return e;
    if ((e = dev_alloc(g, &T.count, nseg))) return e;
    if ((e = dev_alloc(g, &T.off, nseg + 1))) return e;
    if ((e = dev_alloc(g, &T.sbeg, kXcds + 1))) return e;
    if ((e = dev_alloc(g, &T.xitem, (size_t)kXcds * T.xstride))) return e;
    if ((e = dev_alloc(g, &T.queue, (size_t)2 * kXcds * 16))) return e;
    HIP_TRY(hipMemcpy(T.start, start.data(), sizeof(uint64_t) * (nseg + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(T.path, path.data(), sizeof(uint32_t) * nseg, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(T.wseg, wseg.data(), sizeof(uint32_t) * (nwin + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(T.sbeg, sbeg.data(), sizeof(uint32_t) * (kXcds + 1), hipMemcpyHostToDevice));
    HIP_TRY(launch_fill_u32(T.count, nseg, 0u, s));  // the histogram must start at zero
    return PGSGD_OK;
  }();
  if (st) {
    free_set(g, set);
    T.start = nullptr;
    T.shift = 0;
  }
  return st;
}

// Segments of the window-major sampled path stress (R21): the windows of the
// windowed schedule.
pgsgd_status ensure_sps_windowed(pgsgd_graph* g, hipStream_t s) {
  return ensure_seg_tables(g, g->sps, window_shift(g->S), s);
}

// Tiles of the loss adjoint: the loss's segments grouped by the lowest device
// node id their steps visit, in units of kTileNodes ids; a tile (at most
// kTileMaxSeg segments; a fuller group is split) accumulates the gradient of
// the 2 * kTileNodes ids from its base in LDS.
pgsgd_status ensure_loss_tiles(pgsgd_graph* g, hipStream_t s) {
  const SegTables& T = g->loss;
  if (g->d_tile_seg && g->tile_shift == T.shift) return PGSGD_OK;
  HIP_TRY(hipStreamSynchronize(s));
  const auto set = {(void**)&g->d_tile_seg, (void**)&g->d_tile_off, (void**)&g->d_tile_base,
                    (void**)&g->d_tile_queue};
  free_set(g, set);
  g->tile_shift = 0;
  const uint32_t nseg = T.nseg;
  pgsgd_status st;
  if ((st = dev_alloc(g, &g->d_tile_seg, std::max<uint32_t>(nseg, 1)))) return st;
  std::vector<uint32_t> lo(nseg);
  if (nseg) {
    HIP_TRY(launch_segment_min_node(g->d_rec, T.start, nseg, g->d_tile_seg, s));
    HIP_TRY(hipMemcpyAsync(lo.data(), g->d_tile_seg, sizeof(uint32_t) * nseg, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  // segments in order of their tile key (counting sort), then cut into tiles
  const uint32_t n_keys = (uint32_t)(g->n_nodes / kTileNodes + 1);
  std::vector<uint32_t> kb(n_keys + 1, 0), order(nseg);
  for (uint32_t k = 0; k < nseg; ++k) ++kb[lo[k] / kTileNodes + 1];
  for (uint32_t k = 0; k < n_keys; ++k) kb[k + 1] += kb[k];
  std::vector<uint32_t> cur(kb.begin(), kb.end() - 1);
  for (uint32_t k = 0; k < nseg; ++k) order[cur[lo[k] / kTileNodes]++] = k;
  std::vector<uint32_t> toff(1, 0), tbase;
  for (uint32_t key = 0; key < n_keys; ++key)
    for (uint32_t a = kb[key]; a < kb[key + 1]; a += kTileMaxSeg) {
      toff.push_back(std::min(kb[key + 1], a + kTileMaxSeg));
      tbase.push_back(key * kTileNodes);
    }
  const uint32_t nt = (uint32_t)tbase.size();
  st = [&]() -> pgsgd_status {
    pgsgd_status e;
    if ((e = dev_alloc(g, &g->d_tile_off, nt + 1))) return e;
    if ((e = dev_alloc(g, &g->d_tile_base, std::max<uint32_t>(nt, 1)))) return e;
    if ((e = dev_alloc(g, &g->d_tile_queue, 64))) return e;
    if (nseg) HIP_TRY(hipMemcpy(g->d_tile_seg, order.data(), sizeof(uint32_t) * nseg, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(g->d_tile_off, toff.data(), sizeof(uint32_t) * (nt + 1), hipMemcpyHostToDevice));
    if (nt) HIP_TRY(hipMemcpy(g->d_tile_base, tbase.data(), sizeof(uint32_t) * nt, hipMemcpyHostToDevice));
    return PGSGD_OK;
  }();
  if (st) {
    free_set(g, set);
    return st;
  }
  g->n_tiles = nt;
  g->tile_shift = T.shift;
  return PGSGD_OK;
}

// Automatic wave cap of the windowed schedule (see kLocalNodesPerWave; the
// all-cooling iterations use kLocalNodesPerWaveCooling).
uint64_t auto_local_waves(const pgsgd_graph* g, bool cooling = false) {
  const uint32_t sh = window_shift(g->S);
  const double nodes_w = std::min<double>((double)g->n_nodes,
                                          std::ldexp(1.0, (int)sh) * (double)g->n_nodes * g->n_paths / (double)g->S);
  const uint64_t w = (uint64_t)(nodes_w / (double)(cooling ? kLocalNodesPerWaveCooling : kLocalNodesPerWave));
  return std::max<uint64_t>(1, std::min(w, auto_inflight_waves(g)));
}

// Grid of k_layout_local: the in-flight wave cap (params.max_inflight_waves,
// automatic: auto_local_waves) and occupancy give the waves; 256-thread
// blocks in a multiple of 8 (one share per XCD), or 64-thread blocks below 32
// waves.  cooling: the grid of the iterations whose terms all have power-law
// partners (t >= n_iters / 2).
pgsgd_status local_grid(pgsgd_graph* g, const pgsgd_params* p, size_t lds, uint32_t* blocks, uint32_t* threads,
                        bool cooling = false) {
  int nb = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, layout_local_kernel(), 256, lds));
  uint64_t waves = (uint64_t)g->n_cu * (uint64_t)std::max(nb, 1) * 4;
  const uint64_t cap = p->max_inflight_waves ? p->max_inflight_waves : auto_local_waves(g, cooling);
  waves = std::max<uint64_t>(1, std::min(waves, cap));
  if (waves >= 4ull * kXcds) {
    *threads = 256;
    *blocks = (uint32_t)((waves / 4) / kXcds * kXcds);
  } else {
    *threads = 64;
    *blocks = (uint32_t)waves;
  }
  return PGSGD_OK;
}

// Scratch, grid and launch arguments of the windowed schedule for graph g
// (L: the sampling arguments of make_layout_launch).
pgsgd_status local_plan(pgsgd_graph* g, const pgsgd_params* p, size_t lds, const LayoutLaunch& L, hipStream_t s,
                        LocalLaunch* W, uint32_t* blocks, uint32_t* threads) {
  pgsgd_status st;
  if ((st = ensure_local(g, kLocalStreams, s))) return st;
  if ((st = local_grid(g, p, lds, blocks, threads))) return st;
  *W = LocalLaunch{};
  W->L = L;
  W->n_win = g->loc_nwin;
  W->win_shift = g->loc_shift;
  W->count_blocks = (uint32_t)g->n_cu * 2;
  W->xstride = g->loc_xstride;
  W->wcount = g->d_lcount;
  W->woff = g->d_loff;
  W->xitem = g->d_lxitem;
  W->queue = g->d_lqueue;
  W->worder = g->d_lorder;
  W->sbeg = g->d_lsbeg;
  W->wpath = g->d_lwpath;
  W->streams = kLocalStreams;
  W->grab = kLocalGrab;
  return PGSGD_OK;
}

// Byte offsets of the window tables inside one contiguous scratch region
// (every table 256-byte aligned).
struct ScratchCarve {
  size_t wcount, woff, xitem, queue, worder, sbeg, wpath, total;
};

ScratchCarve carve_scratch(uint32_t nwin, uint32_t runs, uint32_t xstride) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  ScratchCarve c{};
  size_t o = 0;
  c.wcount = o, o = up(o + 4ull * nwin);
  c.woff = o, o = up(o + 8ull * (nwin + 1));
  c.xitem = o, o = up(o + 8ull * runs * xstride);
  c.queue = o, o = up(o + 8ull * runs * 16);
  c.worder = o, o = up(o + 4ull * nwin);
  c.sbeg = o, o = up(o + 4ull * (runs + 1));
  c.wpath = o, o = up(o + 4ull * nwin);
  c.total = o;
  return c;
}

// As local_plan, with the window tables in the caller-provided device region
// `scratch` of `scratch_bytes` (nothing allocated): the host tables are copied
// in and the histogram cleared on stream s, in stream order before the
// iterations that read them.
pgsgd_status local_plan_scratch(pgsgd_graph* g, const pgsgd_params* p, size_t lds, const LayoutLaunch& L,
                                hipStream_t s, void* scratch, size_t scratch_bytes, LocalLaunch* W,
                                uint32_t* blocks, uint32_t* threads) {
  pgsgd_status st;
  if ((st = local_host_tables(g, kLocalStreams))) return st;
  if ((st = local_grid(g, p, lds, blocks, threads))) return st;
  const uint32_t nwin = (uint32_t)g->h_lwpath.size();
  const uint32_t runs = kXcds * kLocalStreams;
  const ScratchCarve c = carve_scratch(nwin, runs, g->h_loc_xstride);
  if (c.total > scratch_bytes)
    return fail(PGSGD_ERR_RANGE, "the window tables of this graph need %zu bytes of scratch, above the %zu available",
                c.total, scratch_bytes);
  char* base = static_cast<char*>(scratch);
  *W = LocalLaunch{};
  W->L = L;
  W->n_win = nwin;
  W->win_shift = g->h_loc_shift;
  W->count_blocks = (uint32_t)g->n_cu * 2;
  W->xstride = g->h_loc_xstride;
  W->wcount = reinterpret_cast<uint32_t*>(base + c.wcount);
  W->woff = reinterpret_cast<uint64_t*>(base + c.woff);
  W->xitem = reinterpret_cast<uint64_t*>(base + c.xitem);
  W->queue = reinterpret_cast<uint64_t*>(base + c.queue);
  W->worder = reinterpret_cast<const uint32_t*>(base + c.worder);
  W->sbeg = reinterpret_cast<const uint32_t*>(base + c.sbeg);
  W->wpath = reinterpret_cast<const uint32_t*>(base + c.wpath);
  W->streams = kLocalStreams;
  W->grab = kLocalGrab;
  // the host tables live as long as the graph, so the copies may stay in flight
  HIP_TRY(hipMemcpyAsync(base + c.worder, g->h_lorder.data(), sizeof(uint32_t) * nwin, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + c.sbeg, g->h_lsbeg.data(), sizeof(uint32_t) * (runs + 1), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + c.wpath, g->h_lwpath.data(), sizeof(uint32_t) * nwin, hipMemcpyHostToDevice, s));
  HIP_TRY(launch_fill_u32(W->wcount, nwin, 0u, s));  // the histogram must start at zero
  return PGSGD_OK;
}

// The layout part of a windowed iteration whose counts and offsets are in W:
// run counters cleared, layout kernel.  With e_mid set, an event is recorded
// right before the layout kernel.
hipError_t local_layout(const LocalLaunch& W, uint32_t blocks, uint32_t threads, hipStream_t s,
                        hipEvent_t e_mid = nullptr) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(W.queue), 2ull * kXcds * W.streams * 16, 0u, s);
  if (!e && e_mid) e = hipEventRecord(e_mid, s);
  if (!e) e = launch_layout_local(W, blocks, threads, s);
  return e;
}

// One windowed iteration (W.L.iter, cool_all and eta set) on one stream:
// counts and offsets, then the layout part.
hipError_t local_iteration(const LocalLaunch& W, uint32_t blocks, uint32_t threads, hipStream_t s,
                           hipEvent_t e_mid = nullptr) {
  hipError_t e = launch_local_count_scan(W, s);
  if (!e) e = local_layout(W, blocks, threads, s, e_mid);
  return e;
}

// The layout loop.  With iter_ms set, HIP events bracket every iteration and
// every launch of the dominant kernel, and the durations are written out
// (synchronising).  With trace_f set (windowed schedule), iteration first_iter
// is recorded instead of applied; with apply_mask set (plain or windowed),
// iteration first_iter applies only the terms of [sub_begin, sub_begin +
// sub_count) that the mask selects.
struct LayoutHook {
  uint64_t* trace_i = nullptr;
  uint64_t* trace_j = nullptr;
  uint8_t* trace_f = nullptr;
  uint8_t* trace_o = nullptr;
  const uint8_t* apply_mask = nullptr;
  uint64_t sub_begin = 0, sub_count = 0;
};

pgsgd_status layout_impl(pgsgd_graph* g, const pgsgd_params* p, float* coords, float* iter_ms, float* main_ms,
                         uint32_t* main_launches, void* stream, const LayoutHook& hook = LayoutHook(),
                         void* scratch = nullptr, size_t scratch_bytes = 0) {
  const bool tracing = hook.trace_f != nullptr;
  const bool subset = tracing || hook.apply_mask != nullptr;
  if (!g || (!coords && !tracing)) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (coords && ((uintptr_t)coords & 15u) != 0) return fail(PGSGD_ERR_INVALID_ARG, "coords must be 16-byte aligned");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if ((uint64_t)p->terms_per_step * g->S >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "term count >= 2^48");
  const uint32_t last = p->last_iter == 0 ? p->n_iters : p->last_iter;
  const uint32_t n_run = last - p->first_iter;
  if (iter_ms)
    for (uint32_t k = 0; k < n_run; ++k) iter_ms[k] = 0.0f;
  if (main_ms)
    for (uint32_t k = 0; k < n_run; ++k) main_ms[k] = 0.0f;
  if (main_launches) *main_launches = 0;
  if (g->S == 0 || p->n_iters == 0 || n_run == 0) return ok();
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  size_t lds;
  if ((st = layout_prepare(g, p, s, &lds))) return st;
  std::vector<float> eta;
  build_schedule(p->n_iters, eta_max_of(p, g->d_max), p->eta_min, eta);
  LayoutLaunch L = make_layout_launch(g, p);
  L.t_begin = 0;
  L.t_end = L.n_terms;
  L.g_begin = 0;
  L.g_end = L.n_groups;
  const bool reuse = p->reuse_factor > 1 || p->step_reduction > 1;
  const bool windowed = resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED;
  if (tracing && !windowed) return fail(PGSGD_ERR_INVALID_ARG, "recording through the layout loop needs WINDOWED");
  uint32_t blocks = 0, threads = 256, blocks_c = 0, threads_c = 256;
  LocalLaunch W{};
  if (windowed && scratch) {
    if ((st = local_plan_scratch(g, p, lds, L, s, scratch, scratch_bytes, &W, &blocks, &threads))) return st;
    if ((st = local_grid(g, p, lds, &blocks_c, &threads_c, true))) return st;
  } else if (windowed) {
    if ((st = local_plan(g, p, lds, L, s, &W, &blocks, &threads))) return st;
    if ((st = local_grid(g, p, lds, &blocks_c, &threads_c, true))) return st;
  } else {
    if ((st = layout_grid(g, p, lds, L.n_groups, &blocks, &threads))) return st;
    L.wave_stride = (uint64_t)blocks * (threads / 64);
  }
  L.trace_i = hook.trace_i;
  L.trace_j = hook.trace_j;
  L.trace_f = hook.trace_f;
  L.trace_o = hook.trace_o;
  L.apply_mask = hook.apply_mask;
  if (subset) {
    L.t_begin = hook.sub_begin;
    L.t_end = hook.sub_begin + hook.sub_count;
    if (!windowed) {  // the plain kernel walks the groups of the range only
      L.g_begin = L.t_begin >> 6;
      L.g_end = (L.t_end + 63) >> 6;
    }
  }
  if (main_launches) *main_launches = 1;
  std::vector<hipEvent_t> ev;
  const size_t ev_per_iter = 3;
  if (iter_ms) {
    ev.resize(n_run * ev_per_iter + 1);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  }
  struct EventsFree {
    std::vector<hipEvent_t>& v;
    ~EventsFree() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } events_free{ev};
  if (!tracing) HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  // With PGSGD_FLAG_COUNT_AHEAD a windowed layout of several iterations
  // counts iteration it + 1 on the graph's counting stream while iteration it
  // is laid out, alternating between two count/offset sets: a set is
  // rewritten only after the layout that read it (two iterations earlier) has
  // finished.  By default the passes stay in order: measured on MI355X the
  // overlap saved nothing on the chromosome graph and made a mid-size graph's
  // layout 74% slower.
  const bool ahead = (p->flags & PGSGD_FLAG_COUNT_AHEAD) != 0;
  const bool overlap = windowed && !subset && !scratch && n_run > 1 && ahead;
  LocalLaunch Wset[2] = {W, W};
  hipStream_t s2 = nullptr;
  bool set_used[2] = {false, false};
  auto count_into = [&](uint32_t it, uint32_t k) -> hipError_t {
    LocalLaunch C = Wset[k];
    C.L.iter = it;
    hipError_t e = set_used[k] ? hipStreamWaitEvent(s2, g->ev_layout[k], 0) : hipSuccess;
    if (!e) e = launch_local_count_scan(C, s2);
    if (!e) e = hipEventRecord(g->ev_count[k], s2);
    return e;
  };
  if (overlap) {
    if ((st = ensure_count_stream(g))) return st;
    s2 = g->count_stream;
    Wset[1].wcount = g->d_lcount2;
    Wset[1].woff = g->d_loff2;
    Wset[1].xitem = g->d_lxitem2;
    Wset[1].queue = g->d_lqueue2;
    // the counting stream starts after all earlier work on the caller's stream
    HIP_TRY(hipEventRecord(g->ev_start, s));
    HIP_TRY(hipStreamWaitEvent(s2, g->ev_start, 0));
    HIP_TRY(count_into(p->first_iter, 0));
  }
  for (uint32_t it = p->first_iter; it < last; ++it) {
    const size_t e0 = (size_t)(it - p->first_iter) * ev_per_iter;
    L.iter = it;
    L.cool_all = it >= p->n_iters / 2 ? 1u : 0u;
    L.eta = eta[it];
    if (iter_ms) HIP_TRY(hipEventRecord(ev[e0], s));
    if (overlap) {
      const uint32_t k = (it - p->first_iter) & 1u;
      HIP_TRY(hipStreamWaitEvent(s, g->ev_count[k], 0));
      if (it + 1 < last) HIP_TRY(count_into(it + 1, k ^ 1u));
      LocalLaunch Wi = Wset[k];
      Wi.L = L;
      HIP_TRY(local_layout(Wi, L.cool_all ? blocks_c : blocks, L.cool_all ? threads_c : threads, s,
                           iter_ms ? ev[e0 + 1] : nullptr));
      HIP_TRY(hipEventRecord(g->ev_layout[k], s));
      set_used[k] = true;
      if (iter_ms) HIP_TRY(hipEventRecord(ev[e0 + 2], s));
    } else if (windowed) {
      W.L = L;
      HIP_TRY(local_iteration(W, L.cool_all ? blocks_c : blocks, L.cool_all ? threads_c : threads, s,
                              iter_ms ? ev[e0 + 1] : nullptr));
      if (iter_ms) HIP_TRY(hipEventRecord(ev[e0 + 2], s));
    } else {
      if (iter_ms) HIP_TRY(hipEventRecord(ev[e0 + 1], s));
      if (reuse) HIP_TRY(launch_layout_reuse(L, blocks, threads, s));
      else HIP_TRY(launch_layout_iter(L, blocks, threads, s));
      if (iter_ms) HIP_TRY(hipEventRecord(ev[e0 + 2], s));
    }
    if (subset) break;
  }
  if (iter_ms) HIP_TRY(hipEventRecord(ev.back(), s));
  if (!tracing) HIP_TRY(launch_from_work(g->d_work, coords, g->n_nodes, g->d_inv, s));
  if (iter_ms) {
    HIP_TRY(hipEventSynchronize(ev.back()));
    for (uint32_t k = 0; k < n_run; ++k) {
      const size_t e0 = (size_t)k * ev_per_iter;
      const hipEvent_t end = (k + 1 < n_run) ? ev[e0 + ev_per_iter] : ev.back();
      HIP_TRY(hipEventElapsedTime(&iter_ms[k], ev[e0], end));
      if (main_ms) HIP_TRY(hipEventElapsedTime(&main_ms[k], ev[e0 + 1], ev[e0 + 2]));
    }
  }
  return ok();
}

// Scratch of pgsgd_layout_noalloc: the window tables of one windowed layout
// at a time per device (at most 4 MiB, enough for the 32,768 windows the
// schedule allows: about 2.7 MiB).  Host code must not use the array's name
// as a device address; noalloc_scratch gives each device's copy.
constexpr size_t kNoAllocScratchBytes = 4u << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
pgsgd_status noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(PGSGD_ERR_UNSUPPORTED, "device %d: the allocation-free entry point supports devices 0..%d", device,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[device]) {
    DeviceGuard guard(device);
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(PGSGD_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                  hipGetErrorString(e));
    }
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return PGSGD_OK;
}

// The data-reuse kernel in recording mode over the terms of [t_begin, t_begin
// + count) (t_begin a multiple of 64), with the layout's launch shape.
hipError_t sample_reuse(pgsgd_graph* g, const pgsgd_params* p, hipStream_t s, size_t lds, uint32_t iter,
                        uint64_t t_begin, uint64_t count, uint64_t* i_out, uint64_t* j_out, uint8_t* f_out,
                        uint8_t* o_out) {
  LayoutLaunch L = make_layout_launch(g, p);
  uint32_t blocks, threads;
  if (layout_grid(g, p, lds, L.n_groups, &blocks, &threads) != PGSGD_OK) return hipErrorUnknown;
  L.wave_stride = (uint64_t)blocks * (threads / 64);
  L.iter = iter;
  L.cool_all = iter >= p->n_iters / 2 ? 1u : 0u;
  L.t_begin = t_begin;
  L.t_end = t_begin + count;
  L.g_begin = t_begin >> 6;
  L.g_end = (t_begin + count + 63) >> 6;
  L.trace_i = i_out;
  L.trace_j = j_out;
  L.trace_f = f_out;
  L.trace_o = o_out;
  return launch_layout_reuse(L, blocks, threads, s);
}

}  // namespace

extern "C" {

pgsgd_status pgsgd_sample_terms_reuse(pgsgd_graph* g, const pgsgd_params* p, uint32_t iter, uint64_t t_begin,
                                      uint64_t count, uint64_t* i_out, uint64_t* j_out, uint8_t* flags_out,
                                      uint8_t* offsets_out, void* stream) {
  if (!g || !i_out || !j_out || !flags_out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (iter >= p->n_iters) return fail(PGSGD_ERR_INVALID_ARG, "iter %u >= n_iters %u", iter, p->n_iters);
  if (t_begin + count < t_begin || t_begin + count >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "term range too large");
  if (count == 0 || g->S == 0) return ok();
  if (resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    // the windowed kernels record the slots; offsets_out gets the offsets of
    // each recorded slot's group, reuse_factor - 1 bytes per slot
    const uint64_t srf = p->step_reduction > 1 ? p->step_reduction : 1;
    if (t_begin + count > ((uint64_t)p->terms_per_step * g->S + srf - 1) / srf)
      return fail(PGSGD_ERR_INVALID_ARG, "the windowed schedule records slots of the iteration only");
    pgsgd_params q = *p;
    q.first_iter = iter;
    q.last_iter = iter + 1;
    q.schedule = PGSGD_SCHEDULE_WINDOWED;
    LayoutHook h;
    h.trace_i = i_out;
    h.trace_j = j_out;
    h.trace_f = flags_out;
    h.trace_o = p->reuse_factor > 1 ? offsets_out : nullptr;
    h.sub_begin = t_begin;
    h.sub_count = count;
    return layout_impl(g, &q, nullptr, nullptr, nullptr, nullptr, stream, h);
  }
  if (t_begin % 64) return fail(PGSGD_ERR_INVALID_ARG, "t_begin must be a multiple of 64");
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  size_t lds;
  if ((st = layout_prepare(g, p, s, &lds))) return st;
  HIP_TRY(sample_reuse(g, p, s, lds, iter, t_begin, count, i_out, j_out, flags_out, offsets_out));
  return ok();
}

pgsgd_status pgsgd_layout(pgsgd_graph* g, const pgsgd_params* p, float* coords, void* stream) {
  return layout_impl(g, p, coords, nullptr, nullptr, nullptr, stream);
}

pgsgd_status pgsgd_layout_noalloc(pgsgd_graph* g, const pgsgd_params* p, float* coords, void* stream) {
  if (!g || !p) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (p->flags & PGSGD_FLAG_COUNT_AHEAD)
    return fail(PGSGD_ERR_INVALID_ARG,
                "pgsgd_layout_noalloc counts every iteration in order: PGSGD_FLAG_COUNT_AHEAD needs buffers it does "
                "not allocate");
  void* base = nullptr;
  pgsgd_status st = noalloc_scratch(g->device, &base);
  if (st) return st;
  return layout_impl(g, p, coords, nullptr, nullptr, nullptr, stream, LayoutHook(), base, kNoAllocScratchBytes);
}

pgsgd_status pgsgd_layout_timed(pgsgd_graph* g, const pgsgd_params* p, float* coords, float* iter_ms,
                                float* main_ms, uint32_t* main_launches, void* stream) {
  if (!iter_ms) return fail(PGSGD_ERR_INVALID_ARG, "iter_ms is NULL");
  return layout_impl(g, p, coords, iter_ms, main_ms, main_launches, stream);
}

pgsgd_status pgsgd_sample_terms(pgsgd_graph* g, const pgsgd_params* p, uint32_t iter, uint64_t t_begin,
                                uint64_t count, uint64_t* i_out, uint64_t* j_out, uint8_t* flags_out,
                                void* stream) {
  if (!g || !i_out || !j_out || !flags_out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (iter >= p->n_iters) return fail(PGSGD_ERR_INVALID_ARG, "iter %u >= n_iters %u", iter, p->n_iters);
  if (t_begin + count < t_begin || t_begin + count >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "term range too large");
  if (count == 0 || g->S == 0) return ok();
  const uint32_t sched = resolve_schedule(p);
  if (sched == PGSGD_SCHEDULE_WINDOWED) {
    // the window counting kernels and the layout kernel process the whole
    // iteration; the window-major slots of [t_begin, t_begin + count) are
    // recorded
    const uint64_t srf = p->step_reduction > 1 ? p->step_reduction : 1;
    if (t_begin + count > ((uint64_t)p->terms_per_step * g->S + srf - 1) / srf)
      return fail(PGSGD_ERR_INVALID_ARG, "this schedule records terms of the iteration only (t < T)");
    pgsgd_params q = *p;
    q.first_iter = iter;
    q.last_iter = iter + 1;
    q.schedule = sched;
    LayoutHook h;
    h.trace_i = i_out;
    h.trace_j = j_out;
    h.trace_f = flags_out;
    h.sub_begin = t_begin;
    h.sub_count = count;
    return layout_impl(g, &q, nullptr, nullptr, nullptr, nullptr, stream, h);
  }
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  size_t lds;
  if ((st = layout_prepare(g, p, s, &lds))) return st;
  if (p->reuse_factor > 1 || p->step_reduction > 1) {
    hipError_t e = sample_reuse(g, p, s, lds, iter, t_begin, count, i_out, j_out, flags_out, nullptr);
    HIP_TRY(e);
    return ok();
  }
  // the layout kernel itself, in recording mode, with the layout's launch shape
  LayoutLaunch L = make_layout_launch(g, p);
  uint32_t blocks, threads;
  if ((st = layout_grid(g, p, lds, L.n_groups, &blocks, &threads))) return st;
  L.wave_stride = (uint64_t)blocks * (threads / 64);
  L.iter = iter;
  L.cool_all = iter >= p->n_iters / 2 ? 1u : 0u;
  L.t_begin = t_begin;
  L.t_end = t_begin + count;
  L.g_begin = t_begin >> 6;
  L.g_end = (t_begin + count + 63) >> 6;
  L.trace_i = i_out;
  L.trace_j = j_out;
  L.trace_f = flags_out;
  HIP_TRY(launch_layout_iter(L, blocks, threads, s));
  return ok();
}

pgsgd_status pgsgd_apply_terms(pgsgd_graph* g, float eta, const uint64_t* i, const uint64_t* j,
                               const uint8_t* flags, uint64_t count, float* coords, void* stream) {
  if (!g || !i || !j || !flags || !coords) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (count == 0) return ok();
  if (count >= (1ull << 40)) return fail(PGSGD_ERR_RANGE, "count too large");
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  HIP_TRY(launch_apply_terms(g->d_rec, g->d_work, eta, i, j, flags, count, s));
  HIP_TRY(launch_from_work(g->d_work, coords, g->n_nodes, g->d_inv, s));
  return ok();
}

pgsgd_status pgsgd_apply_slots(pgsgd_graph* g, const pgsgd_params* p, uint32_t iter, uint64_t t_begin,
                               uint64_t count, const uint8_t* mask, float* coords, void* stream) {
  if (!g || !mask || !coords) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (p->reuse_factor > 1 || p->step_reduction > 1)
    return fail(PGSGD_ERR_INVALID_ARG, "the data-reuse variant pairs lanes across terms: no subset can be applied");
  if (iter >= p->n_iters) return fail(PGSGD_ERR_INVALID_ARG, "iter %u >= n_iters %u", iter, p->n_iters);
  if (t_begin + count < t_begin || t_begin + count > (uint64_t)p->terms_per_step * g->S)
    return fail(PGSGD_ERR_INVALID_ARG, "the range must lie inside the iteration's terms");
  if (count == 0) return ok();
  pgsgd_params q = *p;
  q.first_iter = iter;
  q.last_iter = iter + 1;
  LayoutHook h;
  h.apply_mask = mask;
  h.sub_begin = t_begin;
  h.sub_count = count;
  return layout_impl(g, &q, coords, nullptr, nullptr, nullptr, stream, h);
}

namespace {

// Launch arguments of the window-major passes over the graph's segments
// (ensure_sps_windowed done): slots drawn from Philox stream slot_stream;
// loss_pairs > 0 counts the loss's plain pairs instead of Eq. 2's.
SpsWinLaunch sps_win_launch(const pgsgd_graph* g, const SegTables& T, const StressLaunch& P, uint32_t slot_stream,
                            uint32_t graph_id, uint64_t loss_pairs) {
  SpsWinLaunch W{};
  W.P = P;
  W.slot_c3 = (slot_stream << 24) | (graph_id & 0xFFFFFFu);
  W.win_shift = T.shift;
  W.n_seg = T.nseg;
  W.xstride = T.xstride;
  W.count_blocks = (uint32_t)g->n_cu * 2;
  W.seg_start = T.start;
  W.seg_path = T.path;
  W.wseg = T.wseg;
  W.count = T.count;
  W.seg_off = T.off;
  W.sbeg = T.sbeg;
  W.xitem = T.xitem;
  W.queue = T.queue;
  W.loss_pairs = loss_pairs;
  return W;
}

// Segments and their counts for the loss's window-major pairs (reading R22) of
// one optimiser step: validates what the window-major loss needs.
pgsgd_status loss_win_prepare(pgsgd_graph* g, const pgsgd_params* p, const StressLaunch& P, uint64_t n_pairs,
                              hipStream_t s, SpsWinLaunch* W, bool offsets_only) {
  pgsgd_status st = ensure_seg_tables(g, g->loss, loss_shift(g->S), s);
  if (st) return st;
  if ((size_t)g->path_slots * 8 + (size_t)g->loss.nseg * 4 > g->lds_limit)
    return fail(PGSGD_ERR_UNSUPPORTED, "the segment histogram (%u segments) exceeds the %zu-byte LDS of a block",
                g->loss.nseg, g->lds_limit);
  if (n_pairs >= (1ull << 32))
    return fail(PGSGD_ERR_UNSUPPORTED, "n_pairs %llu too large for 32-bit segment counts (the PLAIN order has no "
                "such limit)", (unsigned long long)n_pairs);
  *W = sps_win_launch(g, g->loss, P, kStreamLossSlot, p->graph_id, n_pairs);
  // the tile passes read only the segment offsets: those of the same step are
  // still in the tables when the backward follows its forward
  auto& key = g->loss_key;
  if (offsets_only && key.tables == g->loss.start && key.n_pairs == n_pairs && key.word2 == P.word2 &&
      key.c3 == P.c3 && key.k0 == P.k0 && key.k1 == P.k1)
    return PGSGD_OK;
  key.tables = nullptr;
  HIP_TRY(launch_sps_win_count_scan(*W, s));
  key.tables = g->loss.start;
  key.n_pairs = n_pairs;
  key.word2 = P.word2;
  key.c3 = P.c3;
  key.k0 = P.k0;
  key.k1 = P.k1;
  return PGSGD_OK;
}

}  // namespace

namespace {

struct OutlierSink {
  double threshold = 0.0;
  uint64_t max_out = 0;
  uint64_t *i = nullptr, *j = nullptr;
  uint8_t* e = nullptr;
  double* s = nullptr;
  uint64_t* n_host = nullptr;
};

pgsgd_status path_stress_impl(pgsgd_graph* g, const float* coords, uint32_t m, uint64_t seed, uint32_t graph_id,
                              uint32_t pair_mode, double zipf_theta, uint32_t zipf_window, pgsgd_stress_result* out,
                              void* stream, const OutlierSink* sink, const float* coords_b = nullptr,
                              pgsgd_stress_compare_result* cmp = nullptr);

}  // namespace

pgsgd_status pgsgd_path_stress_pairs(pgsgd_graph* g, const float* coords, uint32_t m, uint64_t seed,
                                     uint32_t graph_id, uint32_t pair_mode, double zipf_theta, uint32_t zipf_window,
                                     pgsgd_stress_result* out, void* stream) {
  return path_stress_impl(g, coords, m, seed, graph_id, pair_mode, zipf_theta, zipf_window, out, stream, nullptr);
}

pgsgd_status pgsgd_path_stress_compare(pgsgd_graph* g, const float* coords_a, const float* coords_b, uint32_t m,
                                       uint64_t seed, uint32_t graph_id, uint32_t pair_mode, double zipf_theta,
                                       uint32_t zipf_window, pgsgd_stress_compare_result* out, void* stream) {
  if (!coords_b || !out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (g && ((uintptr_t)coords_b & 15u) != 0) return fail(PGSGD_ERR_INVALID_ARG, "coords must be 16-byte aligned");
  std::memset(out, 0, sizeof(*out));
  pgsgd_stress_result tmp;
  return path_stress_impl(g, coords_a, m, seed, graph_id, pair_mode, zipf_theta, zipf_window, &tmp, stream, nullptr,
                          coords_b, out);
}

pgsgd_status pgsgd_path_stress_outliers(pgsgd_graph* g, const float* coords, uint32_t m, uint64_t seed,
                                        uint32_t graph_id, uint32_t pair_mode, double zipf_theta,
                                        uint32_t zipf_window, double threshold, uint64_t max_out, uint64_t* i_out,
                                        uint64_t* j_out, uint8_t* e_out, double* s_out, uint64_t* n_out,
                                        pgsgd_stress_result* out, void* stream) {
  if (!n_out || (max_out && (!i_out || !j_out || !e_out || !s_out)))
    return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (!std::isfinite(threshold)) return fail(PGSGD_ERR_INVALID_ARG, "threshold must be finite");
  OutlierSink sink;
  sink.threshold = threshold;
  sink.max_out = max_out;
  sink.i = i_out;
  sink.j = j_out;
  sink.e = e_out;
  sink.s = s_out;
  sink.n_host = n_out;
  pgsgd_stress_result tmp;
  return path_stress_impl(g, coords, m, seed, graph_id, pair_mode, zipf_theta, zipf_window, out ? out : &tmp, stream,
                          &sink);
}

namespace {

pgsgd_status path_stress_impl(pgsgd_graph* g, const float* coords, uint32_t m, uint64_t seed, uint32_t graph_id,
                              uint32_t pair_mode, double zipf_theta, uint32_t zipf_window, pgsgd_stress_result* out,
                              void* stream, const OutlierSink* sink, const float* coords_b,
                              pgsgd_stress_compare_result* cmp) {
  if (!g || !coords || !out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (sink) *sink->n_host = 0;
  if (pair_mode > PGSGD_PAIRS_UNIFORM_WINDOWED) return fail(PGSGD_ERR_INVALID_ARG, "unknown pair mode %u", pair_mode);
  if (pair_mode == PGSGD_PAIRS_POWER_LAW) {
    if (zipf_window < 1 || zipf_window > 65535)
      return fail(PGSGD_ERR_INVALID_ARG, "zipf_window %u outside [1, 65535]", zipf_window);
    if (!(zipf_theta >= 0.0) || !std::isfinite(zipf_theta))
      return fail(PGSGD_ERR_INVALID_ARG, "zipf_theta must be finite and >= 0");
  }
  if (m == 0) return fail(PGSGD_ERR_INVALID_ARG, "pairs_per_step must be >= 1");
  if (graph_id >= (1u << 24)) return fail(PGSGD_ERR_INVALID_ARG, "graph_id must be < 2^24");
  if ((double)m * (double)g->S >= 18446744073709551615.0) return fail(PGSGD_ERR_RANGE, "too many pairs");
  std::memset(out, 0, sizeof(*out));
  if (g->S == 0) return ok();
  const int mode = (int)pair_mode;
  const size_t lds = (size_t)g->path_slots * 8 +
                     (mode == 1 ? (size_t)(zipf_window + 1) * 4 + (size_t)(kGuideSize + 1) * 2 : 0);
  if (lds > g->lds_limit) return fail(PGSGD_ERR_UNSUPPORTED, "too many paths for LDS");
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  if (mode == 1) {
    pgsgd_status st = ensure_zipf(g, zipf_theta, zipf_window, s);
    if (st) return st;
  }
  StressLaunch P = make_stress_launch(g, coords, kStreamSps, graph_id, seed);
  P.m = m;
  P.count = g->S;
  P.W = zipf_window;
  P.work = g->d_work;
  if (sink) {
    P.out_count = g->d_out_n + 3;  // d_out_n[3]: the outlier counter
    P.out_max = sink->max_out;
    P.out_threshold = sink->threshold;
    P.out_i = sink->i;
    P.out_j = sink->j;
    P.out_e = sink->e;
    P.out_s = sink->s;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(P.out_count), 2, 0u, s));
  }
  if (coords_b) {  // the second layout of a paired evaluation
    if (!g->d_work2) {
      pgsgd_status st = dev_alloc(g, &g->d_work2, 2ull * g->n_nodes);
      if (st) return st;
    }
    P.work2 = g->d_work2;
  }
  SpsWinLaunch W{};
  const bool windowed = mode == PGSGD_PAIRS_UNIFORM_WINDOWED;
  if (windowed) {
    pgsgd_status st = ensure_sps_windowed(g, s);
    if (st) return st;
    if ((size_t)g->path_slots * 8 + (size_t)g->sps.nseg * 4 > g->lds_limit)
      return fail(PGSGD_ERR_UNSUPPORTED, "the segment histogram (%u segments) exceeds the %zu-byte LDS of a block",
                  g->sps.nseg, g->lds_limit);
    if (((uint64_t)m << (g->sps.shift + 1)) >= (1ull << 32))
      return fail(PGSGD_ERR_UNSUPPORTED, "pairs_per_step %u too large for 32-bit segment counts", m);
    W = sps_win_launch(g, g->sps, P, kStreamSpsSlot, graph_id, 0);
  }
  auto pass = [&](int k, const double* mean_dev, uint64_t* part_n, uint64_t* part_skip) -> hipError_t {
    return windowed ? launch_sps_win_pass(W, k, mean_dev, g->d_part_f, part_n, part_skip, kStressBlocks, s)
                    : launch_sps_pass(P, k, mode, mean_dev, g->d_part_f, part_n, part_skip, s);
  };
  auto reduce = [&](uint32_t part, double* out_f) -> hipError_t {  // sum of one of the three partial arrays
    return launch_reduce_parts(g->d_part_f + (size_t)part * kStressBlocks, nullptr, nullptr, kStressBlocks, out_f,
                               nullptr, nullptr, nullptr, nullptr, s);
  };
  HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  if (coords_b) HIP_TRY(launch_to_work(coords_b, g->d_work2, g->n_nodes, g->d_inv, s));
  if (windowed) HIP_TRY(launch_sps_win_count_scan(W, s));
  HIP_TRY(pass(1, nullptr, g->d_part_n, g->d_part_skip));
  HIP_TRY(launch_reduce_parts(g->d_part_f, g->d_part_n, g->d_part_skip, kStressBlocks, g->d_out_f, g->d_out_n,
                              g->d_mean, nullptr, nullptr, s));
  double sum_b = 0.0;
  if (coords_b) {  // pass 2 needs both means and the ratio: one round trip
    HIP_TRY(reduce(1, g->d_out_f + 2));
    double f0[3];
    uint64_t n0;
    HIP_TRY(hipMemcpyAsync(f0, g->d_out_f, sizeof(f0), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&n0, g->d_out_n, sizeof(n0), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    sum_b = f0[2];
    const double mean3[3] = {n0 ? f0[0] / (double)n0 : 0.0, n0 ? sum_b / (double)n0 : 0.0,
                             sum_b > 0.0 ? f0[0] / sum_b : 0.0};
    HIP_TRY(hipMemcpyAsync(g->d_mean, mean3, sizeof(mean3), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // mean3 lives on this stack frame
  }
  HIP_TRY(pass(2, g->d_mean, nullptr, nullptr));
  HIP_TRY(reduce(0, g->d_out_f + 1));
  if (coords_b) {
    HIP_TRY(reduce(1, g->d_out_f + 3));
    HIP_TRY(reduce(2, g->d_out_f + 4));
  }
  double f[5];
  uint64_t n[2];
  HIP_TRY(hipMemcpyAsync(f, g->d_out_f, sizeof(f), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(n, g->d_out_n, sizeof(n), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->sum = f[0];
  out->sumsq_dev = f[1];
  out->n_valid = n[0];
  out->n_skipped = n[1];
  out->mean = n[0] ? f[0] / (double)n[0] : 0.0;
  out->stddev = n[0] > 1 ? std::sqrt(f[1] / (double)(n[0] - 1)) : 0.0;
  const double half = n[0] ? 1.96 * out->stddev / std::sqrt((double)n[0]) : 0.0;
  out->ci_lo = out->mean - half;
  out->ci_hi = out->mean + half;
  if (cmp) {
    const uint64_t nv = n[0];
    cmp->mean_a = out->mean;
    cmp->mean_b = nv ? sum_b / (double)nv : 0.0;
    cmp->ratio = sum_b > 0.0 ? f[0] / sum_b : 0.0;
    cmp->sd_a = out->stddev;
    cmp->sd_b = nv > 1 ? std::sqrt(f[3] / (double)(nv - 1)) : 0.0;
    cmp->sd_diff = nv > 1 ? std::sqrt(f[4] / (double)(nv - 1)) : 0.0;
    const double h = (nv && cmp->mean_b > 0.0) ? 1.96 * cmp->sd_diff / (std::sqrt((double)nv) * cmp->mean_b) : 0.0;
    cmp->ratio_ci_lo = cmp->ratio - h;
    cmp->ratio_ci_hi = cmp->ratio + h;
    cmp->sum_a = f[0];
    cmp->sum_b = sum_b;
    cmp->n_valid = nv;
    cmp->n_skipped = n[1];
  }
  if (sink) {
    HIP_TRY(hipMemcpy(sink->n_host, P.out_count, sizeof(uint64_t), hipMemcpyDeviceToHost));
  }
  return ok();
}

}  // namespace

pgsgd_status pgsgd_path_stress(pgsgd_graph* g, const float* coords, uint32_t m, uint64_t seed, uint32_t graph_id,
                               pgsgd_stress_result* out, void* stream) {
  return pgsgd_path_stress_pairs(g, coords, m, seed, graph_id, PGSGD_PAIRS_UNIFORM, 0.99, 1000, out, stream);
}

pgsgd_status pgsgd_path_stress_exact(pgsgd_graph* g, const float* coords, double* mean_out, uint64_t* pairs_out,
                                     void* stream) {
  if (!g || !coords || !mean_out) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  *mean_out = 0.0;
  if (pairs_out) *pairs_out = 0;
  if (g->S == 0) return ok();
  if ((size_t)g->path_slots * 8 > g->lds_limit) return fail(PGSGD_ERR_UNSUPPORTED, "too many paths for LDS");
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  StressLaunch P = make_stress_launch(g, coords, kStreamSps, 0, 0);
  P.work = g->d_work;
  HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  HIP_TRY(launch_path_stress_exact(P, g->d_part_f, g->d_part_n, s));
  HIP_TRY(launch_reduce_parts(g->d_part_f, g->d_part_n, nullptr, kStressBlocks, g->d_out_f, g->d_out_n, nullptr,
                              nullptr, nullptr, s));
  double f = 0.0;
  uint64_t n = 0;
  HIP_TRY(hipMemcpyAsync(&f, g->d_out_f, sizeof(f), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&n, g->d_out_n, sizeof(n), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *mean_out = n ? f / (double)n : 0.0;
  if (pairs_out) *pairs_out = n;
  return ok();
}

pgsgd_status pgsgd_stress_forward(pgsgd_graph* g, const pgsgd_params* p, const float* coords, uint64_t n_pairs,
                                  uint32_t step, float* loss_dev, uint64_t* n_valid_dev, void* stream) {
  if (!g || !coords || !loss_dev || !n_valid_dev) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (n_pairs >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "n_pairs too large");
  const size_t lds = layout_lds_bytes(g->path_slots, p->zipf_window);
  if (lds > g->lds_limit) return fail(PGSGD_ERR_UNSUPPORTED, "LDS image exceeds the block limit");
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure_zipf(g, p->zipf_theta, p->zipf_window, s))) return st;
  StressLaunch P = make_stress_launch(g, coords, kStreamPairs, p->graph_id, p->seed);
  P.W = p->zipf_window;
  P.word2 = step;
  P.count = g->S ? n_pairs : 0;
  P.work = g->d_work;
  if (P.count) HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  uint32_t parts = kStressBlocks;
  if (P.count && resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    SpsWinLaunch W;
    const bool tiles = loss_tile_lds_bytes(p->zipf_window, true) + kTileStaticLds <= g->lds_limit;
    if ((st = loss_win_prepare(g, p, P, n_pairs, s, &W, tiles))) return st;
    if (tiles) {
      if ((st = ensure_loss_tiles(g, s))) return st;
      parts = std::max<uint32_t>(1, std::min<uint32_t>(g->n_tiles, 2u * (uint32_t)g->n_cu));
      HIP_TRY(launch_fill_u32(g->d_tile_queue, 1, 0u, s));
      const TileLaunch T{g->d_tile_seg, g->d_tile_off, g->d_tile_base, g->n_tiles, g->d_tile_queue};
      HIP_TRY(launch_loss_tile_fwd(W, T, g->d_part_f, g->d_part_n, parts, s));
    } else {
      HIP_TRY(launch_loss_win_fwd(W, g->d_part_f, g->d_part_n, kStressBlocks, s));
    }
  } else {
    HIP_TRY(launch_stress_fwd(P, g->d_part_f, g->d_part_n, s));
  }
  HIP_TRY(launch_reduce_parts(g->d_part_f, g->d_part_n, nullptr, parts, nullptr, nullptr, nullptr, loss_dev,
                              n_valid_dev, s));
  return ok();
}

pgsgd_status pgsgd_stress_backward(pgsgd_graph* g, const pgsgd_params* p, const float* coords, uint64_t n_pairs,
                                   uint32_t step, const float* grad_out_dev, const uint64_t* n_valid_dev,
                                   float* grad_coords, void* stream) {
  if (!g || !coords || !grad_out_dev || !n_valid_dev || !grad_coords)
    return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (n_pairs >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "n_pairs too large");
  const size_t lds = layout_lds_bytes(g->path_slots, p->zipf_window);
  if (lds > g->lds_limit) return fail(PGSGD_ERR_UNSUPPORTED, "LDS image exceeds the block limit");
  if (g->S == 0 || n_pairs == 0) return ok();
  DeviceGuard guard(g->device);
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure_zipf(g, p->zipf_theta, p->zipf_window, s))) return st;
  StressLaunch P = make_stress_launch(g, coords, kStreamPairs, p->graph_id, p->seed);
  P.W = p->zipf_window;
  P.word2 = step;
  P.count = n_pairs;
  P.work = g->d_work;
  HIP_TRY(launch_to_work(coords, g->d_work, g->n_nodes, g->d_inv, s));
  if (resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    SpsWinLaunch W;
    // by tiles when their LDS image fits a block (it does for every window W up to ~10^4)
    const bool tiles = loss_tile_lds_bytes(p->zipf_window, true) + kTileStaticLds <= g->lds_limit;
    if ((st = loss_win_prepare(g, p, P, n_pairs, s, &W, tiles))) return st;
    if (tiles) {
      if ((st = ensure_loss_tiles(g, s))) return st;
      if (g->n_tiles) {
        HIP_TRY(launch_fill_u32(g->d_tile_queue, 1, 0u, s));
        const TileLaunch T{g->d_tile_seg, g->d_tile_off, g->d_tile_base, g->n_tiles, g->d_tile_queue};
        const uint32_t blocks = std::min<uint32_t>(g->n_tiles, 2u * (uint32_t)g->n_cu);
        HIP_TRY(launch_loss_tile_bwd(W, T, grad_out_dev, n_valid_dev, grad_coords, blocks, s));
      }
    } else {
      HIP_TRY(launch_loss_win_bwd(W, grad_out_dev, n_valid_dev, grad_coords, kStressBlocks, s));
    }
  } else {
    HIP_TRY(launch_stress_bwd(P, grad_out_dev, n_valid_dev, grad_coords, s));
  }
  return ok();
}

pgsgd_status pgsgd_adam_step(float* x, const float* grad, float* m, float* v, uint64_t n, float lr, float beta1,
                             float beta2, float eps, uint32_t t, void* stream) {
  if (!x || !grad || !m || !v) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  if (t < 1) return fail(PGSGD_ERR_INVALID_ARG, "t must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
    return fail(PGSGD_ERR_INVALID_ARG, "betas must be in [0, 1)");
  if (n == 0) return ok();
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  HIP_TRY(launch_adam(x, grad, m, v, n, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------
struct pgsgd_batch {
  int device = 0;
  uint32_t n_graphs = 0;
  pgsgd_tune tune{};
  pgsgd_params params{};
  BatchGraph* d_graphs = nullptr;
  uint64_t* d_seg_off = nullptr;
  uint64_t* d_path_blob = nullptr;
  float* d_eta = nullptr;
  uint32_t* d_zipf = nullptr;
  uint16_t* d_guide = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchLaunch launch{};
  std::vector<float*> coords;
  std::vector<float2*> work;
  std::vector<uint64_t> n_nodes;
  uint32_t blocks = 0;
  uint64_t total_terms = 0;
  // windowed form: per graph its launch arguments, grid and schedule; the
  // graphs run on `branches` concurrent branches of the captured HIP graph
  bool windowed = false;
  std::vector<pgsgd_graph*> graphs;
  std::vector<LocalLaunch> wl;
  std::vector<uint32_t> wblocks, wthreads, wblocks_c, wthreads_c;  // grids of mixed and all-cooling iterations
  std::vector<std::vector<float>> weta;
  std::vector<std::vector<uint32_t>> branch_graphs;

  ~pgsgd_batch() {
    DeviceGuard g(device);
    (void)hipDeviceSynchronize();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (void* p : {(void*)d_graphs, (void*)d_seg_off, (void*)d_path_blob, (void*)d_eta, (void*)d_zipf,
                    (void*)d_guide})
      if (p) (void)hipFree(p);
  }
};

namespace {

pgsgd_status check_tune(const pgsgd_tune* t) {
  if (t->block_threads < 64 || t->block_threads > 1024 || t->block_threads % 64)
    return fail(PGSGD_ERR_INVALID_ARG, "tune.block_threads must be a multiple of 64 in [64, 1024]");
  if (t->groups_per_item < 1) return fail(PGSGD_ERR_INVALID_ARG, "tune.groups_per_item must be >= 1");
  if (t->blocks_per_cu < 1) return fail(PGSGD_ERR_INVALID_ARG, "tune.blocks_per_cu must be >= 1");
  if (t->phases < 1 || t->phases > 64) return fail(PGSGD_ERR_INVALID_ARG, "tune.phases must be in [1, 64]");
  if (t->branches > kMaxBranches) return fail(PGSGD_ERR_INVALID_ARG, "tune.branches must be at most %u", kMaxBranches);
  return PGSGD_OK;
}

// Graphs of a windowed batch per concurrent branch: longest first, each to
// the branch with the fewest steps so far.
std::vector<std::vector<uint32_t>> assign_branches(pgsgd_graph* const* graphs, uint32_t n, uint32_t nb) {
  std::vector<uint32_t> order(n);
  for (uint32_t k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return graphs[a]->S > graphs[b]->S; });
  std::vector<std::vector<uint32_t>> out(nb);
  std::vector<uint64_t> load(nb, 0);
  for (uint32_t k : order) {
    const uint32_t j = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    out[j].push_back(k);
    load[j] += graphs[k]->S;
  }
  // odd branches run their graphs smallest first, so large graphs (whose
  // wave caps fill much of the GPU) tend to run beside small ones rather than
  // beside each other
  for (uint32_t j = 1; j < nb; j += 2) std::reverse(out[j].begin(), out[j].end());
  return out;
}

// The windowed batch: every graph keeps its own windowed plan (graph_id + k);
// with capture, one HIP graph runs the branches concurrently, each branch its
// graphs one after another (work copy in, all iterations, work copy out).
pgsgd_status batch_build_windowed(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p,
                                  float* const* coords, const pgsgd_tune& t, bool capture, pgsgd_batch** out) {
  const int dev = graphs[0]->device;
  DeviceGuard guard(dev);
  pgsgd_batch* b = new (std::nothrow) pgsgd_batch();
  if (!b) return fail(PGSGD_ERR_OOM, "host allocation failed");
  b->device = dev;
  b->n_graphs = n;
  b->tune = t;
  b->params = *p;
  b->windowed = true;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e) {
    delete b;
    return fail(PGSGD_ERR_DEVICE, "stream create: %s", hipGetErrorString(e));
  }
  pgsgd_status st = PGSGD_OK;
  for (uint32_t k = 0; k < n && !st; ++k) {
    pgsgd_graph* g = graphs[k];
    pgsgd_params q = *p;
    q.graph_id = p->graph_id + k;
    q.schedule = PGSGD_SCHEDULE_WINDOWED;
    size_t lds = 0;
    if ((st = layout_prepare(g, &q, cs, &lds))) break;
    LayoutLaunch L = make_layout_launch(g, &q);
    L.t_begin = 0;
    L.t_end = L.n_terms;
    L.g_begin = 0;
    L.g_end = L.n_groups;
    LocalLaunch W;
    uint32_t blk = 0, thr = 0, blk_c = 0, thr_c = 0;
    if ((st = local_plan(g, &q, lds, L, cs, &W, &blk, &thr))) break;
    if ((st = local_grid(g, &q, lds, &blk_c, &thr_c, true))) break;
    std::vector<float> eta;
    build_schedule(q.n_iters, eta_max_of(&q, g->d_max), q.eta_min, eta);
    b->graphs.push_back(g);
    b->wl.push_back(W);
    b->wblocks.push_back(blk);
    b->wthreads.push_back(thr);
    b->wblocks_c.push_back(blk_c);
    b->wthreads_c.push_back(thr_c);
    b->weta.push_back(eta);
    b->coords.push_back(coords[k]);
    b->total_terms += L.n_terms;
  }
  // the batch keeps its own power-law table: the graphs' cached tables are
  // rebuilt in place by later calls with another theta or window
  if (!st) {
    std::vector<uint32_t> C;
    std::vector<uint16_t> guide;
    build_zipf(p->zipf_theta, p->zipf_window, C, guide);
    e = hipMalloc((void**)&b->d_zipf, sizeof(uint32_t) * C.size());
    if (!e) e = hipMalloc((void**)&b->d_guide, sizeof(uint16_t) * guide.size());
    if (!e) e = hipMemcpy(b->d_zipf, C.data(), sizeof(uint32_t) * C.size(), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(b->d_guide, guide.data(), sizeof(uint16_t) * guide.size(), hipMemcpyHostToDevice);
    if (e) {
      (void)hipGetLastError();
      st = fail(e == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE, "batch power-law table: %s",
                hipGetErrorString(e));
    }
    for (LocalLaunch& W : b->wl) {
      W.L.zipf = b->d_zipf;
      W.L.guide = b->d_guide;
    }
  }
  if (st) {
    (void)hipStreamDestroy(cs);
    delete b;
    return st;
  }
  const uint32_t nb = std::min<uint32_t>(t.branches ? t.branches : kAutoBranches, n);
  b->branch_graphs = assign_branches(graphs, n, nb);
  if (capture) {
    const uint32_t last = p->last_iter == 0 ? p->n_iters : p->last_iter;
    std::vector<hipStream_t> bs(nb, nullptr);
    std::vector<hipEvent_t> join(nb, nullptr);
    hipEvent_t fork = nullptr;
    e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (uint32_t j = 0; j < nb && !e; ++j) {
      e = hipStreamCreateWithFlags(&bs[j], hipStreamNonBlocking);
      if (!e) e = hipEventCreateWithFlags(&join[j], hipEventDisableTiming);
    }
    bool capturing = false;
    if (!e) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (!e) {
      capturing = true;
      e = hipEventRecord(fork, cs);
    }
    for (uint32_t j = 0; j < nb && !e; ++j) {
      e = hipStreamWaitEvent(bs[j], fork, 0);
      for (uint32_t k : b->branch_graphs[j]) {
        pgsgd_graph* g = graphs[k];
        if (!e) e = launch_to_work(coords[k], g->d_work, g->n_nodes, g->d_inv, bs[j]);
        for (uint32_t it = p->first_iter; it < last && !e; ++it) {
          LocalLaunch W = b->wl[k];
          W.L.iter = it;
          W.L.cool_all = it >= p->n_iters / 2 ? 1u : 0u;
          W.L.eta = b->weta[k][it];
          e = local_iteration(W, W.L.cool_all ? b->wblocks_c[k] : b->wblocks[k],
                              W.L.cool_all ? b->wthreads_c[k] : b->wthreads[k], bs[j]);
        }
        if (!e) e = launch_from_work(g->d_work, coords[k], g->n_nodes, g->d_inv, bs[j]);
      }
      if (!e) e = hipEventRecord(join[j], bs[j]);
      if (!e) e = hipStreamWaitEvent(cs, join[j], 0);
    }
    if (capturing) {
      hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
      if (!e) e = e2;
    }
    if (!e) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    for (uint32_t j = 0; j < nb; ++j) {
      if (bs[j]) (void)hipStreamDestroy(bs[j]);
      if (join[j]) (void)hipEventDestroy(join[j]);
    }
    if (fork) (void)hipEventDestroy(fork);
  }
  (void)hipStreamDestroy(cs);
  if (e) {
    (void)hipGetLastError();
    delete b;
    return fail(PGSGD_ERR_DEVICE, "windowed batch setup: %s", hipGetErrorString(e));
  }
  *out = b;
  return PGSGD_OK;
}

// Measured on MI355X (24 chromosome-like graphs): 256 threads, one group per
// item, 2 blocks per CU and graph-major order are the fastest.
pgsgd_tune default_tune() {
  pgsgd_tune t{};
  t.block_threads = 256;
  t.groups_per_item = 1;
  t.blocks_per_cu = 2;
  t.phases = 1;
  return t;
}

// Builds a batch; group_div > 1 restricts every graph to the first 1/group_div
// of its groups (tuning runs only).  capture = false skips the HIP graph.
pgsgd_status batch_build(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p, float* const* coords,
                         const pgsgd_tune* tune, uint32_t group_div, bool capture, pgsgd_batch** out,
                         uint64_t* const* trace_i = nullptr, uint64_t* const* trace_j = nullptr,
                         uint8_t* const* trace_f = nullptr) {
  *out = nullptr;
  if (!graphs || !coords || n == 0) return fail(PGSGD_ERR_INVALID_ARG, "empty or NULL graph list");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if ((uint64_t)p->graph_id + n > (1u << 24)) return fail(PGSGD_ERR_INVALID_ARG, "graph_id + n must be <= 2^24");
  pgsgd_tune t = tune ? *tune : default_tune();
  if ((st = check_tune(&t))) return st;
  const int dev = graphs[0] ? graphs[0]->device : 0;
  uint32_t slots_total = 0;
  for (uint32_t k = 0; k < n; ++k) {
    if (!graphs[k] || !coords[k]) return fail(PGSGD_ERR_INVALID_ARG, "graph or coords %u is NULL", k);
    if (graphs[k]->device != dev) return fail(PGSGD_ERR_INVALID_ARG, "graphs on different devices");
    for (uint32_t q = 0; q < k; ++q)
      if (graphs[q] == graphs[k]) return fail(PGSGD_ERR_INVALID_ARG, "graph %u appears twice in the batch", k);
    if (((uintptr_t)coords[k] & 15u) != 0) return fail(PGSGD_ERR_INVALID_ARG, "coords %u not 16-byte aligned", k);
    if ((uint64_t)p->terms_per_step * graphs[k]->S >= kMaxTerms) return fail(PGSGD_ERR_RANGE, "term count >= 2^48");
    slots_total += graphs[k]->path_slots;
  }
  if (p->reuse_factor > 1 || p->step_reduction > 1)
    return fail(PGSGD_ERR_INVALID_ARG, "the batched form does not run the data-reuse variant");
  if (resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    if (trace_f) return fail(PGSGD_ERR_INVALID_ARG, "internal: windowed batches record through the graph path");
    return batch_build_windowed(graphs, n, p, coords, t, capture, out);
  }
  if (resolve_schedule(p) != PGSGD_SCHEDULE_PLAIN)
    return fail(PGSGD_ERR_INVALID_ARG, "the batched form runs the windowed or the plain schedule");
  const size_t lds = batch_lds_bytes(n, t.phases, slots_total, p->zipf_window);
  if (lds > graphs[0]->lds_limit)
    return fail(PGSGD_ERR_UNSUPPORTED, "batched LDS image of %zu bytes exceeds the %zu-byte block limit", lds,
                graphs[0]->lds_limit);
  DeviceGuard guard(dev);
  pgsgd_batch* b = new (std::nothrow) pgsgd_batch();
  if (!b) return fail(PGSGD_ERR_OOM, "host allocation failed");
  b->device = dev;
  b->n_graphs = n;
  b->tune = t;
  b->params = *p;
  std::vector<BatchGraph> hdr(n);
  std::vector<uint64_t> seg_off((size_t)t.phases * n + 1, 0), blob;
  std::vector<float> eta_all;
  blob.reserve(slots_total);
  for (uint32_t k = 0; k < n; ++k) {
    const pgsgd_graph* g = graphs[k];
    BatchGraph& h = hdr[k];
    h.rec = g->d_rec;
    h.work = g->d_work;
    h.n_nodes = g->n_nodes;
    h.S = g->S;
    h.n_terms = (uint64_t)p->terms_per_step * g->S;
    const uint64_t groups = (h.n_terms + 63) / 64;
    h.n_groups_run = group_div > 1 ? (groups + group_div - 1) / group_div : groups;
    h.path_base = (uint32_t)blob.size();
    h.path_top = g->path_top;
    h.c3 = (kStreamLayout << 24) | (p->graph_id + k);
    h.eta = 0.0f;
    h.trace_i = trace_i ? trace_i[k] : nullptr;
    h.trace_j = trace_j ? trace_j[k] : nullptr;
    h.trace_f = trace_f ? trace_f[k] : nullptr;
    for (uint32_t q = 0; q < g->path_slots; ++q) blob.push_back(q <= g->n_paths ? g->h_path_off[q] : ~0ull);
    h.n_items = (h.n_groups_run + t.groups_per_item - 1) / t.groups_per_item;
    b->total_terms += std::min<uint64_t>(h.n_terms, h.n_groups_run * 64);
    std::vector<float> eta;
    build_schedule(p->n_iters, eta_max_of(p, g->d_max), p->eta_min, eta);
    eta_all.insert(eta_all.end(), eta.begin(), eta.end());
  }
  // segment (phase r, graph k) holds items [floor(r I_k / R), floor((r+1) I_k / R)) of graph k
  const uint32_t R = t.phases;
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t k = 0; k < n; ++k) {
      const uint64_t I = hdr[k].n_items;
      const uint64_t sz = ((r + 1) * I) / R - (r * I) / R;
      const size_t sidx = (size_t)r * n + k;
      seg_off[sidx + 1] = seg_off[sidx] + sz;
    }
  std::vector<uint32_t> C;
  std::vector<uint16_t> guide;
  build_zipf(p->zipf_theta, p->zipf_window, C, guide);
  auto alloc_copy = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    hipError_t e = hipMalloc(dst, bytes ? bytes : 1);
    if (e) return e;
    return bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e;
  if ((e = alloc_copy((void**)&b->d_graphs, hdr.data(), sizeof(BatchGraph) * n)) ||
      (e = alloc_copy((void**)&b->d_seg_off, seg_off.data(), sizeof(uint64_t) * seg_off.size())) ||
      (e = alloc_copy((void**)&b->d_path_blob, blob.data(), sizeof(uint64_t) * blob.size())) ||
      (e = alloc_copy((void**)&b->d_eta, eta_all.data(), sizeof(float) * eta_all.size())) ||
      (e = alloc_copy((void**)&b->d_zipf, C.data(), sizeof(uint32_t) * C.size())) ||
      (e = alloc_copy((void**)&b->d_guide, guide.data(), sizeof(uint16_t) * guide.size()))) {
    (void)hipGetLastError();
    delete b;
    return fail(e == hipErrorOutOfMemory ? PGSGD_ERR_OOM : PGSGD_ERR_DEVICE, "batch setup: %s",
                hipGetErrorString(e));
  }
  int n_cu = graphs[0]->n_cu;
  int max_bpc = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&max_bpc, layout_batch_kernel(), (int)t.block_threads, lds);
  if (e != hipSuccess || max_bpc < 1) {
    (void)hipGetLastError();
    delete b;
    return fail(PGSGD_ERR_UNSUPPORTED, "batched kernel cannot run with %u threads and %zu bytes of LDS",
                t.block_threads, lds);
  }
  const uint32_t bpc = std::min<uint32_t>(t.blocks_per_cu, (uint32_t)max_bpc);
  b->blocks = (uint32_t)n_cu * bpc;
  if (t.max_blocks) b->blocks = std::min(b->blocks, t.max_blocks);
  BatchLaunch& L = b->launch;
  L.graphs = b->d_graphs;
  L.seg_off = b->d_seg_off;
  L.path_blob = b->d_path_blob;
  L.eta_all = b->d_eta;
  L.zipf = b->d_zipf;
  L.guide = b->d_guide;
  L.wave_stride = (uint64_t)b->blocks * (t.block_threads / 64);
  L.groups_per_item = t.groups_per_item;
  L.n_graphs = n;
  L.path_slots_total = slots_total;
  L.W = p->zipf_window;
  L.n_iters = p->n_iters;
  L.k0 = (uint32_t)p->seed;
  L.k1 = (uint32_t)(p->seed >> 32);
  L.phases = t.phases;
  if (capture) {
    hipStream_t cs;
    if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking))) {
      delete b;
      return fail(PGSGD_ERR_DEVICE, "stream create: %s", hipGetErrorString(e));
    }
    const uint32_t last = p->last_iter == 0 ? p->n_iters : p->last_iter;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (uint32_t k = 0; k < n && e == hipSuccess; ++k)
      e = launch_to_work(coords[k], graphs[k]->d_work, graphs[k]->n_nodes, graphs[k]->d_inv, cs);
    for (uint32_t it = p->first_iter; it < last && e == hipSuccess; ++it) {
      BatchLaunch Li = L;
      Li.iter = it;
      Li.cool_all = it >= p->n_iters / 2 ? 1u : 0u;
      e = launch_layout_batch(Li, b->blocks, t.block_threads, cs);
    }
    for (uint32_t k = 0; k < n && e == hipSuccess; ++k)
      e = launch_from_work(graphs[k]->d_work, coords[k], graphs[k]->n_nodes, graphs[k]->d_inv, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete b;
      return fail(PGSGD_ERR_DEVICE, "HIP graph capture: %s", hipGetErrorString(e));
    }
  }
  *out = b;
  return PGSGD_OK;
}

}  // namespace

extern "C" {

pgsgd_status pgsgd_batch_create(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p,
                                float* const* coords, const pgsgd_tune* tune, pgsgd_batch** out) {
  if (!out) return fail(PGSGD_ERR_INVALID_ARG, "out is NULL");
  pgsgd_status st = batch_build(graphs, n, p, coords, tune, 1, true, out);
  return st ? st : ok();
}

pgsgd_status pgsgd_batch_run(pgsgd_batch* b, void* stream) {
  if (!b) return fail(PGSGD_ERR_INVALID_ARG, "batch is NULL");
  DeviceGuard guard(b->device);
  if (b->exec) HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return ok();
}

void pgsgd_batch_destroy(pgsgd_batch* b) { delete b; }

pgsgd_status pgsgd_layout_batched(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p,
                                  float* const* coords, const pgsgd_tune* tune, void* stream) {
  pgsgd_batch* b = nullptr;
  pgsgd_status st = pgsgd_batch_create(graphs, n, p, coords, tune, &b);
  if (st) return st;
  st = pgsgd_batch_run(b, stream);
  if (!st) {
    DeviceGuard guard(b->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) st = fail(PGSGD_ERR_DEVICE, "batched run: %s", hipGetErrorString(e));
  }
  pgsgd_batch_destroy(b);
  return st ? st : ok();
}

pgsgd_status pgsgd_batch_sample_terms(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p, uint32_t iter,
                                      const pgsgd_tune* tune, uint64_t* const* i_out, uint64_t* const* j_out,
                                      uint8_t* const* flags_out, void* stream) {
  if (!i_out || !j_out || !flags_out || !graphs || n == 0) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  pgsgd_status st = check_params(p);
  if (st) return st;
  if (iter >= p->n_iters) return fail(PGSGD_ERR_INVALID_ARG, "iter %u >= n_iters %u", iter, p->n_iters);
  for (uint32_t k = 0; k < n; ++k)
    if (!i_out[k] || !j_out[k] || !flags_out[k]) return fail(PGSGD_ERR_INVALID_ARG, "trace buffer %u is NULL", k);
  if (resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    // a windowed batch runs every graph's own windowed kernels (graph_id + k):
    // record each graph's slots with them
    for (uint32_t k = 0; k < n; ++k) {
      if (!graphs[k]) return fail(PGSGD_ERR_INVALID_ARG, "graph %u is NULL", k);
      pgsgd_params q = *p;
      q.graph_id = p->graph_id + k;
      q.schedule = PGSGD_SCHEDULE_WINDOWED;
      q.first_iter = iter;
      q.last_iter = iter + 1;
      const uint64_t T = (uint64_t)p->terms_per_step * graphs[k]->S;
      if (T == 0) continue;
      LayoutHook h;
      h.trace_i = i_out[k];
      h.trace_j = j_out[k];
      h.trace_f = flags_out[k];
      h.sub_count = T;
      if ((st = layout_impl(graphs[k], &q, nullptr, nullptr, nullptr, nullptr, stream, h))) return st;
    }
    return ok();
  }
  // the coordinates are never touched in trace mode; any aligned pointer will do
  std::vector<float*> dummy(n, reinterpret_cast<float*>(16));
  pgsgd_batch* b = nullptr;
  if ((st = batch_build(graphs, n, p, dummy.data(), tune, 1, false, &b, i_out, j_out, flags_out))) return st;
  DeviceGuard guard(b->device);
  BatchLaunch L = b->launch;
  L.iter = iter;
  L.cool_all = iter >= p->n_iters / 2 ? 1u : 0u;
  hipError_t e = launch_layout_batch(L, b->blocks, b->tune.block_threads, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  delete b;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PGSGD_ERR_DEVICE, "batched sampling: %s", hipGetErrorString(e));
  }
  return ok();
}

}  // extern "C"

namespace {

// Windowed batches: times one iteration of all graphs for 1, 2, 3, 4, 6 and 8
// concurrent branches (launched directly, not captured) and keeps the fastest.
pgsgd_status autotune_windowed(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p, float* const* coords,
                               pgsgd_tune* best, float* ms_out, hipStream_t s) {
  pgsgd_params pt = *p;
  pt.first_iter = 0;
  pt.last_iter = 1;
  pgsgd_tune t0 = default_tune();
  t0.max_blocks = best->max_blocks;
  pgsgd_batch* b = nullptr;
  pgsgd_status st = batch_build(graphs, n, &pt, coords, &t0, 1, false, &b);
  if (st) return st;
  std::vector<hipStream_t> bs(kMaxBranches, nullptr);
  std::vector<hipEvent_t> join(kMaxBranches, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (!e) e = hipEventCreate(&e1);
  for (uint32_t j = 0; j < kMaxBranches && !e; ++j) {
    e = hipStreamCreateWithFlags(&bs[j], hipStreamNonBlocking);
    if (!e) e = hipEventCreateWithFlags(&join[j], hipEventDisableTiming);
  }
  // the caller's coordinates are loaded into the working copies and never written back
  for (uint32_t k = 0; k < n && !e; ++k) e = launch_to_work(coords[k], graphs[k]->d_work, graphs[k]->n_nodes, graphs[k]->d_inv, s);
  // one iteration with uniform partners and one cooling iteration (their costs differ by almost 2x)
  const uint32_t probe_iters[2] = {0u, p->n_iters / 2};
  auto run = [&](uint32_t nb, float* ms) -> hipError_t {
    const auto br = assign_branches(graphs, n, nb);
    hipError_t r = hipEventRecord(e0, s);
    for (uint32_t j = 0; j < nb && !r; ++j) {
      r = hipStreamWaitEvent(bs[j], e0, 0);
      for (uint32_t k : br[j])
        for (uint32_t it : probe_iters) {
          LocalLaunch W = b->wl[k];
          W.L.iter = it;
          W.L.cool_all = it >= p->n_iters / 2 ? 1u : 0u;
          W.L.eta = b->weta[k][std::min<uint32_t>(it, (uint32_t)b->weta[k].size() - 1)];
          if (!r)
            r = local_iteration(W, W.L.cool_all ? b->wblocks_c[k] : b->wblocks[k],
                                W.L.cool_all ? b->wthreads_c[k] : b->wthreads[k], bs[j]);
        }
      if (!r) r = hipEventRecord(join[j], bs[j]);
      if (!r) r = hipStreamWaitEvent(s, join[j], 0);
    }
    if (!r) r = hipEventRecord(e1, s);
    if (!r) r = hipEventSynchronize(e1);
    if (!r && ms) r = hipEventElapsedTime(ms, e0, e1);
    return r;
  };
  float best_ms = 1e30f;
  uint32_t best_nb = 0;
  if (!e) e = run(1, nullptr);  // warm-up
  for (uint32_t nb : {1u, 2u, 3u, 4u, 6u, 8u}) {
    if (e || nb > n) break;
    float ms = 0.0f;
    e = run(nb, &ms);
    if (!e && ms < best_ms) {
      best_ms = ms;
      best_nb = nb;
    }
  }
  (void)hipStreamSynchronize(s);
  for (uint32_t j = 0; j < kMaxBranches; ++j) {
    if (bs[j]) (void)hipStreamDestroy(bs[j]);
    if (join[j]) (void)hipEventDestroy(join[j]);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  delete b;
  if (e) {
    (void)hipGetLastError();
    return fail(PGSGD_ERR_DEVICE, "windowed tuning: %s", hipGetErrorString(e));
  }
  *best = t0;
  best->branches = best_nb;
  if (ms_out) *ms_out = best_ms;
  return PGSGD_OK;
}

}  // namespace

extern "C" {

pgsgd_status pgsgd_autotune_batched(pgsgd_graph* const* graphs, uint32_t n, const pgsgd_params* p,
                                    float* const* coords, pgsgd_tune* best, float* ms_out, void* stream) {
  if (!best || !graphs || !coords || n == 0) return fail(PGSGD_ERR_INVALID_ARG, "NULL argument");
  const uint32_t tune_cap = best->max_blocks;  // a caller's concurrency cap is kept
  pgsgd_status st = check_params(p);
  if (st) return st;
  const int dev = graphs[0] ? graphs[0]->device : 0;
  DeviceGuard guard(dev);
  hipStream_t s = (hipStream_t)stream;
  // Tuning runs load the caller's coordinates into the graphs' working copies
  // and never write them back, so the caller's buffers are left unchanged.
  for (uint32_t k = 0; k < n; ++k)
    if (!graphs[k] || !coords[k]) return fail(PGSGD_ERR_INVALID_ARG, "graph or coords %u is NULL", k);
  if (resolve_schedule(p) == PGSGD_SCHEDULE_WINDOWED) {
    st = autotune_windowed(graphs, n, p, coords, best, ms_out, s);
    return st ? st : ok();
  }
  pgsgd_params pt = *p;
  pt.first_iter = 0;
  pt.last_iter = 1;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const uint32_t threads_c[] = {256, 512};
  const uint32_t gpi_c[] = {1, 4, 16};
  const uint32_t bpc_c[] = {1, 2, 4};
  const uint32_t phase_c[] = {1, 4};
  float best_ms = 1e30f;
  pgsgd_tune best_t = default_tune();
  best_t.max_blocks = tune_cap;
  bool any = false;
  for (uint32_t ph : phase_c)
  for (uint32_t th : threads_c)
    for (uint32_t gpi : gpi_c)
      for (uint32_t bpc : bpc_c) {
        if (bpc * th / 64 > 32) continue;  // more waves than a CU holds
        pgsgd_tune t{th, gpi, bpc, tune_cap, ph};
        pgsgd_batch* b = nullptr;
        if (batch_build(graphs, n, &pt, coords, &t, 16, false, &b) != PGSGD_OK) continue;
        BatchLaunch L = b->launch;
        L.iter = 0;
        L.cool_all = 0;
        float ms = 0.0f;
        bool good = true;
        for (uint32_t k = 0; k < n && good; ++k)
          good = launch_to_work(coords[k], graphs[k]->d_work, graphs[k]->n_nodes, graphs[k]->d_inv, s) == hipSuccess;
        if (good) good = launch_layout_batch(L, b->blocks, th, s) == hipSuccess;  // warm-up
        if (good) good = hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; r < 2 && good; ++r) good = launch_layout_batch(L, b->blocks, th, s) == hipSuccess;
        if (good) good = hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        if (good) good = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        delete b;
        if (!good) {
          (void)hipGetLastError();
          continue;
        }
        ms *= 0.5f;
        if (ms < best_ms) {
          best_ms = ms;
          best_t = t;
          any = true;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  if (!any) return fail(PGSGD_ERR_DEVICE, "no tuning candidate could run");
  *best = best_t;
  if (ms_out) *ms_out = best_ms;
  return ok();
}

}  // extern "C"
