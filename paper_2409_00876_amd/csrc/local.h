// Window-major schedule: the structures shared by the host runtime and the
// kernels of local_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pgsgd {

constexpr uint32_t kStreamWindow = 5;       // Philox stream of the window-slot draws
constexpr uint32_t kLocalShift = 14;        // preferred window: 2^14 steps (about 1 MB of records and coordinates)
constexpr uint32_t kLocalMinWindows = 16;   // smaller windows for small graphs, down to 2^6 steps
constexpr uint32_t kLocalMaxWindows = 32768;
constexpr uint32_t kLocalStreams = 1;       // runs per XCD worked on at the same time
constexpr uint32_t kLocalMaxStreams = 16;
constexpr uint32_t kLocalGrab = 4;          // items a wave takes from its run's counter at once
// Automatic wave cap: waves <= nodes_w / 8, nodes_w ~ 2^shift * n_nodes *
// n_paths / S the node ids a window spans (an XCD's in-flight terms then
// number about as many as its window's node ids), never above the plain cap.
// With the far-first update order of uniform-partner terms, layout quality on
// locality-ordered graphs is flat up to this cap.
constexpr uint64_t kLocalNodesPerWave = 8;
// In the iterations whose terms all have power-law partners (t >= n_iters /
// 2) both endpoints of every in-flight term lie in the XCD's active window, so
// lost Hogwild updates concentrate there: the automatic cap is nodes_w / 32
// (measured on a 9.9M-node, 90-path graph against the oracle's layout, on the
// same pairs of Eq. 2 at m = 3000: nodes_w / 8 left 5.3% more stress, nodes_w /
// 32 2.6%, for 0.6 s more per layout of 3.5 s).
constexpr uint64_t kLocalNodesPerWaveCooling = 32;

// log2 of the window length for S steps: 2^14, halved while there would be
// fewer than 16 windows (not below 2^6), doubled while there would be more
// than 32768.  Part of the sampling definition (the slot draws depend on it).
inline uint32_t window_shift(uint64_t S) {
  auto n = [&](uint32_t sh) { return (S + (1ull << sh) - 1) >> sh; };
  uint32_t sh = kLocalShift;
  while (sh > 6 && n(sh) < kLocalMinWindows) --sh;
  while (n(sh) > kLocalMaxWindows) ++sh;
  return sh;
}

// log2 of the segment length of the loss's window-major pairs (reading R22):
// 2^10 steps, halved while there would be fewer than 16 windows (not below
// 2^6), doubled while there would be more than 32768.  Part of the loss's pair
// definition.
inline uint32_t loss_shift(uint64_t S) {
  auto n = [&](uint32_t sh) { return (S + (1ull << sh) - 1) >> sh; };
  uint32_t sh = 10;
  while (sh > 6 && n(sh) < kLocalMinWindows) --sh;
  while (n(sh) > kLocalMaxWindows) ++sh;
  return sh;
}

// Processing order: kXcds * streams runs of windows; run sigma = x * streams +
// r is stream r of XCD x and holds the windows starting in piece sigma of
// every path (paths cut into kXcds * streams equal pieces), in id order.
struct LocalLaunch {
  LayoutLaunch L;          // sampling parameters, coordinates, trace pointers (trace range in slot order)
  uint32_t n_win;          // ceil(S / 2^win_shift)
  uint32_t win_shift;
  uint32_t count_blocks;   // grid of the count kernel
  uint32_t streams;        // concurrent window streams per XCD
  uint32_t xstride;        // row length of xitem
  uint32_t grab;           // items a wave takes from its stream's counter at once
  uint32_t* wcount;        // [n_win] histogram (zeroed by the scan for the next iteration)
  uint64_t* woff;          // [n_win + 1] first slot of every window (window-id order)
  const uint32_t* worder;  // [n_win] windows in region order
  const uint32_t* sbeg;    // [kXcds * streams + 1] first position in worder of every run
  const uint32_t* wpath;   // [n_win] path holding the whole window, or bit 31 set if it spans paths
  uint64_t* xitem;         // [kXcds * streams][xstride] prefix of 64-slot groups over the windows of each run
  uint64_t* queue;         // [kXcds * streams * 16] item counters, one per run on its own 128-byte line
};

hipError_t launch_local_count_scan(const LocalLaunch& P, hipStream_t s);
hipError_t launch_layout_local(const LocalLaunch& P, uint32_t blocks, uint32_t threads, hipStream_t s);
const void* layout_local_kernel();

}  // namespace pgsgd
