// Device-side building blocks of the PG-SGD layout for gfx950 (CDNA4, wave64).
//
// Everything here runs per lane in registers: the counter-based Philox draw,
// the step / path / partner selection of Alg. 1 (Section "Path-Guided SGD
// Algorithm"), the nucleotide reference distance and the clamped update.  Only
// per-block path metadata and the power-law table live in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgsgd {

// One path step as the kernels read it: 16 bytes, one dwordx4 load.
//   pos      nucleotide offset of the step from the start of its path
//   node_rev node id, bit 31 = reverse-strand visit
//   len      nucleotide length of the node (kept here so a term needs no
//            separate node-length gather: the lean structure of the paper's
//            base kernel, packed per step)
struct alignas(16) StepRec {
  int64_t pos;
  uint32_t node_rev;
  uint32_t len;
};
static_assert(sizeof(StepRec) == 16, "step record must be 16 bytes");

constexpr uint32_t kRevBit = 0x80000000u;
constexpr uint32_t kNodeMask = 0x7FFFFFFFu;
constexpr int kGuideBits = 10;                 // power-law guide table: 2^10 buckets of u
constexpr uint32_t kGuideSize = 1u << kGuideBits;

enum : uint32_t { kStreamLayout = 0, kStreamSps = 1, kStreamPairs = 2, kStreamInit = 3 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products; the key advances by a Weyl sequence between rounds.
// ---------------------------------------------------------------------------
struct Rand4 {
  uint32_t r0, r1, r2, r3;
};

__device__ __forceinline__ Rand4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Rand4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }
__device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) { return __umulhi(a, b); }

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Exclusive prefix of v over the block (blockDim.x = 1024: 16 waves): wave
// scans with shuffles, then one wave scans the 16 wave totals.  *total gets
// the block sum.  Every thread calls it.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* lds16, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) lds16[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint64_t t = lane < 16 ? lds16[lane] : 0;
#pragma unroll
    for (uint32_t d = 1; d < 16; d <<= 1) {
      const uint64_t y = __shfl_up(t, d, 64);
      if (lane >= d) t += y;
    }
    if (lane < 16) lds16[lane] = t;  // inclusive prefix of the wave totals
  }
  __syncthreads();
  const uint64_t before = wave ? lds16[wave - 1] : 0;
  *total = lds16[15];
  __syncthreads();  // lds16 may be reused by the caller
  return before + x - v;
}

// Largest p in [0, n_paths) with off[p] <= i (off is non-decreasing and
// off[n_paths] = S > i).  Fixed trip count: log2 of the power of two >= n_paths.
__device__ __forceinline__ uint32_t find_path(const uint64_t* __restrict__ off, uint32_t top_bit, uint64_t i) {
  uint32_t p = 0;
  for (uint32_t step = top_bit; step != 0; step >>= 1) {
    const uint32_t q = p + step;
    // off has n_paths+1 valid entries padded with UINT64_MAX up to 2*top_bit
    if (off[q] <= i) p = q;
  }
  return p;
}

// Smallest k in [1, n] with C[k] > u, where u = floor(r * C[n] / 2^32); the
// guide table bounds the search to the keys of u's top kGuideBits bits.
__device__ __forceinline__ uint32_t zipf_draw(const uint32_t* __restrict__ C, const uint16_t* __restrict__ guide,
                                              uint32_t n, uint32_t r) {
  const uint32_t u = mulhi32(r, C[n]);
  const uint32_t b = u >> (32 - kGuideBits);
  uint32_t lo = guide[b];
  uint32_t hi = min((uint32_t)guide[b + 1], n);
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (C[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Power-law partner of step i in a path [start, start+len): direction from bit
// 2 of r3 (0 = towards the end), flipped when there is no room that way; the
// hop z ~ Zipf on [1, min(W, room)].  Returns false when the path has a single
// step (no partner exists).
__device__ __forceinline__ bool partner_power_law(uint64_t i, uint64_t start, uint64_t len, uint32_t r2,
                                                  uint32_t r3, const uint32_t* __restrict__ C,
                                                  const uint16_t* __restrict__ guide, uint32_t W, uint64_t& j) {
  const uint64_t room_plus = start + len - 1 - i;
  const uint64_t room_minus = i - start;
  bool down = (r3 >> 2) & 1u;
  if (!down && room_plus == 0) down = true;
  else if (down && room_minus == 0) down = false;
  const uint64_t room = down ? room_minus : room_plus;
  if (room == 0) {
    j = i;
    return false;
  }
  const uint32_t n = room < (uint64_t)W ? (uint32_t)room : W;
  const uint32_t z = zipf_draw(C, guide, n, r2);
  j = down ? i - z : i + z;
  return true;
}

// Path coordinate of endpoint e of a step: the start endpoint is met first on
// a forward visit and last on a reverse one.
__device__ __forceinline__ int64_t endpoint_pos(const StepRec& s, uint32_t e) {
  return s.pos + (int64_t)s.len * (int64_t)(e ^ (s.node_rev >> 31));
}

__device__ __forceinline__ StepRec load_rec(const StepRec* __restrict__ rec, uint64_t s) {
  const uint4 v = *reinterpret_cast<const uint4*>(rec + s);
  StepRec r;
  r.pos = (int64_t)((uint64_t)v.x | ((uint64_t)v.y << 32));
  r.node_rev = v.z;
  r.len = v.w;
  return r;
}

// One sampled term of an iteration.
struct Term {
  uint64_t i, j;
  uint32_t flags;  // bit0 e_i, bit1 e_j, bit2 cooling, bit3 skipped by sampling
};

// Gathers the two step records, forms the slots and the reference distance.
// Returns false if the term is skipped (same slot or zero distance).
__device__ __forceinline__ bool resolve_term(const StepRec* __restrict__ rec, const Term& T, uint64_t& a,
                                             uint64_t& b, float& d) {
  const StepRec si = load_rec(rec, T.i);
  const StepRec sj = load_rec(rec, T.j);
  const uint32_t ei = T.flags & 1u, ej = (T.flags >> 1) & 1u;
  a = 2ull * (si.node_rev & kNodeMask) + ei;
  b = 2ull * (sj.node_rev & kNodeMask) + ej;
  const int64_t dd = endpoint_pos(si, ei) - endpoint_pos(sj, ej);
  d = (float)(dd < 0 ? -dd : dd);
  return a != b && dd != 0;
}

// The clamped SGD step for one pair of points a, b with reference distance d
// (Zheng et al.'s update, which the paper follows for "move against the
// gradient"): mu = min(eta / d^2, 1), r = mu (mag - d) / (2 mag) and disp =
// r (a - b); a moves by -disp and b by +disp.  Returns false (disp unset)
// when the points coincide.  FP32 throughout.  Every layout kernel (plain,
// window-major, data reuse, batched, the parity hook) takes its updates from
// this one function.
__device__ __forceinline__ bool clamped_step(float2 pa, float2 pb, float d, float eta, float2& disp) {
  const float dx = pa.x - pb.x, dy = pa.y - pb.y;
  const float mag = sqrtf(dx * dx + dy * dy);
  if (mag == 0.0f) return false;
  const float mu = fminf(eta / (d * d), 1.0f);
  const float r = mu * (mag - d) / (2.0f * mag);
  disp = make_float2(r * dx, r * dy);
  return true;
}

// One term's update on the interleaved working copy of the coordinates, with
// unlocked loads and stores (Hogwild).  W[2n+e] = (x, y) of endpoint e of node
// n, so each endpoint is one 8-byte access (one cache line) and a node's two
// endpoints share 16 bytes.
__device__ __forceinline__ void apply_update(float2* __restrict__ W, uint64_t a, uint64_t b, float d, float eta) {
  const float2 pa = W[a], pb = W[b];
  float2 m;
  if (!clamped_step(pa, pb, d, eta, m)) return;
  W[a] = make_float2(pa.x - m.x, pa.y - m.y);
  W[b] = make_float2(pb.x + m.x, pb.y + m.y);
}

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

// Sampling of one term from its draw (all integer): step i, partner j, flags.
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

}  // namespace pgsgd
