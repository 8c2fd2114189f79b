/*
 * Seeded synthetic variation-graph generator.
 *
 * This module produces INPUT DATA only (node lengths and path step lists) for
 * both the CPU oracle and the GPU library.  It holds none of the layout
 * method's arithmetic: no positions, no distances, no sampling of terms.
 *
 * Model (a stand-in for the HPRC chromosome graphs, whose data is not
 * available here):
 *   - backbone nodes 0..B-1 in a chain; each backbone node has length
 *     1 + Geometric(p) where the geometric variable counts failures before the
 *     first success (so the mean length is 1/p);
 *   - every haplotype path walks the backbone; at each visited position k,
 *     independently:
 *       * with prob. p_snp it visits the SNP alternative node of k (length 1,
 *         shared by every path that takes it, created on first use) instead of k;
 *       * with prob. p_skip it then skips the next U{1..max_run} positions;
 *       * with prob. p_inv it then traverses the next U{1..max_run} positions in
 *         reverse order on the reverse strand (an inversion);
 *   - final node ids are in backbone order with each used SNP alternative
 *     placed right after its backbone node, i.e. the ids are already ordered
 *     for locality the way a path-guided sort orders a real graph.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
 * one independent stream per path and one for node lengths, so the output is a
 * pure function of the arguments.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t splitmix64(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Probability q in [0,1] -> 64-bit threshold such that P(u < thr) = q. */
static uint64_t prob_threshold(double q) {
  if (q <= 0.0) return 0;
  if (q >= 1.0) return UINT64_MAX;
  return (uint64_t)(q * 18446744073709551616.0);
}

/* Uniform integer in [1, m]. */
static inline uint32_t uniform_1m(uint64_t *st, uint32_t m) {
  uint64_t u = splitmix64(st) >> 32;
  return 1u + (uint32_t)((u * (uint64_t)m) >> 32);
}

static uint64_t stream_seed(uint64_t seed, uint64_t which) {
  uint64_t s = seed ^ (0xD1B54A32D192ED03ull * (which + 1));
  (void)splitmix64(&s);
  return s;
}

#define REV_BIT 0x80000000u

/*
 * Generate one graph.
 *   node_len   : capacity 2*B entries (filled with n_nodes entries)
 *   path_off   : n_paths+1 entries
 *   step_node  : capacity n_paths*B entries (filled with n_steps entries);
 *                bit 31 marks a reverse-strand visit
 *   stats[0..3]: SNP-alternative visits, reverse-strand visits, skipped
 *                backbone positions, number of SNP alternative nodes
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
int synth_generate(uint64_t B, double p_len, uint32_t n_paths, uint64_t seed,
                   double p_snp, double p_skip, double p_inv, uint32_t max_run,
                   uint32_t *node_len, uint64_t *path_off, uint32_t *step_node,
                   uint64_t *n_nodes_out, uint64_t *n_steps_out, uint64_t *stats) {
  if (B == 0 || B >= (1ull << 29) || !(p_len > 0.0 && p_len <= 1.0) || max_run == 0 ||
      !node_len || !path_off || (!step_node && n_paths > 0) || !n_nodes_out || !n_steps_out)
    return -1;
  const uint64_t thr_len = prob_threshold(p_len);
  const uint64_t thr_snp = prob_threshold(p_snp);
  const uint64_t thr_skip = prob_threshold(p_skip);
  const uint64_t thr_inv = prob_threshold(p_inv);

  /* provisional ids: backbone k -> 2k, SNP alternative of k -> 2k+1 */
  uint8_t *alt_used = (uint8_t *)calloc(B, 1);
  if (!alt_used) return -2;
  uint64_t n_snp = 0, n_rev = 0, n_skipped = 0;
  uint64_t s = 0;
  path_off[0] = 0;
  for (uint32_t h = 0; h < n_paths; ++h) {
    uint64_t st = stream_seed(seed, 1000 + (uint64_t)h);
    uint64_t k = 0;
    while (k < B) {
      if (splitmix64(&st) < thr_snp) {
        step_node[s++] = (uint32_t)(2 * k + 1);
        alt_used[k] = 1;
        ++n_snp;
      } else {
        step_node[s++] = (uint32_t)(2 * k);
      }
      k += 1;
      if (splitmix64(&st) < thr_skip) {
        uint64_t L = uniform_1m(&st, max_run);
        uint64_t e = k + L < B ? k + L : B;
        n_skipped += e - k;
        k = e;
      }
      if (splitmix64(&st) < thr_inv) {
        uint64_t L = uniform_1m(&st, max_run);
        uint64_t e = k + L < B ? k + L : B;
        for (uint64_t q = e; q > k; --q) {
          step_node[s++] = (uint32_t)(2 * (q - 1)) | REV_BIT;
          ++n_rev;
        }
        k = e;
      }
    }
    path_off[h + 1] = s;
  }

  /* compact provisional ids into final ids */
  uint32_t *remap = (uint32_t *)malloc(sizeof(uint32_t) * 2 * B);
  if (!remap) { free(alt_used); return -2; }
  uint64_t st_len = stream_seed(seed, 0);
  uint64_t n = 0, n_alt = 0;
  for (uint64_t k = 0; k < B; ++k) {
    uint32_t len = 1;
    while (splitmix64(&st_len) >= thr_len) ++len;
    remap[2 * k] = (uint32_t)n;
    node_len[n++] = len;
    if (alt_used[k]) {
      remap[2 * k + 1] = (uint32_t)n;
      node_len[n++] = 1;
      ++n_alt;
    } else {
      remap[2 * k + 1] = UINT32_MAX;
    }
  }
  for (uint64_t q = 0; q < s; ++q) {
    uint32_t v = step_node[q];
    step_node[q] = remap[v & ~REV_BIT] | (v & REV_BIT);
  }
  free(remap);
  free(alt_used);
  *n_nodes_out = n;
  *n_steps_out = s;
  if (stats) {
    stats[0] = n_snp;
    stats[1] = n_rev;
    stats[2] = n_skipped;
    stats[3] = n_alt;
  }
  return 0;
}
