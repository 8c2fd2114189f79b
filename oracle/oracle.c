/*
 * CPU oracle for PG-SGD pangenome graph layout — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference of what the GPU library computes,
 * written from the paper ("Rapid GPU-Based Pangenome Graph Layout", SC24):
 *   - the layout loop of Alg. 1 (Section "Path-Guided SGD Algorithm"),
 *   - the path stress of Eq. 1 and the sampled path stress of Eq. 2 with its
 *     95% confidence interval (Section "A Quantitative Metric for Pangenome
 *     Layouts"),
 * plus the sampling definition that makes the random choices of Alg. 1
 * reproducible (a counter-based Philox4x32-10 draw per term).  Coordinates
 * are stored in FP32 and every update is computed in FP64; a pure-FP64 batch
 * update exists for the deterministic-batch check.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header or table generator with
 * the GPU library; both implement the same published definitions.
 *
 * Readings of points the paper leaves open (each is stated where used):
 *   R1  N_iters iterations t = 0..N-1 (Alg. 1 loop bounds).
 *   R2  cooling when t >= floor(N/2), or by a fair coin shared by each
 *       aligned group of 64 consecutive terms (warp merging, Section
 *       "Warp Merging", made part of the definition).
 *   R3  "p ∝ |p|, then a step of p" is drawn as one uniform global step.
 *   R4  power-law partner: j = i ± z, z ~ Zipf(theta) truncated to the room
 *       left in the path and to a window W (hop distance counted in steps).
 *   R5  d_ref is the nucleotide distance between the chosen endpoints along
 *       the path: endpoint e of step s sits at pos[s] + len*(e XOR reverse).
 *   R6  the update is the clamped SGD step of Zheng et al. that the paper
 *       follows for "move against the gradient": mu = min(eta/d^2, 1),
 *       each point moves by mu*(mag-d)/2 along the pair direction.
 *   R7  schedule eta_t = eta_max * exp(-lambda t), eta_max = d_max^2,
 *       eta_min = 0.01, lambda = ln(eta_max/eta_min)/(N-1).
 *   R8  terms whose two points coincide as coordinate slots, or whose d is 0,
 *       are skipped (still counted as sampled terms).
 *   R9  sampled path stress draws exactly m*|p| uniform pairs per path,
 *       excludes pairs with d = 0 and pools all paths (Eq. 2).
 *   R17 the data-reuse variant (described in words only) on the plain order.
 *   R18 the window-major order of an iteration's terms (same law of terms).
 *   R19 a sampled stress with the power-law partner instead of a uniform one.
 *   R20 the data-reuse variant on the window-major order.
 *   R21 Eq. 2's pairs visited in window-major order (same law of pairs).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies and xors with a
 * Weyl-sequence key schedule.
 * ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream ids placed in the top byte of counter word 3. */
enum { STREAM_LAYOUT = 0, STREAM_SPS = 1, STREAM_PAIRS = 2, STREAM_INIT = 3 };

static void draw(uint64_t seed, uint64_t index, uint32_t word2, uint32_t stream, uint32_t graph_id,
                 uint32_t r[4]) {
  uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), word2, (stream << 24) | (graph_id & 0xFFFFFFu)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox4x32_10(ctr, key, r);
}

/* floor(a * b / 2^64) and floor(a * b / 2^32): range reduction without rejection. */
static uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }
static uint32_t mulhi32(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

/* ---------------------------------------------------------------------------
 * Zipf (power-law) hop distance, reading R4.  F[k] = sum_{z=1..k} z^-theta in
 * FP64 in increasing z; C[k] = floor(F[k]/F[W] * (2^32-1)) with C[0] = 0.  A
 * draw from 32 random bits r on [1, n] is the smallest k with C[k] > u where
 * u = floor(r * C[n] / 2^32).
 * ------------------------------------------------------------------------- */
void or_zipf_table(double theta, uint32_t W, uint32_t *C) {
  double *F = (double *)malloc(sizeof(double) * ((size_t)W + 1));
  F[0] = 0.0;
  for (uint32_t k = 1; k <= W; ++k) F[k] = F[k - 1] + pow((double)k, -theta);
  C[0] = 0;
  for (uint32_t k = 1; k <= W; ++k) C[k] = (uint32_t)floor(F[k] / F[W] * 4294967295.0);
  free(F);
}

uint32_t or_zipf_draw(const uint32_t *C, uint32_t n, uint32_t r) {
  uint32_t u = mulhi32(r, C[n]);
  /* smallest k in [1, n] with C[k] > u; C[n] > u guarantees one exists */
  uint32_t lo = 1, hi = n;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (C[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* ---------------------------------------------------------------------------
 * Learning-rate schedule S of Alg. 1, reading R7.
 * ------------------------------------------------------------------------- */
void or_schedule(uint32_t n_iters, double eta_max, double eta_min, double *eta) {
  if (n_iters == 0) return;
  if (n_iters == 1) { eta[0] = eta_max; return; }
  double lambda = log(eta_max / eta_min) / (double)(n_iters - 1);
  for (uint32_t t = 0; t < n_iters; ++t) eta[t] = eta_max * exp(-lambda * (double)t);
}

/* ---------------------------------------------------------------------------
 * Graph: only node lengths and path step lists enter the layout (Alg. 1 reads
 * P and L; the lean structure stores node lengths, Section "CUDA Kernel for
 * Pangenome Graph Layout").  pos[s] is the nucleotide offset of step s from
 * the start of its path: the sum of the lengths of the earlier steps.
 * ------------------------------------------------------------------------- */
#define REV_BIT 0x80000000u

typedef struct {
  uint32_t n_nodes, n_paths;
  const uint32_t *node_len;   /* borrowed */
  const uint64_t *path_off;   /* borrowed */
  const uint32_t *step_node;  /* borrowed */
  uint64_t S;
  int64_t *pos;               /* owned */
  int64_t *path_nt;           /* owned */
  int64_t d_max;
} or_graph;

or_graph *or_graph_new(uint32_t n_nodes, const uint32_t *node_len, uint32_t n_paths, const uint64_t *path_off,
                       const uint32_t *step_node) {
  or_graph *g = (or_graph *)calloc(1, sizeof(or_graph));
  g->n_nodes = n_nodes; g->n_paths = n_paths;
  g->node_len = node_len; g->path_off = path_off; g->step_node = step_node;
  g->S = path_off[n_paths];
  g->pos = (int64_t *)malloc(sizeof(int64_t) * (g->S ? g->S : 1));
  g->path_nt = (int64_t *)malloc(sizeof(int64_t) * (n_paths ? n_paths : 1));
  g->d_max = 0;
  for (uint32_t p = 0; p < n_paths; ++p) {
    int64_t acc = 0;
    for (uint64_t s = path_off[p]; s < path_off[p + 1]; ++s) {
      g->pos[s] = acc;
      acc += node_len[step_node[s] & ~REV_BIT];
    }
    g->path_nt[p] = acc;
    if (acc > g->d_max) g->d_max = acc;
  }
  return g;
}

void or_graph_free(or_graph *g) {
  if (!g) return;
  free(g->pos); free(g->path_nt); free(g);
}

const int64_t *or_graph_pos(const or_graph *g) { return g->pos; }
const int64_t *or_graph_path_nt(const or_graph *g) { return g->path_nt; }
int64_t or_graph_d_max(const or_graph *g) { return g->d_max; }

static uint32_t step_node_id(const or_graph *g, uint64_t s) { return g->step_node[s] & ~REV_BIT; }
static uint32_t step_rev(const or_graph *g, uint64_t s) { return g->step_node[s] >> 31; }

/* Reading R5: path coordinate of endpoint e (0 start, 1 end) of step s. */
int64_t or_endpoint_pos(const or_graph *g, uint64_t s, uint32_t e) {
  int64_t len = g->node_len[step_node_id(g, s)];
  return g->pos[s] + len * (int64_t)(e ^ step_rev(g, s));
}

/* Largest p with path_off[p] <= i (empty paths are never returned for i < S). */
static uint32_t path_of_step(const or_graph *g, uint64_t i) {
  uint32_t lo = 0, hi = g->n_paths - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo + 1) / 2;
    if (g->path_off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* ---------------------------------------------------------------------------
 * One term of Alg. 1: step selection (R3), cooling (R2), partner (R4),
 * endpoint coins, and the skip conditions of R8.
 * flags: bit0 e_i, bit1 e_j, bit2 cooling, bit3 skipped.
 * ------------------------------------------------------------------------- */
typedef struct {
  uint32_t n_iters;
  uint32_t zipf_window;
  uint64_t seed;
  uint32_t graph_id;
  const uint32_t *zipf;  /* C[0..W] */
} sampler;

static void partner_power_law(const or_graph *g, const sampler *sp, uint64_t i, uint64_t start, uint64_t len,
                              uint32_t r2, uint32_t r3, uint64_t *j, int *skip) {
  uint64_t room_plus = start + len - 1 - i;
  uint64_t room_minus = i - start;
  uint32_t dir = (r3 >> 2) & 1u;         /* 0: towards the path end, 1: towards its start */
  if (dir == 0 && room_plus == 0) dir = 1;
  else if (dir == 1 && room_minus == 0) dir = 0;
  uint64_t room = dir == 0 ? room_plus : room_minus;
  if (room == 0) { *j = i; *skip = 1; return; }
  uint32_t n = room < sp->zipf_window ? (uint32_t)room : sp->zipf_window;
  uint32_t z = or_zipf_draw(sp->zipf, n, r2);
  *j = dir == 0 ? i + z : i - z;
  (void)g;
}

/* Everything of a term after its step i: partner, endpoint coins, skips;
 * r is the term's draw (words 2 and 3 are used). */
static void term_from_step(const or_graph *g, const sampler *sp, uint32_t iter, uint64_t i, const uint32_t r[4],
                           uint32_t group_coin, uint64_t *i_out, uint64_t *j_out, uint32_t *flags) {
  uint32_t p = path_of_step(g, i);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  uint32_t cooling = (iter >= sp->n_iters / 2) || group_coin;
  uint32_t e_i = r[3] & 1u, e_j = (r[3] >> 1) & 1u;
  uint64_t j;
  int skip = 0;
  if (cooling) partner_power_law(g, sp, i, start, len, r[2], r[3], &j, &skip);
  else j = start + mulhi32(r[2], (uint32_t)len);
  if (!skip) {
    uint64_t a = 2ull * step_node_id(g, i) + e_i, b = 2ull * step_node_id(g, j) + e_j;
    int64_t d = or_endpoint_pos(g, i, e_i) - or_endpoint_pos(g, j, e_j);
    if (a == b || d == 0) skip = 1;
  }
  *i_out = i; *j_out = j;
  *flags = e_i | (e_j << 1) | (cooling << 2) | ((uint32_t)skip << 3);
}

static void sample_term(const or_graph *g, const sampler *sp, uint32_t iter, uint64_t t, uint32_t group_coin,
                        uint64_t *i_out, uint64_t *j_out, uint32_t *flags) {
  uint32_t r[4];
  draw(sp->seed, t, iter, STREAM_LAYOUT, sp->graph_id, r);
  uint64_t i = mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), g->S);
  term_from_step(g, sp, iter, i, r, group_coin, i_out, j_out, flags);
}

/* The fair coin of R2 for the 64-term group containing t: bit 3 of word 3 of
 * the group's first term. */
static uint32_t group_coin_of(const sampler *sp, uint32_t iter, uint64_t t) {
  uint32_t r[4];
  draw(sp->seed, t - (t % 64), iter, STREAM_LAYOUT, sp->graph_id, r);
  return (r[3] >> 3) & 1u;
}

static void make_sampler(sampler *sp, uint32_t n_iters, double theta, uint32_t W, uint64_t seed, uint32_t graph_id) {
  sp->n_iters = n_iters; sp->zipf_window = W; sp->seed = seed; sp->graph_id = graph_id;
  uint32_t *C = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)W + 1));
  or_zipf_table(theta, W, C);
  sp->zipf = C;
}

void or_sample_terms(const or_graph *g, uint32_t n_iters, double theta, uint32_t W, uint64_t seed, uint32_t graph_id,
                     uint32_t iter, uint64_t t_begin, uint64_t count, uint64_t *i_out, uint64_t *j_out,
                     uint8_t *flags_out) {
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  for (uint64_t k = 0; k < count; ++k) {
    uint64_t t = t_begin + k;
    uint32_t fl;
    sample_term(g, &sp, iter, t, group_coin_of(&sp, iter, t), &i_out[k], &j_out[k], &fl);
    flags_out[k] = (uint8_t)fl;
  }
  free((void *)sp.zipf);
}

/* ---------------------------------------------------------------------------
 * The update of one term, reading R6.  Points a and b are coordinate slots
 * 2*node+endpoint in the X and Y planes.  Returns 1 if applied.
 * ------------------------------------------------------------------------- */
static int update_f32(float *X, float *Y, uint64_t a, uint64_t b, int64_t d_int, double eta) {
  double d = (double)d_int;
  double dx = (double)X[a] - (double)X[b];
  double dy = (double)Y[a] - (double)Y[b];
  double mag = sqrt(dx * dx + dy * dy);
  if (mag == 0.0) return 0;
  double mu = eta / (d * d);
  if (mu > 1.0) mu = 1.0;
  double r = mu * (mag - d) / (2.0 * mag);
  X[a] = (float)((double)X[a] - r * dx);
  Y[a] = (float)((double)Y[a] - r * dy);
  X[b] = (float)((double)X[b] + r * dx);
  Y[b] = (float)((double)Y[b] + r * dy);
  return 1;
}

static int update_f64(double *X, double *Y, uint64_t a, uint64_t b, int64_t d_int, double eta) {
  double d = (double)d_int;
  double dx = X[a] - X[b];
  double dy = Y[a] - Y[b];
  double mag = sqrt(dx * dx + dy * dy);
  if (mag == 0.0) return 0;
  double mu = eta / (d * d);
  if (mu > 1.0) mu = 1.0;
  double r = mu * (mag - d) / (2.0 * mag);
  X[a] -= r * dx; Y[a] -= r * dy;
  X[b] += r * dx; Y[b] += r * dy;
  return 1;
}

static int64_t term_distance(const or_graph *g, uint64_t i, uint64_t j, uint32_t flags) {
  int64_t d = or_endpoint_pos(g, i, flags & 1u) - or_endpoint_pos(g, j, (flags >> 1) & 1u);
  return d < 0 ? -d : d;
}

/* Coordinates use the boundary layout [2][n_nodes][2]: the X plane, then the
 * Y plane, endpoint e of node n at index 2n+e. */

/* ---------------------------------------------------------------------------
 * The layout loop of Alg. 1, one thread, terms in order.  Iterations
 * [first, last) of an n_iters schedule; terms_per_step * S terms per
 * iteration (Alg. 1 uses 10).  Returns the number of applied updates.
 * ------------------------------------------------------------------------- */
uint64_t or_layout(const or_graph *g, uint32_t n_iters, uint32_t terms_per_step, double eta_max, double eta_min,
                   double theta, uint32_t W, uint64_t seed, uint32_t graph_id, uint32_t first, uint32_t last,
                   float *coords) {
  if (g->S == 0 || n_iters == 0) return 0;
  if (eta_max <= 0.0) eta_max = (double)g->d_max * (double)g->d_max;
  double *eta = (double *)malloc(sizeof(double) * n_iters);
  or_schedule(n_iters, eta_max, eta_min, eta);
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint64_t T = (uint64_t)terms_per_step * g->S, applied = 0;
  if (last == 0 || last > n_iters) last = n_iters;
  for (uint32_t it = first; it < last; ++it) {
    uint32_t coin = 0;
    for (uint64_t t = 0; t < T; ++t) {
      if (t % 64 == 0) coin = group_coin_of(&sp, it, t);
      uint64_t i, j;
      uint32_t fl;
      sample_term(g, &sp, it, t, coin, &i, &j, &fl);
      if (fl & 8u) continue;
      uint64_t a = 2ull * step_node_id(g, i) + (fl & 1u), b = 2ull * step_node_id(g, j) + ((fl >> 1) & 1u);
      applied += update_f32(X, Y, a, b, term_distance(g, i, j, fl), eta[it]);
    }
  }
  free((void *)sp.zipf);
  free(eta);
  return applied;
}

/* Threaded Hogwild mode (Section "Data-level Parallelism"): T threads take
 * contiguous term ranges and update without locks.  Loads and stores of a
 * coordinate are relaxed atomics on its bit pattern so the races are
 * well-defined; results are not deterministic. */
typedef struct {
  const or_graph *g; const sampler *sp; const double *eta; float *coords;
  uint32_t first, last; uint64_t T, t0, t1; uint64_t applied;
} hw_job;

static float ld_relaxed(const float *p) {
  uint32_t u = __atomic_load_n((const uint32_t *)p, __ATOMIC_RELAXED);
  float f; memcpy(&f, &u, 4); return f;
}
static void st_relaxed(float *p, float f) {
  uint32_t u; memcpy(&u, &f, 4);
  __atomic_store_n((uint32_t *)p, u, __ATOMIC_RELAXED);
}

static void *hogwild_worker(void *arg) {
  hw_job *jb = (hw_job *)arg;
  const or_graph *g = jb->g;
  float *X = jb->coords, *Y = jb->coords + 2ull * g->n_nodes;
  for (uint32_t it = jb->first; it < jb->last; ++it) {
    uint32_t coin = 0;
    for (uint64_t t = jb->t0; t < jb->t1; ++t) {
      if (t == jb->t0 || t % 64 == 0) coin = group_coin_of(jb->sp, it, t);
      uint64_t i, j;
      uint32_t fl;
      sample_term(g, jb->sp, it, t, coin, &i, &j, &fl);
      if (fl & 8u) continue;
      uint64_t a = 2ull * step_node_id(g, i) + (fl & 1u), b = 2ull * step_node_id(g, j) + ((fl >> 1) & 1u);
      double d = (double)term_distance(g, i, j, fl);
      double xa = ld_relaxed(&X[a]), ya = ld_relaxed(&Y[a]), xb = ld_relaxed(&X[b]), yb = ld_relaxed(&Y[b]);
      double dx = xa - xb, dy = ya - yb, mag = sqrt(dx * dx + dy * dy);
      if (mag == 0.0) continue;
      double mu = jb->eta[it] / (d * d);
      if (mu > 1.0) mu = 1.0;
      double r = mu * (mag - d) / (2.0 * mag);
      st_relaxed(&X[a], (float)(xa - r * dx)); st_relaxed(&Y[a], (float)(ya - r * dy));
      st_relaxed(&X[b], (float)(xb + r * dx)); st_relaxed(&Y[b], (float)(yb + r * dy));
      jb->applied++;
    }
  }
  return NULL;
}

/* Runs iterations [first,last) on n_threads threads.  With term_limit > 0 only
 * the first term_limit terms of each iteration are processed (a bounded sample
 * for timing).  Threads synchronise only between iterations. */
uint64_t or_layout_threaded(const or_graph *g, uint32_t n_iters, uint32_t terms_per_step, double eta_max,
                            double eta_min, double theta, uint32_t W, uint64_t seed, uint32_t graph_id,
                            uint32_t first, uint32_t last, float *coords, uint32_t n_threads, uint64_t term_limit) {
  if (g->S == 0 || n_iters == 0 || n_threads == 0) return 0;
  if (eta_max <= 0.0) eta_max = (double)g->d_max * (double)g->d_max;
  double *eta = (double *)malloc(sizeof(double) * n_iters);
  or_schedule(n_iters, eta_max, eta_min, eta);
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  uint64_t T = (uint64_t)terms_per_step * g->S;
  if (term_limit > 0 && term_limit < T) T = term_limit;
  if (last == 0 || last > n_iters) last = n_iters;
  hw_job *jobs = (hw_job *)calloc(n_threads, sizeof(hw_job));
  pthread_t *th = (pthread_t *)calloc(n_threads, sizeof(pthread_t));
  uint64_t applied = 0;
  for (uint32_t it = first; it < last; ++it) {
    for (uint32_t k = 0; k < n_threads; ++k) {
      jobs[k] = (hw_job){g, &sp, eta, coords, it, it + 1, T, T * k / n_threads, T * (k + 1) / n_threads, 0};
      pthread_create(&th[k], NULL, hogwild_worker, &jobs[k]);
    }
    for (uint32_t k = 0; k < n_threads; ++k) {
      pthread_join(th[k], NULL);
      applied += jobs[k].applied;
    }
  }
  free(jobs); free(th); free((void *)sp.zipf); free(eta);
  return applied;
}

/* Pure-FP64 application of a given batch of terms, in order (the
 * deterministic-batch check).  coords64 uses the boundary layout in FP64. */
uint64_t or_apply_terms_f64(const or_graph *g, double eta, const uint64_t *i, const uint64_t *j,
                            const uint8_t *flags, uint64_t count, double *coords64) {
  double *X = coords64, *Y = coords64 + 2ull * g->n_nodes;
  uint64_t applied = 0;
  for (uint64_t k = 0; k < count; ++k) {
    if (flags[k] & 8u) continue;
    uint64_t a = 2ull * step_node_id(g, i[k]) + (flags[k] & 1u);
    uint64_t b = 2ull * step_node_id(g, j[k]) + ((flags[k] >> 1) & 1u);
    applied += update_f64(X, Y, a, b, term_distance(g, i[k], j[k], flags[k]), eta);
  }
  return applied;
}

/* The FP64 batch with every update's r multiplied by r_scale: a deliberately
 * wrong update, used only to measure how small an error of the update the
 * batch check can detect (r_scale = 1 is or_apply_terms_f64). */
uint64_t or_apply_terms_f64_scaled(const or_graph *g, double eta, double r_scale, const uint64_t *i,
                                   const uint64_t *j, const uint8_t *flags, uint64_t count, double *coords64) {
  double *X = coords64, *Y = coords64 + 2ull * g->n_nodes;
  uint64_t applied = 0;
  for (uint64_t k = 0; k < count; ++k) {
    if (flags[k] & 8u) continue;
    uint64_t a = 2ull * step_node_id(g, i[k]) + (flags[k] & 1u);
    uint64_t b = 2ull * step_node_id(g, j[k]) + ((flags[k] >> 1) & 1u);
    double d = (double)term_distance(g, i[k], j[k], flags[k]);
    double dx = X[a] - X[b], dy = Y[a] - Y[b];
    double mag = sqrt(dx * dx + dy * dy);
    if (mag == 0.0) continue;
    double mu = eta / (d * d);
    if (mu > 1.0) mu = 1.0;
    double r = r_scale * mu * (mag - d) / (2.0 * mag);
    X[a] -= r * dx; Y[a] -= r * dy;
    X[b] += r * dx; Y[b] += r * dy;
    ++applied;
  }
  return applied;
}

/* Same, with FP32 storage and FP64 math (what one oracle term does). */
uint64_t or_apply_terms_f32(const or_graph *g, double eta, const uint64_t *i, const uint64_t *j,
                            const uint8_t *flags, uint64_t count, float *coords) {
  float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint64_t applied = 0;
  for (uint64_t k = 0; k < count; ++k) {
    if (flags[k] & 8u) continue;
    uint64_t a = 2ull * step_node_id(g, i[k]) + (flags[k] & 1u);
    uint64_t b = 2ull * step_node_id(g, j[k]) + ((flags[k] >> 1) & 1u);
    applied += update_f32(X, Y, a, b, term_distance(g, i[k], j[k], flags[k]), eta);
  }
  return applied;
}

/* ---------------------------------------------------------------------------
 * Data-reuse variant (Section "A Case Study: Explore the Performance-Quality
 * Trade-off with Sampled Path Stress"): each sampled step yields DRF updates
 * and the number of sampled steps per iteration is divided by SRF.  Reading
 * R17 (the paper gives no formula):
 *   - an iteration has ceil(terms_per_step * S / SRF) sampled terms, in aligned
 *     groups of 64; the group's path is the path of the global step drawn by
 *     its first term (so paths are still chosen with probability ∝ |p|), and
 *     every term t of the group draws its own step uniformly in that path:
 *     i = start + floor(u64(t) * |p| / 2^64); its partner, endpoint coins,
 *     cooling and skips are those of the plain definition;
 *   - after the group's primary updates (terms in order), reuse rounds
 *     k = 1..DRF-1 pair, for every lane l in order, the i-endpoint of lane l
 *     with the j-endpoint of lane (l + o_k) mod 64, o_k = 1 + (byte k-1 of the
 *     words of Philox stream 4 at counter (group, 0, iter)) mod 63, when both
 *     terms exist and are not skipped; d_ref is the path distance of those two
 *     endpoints; pairs with the same slot or d = 0 are skipped.
 * With DRF = 1 and SRF = 1 the loop is or_layout's with group-shared paths.
 * ------------------------------------------------------------------------- */
enum { STREAM_REUSE = 4 };

static void sample_group_term(const or_graph *g, const sampler *sp, uint32_t iter, uint64_t t, uint32_t p,
                              uint32_t group_coin, uint64_t *i_out, uint64_t *j_out, uint32_t *flags) {
  uint32_t r[4];
  draw(sp->seed, t, iter, STREAM_LAYOUT, sp->graph_id, r);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  uint64_t i = start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), len);
  uint32_t cooling = (iter >= sp->n_iters / 2) || group_coin;
  uint32_t e_i = r[3] & 1u, e_j = (r[3] >> 1) & 1u;
  uint64_t j;
  int skip = 0;
  if (cooling) partner_power_law(g, sp, i, start, len, r[2], r[3], &j, &skip);
  else j = start + mulhi32(r[2], (uint32_t)len);
  if (!skip) {
    uint64_t a = 2ull * step_node_id(g, i) + e_i, b = 2ull * step_node_id(g, j) + e_j;
    int64_t d = or_endpoint_pos(g, i, e_i) - or_endpoint_pos(g, j, e_j);
    if (a == b || d == 0) skip = 1;
  }
  *i_out = i; *j_out = j;
  *flags = e_i | (e_j << 1) | (cooling << 2) | ((uint32_t)skip << 3);
}

/* The group's path and the reuse offsets o_1..o_{DRF-1}. */
static uint32_t group_path(const or_graph *g, const sampler *sp, uint32_t iter, uint64_t t0, uint32_t *coin) {
  uint32_t r[4];
  draw(sp->seed, t0, iter, STREAM_LAYOUT, sp->graph_id, r);
  *coin = (r[3] >> 3) & 1u;
  return path_of_step(g, mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), g->S));
}

static void reuse_offsets(const sampler *sp, uint32_t iter, uint64_t group, uint32_t drf, uint32_t *o) {
  uint32_t r[4];
  draw(sp->seed, group, iter, STREAM_REUSE, sp->graph_id, r);
  for (uint32_t k = 1; k < drf; ++k) {
    uint32_t byte = (r[(k - 1) / 4] >> (8 * ((k - 1) % 4))) & 0xFFu;
    o[k] = 1 + byte % 63;
  }
}

void or_sample_terms_reuse(const or_graph *g, uint32_t n_iters, double theta, uint32_t W, uint64_t seed,
                           uint32_t graph_id, uint32_t iter, uint64_t t_begin, uint64_t count, uint64_t *i_out,
                           uint64_t *j_out, uint8_t *flags_out) {
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  for (uint64_t k = 0; k < count; ++k) {
    uint64_t t = t_begin + k;
    uint32_t coin, fl;
    uint32_t p = group_path(g, &sp, iter, t - (t % 64), &coin);
    sample_group_term(g, &sp, iter, t, p, coin, &i_out[k], &j_out[k], &fl);
    flags_out[k] = (uint8_t)fl;
  }
  free((void *)sp.zipf);
}

void or_reuse_offsets(uint64_t seed, uint32_t graph_id, uint32_t iter, uint64_t group, uint32_t drf, uint32_t *o) {
  sampler sp;
  sp.seed = seed; sp.graph_id = graph_id;
  reuse_offsets(&sp, iter, group, drf, o);
}

uint64_t or_layout_reuse(const or_graph *g, uint32_t n_iters, uint32_t terms_per_step, uint32_t drf, uint32_t srf,
                         double eta_max, double eta_min, double theta, uint32_t W, uint64_t seed, uint32_t graph_id,
                         uint32_t first, uint32_t last, float *coords) {
  if (g->S == 0 || n_iters == 0 || drf < 1 || drf > 16 || srf < 1) return 0;
  if (eta_max <= 0.0) eta_max = (double)g->d_max * (double)g->d_max;
  double *eta = (double *)malloc(sizeof(double) * n_iters);
  or_schedule(n_iters, eta_max, eta_min, eta);
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint64_t T = ((uint64_t)terms_per_step * g->S + srf - 1) / srf, applied = 0;
  if (last == 0 || last > n_iters) last = n_iters;
  uint64_t ti[64], tj[64];
  uint32_t tf[64], o[17];
  for (uint32_t it = first; it < last; ++it) {
    for (uint64_t t0 = 0; t0 < T; t0 += 64) {
      uint32_t n = (uint32_t)(T - t0 < 64 ? T - t0 : 64), coin;
      uint32_t p = group_path(g, &sp, it, t0, &coin);
      for (uint32_t l = 0; l < n; ++l) {
        sample_group_term(g, &sp, it, t0 + l, p, coin, &ti[l], &tj[l], &tf[l]);
        if (tf[l] & 8u) continue;
        uint64_t a = 2ull * step_node_id(g, ti[l]) + (tf[l] & 1u), b = 2ull * step_node_id(g, tj[l]) + ((tf[l] >> 1) & 1u);
        applied += update_f32(X, Y, a, b, term_distance(g, ti[l], tj[l], tf[l]), eta[it]);
      }
      reuse_offsets(&sp, it, t0 / 64, drf, o);
      for (uint32_t k = 1; k < drf; ++k) {
        for (uint32_t l = 0; l < n; ++l) {
          uint32_t m = (l + o[k]) % 64;
          if (m >= n || (tf[l] & 8u) || (tf[m] & 8u)) continue;
          uint32_t ei = tf[l] & 1u, ej = (tf[m] >> 1) & 1u;
          uint64_t a = 2ull * step_node_id(g, ti[l]) + ei, b = 2ull * step_node_id(g, tj[m]) + ej;
          int64_t d = or_endpoint_pos(g, ti[l], ei) - or_endpoint_pos(g, tj[m], ej);
          if (a == b || d == 0) continue;
          applied += update_f32(X, Y, a, b, d < 0 ? -d : d, eta[it]);
        }
      }
    }
  }
  free((void *)sp.zipf);
  free(eta);
  return applied;
}

/* ---------------------------------------------------------------------------
 * Window-major enumeration of an iteration's terms (reading R18).  The steps
 * are cut into windows of 2^shift consecutive global steps, shift =
 * or_window_shift(S).  The iteration's T = terms_per_step * S terms are
 *   - counted per window: n_w = #{t < T : floor(i_t / 2^shift) = w}, i_t the
 *     step of term t of the plain definition (sample_term), so (n_w) is
 *     multinomial(T, |w| / S);
 *   - enumerated as slots, window after window: slot s = off_w + k (off_w the
 *     prefix of the counts, k < n_w) draws Philox stream 5 at counter s; its
 *     step is uniform in the window, i = start_w + floor(u64 * |w| / 2^64), and
 *     the rest follows term_from_step with the draw's words 2 and 3; the
 *     cooling coin is bit 3 of word 3 of slot off_w + 64 * floor(k / 64).
 * A multinomial count of uniform draws per window is T i.i.d. uniform steps,
 * so the terms have the distribution of Alg. 1; only their order differs.
 * ------------------------------------------------------------------------- */
enum { STREAM_WINDOW = 5 };

uint32_t or_window_shift(uint64_t S) {
  uint32_t sh = 14;
  while (sh > 6 && ((S + (1ull << sh) - 1) >> sh) < 16) --sh;
  while (((S + (1ull << sh) - 1) >> sh) > 32768) ++sh;
  return sh;
}

typedef struct {
  const or_graph *g; uint64_t seed; uint32_t graph_id, iter, sh; uint64_t t0, t1, n_win; uint64_t *counts;
} count_job;

static void *count_worker(void *arg) {
  count_job *jb = (count_job *)arg;
  for (uint64_t w = 0; w < jb->n_win; ++w) jb->counts[w] = 0;
  for (uint64_t t = jb->t0; t < jb->t1; ++t) {
    uint32_t r[4];
    draw(jb->seed, t, jb->iter, STREAM_LAYOUT, jb->graph_id, r);
    jb->counts[mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), jb->g->S) >> jb->sh]++;
  }
  return NULL;
}

/* The counts n_w; `threads` threads count contiguous term ranges into their
 * own histograms, which are then summed (the same integers for any count). */
void or_window_counts(const or_graph *g, uint64_t seed, uint32_t graph_id, uint32_t iter, uint64_t T,
                      uint64_t *counts, uint32_t threads) {
  uint32_t sh = or_window_shift(g->S);
  uint64_t n_win = (g->S + (1ull << sh) - 1) >> sh;
  if (threads < 1) threads = 1;
  count_job *jobs = (count_job *)calloc(threads, sizeof(count_job));
  pthread_t *tid = (pthread_t *)calloc(threads, sizeof(pthread_t));
  for (uint32_t k = 0; k < threads; ++k) {
    jobs[k].g = g; jobs[k].seed = seed; jobs[k].graph_id = graph_id; jobs[k].iter = iter; jobs[k].sh = sh;
    jobs[k].t0 = T * k / threads; jobs[k].t1 = T * (k + 1) / threads; jobs[k].n_win = n_win;
    jobs[k].counts = (uint64_t *)malloc(sizeof(uint64_t) * (n_win ? n_win : 1));
    pthread_create(&tid[k], NULL, count_worker, &jobs[k]);
  }
  for (uint64_t w = 0; w < n_win; ++w) counts[w] = 0;
  for (uint32_t k = 0; k < threads; ++k) {
    pthread_join(tid[k], NULL);
    for (uint64_t w = 0; w < n_win; ++w) counts[w] += jobs[k].counts[w];
    free(jobs[k].counts);
  }
  free(jobs);
  free(tid);
}

/* Slot k of window w (first slot off_w). */
static void sample_slot(const or_graph *g, const sampler *sp, uint32_t iter, uint32_t sh, uint64_t w, uint64_t off_w,
                        uint64_t k, uint64_t *i_out, uint64_t *j_out, uint32_t *flags) {
  uint32_t r[4], lead[4];
  draw(sp->seed, off_w + k, iter, STREAM_WINDOW, sp->graph_id, r);
  draw(sp->seed, off_w + k - (k % 64), iter, STREAM_WINDOW, sp->graph_id, lead);
  uint64_t start = w << sh, len = g->S - start < (1ull << sh) ? g->S - start : (1ull << sh);
  uint64_t i = start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), len);
  term_from_step(g, sp, iter, i, r, (lead[3] >> 3) & 1u, i_out, j_out, flags);
}

static uint64_t *window_offsets(const or_graph *g, const sampler *sp, uint32_t iter, uint64_t T,
                                uint64_t *n_win_out) {
  uint32_t sh = or_window_shift(g->S);
  uint64_t n_win = (g->S + (1ull << sh) - 1) >> sh;
  uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n_win + 1));
  or_window_counts(g, sp->seed, sp->graph_id, iter, T, off + 1, 1);
  off[0] = 0;
  for (uint64_t w = 0; w < n_win; ++w) off[w + 1] += off[w];
  *n_win_out = n_win;
  return off;
}

/* Slots [s_begin, s_begin + count) (all below T) given the window offsets
 * off[0..n_win] (the prefix of or_window_counts for the same iteration). */
void or_sample_terms_windowed(const or_graph *g, uint32_t n_iters, double theta, uint32_t W, uint64_t seed,
                              uint32_t graph_id, uint32_t iter, const uint64_t *off, uint64_t s_begin,
                              uint64_t count, uint64_t *i_out, uint64_t *j_out, uint8_t *flags_out) {
  if (g->S == 0) return;
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  uint32_t sh = or_window_shift(g->S);
  uint64_t n_win = (g->S + (1ull << sh) - 1) >> sh, w = 0;
  for (uint64_t k = 0; k < count; ++k) {
    uint64_t s = s_begin + k;
    while (w + 1 < n_win && off[w + 1] <= s) ++w;
    uint32_t fl;
    sample_slot(g, &sp, iter, sh, w, off[w], s - off[w], &i_out[k], &j_out[k], &fl);
    flags_out[k] = (uint8_t)fl;
  }
  free((void *)sp.zipf);
}

/* The layout loop of Alg. 1 with the window-major enumeration, one thread,
 * slots in order.  With drf > 1 or srf > 1 it is the data-reuse variant on
 * that enumeration (reading R20): ceil(terms_per_step * S / srf) slots per
 * iteration (counted from the plain draws t below that number); after the
 * primary updates of an aligned 64-slot group of a window, rounds k = 1..drf-1
 * pair slot l's i-endpoint with slot (l + o_k) mod 64's j-endpoint of the same
 * group (both present and not skipped, steps i of the same path), o_k from
 * Philox stream 4 at counter (the group's first slot, iteration) as in the
 * plain variant; d_ref from the two endpoints' path coordinates, pairs with
 * the same slot or d = 0 skipped. */
uint64_t or_layout_windowed(const or_graph *g, uint32_t n_iters, uint32_t terms_per_step, uint32_t drf, uint32_t srf,
                            double eta_max, double eta_min, double theta, uint32_t W, uint64_t seed, uint32_t graph_id,
                            uint32_t first, uint32_t last, float *coords) {
  if (g->S == 0 || n_iters == 0 || drf < 1 || drf > 16 || srf < 1) return 0;
  if (eta_max <= 0.0) eta_max = (double)g->d_max * (double)g->d_max;
  double *eta = (double *)malloc(sizeof(double) * n_iters);
  or_schedule(n_iters, eta_max, eta_min, eta);
  sampler sp;
  make_sampler(&sp, n_iters, theta, W, seed, graph_id);
  float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint32_t sh = or_window_shift(g->S);
  uint64_t T = ((uint64_t)terms_per_step * g->S + srf - 1) / srf, applied = 0;
  uint64_t ti[64], tj[64];
  uint32_t tf[64], o[17];
  if (last == 0 || last > n_iters) last = n_iters;
  for (uint32_t it = first; it < last; ++it) {
    uint64_t n_win;
    uint64_t *off = window_offsets(g, &sp, it, T, &n_win);
    for (uint64_t w = 0; w < n_win; ++w) {
      uint64_t nw = off[w + 1] - off[w];
      for (uint64_t g0 = 0; g0 < nw; g0 += 64) {
        uint32_t n = (uint32_t)(nw - g0 < 64 ? nw - g0 : 64);
        for (uint32_t l = 0; l < n; ++l) {
          sample_slot(g, &sp, it, sh, w, off[w], g0 + l, &ti[l], &tj[l], &tf[l]);
          if (tf[l] & 8u) continue;
          uint64_t a = 2ull * step_node_id(g, ti[l]) + (tf[l] & 1u);
          uint64_t b = 2ull * step_node_id(g, tj[l]) + ((tf[l] >> 1) & 1u);
          applied += update_f32(X, Y, a, b, term_distance(g, ti[l], tj[l], tf[l]), eta[it]);
        }
        if (drf < 2) continue;
        reuse_offsets(&sp, it, off[w] + g0, drf, o);
        for (uint32_t k = 1; k < drf; ++k) {
          for (uint32_t l = 0; l < n; ++l) {
            uint32_t m = (l + o[k]) % 64;
            if (m >= n || (tf[l] & 8u) || (tf[m] & 8u)) continue;
            if (path_of_step(g, ti[l]) != path_of_step(g, ti[m])) continue;
            uint32_t ei = tf[l] & 1u, ej = (tf[m] >> 1) & 1u;
            uint64_t a = 2ull * step_node_id(g, ti[l]) + ei, b = 2ull * step_node_id(g, tj[m]) + ej;
            int64_t d = or_endpoint_pos(g, ti[l], ei) - or_endpoint_pos(g, tj[m], ej);
            if (a == b || d == 0) continue;
            applied += update_f32(X, Y, a, b, d < 0 ? -d : d, eta[it]);
          }
        }
      }
    }
    free(off);
  }
  free((void *)sp.zipf);
  free(eta);
  return applied;
}

/* ---------------------------------------------------------------------------
 * Sampled path stress, Eq. 2, with the two-pass CI95 (reading R9).  Pair q of
 * path p, q in [m*off[p], m*off[p+1]), draws Philox stream 1 at counter q:
 * i = start + floor(u64 * |p| / 2^64), j = start + floor(r2 * |p| / 2^32),
 * e_i = bit 0, e_j = bit 1 of r3.  stress = ((mag - d)/d)^2 in FP64.
 * out[0..5] = mean, ci_lo, ci_hi, stddev, sum (pass 1), sum of squared
 * deviations (pass 2); counts[0..1] = n_valid, n_skipped (d == 0).
 * ------------------------------------------------------------------------- */
static void sps_pair(const or_graph *g, uint64_t seed, uint32_t graph_id, uint32_t p, uint64_t q,
                     uint64_t *i, uint64_t *j, uint32_t *ei, uint32_t *ej) {
  uint32_t r[4];
  draw(seed, q, 0, STREAM_SPS, graph_id, r);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  *i = start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), len);
  *j = start + mulhi32(r[2], (uint32_t)len);
  *ei = r[3] & 1u;
  *ej = (r[3] >> 1) & 1u;
}

static double pair_stress(const or_graph *g, const float *coords, uint64_t i, uint64_t j, uint32_t ei, uint32_t ej,
                          int *valid) {
  int64_t dd = or_endpoint_pos(g, i, ei) - or_endpoint_pos(g, j, ej);
  if (dd == 0) { *valid = 0; return 0.0; }
  double d = (double)(dd < 0 ? -dd : dd);
  const float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint64_t a = 2ull * step_node_id(g, i) + ei, b = 2ull * step_node_id(g, j) + ej;
  double dx = (double)X[a] - (double)X[b], dy = (double)Y[a] - (double)Y[b];
  double mag = sqrt(dx * dx + dy * dy);
  double e = (mag - d) / d;
  *valid = 1;
  return e * e;
}

/* Pair q with the power-law partner (reading R19): step i and the draw as in
 * sps_pair, j the cooling phase's power-law partner of i; *ok = 0 when the path
 * has a single step. */
static void sps_pair_power_law(const or_graph *g, const sampler *sp, uint32_t p, uint64_t q, uint64_t *i,
                               uint64_t *j, uint32_t *ei, uint32_t *ej, int *ok) {
  uint32_t r[4];
  draw(sp->seed, q, 0, STREAM_SPS, sp->graph_id, r);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  *i = start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), len);
  int skip = 0;
  partner_power_law(g, sp, *i, start, len, r[2], r[3], j, &skip);
  *ok = !skip;
  *ei = r[3] & 1u;
  *ej = (r[3] >> 1) & 1u;
}

/* Eq. 2 with uniform (mode 0) or power-law (mode 1) partners; theta and W
 * are read in mode 1 only. */
void or_sampled_path_stress_pairs(const or_graph *g, const float *coords, uint32_t m, uint64_t seed,
                                  uint32_t graph_id, uint32_t mode, double theta, uint32_t W, double *out,
                                  uint64_t *counts) {
  sampler sp;
  sp.zipf = NULL;
  if (mode == 1) make_sampler(&sp, 1, theta, W, seed, graph_id);
  double sum = 0.0, dev = 0.0, mean = 0.0;
  uint64_t n = 0, skipped = 0;
  for (int pass = 1; pass <= 2; ++pass) {
    for (uint32_t p = 0; p < g->n_paths; ++p) {
      for (uint64_t q = (uint64_t)m * g->path_off[p]; q < (uint64_t)m * g->path_off[p + 1]; ++q) {
        uint64_t i, j; uint32_t ei, ej; int valid = 1;
        if (mode == 1) sps_pair_power_law(g, &sp, p, q, &i, &j, &ei, &ej, &valid);
        else sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
        double s = valid ? pair_stress(g, coords, i, j, ei, ej, &valid) : 0.0;
        if (pass == 1) {
          if (valid) { sum += s; ++n; } else { ++skipped; }
        } else if (valid) {
          dev += (s - mean) * (s - mean);
        }
      }
    }
    if (pass == 1) mean = n ? sum / (double)n : 0.0;
  }
  if (sp.zipf) free((void *)sp.zipf);
  double sd = n > 1 ? sqrt(dev / (double)(n - 1)) : 0.0;
  double half = n ? 1.96 * sd / sqrt((double)n) : 0.0;
  out[0] = mean; out[1] = mean - half; out[2] = mean + half; out[3] = sd; out[4] = sum; out[5] = dev;
  counts[0] = n; counts[1] = skipped;
}

/* ---------------------------------------------------------------------------
 * Eq. 2 in window-major order (reading R21): the same law of pairs as the
 * enumeration above (path p receives exactly m|p| pairs with i and j
 * independent and uniform in p and independent endpoint coins), listed
 * segment by segment.  The segments cut the global windows of 2^h steps (h
 * as for the layout's window-major order) at path boundaries, in step order.
 * Segment g receives n_g slots, the number of the pairs q of its path whose
 * step i (as sps_pair draws it) falls in the segment; slot u (slots numbered
 * consecutively over the segments) draws Philox stream 6 at counter u:
 * i = segment start + floor(u64 * segment length / 2^64), j = path start +
 * floor(r2 * |p| / 2^32), e_i = bit 0, e_j = bit 1 of r3.
 * ------------------------------------------------------------------------- */
enum { STREAM_SPS_SLOT = 6 };

/* The segments: start[0..n] (start[n] = S) and path[0..n-1]; returns n.  With
 * start = NULL only counts them. */
uint64_t or_sps_segments(const or_graph *g, uint64_t *start, uint32_t *path) {
  uint32_t sh = or_window_shift(g->S);
  uint64_t n = 0;
  for (uint32_t p = 0; p < g->n_paths; ++p) {
    uint64_t a = g->path_off[p], b = g->path_off[p + 1];
    while (a < b) {
      uint64_t e = ((a >> sh) + 1) << sh;  /* the next window boundary */
      if (e > b) e = b;
      if (start) { start[n] = a; path[n] = p; }
      ++n;
      a = e;
    }
  }
  if (start) start[n] = g->S;
  return n;
}

/* the segment holding step i: the largest g with start[g] <= i */
static uint64_t segment_of(const uint64_t *start, uint64_t n_seg, uint64_t i) {
  uint64_t lo = 0, hi = n_seg;
  while (hi - lo > 1) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (start[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

/* n_g of every segment (counts[0..n_seg-1]) */
void or_sps_segment_counts(const or_graph *g, uint32_t m, uint64_t seed, uint32_t graph_id, const uint64_t *start,
                           uint64_t n_seg, uint64_t *counts) {
  memset(counts, 0, sizeof(uint64_t) * n_seg);
  for (uint32_t p = 0; p < g->n_paths; ++p)
    for (uint64_t q = (uint64_t)m * g->path_off[p]; q < (uint64_t)m * g->path_off[p + 1]; ++q) {
      uint64_t i, j; uint32_t ei, ej;
      sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
      ++counts[segment_of(start, n_seg, i)];
    }
}

static void sps_slot(const or_graph *g, uint64_t seed, uint32_t graph_id, uint64_t seg_start, uint64_t seg_len,
                     uint32_t p, uint64_t u, uint64_t *i, uint64_t *j, uint32_t *ei, uint32_t *ej) {
  uint32_t r[4];
  draw(seed, u, 0, STREAM_SPS_SLOT, graph_id, r);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  *i = seg_start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), seg_len);
  *j = start + mulhi32(r[2], (uint32_t)len);
  *ei = r[3] & 1u;
  *ej = (r[3] >> 1) & 1u;
}

/* Lists the pairs of slots [u_begin, u_begin + count): i, j and e = e_i | e_j << 1. */
void or_sps_windowed_pairs(const or_graph *g, uint32_t m, uint64_t seed, uint32_t graph_id, uint64_t u_begin,
                           uint64_t count, uint64_t *i_out, uint64_t *j_out, uint8_t *e_out) {
  uint64_t n_seg = or_sps_segments(g, NULL, NULL);
  uint64_t *start = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
  uint32_t *path = (uint32_t *)malloc(sizeof(uint32_t) * (n_seg + 1));
  uint64_t *cnt = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
  or_sps_segments(g, start, path);
  or_sps_segment_counts(g, m, seed, graph_id, start, n_seg, cnt);
  uint64_t u = 0;
  for (uint64_t s = 0; s < n_seg; ++s)
    for (uint64_t k = 0; k < cnt[s]; ++k, ++u) {
      if (u < u_begin || u >= u_begin + count) continue;
      uint64_t i, j; uint32_t ei, ej;
      sps_slot(g, seed, graph_id, start[s], start[s + 1] - start[s], path[s], u, &i, &j, &ei, &ej);
      i_out[u - u_begin] = i;
      j_out[u - u_begin] = j;
      e_out[u - u_begin] = (uint8_t)(ei | (ej << 1));
    }
  free(start); free(path); free(cnt);
}

void or_sampled_path_stress_windowed(const or_graph *g, const float *coords, uint32_t m, uint64_t seed,
                                     uint32_t graph_id, double *out, uint64_t *counts) {
  uint64_t n_seg = or_sps_segments(g, NULL, NULL);
  uint64_t *start = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
  uint32_t *path = (uint32_t *)malloc(sizeof(uint32_t) * (n_seg + 1));
  uint64_t *cnt = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
  or_sps_segments(g, start, path);
  or_sps_segment_counts(g, m, seed, graph_id, start, n_seg, cnt);
  double sum = 0.0, dev = 0.0, mean = 0.0;
  uint64_t n = 0, skipped = 0;
  for (int pass = 1; pass <= 2; ++pass) {
    uint64_t u = 0;
    for (uint64_t s = 0; s < n_seg; ++s)
      for (uint64_t k = 0; k < cnt[s]; ++k, ++u) {
        uint64_t i, j; uint32_t ei, ej; int valid;
        sps_slot(g, seed, graph_id, start[s], start[s + 1] - start[s], path[s], u, &i, &j, &ei, &ej);
        double st = pair_stress(g, coords, i, j, ei, ej, &valid);
        if (pass == 1) {
          if (valid) { sum += st; ++n; } else { ++skipped; }
        } else if (valid) {
          dev += (st - mean) * (st - mean);
        }
      }
    if (pass == 1) mean = n ? sum / (double)n : 0.0;
  }
  free(start); free(path); free(cnt);
  double sd = n > 1 ? sqrt(dev / (double)(n - 1)) : 0.0;
  double half = n ? 1.96 * sd / sqrt((double)n) : 0.0;
  out[0] = mean; out[1] = mean - half; out[2] = mean + half; out[3] = sd; out[4] = sum; out[5] = dev;
  counts[0] = n; counts[1] = skipped;
}

void or_sampled_path_stress(const or_graph *g, const float *coords, uint32_t m, uint64_t seed, uint32_t graph_id,
                            double *out, uint64_t *counts) {
  double sum = 0.0;
  uint64_t n = 0, skipped = 0;
  for (uint32_t p = 0; p < g->n_paths; ++p) {
    for (uint64_t q = (uint64_t)m * g->path_off[p]; q < (uint64_t)m * g->path_off[p + 1]; ++q) {
      uint64_t i, j; uint32_t ei, ej; int valid;
      sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
      double s = pair_stress(g, coords, i, j, ei, ej, &valid);
      if (valid) { sum += s; ++n; } else { ++skipped; }
    }
  }
  double mean = n ? sum / (double)n : 0.0;
  double dev = 0.0;
  for (uint32_t p = 0; p < g->n_paths; ++p) {
    for (uint64_t q = (uint64_t)m * g->path_off[p]; q < (uint64_t)m * g->path_off[p + 1]; ++q) {
      uint64_t i, j; uint32_t ei, ej; int valid;
      sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
      double s = pair_stress(g, coords, i, j, ei, ej, &valid);
      if (valid) dev += (s - mean) * (s - mean);
    }
  }
  double sd = n > 1 ? sqrt(dev / (double)(n - 1)) : 0.0;
  double half = n ? 1.96 * sd / sqrt((double)n) : 0.0;
  out[0] = mean; out[1] = mean - half; out[2] = mean + half; out[3] = sd; out[4] = sum; out[5] = dev;
  counts[0] = n; counts[1] = skipped;
}

/* ---------------------------------------------------------------------------
 * Eq. 2 evaluated by several threads, for the stored results of large
 * layouts: exactly the pairs of or_sampled_path_stress (order 0, pair index q
 * over [0, m*S), path p holding q in [m*off[p], m*off[p+1])) or of
 * or_sampled_path_stress_windowed (order 1, slot index u over [0, m*S)).  The
 * index range is cut into one contiguous piece per thread; each thread sums
 * its piece in FP64 and the pieces are added in thread order, so only the
 * rounding of the sums differs from the one-thread evaluation (the pairs,
 * n_valid and n_skipped are the same).
 * ------------------------------------------------------------------------- */
typedef struct {
  const or_graph *g; const float *coords; uint32_t m, graph_id, order; uint64_t seed;
  uint64_t b, e;                                       /* index range of this thread */
  const uint64_t *seg_start; const uint32_t *seg_path; /* order 1: segments */
  const uint64_t *seg_off; uint64_t n_seg;             /* order 1: first slot of every segment */
  uint64_t *hist;                                      /* order 1, counting: per-segment counts */
  int pass; double mean;
  double sum, dev; uint64_t n, skipped;
} sps_job;

/* the pair of index k in the job's order */
static void sps_job_pair(const sps_job *jb, uint64_t k, uint64_t *seg_hint, uint64_t *i, uint64_t *j, uint32_t *ei,
                         uint32_t *ej) {
  const or_graph *g = jb->g;
  if (jb->order == 0) {
    uint32_t p = path_of_step(g, k / jb->m);
    sps_pair(g, jb->seed, jb->graph_id, p, k, i, j, ei, ej);
    return;
  }
  uint64_t s = *seg_hint;
  while (s + 1 < jb->n_seg && jb->seg_off[s + 1] <= k) ++s;
  *seg_hint = s;
  sps_slot(g, jb->seed, jb->graph_id, jb->seg_start[s], jb->seg_start[s + 1] - jb->seg_start[s], jb->seg_path[s], k,
           i, j, ei, ej);
}

static void *sps_count_worker(void *arg) {
  sps_job *jb = (sps_job *)arg;
  memset(jb->hist, 0, sizeof(uint64_t) * jb->n_seg);
  for (uint64_t q = jb->b; q < jb->e; ++q) {
    uint64_t i, j; uint32_t ei, ej;
    sps_pair(jb->g, jb->seed, jb->graph_id, path_of_step(jb->g, q / jb->m), q, &i, &j, &ei, &ej);
    ++jb->hist[segment_of(jb->seg_start, jb->n_seg, i)];
  }
  return NULL;
}

static void *sps_sum_worker(void *arg) {
  sps_job *jb = (sps_job *)arg;
  uint64_t seg = 0;
  if (jb->order == 1 && jb->b < jb->e) {  /* the segment holding slot b: the largest s with seg_off[s] <= b */
    uint64_t lo = 0, hi = jb->n_seg;
    while (hi - lo > 1) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (jb->seg_off[mid] <= jb->b) lo = mid; else hi = mid;
    }
    seg = lo;
  }
  for (uint64_t k = jb->b; k < jb->e; ++k) {
    uint64_t i, j; uint32_t ei, ej; int valid;
    sps_job_pair(jb, k, &seg, &i, &j, &ei, &ej);
    double s = pair_stress(jb->g, jb->coords, i, j, ei, ej, &valid);
    if (jb->pass == 1) {
      if (valid) { jb->sum += s; ++jb->n; } else { ++jb->skipped; }
    } else if (valid) {
      jb->dev += (s - jb->mean) * (s - jb->mean);
    }
  }
  return NULL;
}

static void sps_run(sps_job *jobs, uint32_t threads, void *(*fn)(void *)) {
  pthread_t *tid = (pthread_t *)calloc(threads, sizeof(pthread_t));
  for (uint32_t k = 0; k < threads; ++k) pthread_create(&tid[k], NULL, fn, &jobs[k]);
  for (uint32_t k = 0; k < threads; ++k) pthread_join(tid[k], NULL);
  free(tid);
}

void or_sampled_path_stress_threaded(const or_graph *g, const float *coords, uint32_t m, uint64_t seed,
                                     uint32_t graph_id, uint32_t order, uint32_t threads, double *out,
                                     uint64_t *counts) {
  if (threads < 1) threads = 1;
  uint64_t total = (uint64_t)m * g->S, n_seg = 0;
  uint64_t *seg_start = NULL, *seg_off = NULL;
  uint32_t *seg_path = NULL;
  sps_job *jobs = (sps_job *)calloc(threads, sizeof(sps_job));
  for (uint32_t k = 0; k < threads; ++k) {
    jobs[k].g = g; jobs[k].coords = coords; jobs[k].m = m; jobs[k].graph_id = graph_id; jobs[k].order = order;
    jobs[k].seed = seed; jobs[k].b = total * k / threads; jobs[k].e = total * (k + 1) / threads;
  }
  if (order == 1) {
    n_seg = or_sps_segments(g, NULL, NULL);
    seg_start = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
    seg_path = (uint32_t *)malloc(sizeof(uint32_t) * (n_seg + 1));
    seg_off = (uint64_t *)calloc(n_seg + 1, sizeof(uint64_t));
    or_sps_segments(g, seg_start, seg_path);
    for (uint32_t k = 0; k < threads; ++k) {
      jobs[k].seg_start = seg_start; jobs[k].seg_path = seg_path; jobs[k].n_seg = n_seg;
      jobs[k].hist = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg ? n_seg : 1));
    }
    sps_run(jobs, threads, sps_count_worker);
    for (uint32_t k = 0; k < threads; ++k) {  /* seg_off = exclusive prefix of the summed counts */
      for (uint64_t s = 0; s < n_seg; ++s) seg_off[s + 1] += jobs[k].hist[s];
      free(jobs[k].hist);
      jobs[k].hist = NULL;
    }
    for (uint64_t s = 0; s < n_seg; ++s) seg_off[s + 1] += seg_off[s];
    for (uint32_t k = 0; k < threads; ++k) jobs[k].seg_off = seg_off;
  }
  double sum = 0.0, dev = 0.0, mean;
  uint64_t n = 0, skipped = 0;
  for (uint32_t k = 0; k < threads; ++k) jobs[k].pass = 1;
  sps_run(jobs, threads, sps_sum_worker);
  for (uint32_t k = 0; k < threads; ++k) { sum += jobs[k].sum; n += jobs[k].n; skipped += jobs[k].skipped; }
  mean = n ? sum / (double)n : 0.0;
  for (uint32_t k = 0; k < threads; ++k) { jobs[k].pass = 2; jobs[k].mean = mean; }
  sps_run(jobs, threads, sps_sum_worker);
  for (uint32_t k = 0; k < threads; ++k) dev += jobs[k].dev;
  free(jobs); free(seg_start); free(seg_path); free(seg_off);
  double sd = n > 1 ? sqrt(dev / (double)(n - 1)) : 0.0;
  double half = n ? 1.96 * sd / sqrt((double)n) : 0.0;
  out[0] = mean; out[1] = mean - half; out[2] = mean + half; out[3] = sd; out[4] = sum; out[5] = dev;
  counts[0] = n; counts[1] = skipped;
}

/* The exact expectation of one pass of the sampled estimator: every
 * (i, j, e_i, e_j) of path p has probability 1/(4|p|^2) per pair and path p
 * receives m|p| of the m*S pairs, so E[sum] / E[n] enumerates all of them
 * weighted by 1/(4|p|).  out[0] = E[sum s]/E[n] (the ratio the pooled mean
 * converges to), out[1] = E[n] / (m*S). */
void or_sps_expectation(const or_graph *g, const float *coords, double *out) {
  double num = 0.0, den = 0.0;
  for (uint32_t p = 0; p < g->n_paths; ++p) {
    uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
    if (len == 0) continue;
    double w = 1.0 / (4.0 * (double)len);
    for (uint64_t i = start; i < start + len; ++i)
      for (uint64_t j = start; j < start + len; ++j)
        for (uint32_t e = 0; e < 4; ++e) {
          int valid;
          double s = pair_stress(g, coords, i, j, e & 1u, e >> 1, &valid);
          if (valid) { num += w * s; den += w; }
        }
  }
  out[0] = den > 0 ? num / den : 0.0;
  out[1] = g->S ? den / (double)g->S : 0.0;
}

/* Path stress, Eq. 1: the mean over all unordered step pairs i < j of the
 * same path of the stress averaged over the four endpoint combinations
 * (combinations with d = 0 are left out of that average; a pair whose four
 * combinations all have d = 0 is left out).  out[0] = path stress, out[1] =
 * number of pairs. */
void or_path_stress_exact(const or_graph *g, const float *coords, double *out) {
  double sum = 0.0;
  uint64_t pairs = 0;
  for (uint32_t p = 0; p < g->n_paths; ++p) {
    for (uint64_t i = g->path_off[p]; i < g->path_off[p + 1]; ++i)
      for (uint64_t j = i + 1; j < g->path_off[p + 1]; ++j) {
        double acc = 0.0;
        int nv = 0;
        for (uint32_t e = 0; e < 4; ++e) {
          int valid;
          double s = pair_stress(g, coords, i, j, e & 1u, e >> 1, &valid);
          if (valid) { acc += s; ++nv; }
        }
        if (nv) { sum += acc / nv; ++pairs; }
      }
  }
  out[0] = pairs ? sum / (double)pairs : 0.0;
  out[1] = (double)pairs;
}

/* ---------------------------------------------------------------------------
 * Initial layout (the paper is silent; it is not part of any parity claim):
 * node n starts on the x axis at the path coordinate of its first visit
 * (paths scanned in order), X[2n] = pos, X[2n+1] = pos + len; never-visited
 * nodes start at 0.  Y[2n+e] = jitter * (u - 1/2) with u = (r0 >> 8) / 2^24
 * from Philox stream 3 at counter 2n+e.
 * ------------------------------------------------------------------------- */
void or_init_coords(const or_graph *g, uint64_t seed, uint32_t graph_id, float jitter, float *coords) {
  float *X = coords, *Y = coords + 2ull * g->n_nodes;
  uint8_t *seen = (uint8_t *)calloc(g->n_nodes ? g->n_nodes : 1, 1);
  for (uint32_t n = 0; n < g->n_nodes; ++n) { X[2ull * n] = 0.0f; X[2ull * n + 1] = 0.0f; }
  for (uint64_t s = 0; s < g->S; ++s) {
    uint32_t n = step_node_id(g, s);
    if (seen[n]) continue;
    seen[n] = 1;
    X[2ull * n] = (float)g->pos[s];
    X[2ull * n + 1] = (float)(g->pos[s] + (int64_t)g->node_len[n]);
  }
  free(seen);
  for (uint64_t k = 0; k < 2ull * g->n_nodes; ++k) {
    uint32_t r[4];
    draw(seed, k, 0, STREAM_INIT, graph_id, r);
    float u = (float)(r[0] >> 8) * (1.0f / 16777216.0f);
    Y[k] = jitter * (u - 0.5f);
  }
}

/* ---------------------------------------------------------------------------
 * Differentiable form: the sampled stress as a loss over n_pairs power-law
 * pairs (the cooling sampler, Philox stream 2, counter word 2 = optimiser
 * step).  L = (1/n_valid) sum ((mag - d)/d)^2; dL/dv_a = (2/n_valid)
 * (mag - d)/d^2 * (v_a - v_b)/mag and dL/dv_b = -dL/dv_a (zero when mag = 0).
 * Pairs skipped by R8 do not count.  grad (FP64, boundary layout) is
 * overwritten.  out[0] = L, out[1] = n_valid.
 * ------------------------------------------------------------------------- */
static int pair_power_law(const or_graph *g, const sampler *sp, uint32_t step, uint64_t q, uint64_t *a, uint64_t *b,
                          double *d) {
  uint32_t r[4];
  draw(sp->seed, q, step, STREAM_PAIRS, sp->graph_id, r);
  uint64_t i = mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), g->S);
  uint32_t p = path_of_step(g, i);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start, j;
  int skip = 0;
  partner_power_law(g, sp, i, start, len, r[2], r[3], &j, &skip);
  if (skip) return 0;
  uint32_t ei = r[3] & 1u, ej = (r[3] >> 1) & 1u;
  *a = 2ull * step_node_id(g, i) + ei;
  *b = 2ull * step_node_id(g, j) + ej;
  int64_t dd = or_endpoint_pos(g, i, ei) - or_endpoint_pos(g, j, ej);
  if (*a == *b || dd == 0) return 0;
  *d = (double)(dd < 0 ? -dd : dd);
  return 1;
}

void or_stress_loss_grad(const or_graph *g, const float *coords, uint64_t n_pairs, double theta, uint32_t W,
                         uint64_t seed, uint32_t graph_id, uint32_t step, double *out, double *grad) {
  sampler sp;
  make_sampler(&sp, 2, theta, W, seed, graph_id);
  const float *X = coords, *Y = coords + 2ull * g->n_nodes;
  double sum = 0.0;
  uint64_t n = 0;
  for (uint64_t q = 0; q < n_pairs; ++q) {
    uint64_t a, b; double d;
    if (!pair_power_law(g, &sp, step, q, &a, &b, &d)) continue;
    double dx = (double)X[a] - (double)X[b], dy = (double)Y[a] - (double)Y[b];
    double mag = sqrt(dx * dx + dy * dy);
    double e = (mag - d) / d;
    sum += e * e;
    ++n;
  }
  out[0] = n ? sum / (double)n : 0.0;
  out[1] = (double)n;
  if (grad) {
    double *GX = grad, *GY = grad + 2ull * g->n_nodes;
    memset(grad, 0, sizeof(double) * 4ull * g->n_nodes);
    for (uint64_t q = 0; q < n_pairs && n > 0; ++q) {
      uint64_t a, b; double d;
      if (!pair_power_law(g, &sp, step, q, &a, &b, &d)) continue;
      double dx = (double)X[a] - (double)X[b], dy = (double)Y[a] - (double)Y[b];
      double mag = sqrt(dx * dx + dy * dy);
      if (mag == 0.0) continue;
      double c = 2.0 / (double)n * (mag - d) / (d * d) / mag;
      GX[a] += c * dx; GY[a] += c * dy;
      GX[b] -= c * dx; GY[b] -= c * dy;
    }
  }
  free((void *)sp.zipf);
}

/* ---------------------------------------------------------------------------
 * The differentiable loss with its pairs in window-major order (reading R22):
 * the law of pairs of or_stress_loss_grad (n_pairs pairs; i uniform over all
 * steps; j the power-law partner of i in its path; independent endpoint
 * coins), listed segment by segment over the loss's own segments: the windows
 * of 2^h steps cut at path boundaries, in step order, with h = or_loss_shift(S)
 * (the rule of or_window_shift started from 2^10 steps instead of 2^14, so the
 * segments are shorter than R21's where the graph allows).  Segment g receives n_g
 * slots, the number of the loss's own pairs q < n_pairs whose step i falls in
 * it; slot u (numbered over the segments in order) draws Philox stream 7 at
 * counter u with word 2 = the optimiser step: i = segment start +
 * floor(u64 * segment length / 2^64), j = the power-law partner of i from
 * words 2 and 3 (as the cooling phase draws it), e_i = bit 0 and e_j = bit 1
 * of word 3.  Multinomial counts of uniform steps per segment followed by a
 * uniform step inside the segment are n_pairs independent uniform steps, and
 * each slot's partner and coins are drawn afresh, so the pairs follow the
 * same law.  Loss and gradient as in or_stress_loss_grad.
 * ------------------------------------------------------------------------- */
enum { STREAM_LOSS_SLOT = 7 };

/* Window shift of the loss's segments: windows of 2^10 steps, halved while
 * there are fewer than 16 (down to 2^6), doubled while there are more than
 * 32768. */
uint32_t or_loss_shift(uint64_t S) {
  uint32_t sh = 10;
  while (sh > 6 && ((S + (1ull << sh) - 1) >> sh) < 16) --sh;
  while (((S + (1ull << sh) - 1) >> sh) > 32768) ++sh;
  return sh;
}

/* The loss's segments: start[0..n] (start[n] = S) and path[0..n-1]; returns n.
 * With start = NULL only counts them. */
uint64_t or_loss_segments(const or_graph *g, uint64_t *start, uint32_t *path) {
  uint32_t sh = or_loss_shift(g->S);
  uint64_t n = 0;
  for (uint32_t p = 0; p < g->n_paths; ++p)
    for (uint64_t a = g->path_off[p], b = g->path_off[p + 1]; a < b; ++n) {
      uint64_t e = ((a >> sh) + 1) << sh;
      if (e > b) e = b;
      if (start) { start[n] = a; path[n] = p; }
      a = e;
    }
  if (start) start[n] = g->S;
  return n;
}

/* n_g of every segment for the loss's pairs of optimiser step `step` */
void or_loss_segment_counts(const or_graph *g, uint64_t n_pairs, uint64_t seed, uint32_t graph_id, uint32_t step,
                            const uint64_t *start, uint64_t n_seg, uint64_t *counts) {
  memset(counts, 0, sizeof(uint64_t) * n_seg);
  for (uint64_t q = 0; q < n_pairs; ++q) {
    uint32_t r[4];
    draw(seed, q, step, STREAM_PAIRS, graph_id, r);
    uint64_t i = mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), g->S);
    ++counts[segment_of(start, n_seg, i)];
  }
}

/* Slot u of segment [seg_start, seg_start + seg_len) of path p.  Returns 0 when
 * the pair is skipped (no partner, the same endpoint slot, or d = 0). */
static int loss_slot(const or_graph *g, const sampler *sp, uint32_t step, uint64_t u, uint64_t seg_start,
                     uint64_t seg_len, uint32_t p, uint64_t *i, uint64_t *j, uint32_t *ei, uint32_t *ej,
                     uint64_t *a, uint64_t *b, double *d) {
  uint32_t r[4];
  draw(sp->seed, u, step, STREAM_LOSS_SLOT, sp->graph_id, r);
  *i = seg_start + mulhi64((uint64_t)r[0] | ((uint64_t)r[1] << 32), seg_len);
  uint64_t start = g->path_off[p], len = g->path_off[p + 1] - start;
  int skip = 0;
  partner_power_law(g, sp, *i, start, len, r[2], r[3], j, &skip);
  *ei = r[3] & 1u;
  *ej = (r[3] >> 1) & 1u;
  if (skip) return 0;
  *a = 2ull * step_node_id(g, *i) + *ei;
  *b = 2ull * step_node_id(g, *j) + *ej;
  int64_t dd = or_endpoint_pos(g, *i, *ei) - or_endpoint_pos(g, *j, *ej);
  if (*a == *b || dd == 0) return 0;
  *d = (double)(dd < 0 ? -dd : dd);
  return 1;
}

typedef struct {
  uint64_t n_seg;
  uint64_t *start, *cnt;
  uint32_t *path;
} loss_segments;

static void loss_segments_make(const or_graph *g, uint64_t n_pairs, uint64_t seed, uint32_t graph_id, uint32_t step,
                               loss_segments *ls) {
  ls->n_seg = or_loss_segments(g, NULL, NULL);
  ls->start = (uint64_t *)malloc(sizeof(uint64_t) * (ls->n_seg + 1));
  ls->path = (uint32_t *)malloc(sizeof(uint32_t) * (ls->n_seg + 1));
  ls->cnt = (uint64_t *)malloc(sizeof(uint64_t) * (ls->n_seg + 1));
  or_loss_segments(g, ls->start, ls->path);
  or_loss_segment_counts(g, n_pairs, seed, graph_id, step, ls->start, ls->n_seg, ls->cnt);
}

static void loss_segments_free(loss_segments *ls) {
  free(ls->start); free(ls->path); free(ls->cnt);
}

/* The slots [u_begin, u_begin + count): i, j and flags e_i | e_j << 1 | skipped << 3. */
void or_loss_windowed_pairs(const or_graph *g, uint64_t n_pairs, double theta, uint32_t W, uint64_t seed,
                            uint32_t graph_id, uint32_t step, uint64_t u_begin, uint64_t count, uint64_t *i_out,
                            uint64_t *j_out, uint8_t *f_out) {
  sampler sp;
  make_sampler(&sp, 2, theta, W, seed, graph_id);
  loss_segments ls;
  loss_segments_make(g, n_pairs, seed, graph_id, step, &ls);
  uint64_t u = 0;
  for (uint64_t s = 0; s < ls.n_seg && u < u_begin + count; ++s)
    for (uint64_t k = 0; k < ls.cnt[s]; ++k, ++u) {
      if (u < u_begin || u >= u_begin + count) continue;
      uint64_t i, j = 0, a, b; uint32_t ei, ej; double d;
      int ok = loss_slot(g, &sp, step, u, ls.start[s], ls.start[s + 1] - ls.start[s], ls.path[s], &i, &j, &ei,
                         &ej, &a, &b, &d);
      i_out[u - u_begin] = i;
      j_out[u - u_begin] = j;
      f_out[u - u_begin] = (uint8_t)(ei | (ej << 1) | (ok ? 0u : 8u));
    }
  loss_segments_free(&ls);
  free((void *)sp.zipf);
}

void or_stress_loss_grad_windowed(const or_graph *g, const float *coords, uint64_t n_pairs, double theta, uint32_t W,
                                  uint64_t seed, uint32_t graph_id, uint32_t step, double *out, double *grad) {
  sampler sp;
  make_sampler(&sp, 2, theta, W, seed, graph_id);
  loss_segments ls;
  loss_segments_make(g, n_pairs, seed, graph_id, step, &ls);
  const float *X = coords, *Y = coords + 2ull * g->n_nodes;
  double sum = 0.0;
  uint64_t n = 0;
  for (int pass = 1; pass <= 2; ++pass) {
    if (pass == 2) {
      if (!grad) break;
      memset(grad, 0, sizeof(double) * 4ull * g->n_nodes);
      if (n == 0) break;
    }
    double *GX = grad, *GY = grad ? grad + 2ull * g->n_nodes : NULL;
    uint64_t u = 0;
    for (uint64_t s = 0; s < ls.n_seg; ++s)
      for (uint64_t k = 0; k < ls.cnt[s]; ++k, ++u) {
        uint64_t i, j, a, b; uint32_t ei, ej; double d;
        if (!loss_slot(g, &sp, step, u, ls.start[s], ls.start[s + 1] - ls.start[s], ls.path[s], &i, &j, &ei, &ej,
                       &a, &b, &d))
          continue;
        double dx = (double)X[a] - (double)X[b], dy = (double)Y[a] - (double)Y[b];
        double mag = sqrt(dx * dx + dy * dy);
        if (pass == 1) {
          double e = (mag - d) / d;
          sum += e * e;
          ++n;
        } else if (mag != 0.0) {
          double c = 2.0 / (double)n * (mag - d) / (d * d) / mag;
          GX[a] += c * dx; GY[a] += c * dy;
          GX[b] -= c * dx; GY[b] -= c * dy;
        }
      }
  }
  out[0] = n ? sum / (double)n : 0.0;
  out[1] = (double)n;
  loss_segments_free(&ls);
  free((void *)sp.zipf);
}

/* ---------------------------------------------------------------------------
 * The pairs of Eq. 2 whose stress exceeds a threshold (for finding the pairs
 * behind a heavy-tailed estimate): the pairs of the given mode (0 uniform,
 * 1 power-law partner, 2 uniform in window-major order) in enumeration order;
 * the first max_out are written (i, j, e = e_i | e_j << 1, stress); returns
 * how many exceed the threshold.
 * ------------------------------------------------------------------------- */
uint64_t or_sps_outliers(const or_graph *g, const float *coords, uint32_t m, uint64_t seed, uint32_t graph_id,
                         uint32_t mode, double theta, uint32_t W, double threshold, uint64_t max_out,
                         uint64_t *i_out, uint64_t *j_out, uint8_t *e_out, double *s_out) {
  uint64_t n_out = 0;
  sampler sp;
  sp.zipf = NULL;
  if (mode == 1) make_sampler(&sp, 1, theta, W, seed, graph_id);
#define OR_KEEP(I, J, EI, EJ, S)                            \
  do {                                                      \
    if ((S) > threshold) {                                  \
      if (n_out < max_out) {                                \
        i_out[n_out] = (I); j_out[n_out] = (J);             \
        e_out[n_out] = (uint8_t)((EI) | ((EJ) << 1));       \
        s_out[n_out] = (S);                                 \
      }                                                     \
      ++n_out;                                              \
    }                                                       \
  } while (0)
  if (mode == 2) {
    uint64_t n_seg = or_sps_segments(g, NULL, NULL);
    uint64_t *start = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
    uint32_t *path = (uint32_t *)malloc(sizeof(uint32_t) * (n_seg + 1));
    uint64_t *cnt = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
    or_sps_segments(g, start, path);
    or_sps_segment_counts(g, m, seed, graph_id, start, n_seg, cnt);
    uint64_t u = 0;
    for (uint64_t s = 0; s < n_seg; ++s)
      for (uint64_t k = 0; k < cnt[s]; ++k, ++u) {
        uint64_t i, j; uint32_t ei, ej; int valid;
        sps_slot(g, seed, graph_id, start[s], start[s + 1] - start[s], path[s], u, &i, &j, &ei, &ej);
        double st = pair_stress(g, coords, i, j, ei, ej, &valid);
        if (valid) OR_KEEP(i, j, ei, ej, st);
      }
    free(start); free(path); free(cnt);
  } else {
    for (uint32_t p = 0; p < g->n_paths; ++p)
      for (uint64_t q = (uint64_t)m * g->path_off[p]; q < (uint64_t)m * g->path_off[p + 1]; ++q) {
        uint64_t i, j; uint32_t ei, ej; int valid = 1;
        if (mode == 1) sps_pair_power_law(g, &sp, p, q, &i, &j, &ei, &ej, &valid);
        else sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
        double st = valid ? pair_stress(g, coords, i, j, ei, ej, &valid) : 0.0;
        if (valid) OR_KEEP(i, j, ei, ej, st);
      }
  }
#undef OR_KEEP
  if (sp.zipf) free((void *)sp.zipf);
  return n_out;
}

/* ---------------------------------------------------------------------------
 * Two layouts compared on the same pairs of Eq. 2 (a paired estimate): for
 * every valid pair the stress s_a in layout a and s_b in layout b.  Pass 1
 * gives the means; pass 2 the spreads and sum (s_a - R s_b)^2 with R =
 * sum s_a / sum s_b.  The ratio's 95% interval is the delta-method one,
 * R +- 1.96 sqrt(sum (s_a - R s_b)^2 / (n - 1)) / (sqrt(n) mean_b).
 * out: mean_a, mean_b, R, R_lo, R_hi, sd_a, sd_b, sd of s_a - R s_b, sum_a,
 * sum_b; counts: n_valid, n_skipped.  Modes as or_sps_outliers.
 * ------------------------------------------------------------------------- */
void or_sps_compare(const or_graph *g, const float *coords_a, const float *coords_b, uint32_t m, uint64_t seed,
                    uint32_t graph_id, uint32_t mode, double theta, uint32_t W, double *out, uint64_t *counts) {
  sampler sp;
  sp.zipf = NULL;
  if (mode == 1) make_sampler(&sp, 1, theta, W, seed, graph_id);
  uint64_t n_seg = 0, *start = NULL, *cnt = NULL;
  uint32_t *path = NULL;
  if (mode == 2) {
    n_seg = or_sps_segments(g, NULL, NULL);
    start = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
    path = (uint32_t *)malloc(sizeof(uint32_t) * (n_seg + 1));
    cnt = (uint64_t *)malloc(sizeof(uint64_t) * (n_seg + 1));
    or_sps_segments(g, start, path);
    or_sps_segment_counts(g, m, seed, graph_id, start, n_seg, cnt);
  }
  double sa = 0.0, sb = 0.0, da = 0.0, db = 0.0, dr = 0.0, ma = 0.0, mb = 0.0, R = 0.0;
  uint64_t n = 0, skipped = 0;
  for (int pass = 1; pass <= 2; ++pass) {
    uint64_t u = 0;
    uint32_t p = 0;
    uint64_t q = 0, seg = 0, k = 0;
    for (;;) {  /* the pairs of the mode, in enumeration order */
      uint64_t i, j; uint32_t ei, ej; int valid = 1;
      if (mode == 2) {
        while (seg < n_seg && k >= cnt[seg]) { ++seg; k = 0; }
        if (seg >= n_seg) break;
        sps_slot(g, seed, graph_id, start[seg], start[seg + 1] - start[seg], path[seg], u, &i, &j, &ei, &ej);
        ++u; ++k;
      } else {
        while (p < g->n_paths && q >= (uint64_t)m * g->path_off[p + 1]) ++p;
        if (p >= g->n_paths) break;
        if (q < (uint64_t)m * g->path_off[p]) q = (uint64_t)m * g->path_off[p];
        if (mode == 1) sps_pair_power_law(g, &sp, p, q, &i, &j, &ei, &ej, &valid);
        else sps_pair(g, seed, graph_id, p, q, &i, &j, &ei, &ej);
        ++q;
      }
      int va = valid, vb = valid;
      double s_a = va ? pair_stress(g, coords_a, i, j, ei, ej, &va) : 0.0;
      double s_b = vb ? pair_stress(g, coords_b, i, j, ei, ej, &vb) : 0.0;
      if (!va) {
        if (pass == 1) ++skipped;
        continue;
      }
      if (pass == 1) {
        sa += s_a; sb += s_b; ++n;
      } else {
        da += (s_a - ma) * (s_a - ma);
        db += (s_b - mb) * (s_b - mb);
        dr += (s_a - R * s_b) * (s_a - R * s_b);
      }
    }
    if (pass == 1) {
      ma = n ? sa / (double)n : 0.0;
      mb = n ? sb / (double)n : 0.0;
      R = sb > 0.0 ? sa / sb : 0.0;
    }
  }
  if (start) { free(start); free(path); free(cnt); }
  if (sp.zipf) free((void *)sp.zipf);
  double sdr = n > 1 ? sqrt(dr / (double)(n - 1)) : 0.0;
  double half = (n && mb > 0.0) ? 1.96 * sdr / (sqrt((double)n) * mb) : 0.0;
  out[0] = ma; out[1] = mb; out[2] = R; out[3] = R - half; out[4] = R + half;
  out[5] = n > 1 ? sqrt(da / (double)(n - 1)) : 0.0;
  out[6] = n > 1 ? sqrt(db / (double)(n - 1)) : 0.0;
  out[7] = sdr; out[8] = sa; out[9] = sb;
  counts[0] = n; counts[1] = skipped;
}
