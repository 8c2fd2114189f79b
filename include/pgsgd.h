/*
 * pgsgd.h — C ABI of the MI355X (gfx950) PG-SGD pangenome graph layout library.
 *
 * The library computes the path-guided SGD layout of a variation graph
 * ("Rapid GPU-Based Pangenome Graph Layout", SC24, Alg. 1 in Section
 * "Path-Guided SGD Algorithm") and its quality metric, the sampled path stress
 * (Eq. 2 and its 95% confidence interval, Section "A Scalable Metric: Sampled
 * Path Stress").  Only the paths and the node lengths of the graph enter the
 * layout (Alg. 1 reads P and L; the lean structure of Section "CUDA Kernel for
 * Pangenome Graph Layout" keeps node lengths only), so edges are not part of
 * this interface.
 *
 * Conventions used by every entry point:
 *   - Every call returns a pgsgd_status; nothing throws across the ABI.  On an
 *     error, pgsgd_last_error() returns a message for the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *     memory on the graph's device (for example torch tensor data_ptr()).
 *   - Coordinates use the layout [2][n_nodes][2] in float32: the X plane, then
 *     the Y plane; endpoint e (0 = start, 1 = end) of node n is element 2n+e of
 *     a plane.  Coordinate buffers are owned by the caller, must be contiguous
 *     and 16-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     enqueued asynchronously on it unless a function says it synchronises.
 *   - One graph handle must not be used from two streams at the same time.
 *   - All argument validation happens on the host before any device work, so
 *     every validation error is reported without touching the GPU.
 *
 * Random choices follow a counter-based definition (Philox4x32-10, Salmon et
 * al., SC'11): draw = Philox(counter = (t mod 2^32, t >> 32, word2,
 * stream << 24 | graph_id), key = (seed mod 2^32, seed >> 32)), with stream 0
 * for layout terms (word2 = iteration), 1 for sampled-path-stress pairs
 * (word2 = 0), 2 for differentiable-loss pairs (word2 = optimiser step) and 3
 * for the initial layout jitter.  Results therefore do not depend on the launch
 * configuration, and a run split into iteration ranges samples exactly the
 * same terms as one full run.
 */
#ifndef PGSGD_H
#define PGSGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pgsgd_status;
enum {
  PGSGD_OK = 0,
  PGSGD_ERR_INVALID_ARG = -1, /* null pointer, malformed graph, bad parameter */
  PGSGD_ERR_RANGE = -2,       /* a size beyond what the library supports */
  PGSGD_ERR_OOM = -3,         /* device or host allocation failed */
  PGSGD_ERR_DEVICE = -4,      /* a HIP runtime error (no device, launch failure, ...) */
  PGSGD_ERR_UNSUPPORTED = -5  /* a valid request this build does not implement */
};

/* Message of the last failing call on this thread ("" if none).  The pointer
 * stays valid until the next call on this thread. */
const char *pgsgd_last_error(void);
const char *pgsgd_version(void);

/* ------------------------------------------------------------------------- */
/* Graph                                                                      */
/* ------------------------------------------------------------------------- */
typedef struct pgsgd_graph pgsgd_graph;

typedef struct {
  uint64_t n_steps;       /* S = total path steps (sum over paths of |p|) */
  uint32_t n_nodes;
  uint32_t n_paths;
  int64_t d_max;          /* longest path, in nucleotides */
  uint64_t device_bytes;  /* device memory held by the handle */
  int32_t device;
  uint32_t max_path_steps;
  uint32_t renumbered;    /* 1 if the device keeps the nodes in the path-guided order (see pgsgd_graph_create_ex) */
} pgsgd_graph_info;

/*
 * Copies a variation graph to the device.
 *   n_nodes       number of nodes, < 2^31
 *   node_len      host, n_nodes entries: nucleotide length of each node, >= 1
 *   n_paths       number of paths, >= 1 and <= 2^20 (kernels stage the path
 *                 offsets in LDS: a launch returns UNSUPPORTED when they do not
 *                 fit the per-block LDS limit, about 3,500 paths on gfx950)
 *   path_offsets  host, n_paths+1 entries: CSR offsets of each path's steps in
 *                 step_node; [0] = 0, non-decreasing; S = path_offsets[n_paths]
 *                 < 2^40 and every path has fewer than 2^32 steps.  Empty paths
 *                 are allowed (they are never sampled).
 *   step_node     host, S entries: node id of each step, bit 31 set for a
 *                 reverse-strand visit
 *   step_pos      host or NULL: nucleotide offset of each step from the start
 *                 of its path.  NULL means "compute it": the sum of the lengths
 *                 of the earlier steps of the path.  If given it must equal
 *                 those sums (PGSGD_ERR_INVALID_ARG otherwise).
 *   device        HIP device ordinal
 *   out           receives the handle (NULL on error)
 * The host arrays are copied; the caller may free them once the call returns.
 * Device memory: 16 B per step (records), 24 B per node (first visit and the
 * interleaved working copy of the coordinates), the path offsets, the
 * power-law table (about 258 KB) and reduction scratch (about 49 KB); the
 * windowed schedule and the window-major sampled path stress add a few words
 * per window on first use.  If the environment variable
 * PGSGD_MAX_DEVICE_BYTES holds a positive decimal number, no graph handle may
 * hold more device memory than that: a creation that would need more fails
 * with OOM before any device work, as does any later allocation of the handle.
 * Errors: INVALID_ARG (null pointer, node id >= n_nodes, length 0, offsets not
 * monotone, step_pos mismatch, n_paths = 0), RANGE (sizes above the limits,
 * a path longer than 2^62 nt), OOM, DEVICE.  Synchronous.
 * Equal to pgsgd_graph_create_ex(..., PGSGD_RENUMBER_AUTO, out).
 */
pgsgd_status pgsgd_graph_create(uint32_t n_nodes, const uint32_t *node_len, uint32_t n_paths,
                                const uint64_t *path_offsets, const uint32_t *step_node, const int64_t *step_pos,
                                int device, pgsgd_graph **out);

/*
 * pgsgd_graph_create with a choice of the node order kept on the device.  The
 * windowed schedule gets its locality from nodes that lie close along the
 * paths having close ids (their coordinates then share cache lines; the
 * cache-friendly data layout of Section "Cache-friendly Data Layout" makes the
 * same point).  Graphs sorted along their paths (as pangenome tools emit them)
 * already have that order; for others the library can renumber the nodes into
 * the path-guided order of pgsgd_path_order.  Renumbering is invisible to the
 * caller: coordinates, gradients and node ids at the interface stay in the
 * caller's order, the sampled terms (steps i, j) and the initial layout are
 * the same, and a one-wave layout gives the same coordinates bit for bit; the
 * device holds 4 more bytes per node and the permutes in and out gather and
 * scatter through it.
 *   renumber  PGSGD_RENUMBER_AUTO: renumber when more than 20% of the
 *             consecutive steps of the paths jump more than 32 ids and the
 *             path-guided order at least halves that fraction;
 *             PGSGD_RENUMBER_NEVER; PGSGD_RENUMBER_ALWAYS.  Other values:
 *             INVALID_ARG.
 */
enum { PGSGD_RENUMBER_AUTO = 0, PGSGD_RENUMBER_NEVER = 1, PGSGD_RENUMBER_ALWAYS = 2 };
pgsgd_status pgsgd_graph_create_ex(uint32_t n_nodes, const uint32_t *node_len, uint32_t n_paths,
                                   const uint64_t *path_offsets, const uint32_t *step_node, const int64_t *step_pos,
                                   int device, uint32_t renumber, pgsgd_graph **out);
/* The device node id of every caller node id (host, n_nodes entries; the
 * identity when the graph is not renumbered).  Errors: INVALID_ARG on NULL. */
pgsgd_status pgsgd_graph_get_order(const pgsgd_graph *g, uint32_t *perm_out);
/*
 * The path-guided node order (host only, no device work), a progressive
 * linearization along the paths: the first path's nodes in path order; then
 * each later path, step by step, inserts every node not placed yet right
 * after the last node of that path already placed (at the front if there is
 * none), so a node first met on a later path lands next to its neighbours
 * there; nodes no path visits come last in id order.  perm_out[n] = new id of
 * node n (host, n_nodes entries).  far_before / far_after (host, may be NULL): the fraction
 * of consecutive steps of a path whose node ids differ by more than 32, in
 * the given and in the new order.  Errors: INVALID_ARG (NULL arrays, a node id
 * >= n_nodes).
 */
pgsgd_status pgsgd_path_order(uint32_t n_nodes, const uint32_t *node_len, uint32_t n_paths,
                              const uint64_t *path_offsets, const uint32_t *step_node, uint32_t *perm_out,
                              double *far_before, double *far_after);
/* Frees the handle and its device memory (synchronises the device first).  NULL-safe. */
void pgsgd_graph_destroy(pgsgd_graph *g);
/* Fills *out (host).  Errors: INVALID_ARG on NULL. */
pgsgd_status pgsgd_graph_get_info(const pgsgd_graph *g, pgsgd_graph_info *out);

/* ------------------------------------------------------------------------- */
/* Reading a graph from GFA text                                              */
/* ------------------------------------------------------------------------- */
/*
 * The layout reads the paths and node lengths of a graph only (Alg. 1 takes P
 * and the node lengths; the kernel of Section "CUDA Kernel for Pangenome Graph
 * Layout" keeps that lean structure), and the paper's inputs are the human
 * pangenome graphs of Section "Experiment Setup" in GFA/ODGI form.  These calls
 * turn GFA 1.0/1.1 text into exactly the arrays pgsgd_graph_create takes:
 *   - S <name> <sequence|*> [LN:i:<len>]  node of length |sequence| (or LN;
 *     both given must agree; '*' needs LN); length >= 1 and < 2^32.  Node ids
 *     follow the order of the S lines: the k-th S line is node k.
 *   - P <name> <seg><+|->,... <overlaps>  a path; '-' is a reverse-strand step
 *     (bit 31 of step_node); '*' is an empty path.
 *   - W <sample> <hap> <seqid> <start> <end> <walk>  a path named
 *     sample#hap#seqid (":start-end" appended unless start is '*'); the walk
 *     is a run of '>seg' (forward) and '<seg' (reverse) steps, '*' = empty.
 *   - L lines are counted (n_links) and otherwise ignored, as are comments
 *     ('#'), headers and all other record types; "\r\n" line ends are accepted.
 * Paths are numbered in file order (P and W lines together); a path may name
 * segments whose S line comes later.  Only uncompressed text is read.
 * Errors (nothing is returned on error): INVALID_ARG for a file that cannot be
 * opened or read, a malformed line, a segment defined twice, a step naming a
 * segment without an S line, a length that is 0, missing or contradicted by
 * LN, a step without orientation, a path name used twice (the message names
 * the line); RANGE for 2^31 or more segments, a path of 2^32 or more steps,
 * 2^40 or more steps, more than 2^20 paths, a segment of 2^32 nt or more;
 * UNSUPPORTED for a GFA 2 header (VN:Z:2.x); OOM.  Host only; no device work.
 */
typedef struct pgsgd_gfa pgsgd_gfa;
typedef struct {
  uint32_t n_nodes;
  uint32_t n_paths;
  uint64_t n_steps;
  uint64_t n_links;                  /* L lines read (edges are not used by the layout) */
  const uint32_t *node_len;          /* n_nodes */
  const uint64_t *path_offsets;      /* n_paths + 1, CSR offsets into step_node */
  const uint32_t *step_node;         /* n_steps; bit 31 = reverse-strand step */
  const char *node_names;            /* NUL-terminated names back to back ... */
  const uint64_t *node_name_offsets; /* ... node k's name starts at node_names + offsets[k]; n_nodes + 1 entries */
  const char *path_names;            /* likewise for paths */
  const uint64_t *path_name_offsets; /* n_paths + 1 entries */
} pgsgd_gfa_view;

/* Reads the GFA file `filename` (host path) into a new handle *out. */
pgsgd_status pgsgd_gfa_read(const char *filename, pgsgd_gfa **out);
/* The same from n_bytes of text in host memory (need not be NUL-terminated). */
pgsgd_status pgsgd_gfa_parse(const char *text, uint64_t n_bytes, pgsgd_gfa **out);
/* Pointers into the handle's arrays (valid until pgsgd_gfa_free); pass
 * node_len, path_offsets and step_node to pgsgd_graph_create. */
pgsgd_status pgsgd_gfa_get_view(const pgsgd_gfa *gfa, pgsgd_gfa_view *out);
/* Frees the handle.  NULL-safe. */
void pgsgd_gfa_free(pgsgd_gfa *gfa);

/* ------------------------------------------------------------------------- */
/* Layout parameters (Alg. 1 inputs: schedule S and N_iters)                  */
/* ------------------------------------------------------------------------- */
typedef struct {
  uint32_t n_iters;           /* N_iters (30); one kernel launch per iteration */
  uint32_t terms_per_step;    /* term updates per iteration = terms_per_step * S (Alg. 1: 10) */
  double eta_max;             /* first learning rate; <= 0 selects d_max^2 */
  double eta_min;             /* last learning rate (0.01) */
  double zipf_theta;          /* power-law exponent of the cooling partner (0.99) */
  uint32_t zipf_window;       /* largest power-law hop, in steps (1000), 1..65535 */
  uint32_t graph_id;          /* enters the random counter; < 2^24 */
  uint64_t seed;              /* Philox key */
  uint32_t first_iter;        /* run iterations [first_iter, last_iter) ... */
  uint32_t last_iter;         /* ... ; last_iter = 0 means n_iters */
  uint32_t max_inflight_waves;/* cap on concurrently running 64-term groups (waves); 0 = automatic */
  uint32_t flags;             /* PGSGD_FLAG_* (0: defaults) */
  uint32_t schedule;          /* processing order of an iteration's terms: PGSGD_SCHEDULE_* */
  uint16_t reuse_factor;      /* data reuse: updates per sampled term (DRF), 0 or 1 = off, at most 16 */
  uint16_t step_reduction;    /* data reuse: sampled terms per iteration divided by this (SRF), 0 or 1 = off */
} pgsgd_params;

/* pgsgd_params.flags.  A WINDOWED layout over several iterations can count
 * iteration t + 1 (its window histogram and offsets, in a second set of
 * buffers) on a stream of the graph's own while iteration t is laid out:
 * PGSGD_FLAG_COUNT_AHEAD asks for that overlap; by default (and with
 * PGSGD_FLAG_COUNT_IN_ORDER) every pass stays on the caller's stream, in
 * order.  The sampled terms and, with one wave, the coordinates are the same
 * either way.  Setting both flags is INVALID_ARG.  Batched layouts keep the
 * passes in order. */
enum { PGSGD_FLAG_COUNT_AHEAD = 1, PGSGD_FLAG_COUNT_IN_ORDER = 2 };

/* Data-reuse variant (Section "A Case Study: Explore the Performance-Quality
 * Trade-off with Sampled Path Stress"), active when reuse_factor > 1 or
 * step_reduction > 1, with the PLAIN or the WINDOWED schedule.  PLAIN:
 *   - an iteration samples ceil(terms_per_step * S / step_reduction) terms in
 *     aligned groups of 64; a group's path is the path of the global step
 *     drawn by its first term (paths stay chosen with probability ∝ |p|), and
 *     each term draws its own step uniformly in that path (partner, coins,
 *     cooling and skips as in pgsgd_layout);
 *   - after the group's primary updates, reuse_factor - 1 rounds pair the
 *     i-endpoint of lane l with the j-endpoint of lane (l + o_k) mod 64,
 *     o_k = 1 + (byte k-1 of Philox stream 4 at counter (group, 0, iter)) mod
 *     63, using the values already loaded (cross-lane shuffles, no new loads);
 *     d_ref is the path distance of the two endpoints; same-slot or d = 0
 *     pairs are skipped.  Each endpoint is stored once at the end.
 * WINDOWED: ceil(terms_per_step * S / step_reduction) slots of the window-major
 *   enumeration (counted from the plain step draws t below that number); a
 *   group is an aligned run of 64 slots of one window, and the reuse rounds
 *   pair lane l's i-endpoint with lane (l + o_k) mod 64's j-endpoint when both
 *   steps i lie on the same path, o_k drawn as above at counter (the group's
 *   first slot, 0, iter).
 * Updates per iteration: up to reuse_factor x the sampled terms. */

/* Processing order of the terms of an iteration.
 *   PLAIN    term groups in index order over a grid capped by
 *            max_inflight_waves
 *   WINDOWED window-major enumeration: the steps are cut into windows of
 *            2^h consecutive global steps (h = 14, decreased while there
 *            would be fewer than 16 windows but not below 6, increased while
 *            there would be more than 32768); window w receives n_w slots,
 *            n_w = the number of the iteration's PLAIN step draws that fall
 *            in it (so (n_w) is multinomial(T, |w| / S)); slot s (windows in
 *            order, s < T) draws Philox stream 5 at counter (s mod 2^32,
 *            s >> 32, iter, 5 << 24 | graph_id), takes its step uniformly in
 *            its window, i = start_w + floor(u64 * |w| / 2^64), and its
 *            partner, endpoint coins and skips as a PLAIN term does from
 *            words 2 and 3; its cooling coin is bit 3 of word 3 of the first
 *            slot of its aligned 64-slot group within the window.  A
 *            multinomial count of uniform draws per window is T i.i.d.
 *            uniform steps: the distribution of terms of Alg. 1, in another
 *            order.  Windows are processed in runs (each path cut into 8
 *            pieces, XCD x takes piece x of every path), a window at a time
 *            per XCD, so its step records and the coordinates of the nodes
 *            it visits stay in the XCD's L2.  max_inflight_waves caps the
 *            waves in every iteration (automatic: about nodes_w / 8, nodes_w =
 *            2^h * n_nodes * n_paths / S the nodes a window visits, and
 *            nodes_w / 32 in the iterations t >= n_iters / 2, whose partners
 *            all lie in the active window; both at most the PLAIN cap).
 *            Uniform-partner updates read the partner first and the window-
 *            local endpoint after it arrived, which keeps the window in which
 *            a concurrent update of a local node can be lost short.  Scratch: a few
 *            words per window, allocated on first use.  pgsgd_sample_terms
 *            records slots [t_begin, t_begin + count) in slot order.
 *   AUTO     WINDOWED
 * The value 2 is reserved (INVALID_ARG). */
enum { PGSGD_SCHEDULE_AUTO = 0, PGSGD_SCHEDULE_PLAIN = 1, PGSGD_SCHEDULE_WINDOWED = 3 };

/* Fills the defaults listed above (seed 24301, graph_id 0). */
void pgsgd_params_default(pgsgd_params *p);

/*
 * The learning rate of every iteration, as the float32 values the kernels use:
 * eta_t = eta_max * exp(-lambda t), lambda = ln(eta_max/eta_min)/(N-1), in FP64
 * then rounded (Alg. 1 input S; exponential annealing of Zheng et al., the
 * update rule the paper follows).  d_max is used when eta_max <= 0.  eta_out:
 * host, n_iters entries.  Host only.
 */
pgsgd_status pgsgd_schedule(const pgsgd_params *p, int64_t d_max, float *eta_out);

/*
 * The power-law (Zipf) cumulative table the cooling branch samples from
 * (Alg. 1, "RandomSelect(p, Powerlaw)"): C[0] = 0 and, for k = 1..W,
 * C[k] = floor(F[k]/F[W] * (2^32-1)) with F[k] = sum_{z=1..k} z^-theta summed
 * in FP64 in increasing z.  C_out: host, W+1 entries.  Host only.
 */
pgsgd_status pgsgd_zipf_table(double theta, uint32_t W, uint32_t *C_out);

/* ------------------------------------------------------------------------- */
/* Layout                                                                     */
/* ------------------------------------------------------------------------- */
/*
 * Initial layout: node n starts on the x axis at the path coordinate of its
 * first visit (paths in order): X[2n] = pos, X[2n+1] = pos + len (0 for nodes
 * never visited); Y[2n+e] = jitter * (u - 1/2), u = (r0 >> 8) / 2^24 from
 * Philox stream 3 at counter 2n+e with this seed and graph_id.  coords: device,
 * overwritten.  Async.
 */
pgsgd_status pgsgd_init_coords(pgsgd_graph *g, uint64_t seed, uint32_t graph_id, float jitter, float *coords,
                               void *stream);

/*
 * Runs iterations [first_iter, last_iter) of the PG-SGD layout (Alg. 1) in
 * place on coords (device).  Each iteration is one kernel launch covering
 * terms_per_step * S term updates, run concurrently with unlocked updates
 * (Hogwild, Section "Data-level Parallelism").  Term t of iteration it:
 *   i  = floor(u64 * S / 2^64), u64 = r0 | r1 << 32 (a uniform global step:
 *        "path with probability proportional to |p|, then a step of it");
 *   cooling = (it >= floor(N/2)) or bit 3 of r3 of term t - (t mod 64)
 *        (one coin per aligned group of 64 terms, as in warp merging);
 *   cooling: j = i +/- z, direction bit 2 of r3 (flipped when there is no room
 *        that way), z ~ Zipf(theta) on [1, min(W, room)] drawn from r2 with the
 *        table of pgsgd_zipf_table; a single-step path is skipped;
 *   otherwise: j = start(p) + floor(r2 * |p| / 2^32);
 *   endpoints e_i = bit 0, e_j = bit 1 of r3; endpoint e of step s lies at path
 *        coordinate pos[s] + len * (e XOR reverse[s]); d_ref = |difference|;
 *   terms with the same coordinate slot, d_ref = 0 or coincident points are
 *        skipped; otherwise mu = min(eta / d^2, 1) and both points move by
 *        mu * (|v_i - v_j| - d) / 2 towards (or away from) each other.
 * The schedule (PGSGD_SCHEDULE_*) sets the order in which an iteration's
 * terms are processed.  Async on stream: work the call places on the graph's
 * own counting stream (see pgsgd_params.flags) starts after the work already
 * on stream and is joined back into stream before the call's last kernel, so
 * stream order holds.  The graph's scratch buffers and working copy are
 * shared by all calls on the graph: order them on one stream.  A graph with
 * S = 0 returns OK without work.
 * Errors: INVALID_ARG (NULL, unknown or conflicting flags, zipf_window out of range, graph_id >=
 * 2^24, first_iter > last_iter), RANGE (term count >= 2^48), UNSUPPORTED (LDS limits), DEVICE, OOM.
 */
pgsgd_status pgsgd_layout(pgsgd_graph *g, const pgsgd_params *p, float *coords, void *stream);

/*
 * pgsgd_layout for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same layout, the same kernels and the same sampled terms, but the
 * window tables of the WINDOWED schedule live in a device array of the
 * library (4 MiB per device, held until the process ends; enough for the
 * 32,768 windows the schedule allows) instead of buffers the graph allocates
 * on first use, and every iteration counts its windows in order on `stream`.
 * The call makes no hipMalloc/hipFree: the graph's working copy and power-law
 * table are allocated by pgsgd_graph_create.  The PLAIN schedule needs no
 * scratch and runs as in pgsgd_layout.
 * All calls on one device share that device's array, and it keeps the last
 * call's contents (the call itself clears what must start at zero): calls
 * that overlap on one device, on any streams or graphs, race and give wrong
 * layouts; order them on one stream.
 * Errors: those of pgsgd_layout, plus INVALID_ARG for PGSGD_FLAG_COUNT_AHEAD
 * (counting ahead needs a second table set), RANGE if a graph's window tables
 * would exceed the array, UNSUPPORTED for a device ordinal >= 64.
 */
pgsgd_status pgsgd_layout_noalloc(pgsgd_graph *g, const pgsgd_params *p, float *coords, void *stream);

/*
 * pgsgd_layout with measurement, by HIP events recorded on `stream`:
 *   iter_ms[k]   duration of iteration first_iter + k (all its kernels)
 *   main_ms[k]   summed duration of that iteration's launches of the dominant
 *                kernel (the fused layout kernel of the schedule in use)
 *   *main_launches  launches of the dominant kernel per iteration
 * iter_ms and main_ms: host, last_iter - first_iter entries (main_ms and
 * main_launches may be NULL).  Synchronises the stream.  Same errors as
 * pgsgd_layout, plus INVALID_ARG when iter_ms is NULL.
 */
pgsgd_status pgsgd_layout_timed(pgsgd_graph *g, const pgsgd_params *p, float *coords, float *iter_ms,
                                float *main_ms, uint32_t *main_launches, void *stream);

/* ------------------------------------------------------------------------- */
/* Sampled path stress (Eq. 2)                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
  double mean;       /* sampled path stress: mean of ((|v_i - v_j| - d)/d)^2 */
  double ci_lo;      /* mean - 1.96 sigma / sqrt(n) */
  double ci_hi;      /* mean + 1.96 sigma / sqrt(n) */
  double stddev;     /* sigma from a second pass: sqrt(sum (s - mean)^2 / (n - 1)) */
  double sum;        /* sum of the stress terms (pass 1) */
  double sumsq_dev;  /* sum of squared deviations (pass 2) */
  uint64_t n_valid;  /* pairs with d > 0 */
  uint64_t n_skipped;/* pairs with d = 0 (left out of the mean) */
} pgsgd_stress_result;

/*
 * Sampled path stress with its 95% confidence interval (Eq. 2; two passes, the
 * second for sigma).  Path p receives exactly pairs_per_step * |p| pairs; pair
 * q of path p (q in [m*off[p], m*off[p+1])) draws Philox stream 1 at counter
 * q: i = start + floor(u64 * |p| / 2^64), j = start + floor(r2 * |p| / 2^32),
 * e_i = bit 0, e_j = bit 1 of r3.  All paths are pooled.  Stress terms are
 * computed in FP64 from the float32 coordinates.  coords: device; out: host.
 * Synchronises the stream.  Errors: INVALID_ARG, DEVICE.
 */
pgsgd_status pgsgd_path_stress(pgsgd_graph *g, const float *coords, uint32_t pairs_per_step, uint64_t seed,
                               uint32_t graph_id, pgsgd_stress_result *out, void *stream);

/* Pair modes of pgsgd_path_stress_pairs. */
enum { PGSGD_PAIRS_UNIFORM = 0, PGSGD_PAIRS_POWER_LAW = 1, PGSGD_PAIRS_UNIFORM_WINDOWED = 2 };

/*
 * pgsgd_path_stress with a choice of partner: PGSGD_PAIRS_UNIFORM is Eq. 2
 * (pgsgd_path_stress); PGSGD_PAIRS_POWER_LAW gives pair q the same step i and
 * draw words, and as j the power-law partner of the layout's cooling phase
 * (direction bit 2 of word 3, hop z ~ Zipf(zipf_theta) on [1, min(zipf_window,
 * room)] from word 2; a single-step path has none and the pair counts as
 * skipped).  The power-law mode measures how well the layout keeps short path
 * distances.  zipf_theta, zipf_window are read in that mode only (same limits
 * as in pgsgd_params).
 * PGSGD_PAIRS_UNIFORM_WINDOWED samples the same law of pairs as
 * PGSGD_PAIRS_UNIFORM (each path exactly pairs_per_step * |p| pairs, i and j
 * independent and uniform in the path, independent coins) in window-major
 * order, for locality: the windows of 2^h global steps (h as for the
 * WINDOWED schedule) cut at path boundaries form segments in step order;
 * segment g receives n_g slots, the number of the uniform mode's pairs of its
 * path whose step i falls in it; slot u (numbered over the segments in order)
 * draws Philox stream 6 at counter u: i = segment start + floor(u64 *
 * segment length / 2^64), j = path start + floor(r2 * |p| / 2^32), e_i = bit
 * 0, e_j = bit 1 of r3.  Its segment tables are allocated on first use (about
 * 20 bytes per segment); it needs 8 bytes per path slot plus 4 bytes per
 * segment of LDS and pairs_per_step * 2^(h+1) < 2^32.  Its waves take the
 * 64-slot groups from shared counters, so sum and sumsq_dev are reproducible
 * only up to the rounding of their FP64 summation order (the pairs, n_valid
 * and n_skipped are exact).
 * Every mode first copies coords into the graph's interleaved working copy,
 * so calls on one graph must be ordered on one stream (as for pgsgd_layout).
 * Synchronises the stream.  Errors: INVALID_ARG (unknown mode, bad Zipf
 * parameters), UNSUPPORTED (LDS, segment counts), DEVICE, OOM.
 */
pgsgd_status pgsgd_path_stress_pairs(pgsgd_graph *g, const float *coords, uint32_t pairs_per_step, uint64_t seed,
                                     uint32_t graph_id, uint32_t pair_mode, double zipf_theta, uint32_t zipf_window,
                                     pgsgd_stress_result *out, void *stream);

/*
 * The pairs behind a sampled path stress (Eq. 2 is a mean over millions of
 * pairs; when a few pairs carry a large share of it, the estimate is heavy
 * tailed and these are the pairs to look at): runs pgsgd_path_stress_pairs
 * with the same arguments (same pairs, same *out; out may be NULL) and lists
 * the valid pairs whose stress exceeds `threshold`:
 *   i_out, j_out  device uint64[max_out]: the pair's steps
 *   e_out         device uint8[max_out]: e_i | e_j << 1
 *   s_out         device double[max_out]: the pair's stress (FP64)
 *   *n_out        host: how many pairs exceed the threshold (the first
 *                 max_out found are written, in no particular order)
 * Synchronises the stream.  Errors: those of pgsgd_path_stress_pairs, plus
 * INVALID_ARG for NULL outputs with max_out > 0 or a non-finite threshold.
 */
pgsgd_status pgsgd_path_stress_outliers(pgsgd_graph *g, const float *coords, uint32_t pairs_per_step, uint64_t seed,
                                        uint32_t graph_id, uint32_t pair_mode, double zipf_theta, uint32_t zipf_window,
                                        double threshold, uint64_t max_out, uint64_t *i_out, uint64_t *j_out,
                                        uint8_t *e_out, double *s_out, uint64_t *n_out, pgsgd_stress_result *out,
                                        void *stream);

/*
 * Two layouts of one graph on the same pairs of Eq. 2 (a paired estimate):
 * every valid pair's stress s_a in coords_a and s_b in coords_b, the means,
 * the ratio R = sum s_a / sum s_b and its 95% interval by the delta method,
 * R +- 1.96 sd(s_a - R s_b) / (sqrt(n) mean_b).  When a few pairs carry much
 * of the estimate in both layouts, the paired interval is far narrower than
 * the two separate ones.  Pairs and modes as pgsgd_path_stress_pairs.  A
 * second working copy of the coordinates (16 B per node) is allocated on
 * first use.  Synchronises the stream.  Errors: those of
 * pgsgd_path_stress_pairs, INVALID_ARG for NULL or misaligned coords_b.
 */
typedef struct {
  double mean_a, mean_b, ratio, ratio_ci_lo, ratio_ci_hi;
  double sd_a, sd_b, sd_diff;  /* spreads of s_a, s_b and s_a - R s_b */
  double sum_a, sum_b;
  uint64_t n_valid, n_skipped;
} pgsgd_stress_compare_result;
pgsgd_status pgsgd_path_stress_compare(pgsgd_graph *g, const float *coords_a, const float *coords_b,
                                       uint32_t pairs_per_step, uint64_t seed, uint32_t graph_id, uint32_t pair_mode,
                                       double zipf_theta, uint32_t zipf_window, pgsgd_stress_compare_result *out,
                                       void *stream);

/*
 * Path stress, Eq. 1 (Section "Path Stress"): over every path and every pair of
 * its steps i < j, the stress averaged over the endpoint combinations with
 * d > 0 (a pair with none is left out), then the mean over all such pairs.
 * Each step pair counts once, so paths weigh with |p|^2 (Eq. 2 weighs them
 * with |p|).  Terms in FP64 from the float32 coordinates.  O(sum |p|^2) work:
 * meant for small graphs and for validating the sampled metric.  coords:
 * device; mean_out (and pairs_out, may be NULL): host.  Synchronises.
 */
pgsgd_status pgsgd_path_stress_exact(pgsgd_graph *g, const float *coords, double *mean_out, uint64_t *pairs_out,
                                     void *stream);

/* ------------------------------------------------------------------------- */
/* Differentiable form: sampled stress as a loss                             */
/* ------------------------------------------------------------------------- */
/*
 * Forward: L = (1/n_valid) sum_q ((|v_a - v_b| - d)/d)^2 over n_pairs pairs
 * drawn with the cooling (power-law) sampler of pgsgd_layout from Philox stream
 * 2, counter word 2 = step, with p->seed, p->graph_id, p->zipf_theta and
 * p->zipf_window.  Skipped pairs (single-step path, same slot, d = 0) do not
 * count.  Writes loss_dev[0] (device float32) and n_valid_dev[0] (device
 * uint64).  Async.
 * p->schedule PLAIN enumerates pair q < n_pairs directly.  WINDOWED (the AUTO
 * choice) lists the same law of pairs window-major: the steps are cut into
 * the loss's segments (windows of 2^h steps cut at path boundaries; h = 10,
 * halved while there would be fewer than 16 windows, not below 6, doubled
 * while there would be more than 32768); segment g receives as many slots as
 * plain pair draws fall in it, and slot u draws Philox stream 7 at counter u
 * (word 2 = step): its step uniform in the segment, its partner and coins as
 * above.  The two orders give two samples of the same loss, not the same
 * value.  WINDOWED needs n_pairs < 2^32 (UNSUPPORTED otherwise).
 */
pgsgd_status pgsgd_stress_forward(pgsgd_graph *g, const pgsgd_params *p, const float *coords, uint64_t n_pairs,
                                  uint32_t step, float *loss_dev, uint64_t *n_valid_dev, void *stream);
/*
 * Backward (adjoint of the forward with the same arguments): ADDS
 * grad_out_dev[0] * dL/dcoords into grad_coords (device, [2][n_nodes][2]
 * float32) with float32 atomics; dL/dv_a = (2/n_valid)(mag - d)/d^2 (v_a - v_b)/mag,
 * dL/dv_b = -dL/dv_a, zero when mag = 0.  n_valid_dev is the forward's count.
 * In the WINDOWED order the segments are grouped into tiles of nearby node
 * ids and most of the adjoint is summed in LDS first; a backward right after
 * the forward of the same step, n_pairs, seed and graph_id reuses that
 * forward's segment offsets.  The order of the float32 additions (not their
 * terms) varies from run to run.
 * Forward and backward read the graph's interleaved working copy of coords,
 * so calls on one graph must be ordered on one stream.  Async.
 */
pgsgd_status pgsgd_stress_backward(pgsgd_graph *g, const pgsgd_params *p, const float *coords, uint64_t n_pairs,
                                   uint32_t step, const float *grad_out_dev, const uint64_t *n_valid_dev,
                                   float *grad_coords, void *stream);
/*
 * One Adam step (Kingma and Ba, 2015) over n float32 parameters in place:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; x -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 * x, grad, m, v: device.  t >= 1.  Async.
 */
pgsgd_status pgsgd_adam_step(float *x, const float *grad, float *m, float *v, uint64_t n, float lr, float beta1,
                             float beta2, float eps, uint32_t t, void *stream);

/* ------------------------------------------------------------------------- */
/* Batched form: many graphs laid out by one captured HIP graph              */
/* ------------------------------------------------------------------------- */
typedef struct {
  uint32_t block_threads;   /* 64..1024, multiple of 64 */
  uint32_t groups_per_item; /* consecutive 64-term groups a wave takes per work item, >= 1 */
  uint32_t blocks_per_cu;   /* persistent blocks per compute unit, >= 1 */
  uint32_t max_blocks;      /* cap on the grid (0 = none): bounds concurrent updates for small graphs */
  uint32_t phases;          /* work-item order, 1..64: 1 = graph after graph (fastest on MI355X: the
                               coordinates of the graph in progress stay in the Infinity Cache);
                               R > 1 interleaves the graphs in R phases (updates spread over graphs) */
  uint32_t branches;        /* windowed batches: graphs laid out concurrently, 0..16 (0 = 4) */
} pgsgd_tune;

typedef struct pgsgd_batch pgsgd_batch;

/*
 * Prepares a batched layout of n graphs (all on the same device).  Graph k
 * uses p->graph_id + k as its graph_id (so its terms equal those of a
 * pgsgd_layout of that graph with that graph_id and the same schedule) and
 * its own learning-rate schedule from its own d_max when p->eta_max <= 0.
 * coords[k] is graph k's coordinate buffer (device).  The iterations are
 * captured once in a HIP graph.  p->schedule (resolved as for pgsgd_layout)
 * selects the form:
 *   WINDOWED  every graph runs its own windowed kernels, with its own wave cap
 *             (max_inflight_waves or automatic); the graphs are spread over
 *             tune->branches concurrent branches of the HIP graph (longest
 *             first, each to the least loaded branch), a branch laying out
 *             its graphs one after another; odd-numbered branches take
 *             theirs smallest first, so large graphs run beside small ones.
 *             Only tune->branches is used.
 *   PLAIN     one persistent launch per iteration covers the terms of all
 *             graphs, in the work order of tune->phases (block_threads,
 *             groups_per_item, blocks_per_cu, max_blocks, phases are used;
 *             max_inflight_waves is ignored).
 * tune = NULL picks defaults (4 branches; 256 threads, 1 group per item, 2
 * blocks per CU, 1 phase).  The sampled terms do not depend on tune.  The
 * data-reuse variant (reuse_factor > 1 or step_reduction > 1) is rejected
 * (INVALID_ARG) for both forms.
 */
pgsgd_status pgsgd_batch_create(pgsgd_graph *const *graphs, uint32_t n, const pgsgd_params *p,
                                float *const *coords, const pgsgd_tune *tune, pgsgd_batch **out);
/* Launches the captured iterations [first_iter, last_iter) on stream.  Async. */
pgsgd_status pgsgd_batch_run(pgsgd_batch *b, void *stream);
/* Frees the batch (synchronises the device first).  NULL-safe. */
void pgsgd_batch_destroy(pgsgd_batch *b);
/* One-shot: create, run, synchronise, destroy. */
pgsgd_status pgsgd_layout_batched(pgsgd_graph *const *graphs, uint32_t n, const pgsgd_params *p,
                                  float *const *coords, const pgsgd_tune *tune, void *stream);
/*
 * Times candidate tunings of the batch (on scratch copies of the coordinates,
 * which are left unchanged) and writes the fastest to *best: for the windowed
 * form 1, 2, 3, 4, 6 or 8 branches, each timed on iteration 0 (uniform
 * partners) plus iteration n_iters / 2 (cooling), whose costs differ by about
 * 2x; for the plain form the persistent kernel's shape, timed on one
 * iteration.  On entry best->max_blocks is a grid cap kept in every plain
 * candidate (0 = none).
 * ms_out (host, may be NULL) receives the best time.  Synchronous.
 */
pgsgd_status pgsgd_autotune_batched(pgsgd_graph *const *graphs, uint32_t n, const pgsgd_params *p,
                                    float *const *coords, pgsgd_tune *best, float *ms_out, void *stream);

/*
 * Parity hook for the batched kernel: runs iteration iter of the batch in a
 * recording mode that writes every sampled term of graph k (t in [0,
 * terms_per_step * S_k)) to i_out[k], j_out[k], flags_out[k] (device arrays of
 * that length, flags as in pgsgd_sample_terms) instead of updating
 * coordinates.  Uses the same kernels, work mapping and tune as
 * pgsgd_batch_run (windowed form: each graph's windowed kernels; the slots
 * of graph k in slot order).  Synchronises the stream (plain form; the
 * windowed form records asynchronously on the stream).
 */
pgsgd_status pgsgd_batch_sample_terms(pgsgd_graph *const *graphs, uint32_t n, const pgsgd_params *p, uint32_t iter,
                                      const pgsgd_tune *tune, uint64_t *const *i_out, uint64_t *const *j_out,
                                      uint8_t *const *flags_out, void *stream);

/* ------------------------------------------------------------------------- */
/* Parity hooks: the sampling and the update as separate kernels             */
/* ------------------------------------------------------------------------- */
/*
 * Writes the terms t in [t_begin, t_begin + count) of iteration iter, sampled
 * exactly as pgsgd_layout samples them: i_out, j_out (device uint64) and
 * flags_out (device uint8: bit0 e_i, bit1 e_j, bit2 cooling, bit3 skipped).
 * The terms are recorded by the layout kernels of the schedule p->schedule
 * resolves to, with the launch shape pgsgd_layout uses: PLAIN records with the
 * plain kernel; WINDOWED runs its counting and layout kernels over the whole
 * iteration (without updating coordinates) and records the slots of the range,
 * which must lie in [0, terms_per_step * S).  With the data-reuse variant active it records that variant's terms
 * (see pgsgd_sample_terms_reuse).  Async.
 */
pgsgd_status pgsgd_sample_terms(pgsgd_graph *g, const pgsgd_params *p, uint32_t iter, uint64_t t_begin,
                                uint64_t count, uint64_t *i_out, uint64_t *j_out, uint8_t *flags_out,
                                void *stream);
/*
 * The data-reuse variant's terms and reuse offsets, recorded by its layout
 * kernel with the layout's launch shape.  PLAIN: terms t in [t_begin, t_begin
 * + count) as in pgsgd_sample_terms (t_begin a multiple of 64), and, when
 * offsets_out (device, may be NULL) is given, the offsets o_1..o_{reuse_factor-1}
 * of every 64-term group of the range (reuse_factor - 1 bytes per group, in
 * group order).  WINDOWED: the slots of the range (below ceil(terms_per_step *
 * S / step_reduction)) and, with offsets_out, the offsets of each slot's group
 * (reuse_factor - 1 bytes per slot).  Async.
 */
pgsgd_status pgsgd_sample_terms_reuse(pgsgd_graph *g, const pgsgd_params *p, uint32_t iter, uint64_t t_begin,
                                      uint64_t count, uint64_t *i_out, uint64_t *j_out, uint8_t *flags_out,
                                      uint8_t *offsets_out, void *stream);

/*
 * Applies count given terms (device arrays as written by pgsgd_sample_terms)
 * with learning rate eta, one thread per term, with the update of
 * pgsgd_layout.  Terms touching the same slot race.  Async.
 */
pgsgd_status pgsgd_apply_terms(pgsgd_graph *g, float eta, const uint64_t *i, const uint64_t *j,
                               const uint8_t *flags, uint64_t count, float *coords, void *stream);

/*
 * The collision-free batch of the update's parity check, applied by the
 * layout kernel itself: runs iteration iter of pgsgd_layout (Alg. 1's inner
 * loop with the update rule of pgsgd_layout) with the kernels and launch shape
 * of the schedule p resolves to, but applies only the terms t (WINDOWED: the
 * slots) of [t_begin, t_begin + count) with mask[t - t_begin] != 0; every
 * other term of the iteration is sampled and dropped.  mask: device, count
 * bytes.  coords: device, updated in place.  The range must lie inside the
 * iteration's terms_per_step * S terms.  Terms of the subset that touch the
 * same slot race, as in pgsgd_layout.  Errors: INVALID_ARG (NULL, range, the
 * data-reuse variant), and those of pgsgd_layout.  Async.
 */
pgsgd_status pgsgd_apply_slots(pgsgd_graph *g, const pgsgd_params *p, uint32_t iter, uint64_t t_begin,
                               uint64_t count, const uint8_t *mask, float *coords, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PGSGD_H */
