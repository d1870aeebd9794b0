/*
 * libshaken -- shaken dynamics on MI355X (gfx950).
 *
 * Shaken dynamics (Apollonio, D'Autilia, Scoppola, Scoppola, Troiani,
 * arXiv:1904.06257) is a parallel Markov chain for an Ising system
 *
 *     H(sigma) = - sum_{{x,y} in E} J_xy sigma_x sigma_y - 2 sum_x lambda_x sigma_x
 *
 * (section 2, equation ham1).  Every undirected edge is given an orientation;
 * the oriented edge set E^o splits the neighbourhood of each site into an
 * in-half {y : (y,x) in E^o} and an out-half {y : (x,y) in E^o} (section 2,
 * construction of the doubling graph from G^o).  One full step is two
 * half-steps (section 2, kernels P^{1->2}, P^{2->1} and P^sh):
 *
 *   half-step 1: every spin is redrawn at once, P(+1) = 1/(1 + exp(-2 beta h)),
 *                h_x = sum_{in-half} J_yx sigma_y + q sigma_x + lambda_x
 *   half-step 2: the same with the out-half, read from the result of step 1.
 *
 * On the L x L torus E^o = {(x, x_up), (x, x_right)}: half-step 1 reads the
 * down and left neighbours (P^dl), half-step 2 the up and right ones (P^ur)
 * (section 3, equations hur, hdl, pasymm, pasymm1).  Torus sites are stored
 * row-major, site (row, col) at row*L + col, "up" = row+1, "right" = col+1.
 *
 * Randomness and thresholds (the paper fixes none; the library's contract,
 * identical on every code path and reproduced bit for bit by an independent
 * CPU implementation):
 *   Philox4x32-10 with key (lo32(seed), hi32(seed)).  A site's new spin is +1
 *   iff u < T, where T in [0, 2^32] is the threshold of its local field
 *       h = ((double)S + q*sigma) + lambda,  e = exp(-((2 beta)|h|)),
 *       t = floor(e/(1+e) * 2^32),  T = (h >= 0) ? 2^32 - t : t,
 *   computed in IEEE double on the host, and u is a 32-bit uniform:
 *     torus:  word w = row*ceil(L/32) + (col>>5), bit b = col & 31,
 *             R_k = word (k&3) of Philox((w, s, replica, k>>2)),
 *             u = sum_k ((R_k >> b) & 1) 2^(31-k)            (bit-sliced)
 *     graph:  u = word (v&3) of Philox((v>>2, s, replica, 0x80000000))
 *   with s the half-step index (0, 1, 2, ... ; even = half-step 1).
 *   A random initial state uses s = 0xFFFFFFFF: torus site +1 iff bit b of
 *   R_0; graph vertex +1 iff bit 31 of its u.
 *
 * Conventions for every call:
 *   - Return codes only; nothing is thrown across the ABI.  On failure the
 *     thread-local message of shaken_last_error() says why.
 *   - Host arrays passed in are copied before the call returns; the caller
 *     keeps ownership.  Device memory belongs to the context until
 *     shaken_free().
 *   - Work is enqueued on the context's HIP stream.  Calls that hand data back
 *     to the host synchronise that stream; the others return as soon as the
 *     work is enqueued.
 *   - A context is not thread-safe.  Distinct contexts are independent.
 */
#ifndef SHAKEN_H
#define SHAKEN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHAKEN_VERSION_MAJOR 0
#define SHAKEN_VERSION_MINOR 1

typedef enum shaken_status {
    SHAKEN_OK = 0,
    SHAKEN_EINVAL = 1,   /* invalid argument (message says which)          */
    SHAKEN_ENOMEM = 2,   /* host or device allocation failed               */
    SHAKEN_EDEVICE = 3,  /* HIP runtime error (message carries its string) */
    SHAKEN_ESTATE = 4    /* call not valid in the context's current state  */
} shaken_status;

/* ------------------------------------------------------------------ inputs */

typedef enum shaken_graph_kind {
    SHAKEN_TORUS = 0,      /* L x L periodic square lattice, E^o = up/right edges */
    SHAKEN_EDGES = 1,      /* arbitrary simple graph given as oriented edges      */
    SHAKEN_TRIANGULAR = 2  /* L x L periodic triangular lattice (section 4)       */
} shaken_graph_kind;

/* The interaction graph with its orientation (Definition 2.1).
 *   kind == SHAKEN_TORUS: L is the side, 3 <= L <= 32768; n, m, src, dst unused.
 *   kind == SHAKEN_TRIANGULAR: L as for the torus; the triangular lattice in
 *     skewed coordinates, site x = (row, col) with the six neighbours x +- e1
 *     (one column), x +- e2 (one row), x +- (e1 + e2); E^o = {(x, x + e1),
 *     (x, x + e2), (x, x + e1 + e2)}, so half-step 1 reads the left, down and
 *     down-left neighbours and half-step 2 the other three.  J: NULL or 3*L*L
 *     uniform entries (index 3x + k, k = right, up, diagonal).  Same spin
 *     layouts, randomness and options as the square torus, except +-J.
 *   kind == SHAKEN_EDGES: n vertices (1 <= n < 2^31), m oriented edges; edge e
 *     is (src[e], dst[e]) in E^o, i.e. dst[e] reads src[e] in half-step 1 and
 *     src[e] reads dst[e] in half-step 2.  Host arrays of m int32 each.
 *     Self-loops, out-of-range ids and an edge given twice (in either
 *     direction) are rejected with SHAKEN_EINVAL. */
typedef struct shaken_graph {
    int32_t kind;
    int32_t L;
    int32_t n;
    int64_t m;
    const int32_t *src;
    const int32_t *dst;
} shaken_graph;

/* External field lambda as a small table of values (section 2, lambda_x).
 *   n_classes in [1, 256]; value[c] = lambda of class c (host doubles);
 *   class_of_vertex: host uint8 per vertex (n entries), or NULL = all class 0.
 *   The torus takes a uniform field only (n_classes == 1, class_of_vertex NULL).
 *   Passing NULL for the whole struct means lambda = 0 everywhere.
 *   lambda enters h with weight 1 and H(sigma) with weight 2 (equations ham1,
 *   hur, hdl). */
typedef struct shaken_field {
    int32_t n_classes;
    const double *value;
    const uint8_t *class_of_vertex;
} shaken_field;

enum {
    SHAKEN_FMT_AUTO = 0,       /* torus: bit-packed; graph: int8              */
    SHAKEN_FMT_INT8 = 1,       /* one int8 (+1 / -1) per site                 */
    SHAKEN_FMT_BITPACKED = 2   /* one bit per site, set = +1: torus
                                  uint32[L][ceil(L/32)] (bit c & 31 of word
                                  (r, c >> 5)); graph uint32[ceil(n/32)] (bit
                                  v & 31 of word v >> 5)                      */
};

enum {
    SHAKEN_INIT_RANDOM = 0,    /* from Philox at s = 0xFFFFFFFF (see above)   */
    SHAKEN_INIT_ALL_UP = 1,
    SHAKEN_INIT_ALL_DOWN = 2,
    SHAKEN_INIT_USER = 3       /* init_spins: host int8, +1/-1, n or L*L      */
};

enum {
    SHAKEN_LAYOUT_AUTO = 0,    /* PACKED when it applies (it carries the ELL
                                  records too); else, up to 65536 vertices,
                                  ELL when it applies; else CSR (on larger
                                  graphs the grid kernels run 1.1-1.4x
                                  faster on CSR than on ELL)                  */
    SHAKEN_LAYOUT_CSR = 1,     /* in-half and out-half CSR (any graph)        */
    SHAKEN_LAYOUT_ELL = 2,     /* couplings +-1 and degree <= 4 only: one
                                  slot-major record per neighbour slot holding
                                  the index, the half it belongs to and the
                                  sign of J                                   */
    SHAKEN_LAYOUT_PACKED = 3   /* ELL plus one 8-byte record per vertex (three
                                  16-bit neighbour indices, their halves,
                                  signs and the field class) read by the
                                  persistent batch kernel; needs couplings
                                  +-1, degree <= 3, n <= 65536 and at most 16
                                  field classes                               */
};

typedef struct shaken_opts {
    int32_t format;            /* SHAKEN_FMT_*                                */
    int32_t init;              /* SHAKEN_INIT_*                               */
    const int8_t *init_spins;  /* SHAKEN_INIT_USER only                       */
    uint32_t replica;          /* third Philox counter word                   */
    int32_t device;            /* HIP device ordinal; -1 = current device     */
    void *stream;              /* hipStream_t; NULL = the null stream         */
    int32_t graph_layout;      /* SHAKEN_LAYOUT_* (graphs only)               */
    int32_t flags;             /* SHAKEN_GRAPH_SPLIT, SHAKEN_ORDER_REVERSED    */
    const uint8_t *frozen;     /* NULL, or host bytes per site (n; torus row-
                                  major): nonzero = the site is in the frozen
                                  set B of section 3.1 and stays +1 (its start
                                  value and every draw are overridden; it
                                  enters its neighbours' fields as +1)        */
} shaken_opts;

/* opts.flags.  SHAKEN_GRAPH_SPLIT: the generalised split of section 5 -- an
 * undirected pair {x, y} may be given in both orientations, (x, y) and (y, x),
 * each with its own coupling, so that the Ising coupling is the sum
 * (matrix form J = J^o + J^o^T).  Each oriented edge then feeds its own half
 * only (in-half of its head, out-half of its tail), e.g. J^o = J / 2 on every
 * orientation gives the symmetric split, whose two half-steps are the same
 * kernel.  Without the flag a pair given twice is SHAKEN_EINVAL (Definition
 * 2.1 orients each undirected edge once); the same oriented edge given twice
 * is SHAKEN_EINVAL either way.  Half-integer splits: scale J, q and lambda by
 * 2 and beta by 1/2. */
enum { SHAKEN_GRAPH_SPLIT = 1, SHAKEN_ORDER_REVERSED = 2, SHAKEN_GRAPH_LDS = 4, SHAKEN_GRAPH_NO_LDS = 8 };
/* SHAKEN_GRAPH_LDS / SHAKEN_GRAPH_NO_LDS (graphs, grid launches): run the
 * half-steps in the kernel that first copies the bit-packed configuration
 * into LDS, so that every neighbour gather is an LDS read instead of a
 * random global load (graphs of at most 1,179,648 vertices; int8 chains then
 * keep a packed mirror of their spins), or never.  Default: that kernel from
 * 131,072 vertices on.  A batch group takes it when all its chains do; with
 * autotune a batch measures both.  Results are identical either way. */
/* SHAKEN_ORDER_REVERSED (torus and graph): the reversed order of section 3,
 * P^{sh'} = P^{2->1} P^{1->2}: the half-step at an even counter reads the
 * out-half (torus: up and right neighbours, P^ur) and the one at an odd
 * counter the in-half.  The uniforms stay keyed by (site, s), so a reversed
 * graph run equals the forward run on the reversed edge set. */

typedef struct shaken_ctx shaken_ctx;

/* ------------------------------------------------------------ single chain */

/* Create a chain: graph g with couplings J and field lambda, self-interaction
 * q >= 0 (Definition 2.2 takes q > 0; q = 0 is accepted) and inverse
 * temperature beta >= 0 (both finite), Philox key `seed`.
 *   J: host int8 per oriented edge (m entries), or NULL = all +1.  For the
 *      torus J is per oriented edge too (2*L*L entries, x = row*L + col:
 *      index 2x is the edge (x, x_up), 2x+1 is (x, x_right)); every entry
 *      must have the same magnitude: a uniform coupling, or +-J with any
 *      signs (the Edwards-Anderson couplings of section 6, kept as two sign
 *      bit-planes); NULL means +1.
 *   opts: NULL = defaults (AUTO format, random init, replica 0, current
 *      device, null stream).
 * The threshold table covers every local field the graph can produce; its
 * size is (2*Smax+1) * 2 * n_classes entries with Smax the largest sum of
 * |J| over a half-neighbourhood; more than 2^24 entries is SHAKEN_EINVAL.
 * Errors: SHAKEN_EINVAL (bad graph, q/beta negative or not finite, torus with
 * couplings of different magnitudes or a non-uniform field), SHAKEN_ENOMEM,
 * SHAKEN_EDEVICE. */
shaken_status shaken_init(shaken_ctx **out, const shaken_graph *g, const int8_t *J,
                          const shaken_field *lambda, double q, double beta,
                          uint64_t seed, const shaken_opts *opts);

/* Release every device and host resource of the context (NULL is a no-op). */
shaken_status shaken_free(shaken_ctx *ctx);

/* Advance n >= 0 half-steps (section 2, P^{1->2} then P^{2->1} alternately).
 * The parity of the context's half-step counter s selects the half: even =
 * half-step 1 (in-half, torus dl), odd = half-step 2 (out-half, torus ur).
 * Asynchronous. */
shaken_status shaken_half_step(shaken_ctx *ctx, int64_t n);

/* Advance n_full >= 0 full steps (P^sh = P^{1->2} P^{2->1}, section 2).
 * If H_out / M_out are non-NULL they receive n_full+1 host int64 values:
 * H(sigma_t) and M(sigma_t) = sum_x sigma_x for t = 0..n_full (t = 0 is the
 * configuration before the call).  H_out requires every 2*lambda to be an
 * integer (else SHAKEN_EINVAL), so that H is exact.  The counter s must be
 * even (else SHAKEN_ESTATE).  Synchronises the stream when logs are asked
 * for. */
shaken_status shaken_sweep(shaken_ctx *ctx, int64_t n_full, int64_t *H_out, int64_t *M_out);

/* Variant of shaken_sweep for callers that cannot allocate memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same half-steps and the same logs, but the per-step partial
 * sums of the observables go to a fixed 4 MiB device buffer of the library
 * (one per device, its address looked up at shaken_init) instead of log space
 * grown on demand, and the logs are written to device memory.  The call
 * allocates nothing, on the device or on the host, and only enqueues work on
 * the context's stream (the one exception: after shaken_batch_set_params
 * changed this context's parameters, the first call re-uploads its tables and
 * synchronises).
 *   H_dev, M_dev: NULL, or device int64 arrays of n_full+1 entries that
 *     receive H(sigma_t) and M(sigma_t), t = 0..n_full, exactly as H_out and
 *     M_out of shaken_sweep (H_dev needs every 2*lambda to be an integer).
 *     With both NULL nothing is logged and the buffer is not used.
 * Limits with logs: at most 32 field classes, and n_full + 1 slots of
 * 8 * 16 * ceil((1 + n_classes) / 16) int64 each within the 2^19 int64 of
 * the buffer -- 4095 full steps per call for up to 15 classes, 2047 for 16 to
 * 31; beyond that SHAKEN_EINVAL, with the bound in the message.
 * The buffer is shared by every context on a device and keeps the last call's
 * contents (each call clears the part it uses first): calls that overlap on
 * one device -- from different streams or threads -- race and corrupt each
 * other's logs.  Other errors as shaken_sweep. */
shaken_status shaken_sweep_noalloc(shaken_ctx *ctx, int64_t n_full, int64_t *H_dev, int64_t *M_dev);

/* Observables of the current configuration. */
typedef struct shaken_obs {
    int64_t half_step;   /* the counter s                                    */
    int64_t n_sites;
    int64_t M;           /* sum_x sigma_x                                    */
    int64_t E_J;         /* sum_{(x,y) in E^o} J_xy sigma_x sigma_y           */
    int64_t E_lambda2;   /* sum_x 2 lambda_x sigma_x, valid iff flags & 1     */
    double H;            /* -E_J - sum_x 2 lambda_x sigma_x (double)         */
    int32_t flags;       /* bit 0: every 2*lambda is an integer              */
    int32_t reserved;
} shaken_obs;

/* Synchronises the stream. */
shaken_status shaken_observables(shaken_ctx *ctx, shaken_obs *out);

/* Change beta and q (rebuilds the threshold table; same validation as init). */
shaken_status shaken_set_params(shaken_ctx *ctx, double beta, double q);

/* Copy the current configuration to / from host int8 (+1/-1), n or L*L
 * entries, row-major for the torus.  get synchronises; set validates
 * entries (SHAKEN_EINVAL unless every value is +1 or -1). */
shaken_status shaken_get_spins(shaken_ctx *ctx, int8_t *out);
shaken_status shaken_set_spins(shaken_ctx *ctx, const int8_t *in);

/* Set the half-step counter s (checkpoint restore); s < 2^32 - 1. */
shaken_status shaken_set_half_step(shaken_ctx *ctx, int64_t s);

/* Copy the threshold table: entry index ((S + Smax)*2 + (sigma > 0)) *
 * n_classes + class holds T (33 bits in a uint64).  If out is NULL only *n
 * is set; otherwise *n must hold the capacity on entry and receives the
 * entry count.  *smax receives Smax when non-NULL. */
shaken_status shaken_get_lut(const shaken_ctx *ctx, uint64_t *out, size_t *n, int32_t *smax);

/* Borrow the device pointer of the current configuration (valid until the
 * next call on the context) and its format (SHAKEN_FMT_INT8 / BITPACKED). */
shaken_status shaken_spins_device(shaken_ctx *ctx, void **ptr, int32_t *format);

/* Block until the context's stream is idle. */
shaken_status shaken_synchronize(shaken_ctx *ctx);

/* ------------------------------------------------------------------ batches */

/* A batch runs many independent chains (each its own graph, J, lambda, beta,
 * q, seed and replica -- the paper's dynamics per chain, unchanged) with
 * fused launches.  Strategies:
 *   SHAKEN_BATCH_GRID:       one launch per half-step covering every chain
 *                            (any size); optionally replayed from a HIP graph.
 *   SHAKEN_BATCH_PERSISTENT: one launch per call; each workgroup takes whole
 *                            chains from a device queue (longest first) and
 *                            keeps their spins in LDS for all the steps.  Tori
 *                            need the bit-packed format and L <= 256; graphs
 *                            n <= 65536 and at most 16 field classes.
 *   SHAKEN_BATCH_AUTO:       persistent when every chain fits, else grid. */
enum { SHAKEN_BATCH_AUTO = 0, SHAKEN_BATCH_GRID = 1, SHAKEN_BATCH_PERSISTENT = 2 };

typedef struct shaken_batch_opts {
    int32_t strategy;      /* SHAKEN_BATCH_*                                  */
    int32_t use_hipgraph;  /* capture the launches in a HIP graph and replay
                              it: grid strategy, 16 full steps of half-step
                              launches per replay (captured on the first
                              sweep, whatever its length; the remainder of
                              a call runs eagerly); persistent strategy, the
                              whole call (one capture for every n_full)      */
    int32_t autotune;      /* 0: fixed launch shapes; 1: measure candidates
                              on the first call and keep the fastest (grid:
                              the block size of every group; persistent: the
                              number of resident workgroups, on trial runs
                              after which every configuration is restored);
                              2: as 1, but a batch of the same shape (device,
                              and every chain's kind, format, sizes, table,
                              couplings, field classes and layout) measured
                              earlier in this process reuses that result
                              without measuring; other values: SHAKEN_EINVAL */
    int32_t record;        /* log H and M of every chain at every full step  */
    void *stream;          /* hipStream_t; NULL = the first chain's stream   */
    int32_t track;         /* persistent strategy: keep, per chain, H of the
                              last configuration and the lowest H (with its
                              configuration) over the full-step
                              configurations of each sweep call; needs every
                              2*lambda to be an integer                      */
    int32_t log_reserve;   /* with record: log space for sweeps of up to this
                              many full steps is allocated at creation, so
                              such sweeps allocate nothing; 0 = allocate on
                              the first sweep that needs more (>= 0)         */
} shaken_batch_opts;

typedef struct shaken_batch shaken_batch;

/* Group n >= 1 contexts into a batch.  Every context must be on the same
 * device and have the same half-step counter s (even).  The contexts stay
 * owned by the caller and must outlive the batch; the batch never frees
 * them.  Errors: SHAKEN_EINVAL, SHAKEN_ESTATE (counters differ or odd),
 * SHAKEN_ENOMEM, SHAKEN_EDEVICE. */
shaken_status shaken_batch_create(shaken_batch **out, shaken_ctx *const *ctx, int32_t n,
                                  const shaken_batch_opts *opts);

/* Advance every chain of the batch by n_full full steps.  With record set,
 * each chain's H/M log of this call (n_full+1 entries) can then be read with
 * shaken_batch_get_log.  Every chain's counter must still be the batch's and
 * even (SHAKEN_ESTATE otherwise: a member stepped on its own, or restored to
 * an odd counter).  Asynchronous. */
shaken_status shaken_batch_sweep(shaken_batch *b, int64_t n_full);

/* Copy chain i's log of the last shaken_batch_sweep (requires record and
 * integer 2*lambda for H).  cap = capacity of H_out / M_out in entries. */
shaken_status shaken_batch_get_log(shaken_batch *b, int32_t i, int64_t *H_out, int64_t *M_out,
                                   int64_t cap);

/* Same log with the coupling energy E_J(sigma_t) = sum over the undirected
 * edges of J_xy sigma_x sigma_y (equation ham1 without the field term) in
 * place of H: exact for any lambda.  EJ_out must be non-NULL, M_out may be
 * NULL; cap as above.  This is what the metastability runs of section 3.2
 * read (lambda = 0.15 there, so H is not an integer). */
shaken_status shaken_batch_get_log_ej(shaken_batch *b, int32_t i, int64_t *EJ_out, int64_t *M_out,
                                      int64_t cap);

/* Every chain's log of the last sweep at once, read from the device with one
 * copy: row i (chain i in batch order) of each non-NULL output, row-major
 * [n_chains][cap], receives that chain's n_full+1 entries of H (integer
 * 2*lambda on every chain required), M and E_J.  SHAKEN_EINVAL if every
 * output is NULL or cap < n_full+1; SHAKEN_ESTATE without a recorded sweep.
 * Host memory: one temporary copy of the call's log space. */
shaken_status shaken_batch_get_logs(shaken_batch *b, int64_t *H_out, int64_t *M_out, int64_t *EJ_out,
                                    int64_t cap);

/* Set beta[i] and q[i] (host arrays, one per chain) for the following sweeps
 * of the batch: the thresholds are rebuilt on the host in double exactly as
 * shaken_set_params does and uploaded.  This is how an annealing schedule
 * (beta_t, q_t) drives the chains (section 6, Theorem 6.1: alternate dynamics
 * as a minimiser).  Synchronises the batch stream.  SHAKEN_EINVAL on a
 * negative or non-finite value. */
shaken_status shaken_batch_set_params(shaken_batch *b, const double *beta, const double *q);

/* After a sweep with opts.track: H_last[i] = H of chain i's configuration at
 * the end of the call, H_best[i] = the lowest H over its full-step
 * configurations of the call (the one it started from included).  best_spins
 * (optional, host int8) receives, concatenated over the chains in batch
 * order, the configuration that reached H_best (n or L*L entries each).
 * Synchronises. */
shaken_status shaken_batch_get_track(shaken_batch *b, int64_t *H_last, int64_t *H_best,
                                     int8_t *best_spins);

/* Strategy the batch uses (after AUTO and autotuning), and the last call's
 * device time in milliseconds measured with HIP events on the batch stream
 * (synchronises). */
shaken_status shaken_batch_info(shaken_batch *b, int32_t *strategy, double *last_ms);

/* Host-side work the batch has done since creation, so that a caller can
 * check that a call did none of it (a timed call, a serving loop):
 *   sweeps:     shaken_batch_sweep calls completed;
 *   captures:   HIP graphs captured and instantiated (grid strategy: one graph
 *               of 16 full steps, captured on the first sweep whatever its
 *               length and again only after the log space or the launch
 *               shapes changed; persistent strategy: one, on the first sweep,
 *               that serves every later call whatever its n_full);
 *   log_allocs: device allocations of log space (a recorded sweep longer than
 *               any before it, beyond opts.log_reserve);
 *   autotunes:  autotuning passes that measured (the first sweep with
 *               opts.autotune; none when autotune = 2 found the shape);
 *   uploads:    refreshes of the device chain descriptors (log space moved,
 *               parameters changed, or a member's spin buffers swapped by
 *               shaken_set_half_step).
 * Never fails on a valid batch. */
typedef struct shaken_batch_counts {
    int64_t sweeps;
    int64_t captures;
    int64_t log_allocs;
    int64_t autotunes;
    int64_t uploads;
} shaken_batch_counts;

shaken_status shaken_batch_counters(shaken_batch *b, shaken_batch_counts *out);

/* Launch shape chain i runs with (after autotuning, if any): the workgroup
 * size of its group's half-step launches on the grid strategy -- 64, 128 or
 * 256, or 1024 for the graph kernel that stages the configuration in LDS --
 * and 0 on the persistent strategy.  SHAKEN_EINVAL for a bad index. */
shaken_status shaken_batch_launch_shape(shaken_batch *b, int32_t i, int32_t *block);

shaken_status shaken_batch_free(shaken_batch *b);


/* ------------------------------------------------- annealing schedule network
 *
 * A small multilayer perceptron that maps per-chain features (size, degree
 * statistics, elapsed fraction of the schedule, current and best energy
 * density, previous beta and q) to the next (log beta, log q) of an annealing
 * schedule for the minimisation use of the dynamics (section 6).  The network
 * is not part of the paper; it only chooses parameters, the sampler's
 * arithmetic is unchanged.
 *
 * Shape: 16 inputs (features padded with zeros) -> 128 -> 128 -> 128 -> 16
 * outputs (the first 2 are used), ReLU after each hidden layer.  Parameters
 * are FP32 masters; every product uses their BF16 (round to nearest even)
 * copies and BF16 activations, accumulated in FP32 on the matrix cores.
 * Parameter vector layout (FP32, SHAKEN_MLP_NPARAM entries): W1[128][16],
 * b1[128], W2[128][128], b2[128], W3[128][128], b3[128], W4[16][128], b4[16]
 * (row-major, W[out][in]); rows 2..15 of W4 and b4[2..15] are kept at zero.
 */
#define SHAKEN_MLP_IN 16
#define SHAKEN_MLP_HIDDEN 128
#define SHAKEN_MLP_OUT 16
#define SHAKEN_MLP_NPARAM (128 * 16 + 128 + 2 * (128 * 128 + 128) + 16 * 128 + 16)

typedef struct shaken_mlp shaken_mlp;

/* Allocate a network (parameters zero) on `device` (-1 = current) with work
 * enqueued on `stream` (hipStream_t, NULL = null stream). */
shaken_status shaken_mlp_create(shaken_mlp **out, int32_t device, void *stream);
shaken_status shaken_mlp_free(shaken_mlp *m);

/* Copy the FP32 parameter vector from / to the host (n = SHAKEN_MLP_NPARAM).
 * Setting also refreshes the BF16 copies and zeroes the Adam moments. */
shaken_status shaken_mlp_set_params(shaken_mlp *m, const float *host, size_t n);
shaken_status shaken_mlp_get_params(shaken_mlp *m, float *host, size_t n);

/* y[batch][16] = f(x[batch][16]); x and y are device FP32 row-major.  Keeps
 * the activations for shaken_mlp_backward.  batch >= 1. */
shaken_status shaken_mlp_forward(shaken_mlp *m, const float *x_dev, int32_t batch, float *y_dev);

/* Gradient of sum_rows w_r * sum_{c<2} (y[r][c] - target[r][c])^2 / sum_r w_r
 * at the last forward: writes the loss to *loss_host (synchronises) and the
 * parameter gradient into the network's FP32 gradient buffer.  target and w
 * are device FP32 ([batch][16] and [batch]; w may be NULL = all ones). */
shaken_status shaken_mlp_loss_backward(shaken_mlp *m, const float *target_dev, const float *w_dev,
                                       int32_t batch, float *loss_host);

/* Backward pass for an arbitrary output gradient dy[batch][16] (device FP32)
 * of the last forward; fills the FP32 gradient buffer. */
shaken_status shaken_mlp_backward(shaken_mlp *m, const float *dy_dev, int32_t batch);

/* Copy the gradient buffer to the host (n = SHAKEN_MLP_NPARAM). */
shaken_status shaken_mlp_get_grads(shaken_mlp *m, float *host, size_t n);

/* One Adam step on the FP32 masters from the gradient buffer (step t >= 1 for
 * the bias corrections), then refresh the BF16 copies. */
shaken_status shaken_mlp_adam(shaken_mlp *m, float lr, float beta1, float beta2, float eps,
                              int32_t t);

/* ------------------------------------------------------ one-call batch runs
 *
 * shaken_batch_run creates a batch over ctx[0..n-1], runs n_full full steps
 * under an optional annealing schedule, fills the requested results and frees
 * the batch; the contexts keep their final configurations (and, with a
 * schedule, the last beta and q).  This is the minimisation use of the
 * dynamics (section 6): at low temperature the pair law concentrates on the
 * minimisers of the pair Hamiltonian, which lie on the diagonal -- minimisers
 * of H -- once q exceeds every half-neighbourhood coupling sum (Theorem 6.1,
 * read as q > max_x sum_{(x,y) in E^o} |J_xy| + |lambda_x|).  The schedule
 * only chooses (beta, q) between chunks of full steps; the sampler's
 * arithmetic is unchanged, and every energy reported is that of a
 * configuration the dynamics reached. */
enum {
    SHAKEN_SCHEDULE_NONE = 0,       /* every chain keeps its own beta and q     */
    SHAKEN_SCHEDULE_GEOMETRIC = 1,  /* beta geometric from beta0 to beta1, q
                                       constant, the same for every chain      */
    SHAKEN_SCHEDULE_MLP = 2         /* the schedule network picks (beta, q) for
                                       every chain and chunk; the geometric
                                       schedule stands in for any chain whose
                                       network output is not finite            */
};

typedef struct shaken_schedule {
    int32_t kind;            /* SHAKEN_SCHEDULE_*                               */
    int32_t chunk_sweeps;    /* full steps per chunk (>= 1, n_full a multiple of
                                it; kinds GEOMETRIC and MLP): (beta, q) change
                                only between chunks                          */
    double beta0, beta1;     /* geometric schedule (> 0, finite): chunk c of C
                                runs at beta = exp(log beta0 + ((c + 1/2) / C)
                                * (log beta1 - log beta0)) (libm log and exp)  */
    double q;                /* geometric schedule: q (>= 0, finite)           */
    shaken_mlp *mlp;         /* kind MLP: the network (same device)            */
} shaken_schedule;

/* The schedule network's inputs, one row of 16 FP32 per chain and chunk c of
 * C (features of the chain before the chunk, zero beyond entry 8):
 *   0  log2(sites) / 16
 *   1  mean degree / 4                (in-half + out-half sizes)
 *   2  std(in-half size - out-half size) / 2, over the sites
 *   3  c / C
 *   4  H(current configuration) / sites
 *   5  lowest H so far / sites
 *   6  log beta of the previous chunk / 3   (0 before the first chunk)
 *   7  log q of the previous chunk / 3      (0 before the first chunk)
 *   8  1
 * each computed in double and rounded to FP32.  Outputs 0 and 1 are
 * (log beta, log q); after the fallback for non-finite rows both are clamped
 * to [log 0.05, log 20] and [log 0.05, log 8]. */

typedef struct shaken_run_result {
    int64_t *H_final;     /* NULL or n: H of each chain's final configuration */
    int64_t *H_best;      /* NULL or n: lowest H over each chain's full-step
                             configurations of the run (the start included) */
    int8_t *best_spins;   /* NULL or, concatenated in chain order, the
                             configuration that first reached H_best (n or
                             L*L int8 each); needs the persistent strategy   */
    double *beta_used;    /* NULL or [chunks][n]: beta of each chain in each
                             chunk (kinds GEOMETRIC and MLP)                 */
    double *q_used;       /* NULL or [chunks][n]: q likewise                  */
    int64_t chunks;       /* out: number of chunks run                        */
    int64_t fallbacks;    /* out: (chunk, chain) pairs where the network's
                             output was not finite                           */
} shaken_run_result;

/* Run n_full full steps of the chains ctx[0..n-1] as one batch (opts as for
 * shaken_batch_create, NULL = defaults; AUTO picks the persistent kernel
 * when every chain fits it) under `sched` (NULL = SHAKEN_SCHEDULE_NONE), and
 * fill what `res` asks for (res may be NULL).  Energies (H_final, H_best,
 * best_spins, and the MLP's features) need every 2*lambda to be an integer;
 * they are tracked on the device (persistent strategy) or read from the
 * observables log (grid strategy).  Allocates the batch and, for the MLP,
 * two small feature buffers; synchronises.  Errors: SHAKEN_EINVAL (bad
 * schedule, n_full not a multiple of chunk_sweeps, best_spins without the
 * persistent strategy, network on another device), SHAKEN_ESTATE, and those
 * of the batch calls. */
shaken_status shaken_batch_run(shaken_ctx *const *ctx, int32_t n, int64_t n_full,
                               const shaken_batch_opts *opts, const shaken_schedule *sched,
                               shaken_run_result *res);

/* -------------------------------------------------------------- diagnostics */

const char *shaken_strerror(shaken_status s);
/* Message of the last failing call on this thread ("" if none). */
const char *shaken_last_error(void);
/* (major << 16) | minor */
int32_t shaken_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SHAKEN_H */
