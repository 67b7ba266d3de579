/*
 * nd.h -- C ABI of the MI355X (gfx950) nucleus-decomposition library.
 *
 * Computes the kappa_s index of every r-clique of a simple undirected graph
 * by the iterated h-index method of Sariyuce, Seshadhri and Pinar, "Local
 * Algorithms for Hierarchical Dense Subgraph Discovery" (PVLDB 12(1), 2019):
 * tau_0 = d_s (the S-degree), tau_{t+1} = U tau_t, where the update operator U
 * (Section 3, Defn. of U) sets, for every r-clique R,
 *     rho(S,R) = min over the other r-cliques R' of S of tau(R')  (S contains R)
 *     U tau(R) = H({rho(S,R)} over all S containing R),
 * H being the h-index (Section 2.2).  The iteration stops at the first sweep
 * that changes nothing; the result is then exactly kappa_s (Theorem 3 and
 * Lemma 2).  Five instances are supported (Section 5 evaluates the first
 * three; the definitions hold for any r < s, Section 2.1):
 *     ND_KCORE      (r,s) = (1,2)  core number of every vertex
 *     ND_KTRUSS     (r,s) = (2,3)  truss number of every edge, counted in
 *                                  triangles (Section 2.1; Cohen's k-truss
 *                                  number is this value + 2)
 *     ND_NUCLEUS34  (r,s) = (3,4)  kappa_4 of every triangle
 *     ND_NUCLEUS13  (r,s) = (1,3)  kappa_3 of every vertex (its triangles)
 *     ND_NUCLEUS24  (r,s) = (2,4)  kappa_4 of every edge (its 4-cliques)
 * under synchronous (SND, Alg. 2) or asynchronous (AND, Alg. 3) updates.
 *
 * Output order.  r-cliques are numbered by the lexicographic order of their
 * sorted vertex tuples: vertices by id; edges (u,v), u<v; triangles (u,v,w),
 * u<v<w.  nd_rcliques() lists them.  An r-clique contained in no s-clique
 * has kappa = 0.
 *
 * Conventions for every entry point.
 *   - All calls return an nd_status; on failure nd_last_error() (per calling
 *     thread) describes it.  No call throws across the ABI.
 *   - `stream` is a hipStream_t passed as void* (NULL = the device's null
 *     stream).  Work is ordered on it.  Every call returns only after its
 *     device work has finished, unless stated otherwise.
 *   - `on_device` != 0 means a pointer argument is a device pointer on the
 *     context's device; 0 means host memory.  Inputs are read during the call
 *     only (the library keeps its own copies); outputs are caller-allocated.
 *   - The library owns every array it derives (canonical CSR, r-clique lists,
 *     incidence lists, tau buffers) and frees them in nd_graph_destroy().
 *   - Device memory is charged to the context's budget; a call that would
 *     exceed it fails with ND_ERR_OOM and leaves the graph unchanged.
 *   - Sizes: vertex ids and r-clique ids are int32 (so n, |E| and the number
 *     of triangles must be below 2^31); offsets and incidence counts are
 *     int64.
 *   - Objects are not thread-safe: calls on one nd_ctx (and its graphs) must
 *     not overlap, except the nd_server_* calls, which are, and graph
 *     creation and destruction, which may run beside a server's threads.
 *     The library captures no stream: the caller may use any stream,
 *     the legacy default one included, while a server is sweeping.
 *
 * Environment (tuning only; results never depend on them).
 *   ND_FRONTIER_SWITCH=d  with use_frontier, notifications start once a sweep
 *                         changes at most 1/d of the swept r-cliques
 *                         (default 8; 0: from the second sweep on).
 *   ND_BATCH_NO_GRAPH=1   batched epochs are launched one by one instead of
 *                         through HIP graphs of eight epochs.
 *   ND_PREP_THREADS=t     host threads building or preparing graphs in
 *                         nd_graphs_from_edges, nd_prepare_many and
 *                         nd_batch_decompose (default 2) and in a server
 *                         (default 4).
 *   ND_TRUSS_NO_LDS=1     the k-truss builder intersects the 64-lane bin
 *                         without the per-source LDS copy (the path taken
 *                         when an out-list exceeds 5120 entries).
 *   ND_TRUSS_NO_TRIBUF=1  the k-truss builder intersects twice instead of
 *                         recording the triangles (the path taken when the
 *                         buffer does not fit the memory budget).
 *   ND_N34_NO_ROWS=1      the (3,4) builder keeps no bit rows: triangles are
 *                         listed by intersection and every pass builds its
 *                         rows again (the path taken when they do not fit a
 *                         quarter of the memory budget left).
 *   ND_LEVELS_BIG=c       nd_levels runs a level on the whole GPU when it has
 *                         at least c candidate r-cliques (default 1024).
 */
#ifndef ND_H
#define ND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ND_OK = 0,
  ND_ERR_INVALID = 1,       /* bad argument or malformed graph */
  ND_ERR_OOM = 2,           /* device-memory budget or device exhausted */
  ND_ERR_DEVICE = 3,        /* a HIP runtime call failed */
  ND_ERR_UNSUPPORTED = 4,   /* kind/mode/option not available */
  ND_ERR_NOT_CONVERGED = 5, /* max_iters reached; output is tau_t >= kappa */
  ND_ERR_BUSY = 6,          /* server queue full */
  ND_ERR_CANCELLED = 7,     /* served request cancelled or stopped early */
  ND_ERR_TIMEOUT = 8        /* nd_server_wait timed out; request still live */
} nd_status;

typedef enum {
  ND_KCORE = 0,
  ND_KTRUSS = 1,
  ND_NUCLEUS34 = 2,
  ND_NUCLEUS13 = 3,
  ND_NUCLEUS24 = 4
} nd_kind;

/* ND_SND: Jacobi-style sweeps, tau_{t+1} = U tau_t from a snapshot (Alg. 2);
 *         every iterate is deterministic.
 * ND_AND: Gauss-Seidel-style sweeps that read the latest values in place
 *         (Alg. 3 without the notification lines); the converged result is
 *         identical, intermediate iterates depend on scheduling. */
typedef enum { ND_SND = 0, ND_AND = 1 } nd_mode;

typedef struct nd_ctx nd_ctx;
typedef struct nd_graph nd_graph;
typedef struct nd_server nd_server;

/* Per-sweep report handed to nd_opts.on_iter. */
typedef struct {
  int32_t iter;           /* sweep number t >= 1; tau_dev holds tau_t */
  int64_t evaluated;      /* r-cliques whose h-index was computed */
  int64_t changed;        /* r-cliques whose value changed in this sweep */
  int64_t active_next;    /* active r-cliques (Section 4.3): those the
                             notifications flag for recomputation in the
                             next sweep (with use_frontier exactly the
                             next sweep's `evaluated`); -1 unless counted
                             (count_active or stop_active_ratio) */
  const int32_t *tau_dev; /* device pointer, valid only during the callback */
  double ms;              /* device time of the sweep */
} nd_iter_info;

/* Return nonzero to stop the iteration after this sweep (the call then
 * returns ND_ERR_NOT_CONVERGED unless the sweep changed nothing). */
typedef int (*nd_iter_cb)(void *user, const nd_iter_info *info);

typedef struct {
  nd_mode mode;
  int32_t max_iters;        /* sweep limit; < 0: run until a sweep changes
                               nothing */
  int32_t use_frontier;     /* 1: recompute only r-cliques notified by a
                               changed neighbour (Section 4.3); results are
                               identical */
  double stop_active_ratio; /* > 0: stop after the first sweep t whose
                               active_next / |R| falls below this ratio
                               (the indicator of Section 5.1.4); the
                               result is then tau_t, an upper bound on
                               kappa_s.  Implies count_active */
  int32_t snapshot_every;   /* on_iter sees every this-many-th sweep (and
                               the last one); <= 1: every sweep */
  int32_t count_active;     /* 1: count active_next after every sweep.
                               Notifications then run from the first sweep
                               (written and counted but not used to skip
                               work when use_frontier is 0); one extra pass
                               over |R| flag bytes per sweep */
  nd_iter_cb on_iter;       /* optional per-sweep callback (snapshots) */
  void *user;
} nd_opts;

/* Defaults: ND_SND, max_iters -1, no frontier, exact, snapshot_every 1, no
 * active counting, no callback. */
void nd_opts_init(nd_opts *opts);

typedef struct {
  int32_t sweeps;      /* sweeps run, the last being the one that observed
                          no change when converged */
  int32_t converged;   /* 1 when the last sweep changed nothing */
  int64_t n_rcliques;  /* |R| */
  int64_t n_incidence; /* P = sum over R of d_s(R) */
  int64_t updates;     /* h-index evaluations summed over sweeps (r-cliques
                          with d_s = 0 are exact from the start and are not
                          evaluated) */
  double ms_prep;      /* device time of prepare work done by this call */
  double ms_iterate;   /* device time of the sweeps */
  int32_t max_sdegree; /* max over R of d_s(R) */
  int32_t tau_bytes;   /* bytes per stored tau value: for one graph 1 when
                          every d_s is below 256, 2 below 32768, else 4;
                          in batches and the server 2 or 4 */
} nd_result;

/* ------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the library may hold for this context (0 = no cap beyond the
 * device).  On success *out owns the context. */
nd_status nd_ctx_create(int device, size_t hbm_budget_bytes, nd_ctx **out);
/* Destroy a context; its graphs and servers must be destroyed first. */
void nd_ctx_destroy(nd_ctx *ctx);
/* Device bytes currently held for graphs of this context (incl. cache). */
size_t nd_ctx_bytes_in_use(const nd_ctx *ctx);

/* --------------------------------------------------------------- graph */

/* Graph from m raw undirected pairs (src[i], dst[i]) on vertices 0..n-1
 * (Section 2: the graph is simple and undirected).  Self-loops are dropped
 * and repeated pairs merged, on the device.  ND_ERR_INVALID if n < 0, m < 0
 * or an endpoint is outside [0,n). */
nd_status nd_graph_from_edges(nd_ctx *ctx, int32_t n, int64_t m,
                              const int32_t *src, const int32_t *dst,
                              int on_device, void *stream, nd_graph **out);

/* count graphs at once, graph i as nd_graph_from_edges(ctx, n[i], m[i],
 * src[i], dst[i], on_device, ...) would build it, on host threads (two by
 * default) with a stream each, ordered after `stream`; their short,
 * launch-bound build phases overlap.  out[i] receives graph i.  On any
 * failure (the first is returned) no graph is kept and every out[i] is
 * NULL. */
nd_status nd_graphs_from_edges(nd_ctx *ctx, int32_t count, const int32_t *n,
                               const int64_t *m, const int32_t *const *src,
                               const int32_t *const *dst, int on_device,
                               void *stream, nd_graph **out);

/* Graph from a canonical CSR: row_off[n+1] (row_off[0] = 0, non-decreasing,
 * row_off[n] = nnz) and col[nnz], each list strictly ascending, no self-loop,
 * symmetric (v in N(u) iff u in N(v)).  Checked on the device;
 * ND_ERR_INVALID if any condition fails. */
nd_status nd_graph_from_csr(nd_ctx *ctx, int32_t n, int64_t nnz,
                            const int64_t *row_off, const int32_t *col,
                            int on_device, void *stream, nd_graph **out);

void nd_graph_destroy(nd_graph *g);

/* Vertex count and stored adjacency entries (2|E|) of the simple graph. */
nd_status nd_graph_dims(const nd_graph *g, int32_t *n, int64_t *nnz);

/* Copy out the canonical CSR: row_off[n+1], col[nnz]. */
nd_status nd_graph_csr(nd_graph *g, int64_t *row_off, int32_t *col,
                       int on_device, void *stream);

/* Build the r-clique list, the s-clique incidence lists and d_s for `kind`
 * (idempotent).  For each r-clique R the incidence list holds, for every
 * s-clique S containing R, the ids of the C(s,r)-1 other r-cliques of S
 * (Defn. of U, step 1); the paper finds these on the fly (Section 5), this
 * library stores them once.  Called implicitly by nd_decompose. */
nd_status nd_prepare(nd_graph *g, nd_kind kind, void *stream);

/* Prepare `count` graphs of one context for `kind`, like nd_prepare on each,
 * on host threads (two by default) with a stream each (ordered after `stream`,
 * which waits for all of them on return), largest graphs first, so that
 * their short, launch-bound build phases overlap.  Graphs already prepared
 * are skipped.  The first failure is returned; graphs prepared before it
 * stay prepared. */
nd_status nd_prepare_many(nd_ctx *ctx, int32_t count, nd_graph *const *graphs,
                          nd_kind kind, void *stream);

/* Sizes for `kind`: |R|, P = sum_R d_s(R), and the device bytes the graph
 * holds after preparing it.  Prepares the graph if needed, except when only
 * |R| is asked for (n_incidence and dev_bytes NULL) and it follows from the
 * graph itself: the vertex count for r = 1, the edge count for r = 2. */
nd_status nd_sizes(nd_graph *g, nd_kind kind, int64_t *n_rcliques,
                   int64_t *n_incidence, size_t *dev_bytes);

/* Copy out the r-clique list: verts[i*r + j] = j-th smallest vertex of
 * r-clique i (r = 1, 2, 3, 1, 2 for the five kinds), lexicographic order. */
nd_status nd_rcliques(nd_graph *g, nd_kind kind, int32_t *verts, int on_device,
                      void *stream);

/* Copy out the incidence lists: off[|R|+1] (in s-cliques, int64) and
 * ids[k * P] with k = C(s,r)-1, the k ids of each s-clique consecutive.
 * Within a list the s-cliques are ordered by their vertex outside R; the
 * exact order is an implementation detail (compare as sets). */
nd_status nd_incidence(nd_graph *g, nd_kind kind, int64_t *off, int32_t *ids,
                       int on_device, void *stream);

/* S-degrees d_s = tau_0 (Alg. 2, initialisation). */
nd_status nd_sdegree(nd_graph *g, nd_kind kind, int32_t *ds, int on_device,
                     void *stream);

/* --------------------------------------------------------- decompose */

/* Run SND or AND from tau_0 = d_s until a sweep changes nothing (or a stop
 * condition in opts) and write kappa[|R|] (int32).  opts may be NULL
 * (defaults).  res may be NULL.  On ND_ERR_NOT_CONVERGED kappa holds the
 * last iterate, an upper bound on kappa_s (Theorem 1). */
nd_status nd_decompose(nd_graph *g, nd_kind kind, const nd_opts *opts,
                       int32_t *kappa, int on_device, void *stream,
                       nd_result *res);

/* nd_decompose for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same contract and results as nd_decompose, except:
 *   - the graph must already be prepared for `kind` (nd_prepare, or any
 *     earlier call that prepared it); otherwise ND_ERR_INVALID;
 *   - every buffer of the iteration (tau buffers, notification flags, sweep
 *     counters, the snapshot handed to on_iter, and the staging of kappa
 *     when it goes to host memory) lives in one static device workspace of
 *     ND_NOALLOC_WORKSPACE_BYTES, reserved on a device when the first
 *     context is created there and held until the process ends.  It needs
 *     about (2b + 2)|R| bytes for SND with notifications (b = bytes per tau,
 *     nd_result.tau_bytes; b|R| fewer for AND, 2|R| fewer without flags),
 *     plus 4|R| with on_iter and 4|R| for a host kappa; a decomposition
 *     that does not fit fails with ND_ERR_OOM before running anything;
 *   - the call allocates no device or host memory.
 * Every call on a device shares that device's workspace, whose contents
 * persist between calls: calls that overlap in time on one device (other
 * threads, other streams) race and give undefined results. */
#define ND_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)
nd_status nd_decompose_noalloc(nd_graph *g, nd_kind kind, const nd_opts *opts,
                               int32_t *kappa, int on_device, void *stream,
                               nd_result *res);

/* Apply the update operator once: tau_out = U tau_in (Section 3, Defn. of U),
 * for an arbitrary tau_in[|R|] with 0 <= tau_in <= d_s (values above d_s are
 * rejected).  Both arrays device or both host per on_device. */
nd_status nd_update(nd_graph *g, nd_kind kind, const int32_t *tau_in,
                    int32_t *tau_out, int on_device, void *stream);

/* PartialAND (Section 4.3, end): AND sweeps that recompute only the
 * r-cliques listed in ids[count] (original ids; repeats allowed), every other
 * r-clique keeping tau_0 = d_s, until a sweep changes none of them (or
 * opts->max_iters sweeps; opts may be NULL).  out[i] receives the final
 * value of ids[i].  The limit is the largest fixed point, below d_s, of the
 * update operator restricted to the set -- the same for any sweep order --
 * and an upper bound on kappa_s there.  ids and out: device pointers if
 * on_device, else host.  opts->mode and use_frontier are ignored (AND, no
 * notifications); stop_active_ratio must be 0 (ND_ERR_UNSUPPORTED).  ND_ERR_INVALID for an id outside [0, |R|);
 * ND_ERR_NOT_CONVERGED (out then holds the current values) when max_iters
 * stopped it.  res (may be NULL): sweeps, and updates = members x sweeps. */
nd_status nd_partial_and(nd_graph *g, nd_kind kind, const int32_t *ids,
                         int64_t count, const nd_opts *opts, int32_t *out,
                         int on_device, void *stream, nd_result *res);

/* Ego-network estimates (the application of PartialAND in Section 5.3): for
 * every query r-clique q = queries[i] (original ids), PartialAND on
 * P(q) = {q} and every r-clique sharing an s-clique with q -- for k-core q
 * and its neighbours, for k-truss q and the other edges of its triangles --
 * each query independently; est[i] = q's resulting value (an upper bound on
 * kappa_s(q), usually equal), sweeps[i] (sweeps may be NULL) the sweeps it
 * took.  max_iters < 0: until convergence.  All queries whose P(q) has at
 * most 4096 r-cliques run in one launch, a workgroup each; larger ones run
 * one at a time as nd_partial_and.  Pointers are device pointers if
 * on_device, else host.  ND_ERR_INVALID for a query outside [0, |R|);
 * ND_ERR_NOT_CONVERGED if some query hit max_iters. */
nd_status nd_ego_estimate(nd_graph *g, nd_kind kind, const int32_t *queries,
                          int64_t count, int32_t max_iters, int32_t *est,
                          int32_t *sweeps, int on_device, void *stream);

/* Degree levels (Defn. 4): level[R] = i for every r-clique R of L_i, in
 * r-clique id order (device pointer if on_device, else host; |R| entries);
 * *num_levels (host) = the number of non-empty levels, which bounds the SND
 * sweeps (the level-i r-cliques are exact after i sweeps; the DL row of
 * Table 3).  L_0 = r-cliques of minimum S-degree; removing an r-clique
 * removes every s-clique containing it; L_i = the minimum-degree r-cliques
 * of what remains.  One workgroup runs the levels in turn; a level with
 * many candidate r-cliques runs on the whole GPU instead (four kernels and
 * a 64-byte read-back). */
nd_status nd_levels(nd_graph *g, nd_kind kind, int32_t *level,
                    int32_t *num_levels, int on_device, void *stream);

/* Decompose `count` graphs together: their r-cliques form one combined work
 * list swept by each launch; a graph stops being swept once one of its sweeps
 * changes nothing.  Graphs not yet prepared are prepared as by
 * nd_prepare_many while those already prepared are being swept, each joining
 * the sweeps as soon as it is ready (graphs needing 32-bit tau are swept in
 * a second combined list).  kappas[i] receives graph i's result (device
 * pointers if on_device), res[i] its statistics (res may be NULL; its
 * ms_iterate is the time of the whole call).  Results equal those of
 * nd_decompose on each graph alone.  opts: mode, max_iters and use_frontier
 * apply to every graph; on_iter and stop_active_ratio give
 * ND_ERR_UNSUPPORTED. */
nd_status nd_batch_decompose(nd_ctx *ctx, int32_t count,
                             nd_graph *const *graphs, nd_kind kind,
                             const nd_opts *opts, int32_t *const *kappas,
                             int on_device, void *stream, nd_result *res);

/* ------------------------------------------------------------ serving */

/* A server serves decomposition requests with continuous batching (the
 * batching of nd_batch_decompose, kept running).  It owns six host threads,
 * each with its own stream.  Four preparation threads build admitted
 * requests' r-cliques and incidence lists (nd_prepare's work) while a slot
 * (max_slots) is free and the device memory fits the context budget -- the
 * lists are allocated at their exact size from the count pass.  A build
 * starts beside others only while the free budget holds twice the largest
 * graph built so far for each of them.  A request that does not fit
 * releases what it built and is retried with no other build running, then
 * waits for a running request to retire, and fails with ND_ERR_OOM if
 * nothing else holds memory.  Two worker threads, one for small requests
 * (fewer than 2^20 incidence entries) and one for the rest, add prepared
 * requests to the running batch of their class, kind and options and keep
 * sweeping, so requests that arrive while others are on the GPU join them
 * without stopping the sweeps, and small ones do not wait at every sweep for
 * the long sweeps of large ones.  A request retires when it converges, hits
 * max_iters or is cancelled, freeing its slot and its device memory.
 * max_queue bounds the requests waiting for a slot. */
nd_status nd_server_create(nd_ctx *ctx, int32_t max_slots, int32_t max_queue,
                           nd_server **out);

/* Submit g for decomposition of `kind`: the server takes ownership of g
 * (destroyed when the request ends) and does nothing with it on the calling
 * thread.  opts: mode, max_iters and use_frontier (NULL: defaults); the
 * other options give ND_ERR_UNSUPPORTED.  ND_ERR_BUSY when max_queue
 * requests are waiting. */
nd_status nd_server_submit(nd_server *srv, nd_graph *g, nd_kind kind,
                           const nd_opts *opts, uint64_t *ticket);

/* How a served request went (nd_server_wait). */
typedef struct {
  double latency_ms;          /* submission to completion (host clock) */
  double prep_ms;             /* host time spent preparing it */
  int64_t epochs_during_prep; /* sweep epochs the server ran, over all
                                 batches, while it was being prepared */
  int64_t epoch_joined;       /* its batch's epoch count when it joined */
  int64_t epoch_done;         /* the same after its last sweep */
  int32_t joined_running;     /* 1: its batch was already sweeping another
                                 request when it joined */
  int32_t peak_members;       /* most requests of its batch swept together
                                 in one epoch chunk while it ran */
} nd_serve_info;

/* Wait up to timeout_us (< 0: forever) for a request and return its final
 * status (ND_ERR_TIMEOUT if still running: call again).  res and info
 * (either may be NULL) receive its statistics.  After ND_OK or
 * ND_ERR_NOT_CONVERGED the result (res->n_rcliques values) is kept until
 * nd_server_result collects it; after any other status the request is gone. */
nd_status nd_server_wait(nd_server *srv, uint64_t ticket, int64_t timeout_us,
                         nd_result *res, nd_serve_info *info);

/* Copy a finished request's kappa into host buffer kappa[capacity] (in
 * r-clique id order; ND_ERR_INVALID if capacity < n_rcliques) and release
 * the request.  kappa = NULL only releases it. */
nd_status nd_server_result(nd_server *srv, uint64_t ticket, int32_t *kappa,
                           int64_t capacity);

/* Cancel a waiting or running request; its wait returns ND_ERR_CANCELLED. */
nd_status nd_server_cancel(nd_server *srv, uint64_t ticket);

/* Stop both threads, cancel what is left, free everything. */
void nd_server_destroy(nd_server *srv);

/* --------------------------------------------------------------- errors */

const char *nd_status_str(nd_status s);
const char *nd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ND_H */
