/*
 * cos.h -- C ABI of the leveled-DAG diagram-summation library for AMD Instinct
 * MI355X (gfx950).
 *
 * The operation (paper Sec. II.B, caption of Fig. combinedgraphflat): a
 * directed graph whose nodes sit on levels l = 0..L, with a single root on
 * level 0 and a single final node on level L, and edges only from level l-1 to
 * level l.  The root holds 1; each edge multiplies the value at its source by
 * its edge factor and adds the product into its destination; the final node
 * then holds the sum, over every root-to-final path, of the product of the
 * path's edge factors (one path = one diagram).  Levels are evaluated in order,
 * each completely before the next (Sec. II.C, "Windowing"), and many sample
 * points (configurations) are evaluated at once (Sec. II.C, "Distributing the
 * task on a grid of blocks").
 *
 * The graph is given in the flattened form of Fig. combinedgraphflat: per edge
 * level, node-agnostic arrays of (src, dst) pairs.  Two kinds of edge factor:
 * the closed-form stand-in
 *       w_e(x) = a_e / (1 + b_e * |x - k_e|^2),    x, k_e in R^3,
 * for the Green's function an edge carries in the paper (cos_create_graph),
 * and the paper's own form, a per-sample table entry times a constant,
 *       w_e(s) = c_e * T_s[slot_e]              (cos_create_graph_lookup).
 *
 * Conventions for every entry point:
 *  - Every call returns a cos_status.  On failure cos_last_error() returns a
 *    message for the calling thread; outputs are then undefined and no handle
 *    is produced.  No C++ exception crosses this boundary.
 *  - "host" pointers are read during the call only and stay owned by the
 *    caller.  "device" pointers are HIP device allocations owned by the
 *    caller, which keeps them alive until the work queued on `stream` ends.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is queued on it asynchronously, in stream order.
 *  - Results are deterministic: the same graph, samples and precision give
 *    bit-identical outputs on every call (no floating-point atomics).
 */
#ifndef COS_H
#define COS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COS_ABI_VERSION 4

typedef enum cos_status {
    COS_OK = 0,
    COS_EINVAL = -1,    /* malformed graph, sizes or pointers */
    COS_ENOMEM = -2,    /* host or device allocation failed, or a request can never fit */
    COS_EDEVICE = -3,   /* a HIP runtime call or kernel launch failed */
    COS_EAGAIN = -4,    /* serving: request not finished yet */
    COS_ECANCELED = -5  /* serving: request was cancelled */
} cos_status;

typedef enum cos_precision {
    /* binary64 node values and edge factors at every level */
    COS_FP64 = 0,
    /* binary32 node values and factors on interior levels with a power-of-two
       rescale per (level, sample); binary64 final-node reduction and exponent
       bookkeeping.  Single precision is the paper's own mode (Sec. III,
       "Numerical stability"); the rescale is this library's addition. */
    COS_FP32_RESCALED = 1,
    /* as COS_FP32_RESCALED without the rescale (the paper's plain FP32) */
    COS_FP32 = 2,
    /* as COS_FP32_RESCALED, with the interior level values stored in IEEE
       binary16 (half the level bytes; arithmetic stays binary32).  The
       per-(level, sample) shift also carries a per-level headroom 2^h computed
       at graph creation from the largest row sum of |a_e|, so that no stored
       value can exceed the binary16 range.  Rational factors only (lookup
       factors have no such bound: COS_EINVAL), streamed and panel plans.  Storage
       rounding makes it less accurate than binary32 (relative rounding 2^-11
       per stored level; the paper's Sec. IV suggests trading precision for
       speed in this direction). */
    COS_FP16_RESCALED = 3,
    /* the same with bfloat16 storage (relative rounding 2^-8 per stored
       level, binary32's exponent range, no headroom needed); both factor
       kinds, streamed and panel plans. */
    COS_BF16_RESCALED = 4
} cos_precision;

typedef struct cos_graph cos_graph;

/* Kernel plan of cos_evaluate (see cos_graph_set_path). */
typedef enum cos_path {
    COS_PATH_AUTO = 0,     /* fused when the widest level fits in LDS, else panel where it applies,
                              else streamed */
    COS_PATH_STREAMED = 1, /* one launch per level, level values streamed through HBM */
    COS_PATH_FUSED = 2,    /* one launch for the whole graph, level values held in LDS */
    COS_PATH_PANEL = 3     /* streamed, binary32 and 16-bit storage precisions of wide graphs (lookup
                              factors: binary32): row panels with their edge records in LDS swept over
                              narrow sample tiles */
} cos_path;

typedef struct cos_graph_info {
    int32_t L;               /* number of edge levels (node levels 0..L) */
    int32_t fused_mask;      /* bit p set: the fused plan fits for cos_precision p */
    int64_t n_nodes;         /* sum of widths; the final node id is n_nodes - 1 */
    int64_t n_edges;
    int64_t max_width;       /* widest interior level (0 when L == 1) */
    int64_t max_in_degree;   /* over interior levels 1..L-1 */
    int64_t final_in_degree; /* in-edges of the final node */
    uint64_t device_bytes;   /* device memory held by the graph */
    int32_t factor_kind;     /* COS_FACTOR_RATIONAL or COS_FACTOR_LOOKUP */
    int32_t n_inputs;        /* rows of the per-sample input x_dev: 3, or n_slots */
    int32_t panel_mask;      /* bit p set: the panel plan applies for cos_precision p */
    int32_t reserved;
} cos_graph_info;

/* Edge-factor kinds. */
#define COS_FACTOR_RATIONAL 0 /* w_e(x) = a_e / (1 + b_e |x - k_e|^2), x the sample's point in R^3 */
#define COS_FACTOR_LOOKUP 1   /* w_e(s) = c_e * T_s[slot_e], T_s the sample's table */

/* Message for the last failed call on this thread ("" if none).  Owned by the
   library; valid until the thread's next call. */
const char *cos_last_error(void);

/* Hash of the sources the library was built from (NUL-terminated, static). */
const char *cos_build_id(void);

/* COS_ABI_VERSION of the built library. */
int32_t cos_abi_version(void);

/*
 * Build a device-resident graph from flattened per-level edge lists
 * (Sec. II.C "Graph flattening", Fig. combinedgraphflat).  The graph is built
 * once and evaluated many times (Sec. II.B: a graph is constructed once
 * before any calculation).
 *
 *   L                 number of edge levels, >= 1
 *   widths   host     int64[L+1]; widths[0] = widths[L] = 1, all >= 1,
 *                     sum < 2^31.  Node ids are global and contiguous level
 *                     by level: level l holds ids off_l .. off_l + widths[l]-1.
 *   edges_per_level   host int64[L]; entry l-1 counts the edges into level l
 *                     (an edge level is named by its destination level).
 *   src, dst host     int32[E], E = sum(edges_per_level), level-major: the
 *                     edges of level 1 first.  src must lie in level l-1 and
 *                     dst in level l.  Any order within a level; parallel
 *                     edges are separate terms; nodes without in-edges hold 0.
 *   a, b     host     float64[E]: finite, b >= 0 (b = 0 gives w = a).
 *   k        host     float64[E][3], finite; 1 + b|k|^2 and 2b|k_i| must be
 *                     finite in binary64 (the library evaluates the
 *                     denominator in the expanded form c0 + b|x|^2 + g.x).
 *   out               receives the handle; release with cos_destroy_graph.
 *
 * The inputs are copied; the caller may free them on return.  Within each
 * level the library stores edges in canonical order: by destination, then
 * source, then the bit patterns of (a, b, k0, k1, k2), so every permutation of
 * the same edge set yields the same device graph and bit-identical results.
 * Errors: COS_EINVAL (validation), COS_ENOMEM, COS_EDEVICE.
 */
cos_status cos_create_graph(int32_t L, const int64_t *widths, const int64_t *edges_per_level,
                            const int32_t *src, const int32_t *dst, const double *a,
                            const double *b, const double *k, cos_graph **out);

/*
 * Build a graph whose edge factors are table lookups, the paper's own form
 * (Sec. II.B: each edge multiplies by the Green's function G_ab between two of
 * the configuration's vertices; Sec. III: per edge the tail value, that Green's
 * function and a -1 when the edge closes a fermion loop).  Edge e multiplies
 * its source value by coef[e] * T_s[slot[e]], where T_s is sample s's table of
 * n_slots values given to cos_evaluate (slot = the vertex pair, coef = the
 * sign or any other finite constant).
 *
 *   L, widths, edges_per_level, src, dst   as for cos_create_graph.
 *   slot     host     int32[E], each in 0 .. n_slots-1.
 *   coef     host     float64[E], finite.
 *   n_slots           >= 1: entries of every sample's table.
 *
 * Copied like cos_create_graph; canonical order by destination, source, slot,
 * then the bit pattern of coef.  Errors: COS_EINVAL, COS_ENOMEM, COS_EDEVICE.
 */
cos_status cos_create_graph_lookup(int32_t L, const int64_t *widths, const int64_t *edges_per_level,
                                   const int32_t *src, const int32_t *dst, const int32_t *slot,
                                   const double *coef, int32_t n_slots, cos_graph **out);

/* Sizes of a graph (see cos_graph_info).  Errors: COS_EINVAL on NULL. */
cos_status cos_graph_get_info(const cos_graph *g, cos_graph_info *info);

/*
 * Choose the kernel plan later cos_evaluate calls on this graph use.  Both
 * plans compute the same arithmetic in the same order and give bit-identical
 * results; the choice only moves the level values between HBM (streamed) and
 * LDS (fused, for graphs whose widest level fits on chip -- the paper's small
 * low-order graphs, Sec. III).  COS_PATH_FUSED on a graph or precision it does
 * not fit makes cos_evaluate fail with COS_EINVAL.  Not thread-safe with
 * respect to concurrent cos_evaluate calls on the same graph.
 * Errors: COS_EINVAL (NULL graph, unknown path).
 */
cos_status cos_graph_set_path(cos_graph *g, cos_path path);

/*
 * Copy the graph's edges back to host arrays of E entries (k: E*3), in the
 * canonical order described at cos_create_graph, with global node ids.
 * Errors: COS_EINVAL on NULL.
 */
cos_status cos_graph_export(const cos_graph *g, int32_t *src, int32_t *dst, double *a, double *b,
                            double *k);

/* The same for a lookup graph: slot int32[E], coef float64[E].  COS_EINVAL for
   a graph with rational factors (and cos_graph_export on a lookup graph). */
cos_status cos_graph_export_lookup(const cos_graph *g, int32_t *src, int32_t *dst, int32_t *slot,
                                   double *coef);

/*
 * Device scratch bytes cos_evaluate needs for S samples at precision p
 * (level buffers, exponent rows and final-node partial sums; for the binary32
 * precisions of a lookup graph also a binary32 copy of the sample tables).
 * Errors: COS_EINVAL.
 */
cos_status cos_evaluate_workspace_size(const cos_graph *g, int64_t S, cos_precision p,
                                       uint64_t *bytes);

/*
 * Evaluate the final-node value for S sample points (Sec. II.B; many
 * configurations at once as in Sec. II.C).
 *
 *   x_dev        device float64[R][S], the per-sample inputs as structure of
 *                arrays: x_dev[c*S + s] is row c of sample s.  R = 3 for
 *                rational factors (the sample's coordinates), R = n_slots for
 *                lookup factors (the sample's table T_s).
 *   S            >= 0 (0: nothing is queued).
 *   p            a cos_precision.  COS_FP16_RESCALED needs rational
 *                factors whose largest level row sum of |a_e| is below 2^110.
 *   out_dev      device float64[S].  Without out_exp_dev: the value V(x_s).
 *   out_exp_dev  device int32[S] or NULL.  When given, the result is returned
 *                as out_dev[s] * 2^out_exp_dev[s] (for values whose magnitude
 *                may leave the binary64 range); always 0 for COS_FP64.
 *   workspace_dev, workspace_bytes
 *                device scratch, 256-byte aligned, used only by work queued
 *                on `stream`: cos_evaluate_workspace_size bytes, or on the
 *                streamed plan less (room for at least 256 samples), in which
 *                case the sweep runs in sample chunks that fit it (the same
 *                results).  NULL: the library allocates and frees it in
 *                stream order (hipMallocAsync / hipFreeAsync).
 *   stream       hipStream_t as void*.
 *
 * Asynchronous: returns once the work is queued.  With a workspace it queues
 * kernel launches only (no allocation, no memset), so it may be captured into
 * a HIP graph on `stream` and replayed; replays read x and write out afresh.
 * Errors: COS_EINVAL (NULL or misaligned pointers, bad S or precision,
 * workspace too small, a binary32 precision for a graph with a parameter
 * (a, b, k or coef) that rounds to infinity in binary32), COS_ENOMEM,
 * COS_EDEVICE (launch failure).
 */
cos_status cos_evaluate(const cos_graph *g, const double *x_dev, int64_t S, cos_precision p,
                        double *out_dev, int32_t *out_exp_dev, void *workspace_dev,
                        uint64_t workspace_bytes, void *stream);

/* Bytes of the fixed device workspace of cos_evaluate_no_alloc (64 MiB). */
#define COS_NO_ALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * cos_evaluate for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same evaluation, arguments and results as cos_evaluate, with the workspace
 * taken from a fixed array of COS_NO_ALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine) and queues
 * kernel launches only.
 *
 * A streamed-plan sweep that needs more than the array holds runs in sample
 * chunks that fit it (the same results).  A graph whose plan does not fit at
 * all -- a fused plan needing more, or fewer than 256 samples per chunk
 * fitting -- is refused with COS_EINVAL and a message naming both sizes.
 *
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (other streams, other threads)
 * race and give undefined results; serialise them.  The first call on a
 * device looks up the array's device address (thread-safe).
 * Errors: those of cos_evaluate, and COS_EDEVICE if the array's address cannot
 * be obtained.
 */
cos_status cos_evaluate_no_alloc(const cos_graph *g, const double *x_dev, int64_t S, cos_precision p,
                                 double *out_dev, int32_t *out_exp_dev, void *stream);

/* Release a graph and its device memory.  Must not race with queued work that
   reads it.  NULL is a no-op.  Errors: COS_EDEVICE if hipFree fails. */
cos_status cos_destroy_graph(cos_graph *g);

/* ------------------------------------------------------------- Monte Carlo
 *
 * Markov-chain walkers over sample configurations: the integration over the
 * vertex coordinates by Monte Carlo sampling (Sec. II.B), with the walkers'
 * configurations evaluated together as the samples of one sweep (Sec. II.C,
 * "Distributing the task on a grid of blocks") and proposal and acceptance
 * done on the device (Sec. IV).  Walker c holds x_c (a column of x_dev) and
 * v_c = V(x_c).  One step t of every walker:
 *
 *   r_0..r_3 = Philox4x64-10 (Salmon et al., SC'11), counter (c, t, 0, 0),
 *              key (seed, 0);  u_i = (r_i >> 11) * 2^-53
 *   x'_i     = x_i + sigma * (2 u_i - 1), i < 3 (product and sum each rounded)
 *   v'       = V(x') at precision p (the level sweep of cos_evaluate)
 *   accept iff u_3 * |v| < |v'|   (Metropolis for the density |V|)
 *   then at the walker's state: acc[0][c] += sign(v), acc[1][c] += |x|^2
 *   (x0 x0 + x1 x1 + x2 x2, left to right), accepted[c] += 1 if accepted.
 *
 * The average of acc[0] over walkers and steps estimates int V / int |V|.
 * Random numbers depend on (seed, c, t) only: splitting a run into calls
 * (step0 = steps already done) or running a subset of walkers gives the same
 * bits.
 */

/* Device scratch bytes cos_mc_run needs for C walkers at precision p (the
   proposals, their values and the sweep's workspace).  Errors: COS_EINVAL. */
cos_status cos_mc_workspace_size(const cos_graph *g, int64_t C, cos_precision p, uint64_t *bytes);

/*
 * Run steps step0 .. step0 + n_steps - 1 of C walkers on a graph with
 * rational factors.
 *
 *   x_dev         device float64[3][C], in/out: the walkers' coordinates.
 *   v_dev         device float64[C], in/out: V(x) of each walker at precision
 *                 p (the caller evaluates the starting points with
 *                 cos_evaluate; the run keeps it current).
 *   accepted_dev  device int64[C], in/out: accepted proposals (added to).
 *   acc_dev       device float64[2][C], in/out: sums of sign(v) and |x|^2
 *                 over the steps (added to).
 *   seed, sigma   generator key; proposal half-width (finite, >= 0).
 *   workspace_dev, workspace_bytes
 *                 at least cos_mc_workspace_size bytes, 256-byte aligned; NULL:
 *                 allocated and freed in stream order.
 *
 * Asynchronous on `stream`.  A graph on the fused plan (see cos_graph_set_path)
 * runs the whole call in one launch; others take a propose launch, a sweep and
 * an accept launch per step; both give the same bits.  Errors: COS_EINVAL (NULL pointers, C outside 1..2^31,
 * negative step0 or n_steps, bad sigma, lookup factors, a precision or plan
 * the graph refuses, small or misaligned workspace), COS_ENOMEM, COS_EDEVICE.
 * On error the walkers' state is unspecified.
 */
cos_status cos_mc_run(const cos_graph *g, cos_precision p, int64_t C, double *x_dev, double *v_dev,
                      int64_t step0, int64_t n_steps, uint64_t seed, double sigma, int64_t *accepted_dev,
                      double *acc_dev, void *workspace_dev, uint64_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ serving
 *
 * A server evaluates requests (graph, samples, precision) submitted at any
 * time against graphs that stay resident on the device -- the paper's picture
 * of thousands of configurations in flight (Sec. II.C, Sec. III) applied to a
 * stream of requests.  Requests are admitted while a slot is free and their
 * device workspace fits in an HBM budget; every admitted request advances by
 * one stage per step, where a step is one level-synchronous launch shared by
 * all admitted requests (replayed from an instantiated HIP graph): a graph whose
 * widest level fits in LDS completes in one step, a wider graph advances one
 * level per step, then its final node in two more (a lookup request at a
 * binary32 precision first takes one step to copy its tables to binary32,
 * as cos_evaluate does).  Requests that arrive while
 * others run join the next step (continuous batching).  Each result is
 * bit-identical to cos_evaluate on the same graph, samples and precision.
 */
typedef struct cos_server cos_server;

typedef struct cos_req_stats {
    int64_t t_submit_ns;  /* steady-clock time stamps (ns); 0 when not reached */
    int64_t t_admit_ns;
    int64_t t_done_ns;
    int32_t status;       /* COS_OK done, COS_EAGAIN queued or running, COS_ECANCELED, or a failure */
    int32_t steps;        /* steps the request took part in */
    int64_t first_step;   /* index of its first step, -1 before admission */
    int64_t footprint;    /* device workspace bytes it holds while admitted */
} cos_req_stats;

/* One step of a server (the step trace).  With the requests' first_step and
   steps (one stage per step, in consecutive steps), it tells which stage of
   which request ran in which launch. */
typedef struct cos_step_record {
    int64_t step;          /* step index */
    int64_t t_launch_ns;   /* steady clock: the step graph was queued */
    int64_t t_done_ns;     /* steady clock: its completion callback ran */
    int32_t n_fused;       /* requests with whole-graph work in the step */
    int32_t n_streamed;    /* requests with a level, final-node or combine stage */
    int64_t items;         /* work items of the step */
} cos_step_record;

typedef struct cos_server_stats {
    int64_t submitted, completed, cancelled, failed;
    int64_t steps;              /* step launches */
    int64_t items;              /* work items over all steps */
    int64_t max_active;         /* most requests admitted at once */
    int64_t max_step_requests;  /* most requests sharing one step */
    uint64_t budget_bytes;      /* HBM budget for request workspaces */
    uint64_t peak_bytes;        /* largest sum of admitted workspaces */
} cos_server_stats;

/*
 * Create a server on the current device.  hbm_budget: bytes of device memory
 * the server allocates once and hands out as request workspaces (a graph whose
 * widest level fits in LDS needs none); max_slots: requests admitted at once,
 * 1..512.  Starts a scheduling thread.  Errors: COS_EINVAL, COS_ENOMEM,
 * COS_EDEVICE.
 */
cos_status cos_server_create(uint64_t hbm_budget, int32_t max_slots, cos_server **out);

/* Register a graph (it must outlive the server) and get its id.  Either
   factor kind: a request on a lookup graph passes its samples' tables as x
   ([n_slots][S], as cos_evaluate).  Errors: COS_EINVAL (NULL, graph on
   another device). */
cos_status cos_server_add_graph(cos_server *srv, const cos_graph *g, int32_t *gid);

/*
 * Queue a request: x_dev device float64[3][S], out_dev device float64[S],
 * out_exp_dev device int32[S] or NULL (as for cos_evaluate).  Every precision
 * is served; 16-bit storage runs on the streamed plan, with cos_evaluate's bits.
 * The caller keeps them alive until the request ends (poll/wait return a
 * final status).  Never blocks.  Errors: COS_EINVAL (unknown gid, S < 1, bad
 * precision or one cos_evaluate would refuse for this graph, S too large for
 * one sweep), COS_ENOMEM (the request's workspace exceeds the whole budget, so
 * it could never be admitted).
 */
cos_status cos_server_submit(cos_server *srv, int32_t gid, const double *x_dev, int64_t S, cos_precision p,
                             double *out_dev, int32_t *out_exp_dev, uint64_t *ticket);

/*
 * Status of a request.  Returns COS_EAGAIN while queued or running; once the
 * request has ended it returns its final status (COS_OK, COS_ECANCELED or the
 * failure), fills *stats (nullable) and forgets the ticket.
 * Errors: COS_EINVAL (unknown ticket).
 */
cos_status cos_server_poll(cos_server *srv, uint64_t ticket, cos_req_stats *stats);

/* As cos_server_poll, but blocks until the request has ended. */
cos_status cos_server_wait(cos_server *srv, uint64_t ticket, cos_req_stats *stats);

/* Cancel a request that has not been admitted yet.  Returns COS_OK, or
   COS_EAGAIN if it is already running (it will complete).  Errors: COS_EINVAL. */
cos_status cos_server_cancel(cos_server *srv, uint64_t ticket);

/* Counters of the server's lifetime.  Errors: COS_EINVAL on NULL. */
cos_status cos_server_get_stats(cos_server *srv, cos_server_stats *stats);

/*
 * Step trace: copy the records of completed steps not read before, oldest
 * first, up to cap of them, into out (host array); *n receives the count.
 * The server keeps the last 65536 unread records (older ones are dropped).
 * Errors: COS_EINVAL (NULL server or n, cap < 0, out NULL with cap > 0).
 */
cos_status cos_server_read_steps(cos_server *srv, cos_step_record *out, int64_t cap, int64_t *n);

/*
 * Failure handling.  A newly admitted request's set-up (its slot entry and
 * exponent rows, written on the device by the first step that includes it)
 * is prepared on the host; a request whose set-up fails ends alone with
 * COS_EDEVICE and its slot and workspace are returned, while the others go on.
 * A failed step launch fails every active request of the server.  For tests
 * of the per-request path without a device fault: make the set-up of the
 * admission with this index (0-based, in admission order; -1: none) fail.
 * Errors: COS_EINVAL (NULL server, index < -1).
 */
cos_status cos_server_fail_admission(cos_server *srv, int64_t admission_index);

/* Cancel queued requests, wait for admitted ones, stop the scheduling thread
   and free the server's device memory.  NULL is a no-op. */
cos_status cos_server_destroy(cos_server *srv);

/*
 * Kernel timing probe (for benchmarks).  While enabled, every kernel the
 * library queues is bracketed by a pair of HIP events recorded on the same
 * stream.  cos_timing_read waits for the recorded events, returns the summed
 * device time in milliseconds and the launch count for kernel class `kind`,
 * and clears that class's records.  Kinds: 0 interior level gather,
 * 1 fused multi-level (LDS-resident), 2 final-node partial sums,
 * 3 final-node combine, 4 scratch fills, 5 serving step, 6 chunk sums of
 * interior nodes of high in-degree.
 * Errors: COS_EINVAL (bad kind), COS_EDEVICE.
 */
cos_status cos_timing_enable(int32_t enable);
cos_status cos_timing_read(int32_t kind, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* COS_H */
