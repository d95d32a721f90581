/*
 * fork.h -- C ABI of the MI355X (gfx950) fork-processing library.
 *
 * A fork-processing pattern (FPP) launches many independent single-source
 * queries on one shared graph (Algorithm 1; Definition 2.2).  This library
 * runs them with the paper's buffered execution model (Section 3, Algorithm
 * 2): the graph is cut into partitions (Definition 2.1), each partition keeps a
 * buffer of pending operations <q, v, val> (Definition 2.3), and the
 * scheduler repeatedly picks partitions (Section 5.2) whose buffered queries
 * are then processed together, with yielding (Section 5.1), until every buffer
 * is empty.
 *
 * Conventions for every entry point:
 *   - Returns FORK_OK (0) or a negative fork_status.  No exception or abort
 *     crosses the ABI.  fork_last_error() gives a message for the last failing
 *     call on the calling thread.
 *   - Pointers are plain host pointers unless a flag says "device".  Input
 *     arrays are only borrowed for the duration of the call (copied).
 *   - The context owns all device memory it allocates until fork_destroy.
 *   - A context is not thread-safe: calls on one context must be serialised.
 */
#ifndef FORK_H
#define FORK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fork_ctx fork_ctx;

typedef enum {
    FORK_OK = 0,
    FORK_E_INVALID = -1,       /* bad argument; nothing changed              */
    FORK_E_NOMEM = -2,         /* device or host allocation failed           */
    FORK_E_DEVICE = -3,        /* HIP runtime error, or no usable GPU        */
    FORK_E_STATE = -4,         /* call not valid in the context's state      */
    FORK_E_CAPACITY = -5,      /* operation pool exhausted, or a visit over the
                                  frontier-spill bound (fork_stats_t.spill_max) */
    FORK_E_NOT_CONVERGED = -6  /* max_passes reached with work still pending */
} fork_status;

/* Query kinds (Section 3 lists the supported FPP queries). */
typedef enum { FORK_SSSP = 1, FORK_BFS = 2, FORK_PPR = 3 } fork_query_type;

/* Inter-partition scheduling policies (Section 5.2; the alternatives are the
 * ones compared in the paper's priority-functor study).  LEARNED replaces the
 * priority functor by an MLP score computed from buffer statistics. */
typedef enum {
    FORK_SCHED_FIFO = 0,      /* oldest pending operation first (paper default) */
    FORK_SCHED_PRIORITY = 1,  /* best buffered-operation priority first        */
    FORK_SCHED_LEARNED = 2,   /* MLP score over partition statistics           */
    FORK_SCHED_RANDOM = 3,    /* any partition with pending work               */
    FORK_SCHED_MAXOPS = 4     /* most buffered operations first                */
} fork_sched;

/* Graph-level configuration, fixed at fork_graph_load.  Zero = automatic. */
typedef struct {
    uint32_t partition_vertices; /* max vertices per partition (<= 65536)      */
    uint32_t partition_edges;    /* max out-edges per partition (edge balance) */
    uint32_t max_queries;        /* queries resident at once (a "wave")        */
    uint64_t pool_bytes;         /* device bytes for the operation pool        */
    int      inputs_on_device;   /* row_ptr/col/weight are device pointers     */
    int      device;             /* HIP device ordinal                          */
    const uint32_t *vertex_order;/* NULL, or uint32[num_vertices]: a permutation
                                    giving each vertex's position in the
                                    library's internal numbering.  Partitions
                                    are contiguous ranges of that numbering, so
                                    an order that keeps neighbours close (2D
                                    tiles of a grid, a space-filling curve of a
                                    road network) cuts fewer edges; the paper's
                                    partitioner study credits locality-aware
                                    partitions with large gains over random
                                    ones (Appendix C).  Sources, results and
                                    digests always use the caller's ids; only
                                    fork_partitions reports internal positions.
                                    Host memory, or device memory when
                                    inputs_on_device.  Not a permutation:
                                    FORK_E_INVALID.                            */
} fork_config;

/* PPR parameters (passed to fork_submit for FORK_PPR).  A vertex is pushed
 * while r[v] > 0 and r[v] >= thr(v), thr(v) = epsilon (eps_mode 0) or
 * epsilon * outdeg(v) (eps_mode 1).
 *
 * l1_target > 0 asks for a certified result: after the push terminates at
 * epsilon, the run lowers this query's threshold and pushes again (from every
 * vertex that then qualifies) until sum_v r[v] <= 0.9 * l1_target.  Forward
 * push keeps p + PPR(r) = PPR(e_s) (Section 4.1's push; the paper gives no
 * formula), and ||PPR(r)||_1 <= ||r||_1, so the returned p is then within
 * l1_target of the exact PPR vector in L1, the last tenth being left for
 * fp32 rounding.  The cost grows as the threshold falls; after 32 reductions
 * fork_run gives FORK_E_NOT_CONVERGED.  Certified queries need partitions of
 * at most 1,024 vertices (fork_config.partition_vertices <= 1024), so that a
 * refinement's re-activated vertices always fit the visit's frontier;
 * fork_run gives FORK_E_INVALID, and runs nothing, for larger partitions. */
typedef struct {
    float alpha;     /* teleport probability, in (0, 1)        */
    float epsilon;   /* push threshold, > 0                    */
    int   eps_mode;  /* 0 = absolute, 1 = degree-scaled        */
    float l1_target; /* 0 = off; else the certified L1 bound   */
} fork_ppr_params;

/* Execution engines (both run Algorithm 2 with the same scheduler):
 *   BUFFERED -- one work item per (partition, query): buffered operations are
 *               chunked lists of <v, val> per (partition, query), consumed into
 *               an LDS copy of the query's state slice (Sections 3-4 as in the
 *               paper, one query per workgroup).
 *   GROUPED  -- one work item per (partition, group of 64 queries of one
 *               type): the state is vertex-major per group (one 256-byte row
 *               per vertex, a lane per query), so a visit reads each out-edge
 *               once for 64 queries; pending operations are consolidated per
 *               (query, vertex) in the state rows (Section 4.2) and tracked by
 *               lane masks.  No certified PPR, traces or persistent kernel. */
enum { FORK_ENGINE_BUFFERED = 0, FORK_ENGINE_GROUPED = 1 };

/* Per-run options.  NULL = defaults (PRIORITY, automatic tuning, stream 0). */
typedef struct {
    int      scheduler;        /* fork_sched                                     */
    uint32_t parts_per_pass;   /* partitions processed per pass (0 = auto)       */
    uint32_t delta;            /* SSSP/BFS yield range Delta of heuristic 2 (0=auto) */
    float    edge_budget_mu;   /* yield after mu*|E_P|/|Q_P| edges (0 = off)     */
    uint64_t max_passes;       /* 0 = unlimited                                  */
    void    *stream;           /* hipStream_t to run on (NULL = default stream)  */
    const float *mlp_weights;  /* 5,313 fp32 (host), for FORK_SCHED_LEARNED      */
    int      persistent;       /* 1 = one persistent kernel with a device queue  */
    uint64_t seed;             /* for FORK_SCHED_RANDOM                          */
    int      profile;          /* 1 = time every pass kernel with HIP events     */
    uint32_t items_per_pass;   /* (partition, query) items queued per pass when
                                  parts_per_pass is 0 (0 = auto)                 */
    int      trace;            /* 1 = record scheduler traces (see fork_trace)   */
    int      window_mode;      /* heuristic 2 window: 0 = the query's best buffered
                                  value over all partitions (dist_min), 1 = the
                                  first value of each visit                     */
    uint32_t window;           /* SSSP batch width inside a visit: vertices with
                                  distance in [lo, lo + window) expand together
                                  (0 = auto)                                     */
    uint32_t slice_slots;      /* LDS copy of a visited partition's query state:
                                  0 = dense (one word per partition vertex);
                                  else a hash table of this many slots (a
                                  multiple of 256, 256..16384) holding only the vertices the
                                  visit touches, so more workgroups fit per CU;
                                  vertices that find no free slot are updated in
                                  place in global memory.  Partitions too large
                                  for the dense slice always use a hashed one
                                  (4096 slots when 0 is given)                    */
    int      engine;           /* FORK_ENGINE_BUFFERED (0) or FORK_ENGINE_GROUPED (1) */
    uint32_t group_threads;    /* grouped engine: threads of the workgroup that
                                  visits one (partition, group) pair: 256, 512
                                  or 1024 (0 = 256)                              */
} fork_run_opts;

/* Counters accumulated over the last fork_run (all waves). */
typedef struct {
    uint64_t passes;           /* scheduling steps                          */
    uint64_t work_items;       /* (partition, query) items processed        */
    uint64_t edges;            /* edges scanned (relaxations / edge pushes) */
    uint64_t improved;         /* state writes that improved a value        */
    uint64_t ops_emitted;      /* operations written to buffers             */
    uint64_t ops_consumed;     /* operations read from buffers              */
    uint64_t vertex_pushes;    /* PPR vertex pushes / SSSP vertex expansions*/
    uint64_t yields;           /* work items that yielded                   */
    uint64_t chunks;           /* pool chunks allocated                     */
    uint64_t waves;            /* query waves                               */
    double   init_ms;          /* state init + seeding, all waves           */
    double   run_ms;           /* buffered processing, all waves            */
    double   digest_ms;        /* digest computation                        */
    double   process_ms;       /* sum of pass-kernel durations (profile=1)  */
    uint64_t process_launches; /* pass kernels timed                        */
    uint64_t intra_edges;      /* edges whose target is in the same partition */
    uint64_t pruned;           /* operations not sent: target already as short */
    uint32_t num_partitions;
    uint32_t weight_bytes;     /* bytes per stored edge weight (0 = none)   */
    uint64_t refine_rounds;    /* certified-PPR threshold reductions, summed
                                  over waves                                */
    uint64_t selected_edges;   /* out-edges of the partitions scheduled, summed
                                  over passes (edge data staged per pass)   */
    uint64_t ppr_edges;        /* the PPR queries' share of `edges`          */
    uint64_t ppr_vertex_pushes;/* the PPR queries' share of `vertex_pushes`  */
    uint64_t spilled;          /* activated vertices retained as buffered
                                  operations because the visit's frontier
                                  was full                                  */
    uint64_t activations;      /* grouped engine: (vertex, group) pairs marked
                                  pending in another partition              */
    uint64_t expansions;       /* grouped engine: vertex expansions, each for
                                  one or more of its group's queries        */
    uint64_t spill_max;        /* most vertices one visit retained as
                                  operations (a visit retaining more than
                                  32,768 stops the run: FORK_E_CAPACITY)    */
    uint64_t rounds;           /* grouped engine: rounds of the visits (one
                                  round expands a set of pending vertices)  */
    uint64_t edge_tasks;       /* grouped engine: 64-edge tasks of the rounds*/
    uint64_t visit_ns[5];      /* grouped engine: workgroup time in the visit
                                  phases, summed over workgroups: [0] bitmap
                                  gather, [1] round take, [2] filter and edge
                                  numbering, [3] edge tasks, [4] yield      */
    double wall_ms;            /* host wall-clock time of the fork_run call */
    double setup_ms;           /* of which before the first wave's device work
                                  (planning, buffer reservation)            */
} fork_stats_t;

/* Per-query digest (fork_fetch field FORK_FIELD_DIGEST).  For SSSP/BFS:
 * count = reached vertices, sum = sum of finite values, hash = sum mod 2^64
 * over reached v of mix64(v * 2^32 + value) with mix64 the SplitMix64
 * finaliser.  For PPR: count = vertices with p > 0, fsum = sum of p,
 * fres = sum of r, fmax = max p. */
typedef struct {
    uint64_t count;
    uint64_t sum;
    uint64_t hash;
    double   fsum, fres, fmax;
} fork_digest;

enum {
    FORK_FIELD_VALUE = 0,  /* int32[V] distance or level                     */
    FORK_FIELD_P = 1,      /* float[V] PPR estimate p                        */
    FORK_FIELD_R = 2,      /* float[V] PPR residual r                        */
    FORK_FIELD_DIGEST = 3  /* fork_digest                                    */
};

/* Sweep cut of one PPR result (fork_sweep).  Sizes count swept vertices. */
#define FORK_SWEEP_MAX 1024
#define FORK_SWEEP_BUCKETS 11
typedef struct {
    uint32_t support;          /* vertices with p > 0 and d > 0                   */
    uint32_t swept;            /* prefixes evaluated: min(support, max_size)      */
    uint32_t best_size;        /* least-conductance prefix (0: none defined)      */
    uint32_t flags;            /* 1 = more than FORK_SWEEP_MAX vertices share the
                                  cut-off key: no result for this query           */
    double   best_conductance; /* +inf when no prefix has one                     */
    uint64_t best_cut;         /* edges leaving the best prefix                   */
    uint64_t best_volume;      /* its volume                                      */
    double   size_min[FORK_SWEEP_BUCKETS]; /* least conductance of prefix sizes in
                                  [2^j, 2^(j+1)); +inf when none                  */
} fork_sweep_t;

/*
 * Load a graph (Definition 2.1 fixes what a partition owns: the out-edges of
 * its vertices).  row_ptr: uint64[num_vertices+1], col: uint32[num_edges],
 * weight: uint32[num_edges] positive integers, or NULL for unit weights.
 * Requires num_edges < 2^32, num_vertices >= 1, every col < num_vertices,
 * row_ptr non-decreasing from 0 to num_edges.  cfg may be NULL.  On success
 * *out owns a new context.
 */
int fork_graph_load(fork_ctx **out, uint32_t num_vertices, uint64_t num_edges,
                    const uint64_t *row_ptr, const uint32_t *col,
                    const uint32_t *weight, const fork_config *cfg);

/*
 * Add n queries of one type from the given source vertices (Algorithm 1:
 * one query per source).  params: NULL for SSSP/BFS, a fork_ppr_params* for
 * PPR.  All-or-nothing: any source >= V, a bad type or bad PPR parameters
 * gives FORK_E_INVALID and enqueues nothing.  Query ids are dense, assigned in
 * submit order from 0; *first_query_id (may be NULL) receives the first id.
 * Submitting after a run starts a new batch (previous results are dropped).
 */
int fork_submit(fork_ctx *ctx, int query_type, const uint32_t *sources,
                uint32_t n, const void *params, uint32_t *first_query_id);

/*
 * Run all submitted queries to completion (Algorithm 2: while any buffer
 * holds operations, schedule a partition and process it).  Queries beyond
 * max_queries run in successive waves; every query gets a digest, and full
 * vectors stay available for the queries of the last wave.  Blocks until done.
 * Results are exact for SSSP/BFS whatever the schedule (Section 5.1: yielded
 * operations are retained, so correctness holds).
 */
int fork_run(fork_ctx *ctx, const fork_run_opts *opts);

/*
 * Plan the waves fork_run would make for the submitted queries under opts
 * and allocate their device buffers (query state, and the grouped engine's
 * rows and pending sets), without running anything; a following fork_run
 * with the same queries and options allocates nothing more for them.  The
 * setup step before Algorithm 2's loop, split off so that a caller can pay
 * the allocation outside a timed or latency-bound region.  Blocks until the
 * buffers are allocated.  Errors as fork_run's (FORK_E_NOMEM when one
 * query's state does not fit in device memory).
 */
int fork_prepare(fork_ctx *ctx, const fork_run_opts *opts);

/*
 * Sweep cuts of resident PPR queries: the NCP application built on the PPR
 * queries (Sections 2 and 6.1; the paper computes the network community
 * profile from one PPR per seed and does not print the sweep).  Reading:
 * the graph is taken as undirected, each directed edge one undirected edge,
 * d(v) = out-degree + in-degree, total volume 2|E|; the vertices with
 * p[v] > 0 and d(v) > 0 are swept in decreasing fp32 p[v]/d(v), equal keys
 * in increasing internal position (the caller's id when no vertex_order was
 * given); prefix S_k has conductance cut(S_k) / min(vol(S_k), 2|E| - vol(S_k)).
 * For queries first_query_id .. first_query_id + n - 1 (all PPR and in the
 * resident wave), evaluates the first min(support, max_size) prefixes,
 * 1 <= max_size <= FORK_SWEEP_MAX, and writes one fork_sweep_t per query to
 * out (host memory, n entries).  The first call builds the graph's reverse
 * adjacency on the device (4|E| + 8|V| bytes, kept until fork_destroy).
 * Errors: FORK_E_INVALID (bad range, type or max_size), FORK_E_STATE (a
 * query that is not resident).
 */
int fork_sweep(fork_ctx *ctx, uint32_t first_query_id, uint32_t n, uint32_t max_size, fork_sweep_t *out);

/*
 * Betweenness centrality from resident BFS or SSSP queries: the BC
 * application (Sections 2 and 6.1: BFSs from sampled sources, then Brandes'
 * accumulation of dependencies; on a weighted graph the same over SSSP).  A
 * BFS query counts unit steps, an SSSP query the graph's weights; shortest
 * paths are counted as edge sequences of the multigraph.  For queries
 * first_query_id .. first_query_id + n - 1 (BFS or SSSP, in the resident
 * wave), writes out[v] = sum over their sources s of delta_s(v), with
 * delta_s(s) = 0, as double[num_vertices] in the caller's ids (host memory).
 * Path counts are kept as natural logarithms in fp64 (a 2048 x 2048 grid has
 * about 10^1230 corner-to-corner shortest paths), so no count overflows.
 * Device scratch: about 20 bytes per vertex per query, allocated for the
 * call; the first call also builds the graph's reverse adjacency.
 * Errors: FORK_E_INVALID (bad range, or a PPR query), FORK_E_STATE (not
 * resident), FORK_E_CAPACITY (a query whose BFS levels or SSSP distances
 * reach 65,536: its vertices are sorted by value with a counting sort of
 * that range; no non-finite value is ever returned).
 */
int fork_bc(fork_ctx *ctx, uint32_t first_query_id, uint32_t n, double *out);

/*
 * Copy one query's result (Algorithm 1: each query of the FPP yields its own
 * result vector, as if run alone; Definition 2.2).  The digest is an addition
 * of this library for batches whose vectors do not all stay resident.
 * Field FORK_FIELD_VALUE (int32[V]), _P or _R
 * (float[V]) or _DIGEST (fork_digest).  dst_bytes must be large enough.
 * dst_on_device != 0: dst is a device pointer (device-to-device copy).
 * FORK_E_STATE if the query has not run, or its vectors are no longer
 * resident (an earlier wave); FORK_E_INVALID for a field that does not match
 * the query type.
 */
int fork_fetch(fork_ctx *ctx, uint32_t query_id, int field, void *dst,
               uint64_t dst_bytes, int dst_on_device);

/*
 * Scheduler trace of the last run made with opts.trace = 1 (the run is done
 * twice per wave: once to learn the final state, once traced).  One record
 * per visited partition per pass, FORK_TRACE_WIDTH floats each:
 *   [0..15] the partition's 16 buffer-statistics features at selection,
 *   [16] useful work of the visits (SSSP/BFS: vertex expansions whose
 *        distance was already final; PPR: vertex pushes),
 *   [17] all work of the visits (expansions / pushes), [18] pass, [19] partition.
 * Writes min(cap, available) records to dst (host); *n gets the available count.
 */
#define FORK_TRACE_WIDTH 20
int fork_trace(fork_ctx *ctx, float *dst, uint64_t cap, uint64_t *n);

/*
 * Learned scheduler network (an addition to the paper's priority functor,
 * Section 5.2): y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, sizes
 * 16 -> 64 -> 64 -> 1, fp32, flat parameters theta[5313] laid out
 * W1[64][16] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.  All pointers are
 * host pointers; the work runs on the current HIP device.  x is [n][16].
 *
 * fork_mlp_forward: y[n] = scores.
 * fork_mlp_grad:    loss = mean (y - t)^2 over the n samples and its gradient
 *                   grad[5313] (forward and backward kernels on the GPU).
 * fork_mlp_train:   `steps` Adam steps (lr, beta 0.9/0.999, eps 1e-8) on
 *                   mini-batches of `batch` samples drawn as seeded epochs;
 *                   theta is updated in place; losses[steps] (may be NULL)
 *                   receives each step's batch loss.
 */
int fork_mlp_forward(const float *theta, const float *x, uint64_t n, float *y);
int fork_mlp_grad(const float *theta, const float *x, const float *t, uint64_t n,
                  float *grad, float *loss);
int fork_mlp_train(float *theta, const float *x, const float *t, uint64_t n,
                   uint32_t steps, uint32_t batch, float lr, uint64_t seed,
                   float *losses);

/*
 * fork_mlp_train without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid it).  The same training as fork_mlp_train, but every pointer is
 * a device pointer on the current device: theta[5313] (updated in place),
 * x[n][16], t[n], losses[steps] (or NULL); the work is queued on `stream`
 * (hipStream_t, NULL = the default stream) and the call returns without
 * waiting for it.  The gradient, Adam's moments and the epoch permutation
 * live in a fixed array of this library in device memory (one per GPU,
 * about 190 KB, held until the process ends), so n is limited to 32,768
 * samples (FORK_E_INVALID beyond).  Calls that overlap on one GPU share that
 * array and race: serialise them (one stream, or wait between calls).
 * Nothing is allocated: no hipMalloc/hipFree, no host allocation; every value
 * that must start at zero is cleared by a kernel at the start of each call.
 */
int fork_mlp_train_noalloc(float *theta, const float *x, const float *t, uint64_t n, uint32_t steps,
                           uint32_t batch, float lr, uint64_t seed, float *losses, void *stream);

/* Copy the counters of the last run into *dst (dst_bytes >= sizeof): the
 * work measures of the paper's evaluation (edges processed, compared with the
 * sequential algorithms' in Section 6.3; operations buffered and consumed,
 * Section 4.2; yields, Section 5.1) and this library's pass timings.
 * FORK_E_INVALID if dst_bytes < sizeof(fork_stats_t). */
int fork_stats(fork_ctx *ctx, void *dst, uint64_t dst_bytes);

/* Partition plan: writes up to cap+1 boundaries; *num_parts receives |P|. */
int fork_partitions(fork_ctx *ctx, uint32_t *starts, uint32_t cap, uint32_t *num_parts);

/* Free the context and all its device memory.  NULL is ignored. */
void fork_destroy(fork_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *fork_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FORK_H */
