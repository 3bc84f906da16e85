/*
 * raks.h -- C ABI of the MI355X (gfx950) library for radial pattern keyword
 * search on knowledge graphs (RAKS; Yang & Tung, "Efficient Radial Pattern
 * Keyword Search on Knowledge Graphs in Parallel").
 *
 * Every call returns RAKS_OK (0) or a negative error code; no exception
 * crosses the ABI.  raks_last_error() gives a message for the last failing
 * call on the calling thread.  All pointers in descriptors are HOST pointers
 * unless stated otherwise; the library copies what it needs before returning
 * and never keeps a caller pointer.  One context owns one graph and its device
 * state on one GPU.  Calls on one context must come from one thread at a
 * time, except raks_submit / raks_poll / raks_wait, which any thread may call
 * while serving runs.
 *
 * The arithmetic is integer once the activation levels are set; every result
 * is bit-for-bit deterministic.
 */
#ifndef RAKS_H
#define RAKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAKS_OK 0
#define RAKS_EINVAL (-1)  /* invalid argument or graph contract violated */
#define RAKS_ENOMEM (-2)  /* device or host allocation failed / budget exceeded */
#define RAKS_EDEVICE (-3) /* HIP runtime error or no usable gfx950 device */
#define RAKS_ESTATE (-4)  /* call not valid in the context's current state */
#define RAKS_EAGAIN (-5)  /* result not ready yet */

#define RAKS_ACT_EDGE 0   /* activation per arc from label frequencies (Section 3.1) */
#define RAKS_ACT_NODE 1   /* activation per node from node weights (same Eqs. 1-3) */

/* Bit flags of raks_results.status */
#define RAKS_STATUS_CG_LEVEL_BOUND 1   /* central run hit max_level with fewer than w CGs */
#define RAKS_STATUS_RPG_LEVEL_BOUND 2  /* marginal run hit max_level before a stop rule */

/* End reasons of a run (raks_query_stats.end_reason) */
#define RAKS_END_NONE 0           /* run not executed */
#define RAKS_END_EXHAUSTED 1      /* frontier became empty */
#define RAKS_END_STOP 2           /* >= w CGs (central run); Theorem 4 or every CG has an RPG (marginal run) */
#define RAKS_END_LEVEL_BOUND 3    /* the level bound was reached */
#define RAKS_END_EMPTY_KEYWORD 4  /* a keyword of the run has no node */

typedef struct raks_ctx raks_ctx;

/* Optional device allocator: returns a device pointer of at least `bytes`
 * bytes aligned to 256, or NULL.  Used for every device buffer the context
 * owns.  Both callbacks may be NULL (then hipMalloc/hipFree are used). */
typedef void* (*raks_alloc_fn)(size_t bytes, void* user);
typedef void (*raks_free_fn)(void* ptr, size_t bytes, void* user);

typedef struct {
    int32_t device;         /* HIP device ordinal */
    void* stream;           /* hipStream_t to run on, or NULL for a library-owned stream */
    raks_alloc_fn alloc;    /* optional device allocator (see above) */
    raks_free_fn free;
    void* alloc_user;
    uint64_t mem_budget;    /* bytes of device memory the context may hold; 0 = no limit */
    int32_t lanes;          /* query lanes, 0..32 (0 = 1); see raks_query_batch */
    /* Initial recovery capacities per (result, keyword) instance (Algorithm 2):
     * recovered nodes, recovered arcs, and work chunks of 256 arcs per layer
     * (0 = 4096, 16384, 65536).  An instance that needs more is grown and its
     * phase repeated, so these only trade memory against repeats. */
    uint32_t rec_nodes, rec_arcs, rec_chunks;
    /* Results whose recovered lists hold more entries than this (0 = 2^20)
     * are merged through bitmaps over all nodes and arcs instead of a
     * one-workgroup sort; the output is the same. */
    uint64_t big_list;
} raks_ctx_opts;

/* Creates a context on opts->device (opts may be NULL: device 0, own stream,
 * hipMalloc, one lane).  A lane is one query's device workspace with its own
 * stream (lane 0 uses opts->stream when given); lanes let the queries of a
 * batch or of the serving loop run on the device at the same time.  Fails
 * with RAKS_EDEVICE when the device is not gfx950.  *out is owned by the
 * caller until raks_destroy. */
int raks_create(raks_ctx** out, const raks_ctx_opts* opts);

/* Frees every device and host resource of the context (NULL-safe). */
int raks_destroy(raks_ctx* ctx);

/* Graph input (Section 2: a bi-directed labelled knowledge graph stored as
 * CSR, Section 4.1).  Contract, checked on the device (RAKS_EINVAL if broken):
 *   - row_ptr[0] = 0, non-decreasing, row_ptr[n_nodes] = n_arcs < 2^32;
 *   - 0 <= col[e] < n_nodes, no self-loops;
 *   - each row sorted strictly increasing by (label, col);
 *   - bi-directed: for every arc (u -> v, l) the arc (v -> u, l) exists;
 *   - keyword t owns kw_nodes[kw_ptr[t] .. kw_ptr[t+1]), strictly increasing
 *     node ids (the keyword -> node mapping of Section 4.1);
 *   - 0 < a_bar <= 100 (average shortest hop count, Section 3.1),
 *     0 < alpha < 1 (Eqs. 1-2).
 * node_weight may be NULL in RAKS_ACT_EDGE mode.  Arrays are copied; the
 * caller may free them on return.  Replaces a previously loaded graph. */
typedef struct {
    int32_t n_nodes;
    int64_t n_arcs;
    const int64_t* row_ptr;      /* [n_nodes + 1] */
    const int32_t* col;          /* [n_arcs] */
    const uint16_t* label;       /* [n_arcs] */
    const uint8_t* node_weight;  /* [n_nodes] (RAKS_ACT_NODE) */
    int32_t n_keywords;
    const int64_t* kw_ptr;       /* [n_keywords + 1] */
    const int32_t* kw_nodes;     /* [kw_ptr[n_keywords]] */
    double a_bar;
    double alpha;
    int32_t act_mode;            /* RAKS_ACT_EDGE or RAKS_ACT_NODE */
} raks_graph_desc;

/* Loads the graph and computes activation levels on the GPU (Section 3.1,
 * Eqs. 1-3): EDGE mode per arc from c = |arcs of src with the label| +
 * |arcs into dst with the label|, rescaled log weights, reward/penalty around
 * a_bar, round half up; NODE mode per node from node_weight min-max rescaled.
 * Errors: RAKS_EINVAL (contract), RAKS_ENOMEM, RAKS_EDEVICE. */
int raks_load_graph(raks_ctx* ctx, const raks_graph_desc* g);

/* Host-only: the activation level (Eqs. 1-3, Section 3.1) of every value in
 * [lo, hi] into out[0 .. hi-lo].  RAKS_ACT_EDGE: the values are label counts
 * c (c = |arcs of the source with the label| + |arcs into the destination
 * with the label|) and [lo, hi] is the range of c over the graph, so the
 * rescaled weight is (ln c - ln lo) / (ln hi - ln lo); RAKS_ACT_NODE: node
 * weights, rescaled (w - lo) / (hi - lo).  Reward below alpha, penalty above,
 * round half up, in IEEE binary64 in the order written; a single-valued range
 * rescales to 0.  raks_load_graph builds this table once per alpha and the
 * device only looks levels up, so every arc with the same count gets the same
 * level.  RAKS_EINVAL for an unknown mode, lo < 1 (EDGE), hi < lo, a range of
 * 2^28 values or more, a_bar <= 0 or alpha outside (0,1). */
int raks_level_table(int32_t mode, int64_t lo, int64_t hi, double a_bar, double alpha,
                     uint8_t* out);
/* Recomputes the activation levels for a new alpha (users adjust the search
 * granularity with alpha, Section 3.1).  RAKS_ESTATE without a graph. */
int raks_set_alpha(raks_ctx* ctx, double alpha);

/* Copies the per-arc activation levels (uint8 [n_arcs]) to host memory
 * `out`.  In NODE mode the level of arc u -> v is that of node v. */
int raks_get_activations(raks_ctx* ctx, uint8_t* out, int64_t n);

/* A radial pattern query (Definition 1) and its parameters (Table 2).
 *   central: 1..16 distinct keyword ids; marginal: 0..16 distinct ids, none
 *   central.  k >= 1 results, beam width w >= k (0 = k) and w <= 256
 *   (Section 3.4); gamma = gamma_num/gamma_den in [0,1] (Eq. 6; 0/0 = 1/2);
 *   max_level in 1..250 (0 = 20, the paper's level bound).
 *   score_mode (Section 3.3 allows a multiplicative combination): 1 ranks
 *   by key = S^c * S^m (without marginal keywords: S^c), and Theorem 4 stops
 *   when the k-th key <= min S^c over CGs without RPG * S^m of the k-th.
 *   rerank (Section 3.3, ties broken by a sum of edge weights): results of
 *   equal key are ordered by weight_sum, the sum of the activation levels of
 *   their arcs, then S^c and CG rank; every RPG whose key does not exceed the
 *   k-th one's is recovered before the first k are kept, and Theorem 4 stops
 *   only on a strict inequality.  Values other than 0/1 give RAKS_EINVAL.
 *   alpha: the granularity of Eqs. 1-2 for this query alone, without
 *   reloading (users tune alpha per search, Section 3.1); the levels for an
 *   alpha are built on first use (one pass over the arcs) and the last few
 *   are cached.
 * Violations give RAKS_EINVAL.  A keyword with no node gives no results. */
typedef struct {
    const int32_t* central;
    int32_t n_central;
    const int32_t* marginal;
    int32_t n_marginal;
    int32_t k;
    int32_t w;
    int32_t gamma_num;
    int32_t gamma_den;
    int32_t max_level;
    double alpha;       /* 0: the context's alpha; else in (0,1) for this query only */
    int32_t score_mode; /* 0: S^r of Eq. 6; 1: the multiplicative combination S^c * S^m */
    int32_t rerank;     /* 1: RPGs of equal score re-ranked by weight_sum */
} raks_query_desc;

typedef struct {
    int32_t src, dst, label;
} raks_arc;

/* One result subgraph: a radial pattern graph (Definition 5) or, without
 * marginal keywords, a central graph (Definition 4).  score_c = S^c (Eq. 4),
 * score_m = S^m (Eq. 5), key = gamma_num*S^c + (gamma_den-gamma_num)*S^m,
 * i.e. gamma_den * S^r (Eq. 6), or S^c * S^m with score_mode 1.  nodes ascending; arcs in CSR order, i.e. by
 * (src, label, dst); each arc points along the search direction (from a
 * keyword node towards the central node / the central-keyword nodes). */
typedef struct {
    int32_t central_node;
    int32_t score_c;
    int32_t score_m;
    int64_t key;
    int64_t weight_sum;     /* sum of the activation levels of the result's arcs */
    int32_t n_nodes;
    const int32_t* nodes;
    int32_t n_arcs;
    const raks_arc* arcs;
} raks_result;

/* Per-run work counters ([0] central run, [1] marginal run). */
typedef struct {
    int32_t levels[2];       /* levels processed (identification passes) */
    int32_t end_reason[2];   /* RAKS_END_* */
    int64_t frontier[2];     /* sum over levels of |frontier| */
    int64_t e_arc[2];        /* arcs scanned: degrees of expanding frontiers */
    int64_t e_alg[2];        /* arcs scanned per (frontier, keyword) pair, as Algorithm 1 counts */
    int64_t gate_pass[2];    /* scanned arcs whose level allowed expansion */
    int64_t h_writes[2];     /* node-keyword matrix entries written */
    int32_t n_cg;            /* central graphs identified by the central run */
    double device_ms;        /* wall time of the query on its device stream */
    double host_ms;          /* call (or submission) to results ready, host clock */
    double queue_ms;         /* submission to start on a lane (serving; 0 otherwise) */
} raks_query_stats;

typedef struct {
    int32_t n;               /* number of results (<= k) */
    raks_result* r;          /* ranked by (key, score_c, CG rank) */
    raks_query_stats stats;
    int32_t status;          /* RAKS_STATUS_* bits */
} raks_results;

/* Caller-owned output of raks_query_noalloc.  The caller sets the arrays and
 * their capacities; the call fills the rest.  r[i].nodes and r[i].arcs point
 * into `nodes` and `arcs`, where the results' lists lie back to back. */
typedef struct {
    raks_result* r;          /* [cap_results] */
    int32_t cap_results;     /* at least the query's k */
    int32_t* nodes;          /* [cap_nodes] */
    int64_t cap_nodes;
    raks_arc* arcs;          /* [cap_arcs] */
    int64_t cap_arcs;
    int32_t n;               /* out: number of results (<= k) */
    int32_t status;          /* out: RAKS_STATUS_* bits */
    int64_t n_nodes;         /* out: node entries of all results (also on a too-small RAKS_ENOMEM) */
    int64_t n_arcs;          /* out: arc entries of all results (likewise) */
    raks_query_stats stats;  /* out */
} raks_results_buf;

/* Runs one query (both runs of Section 4.1 on the GPU: exploration,
 * identification, top-w selection, recovery, marginal run, ranking) and
 * returns its results.  *out is library-owned until raks_results_free. */
int raks_query(raks_ctx* ctx, const raks_query_desc* q, raks_results** out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. tight serving loops or harnesses that forbid it): the same
 * query and results as raks_query, with no device or pinned-host allocation
 * in the call.  It runs on a lane of its own that raks_create sets up; all of
 * its device state lives in one static device array of 256 MiB per GPU that
 * the library holds until the process ends.  That array is shared by every
 * context on the GPU and keeps the last call's contents (the call initialises
 * what it reads), so calls that overlap on one GPU race: issue them one at a
 * time per GPU.  The results are written to the caller's arrays in `out`.
 * Errors: RAKS_EINVAL for NULL arguments, negative capacities, a NULL array
 * with a positive capacity, cap_results < k or an invalid query;
 * RAKS_ESTATE while serving runs, without a graph, or when the levels of the
 * query's alpha have not been built (a raks_query with that alpha builds
 * them); RAKS_ENOMEM when the query's device state would exceed the 256 MiB
 * (graphs of up to about 3M nodes fit), or when the results do not fit the
 * caller's arrays (then out->n_nodes / n_arcs give the sizes needed and out->n
 * is 0).  Event timing (raks_set_timing) does not cover this lane. */
int raks_query_noalloc(raks_ctx* ctx, const raks_query_desc* q, raks_results_buf* out);

/* Runs n queries and returns outs[i] = the results of qs[i], identical to
 * those of raks_query(qs[i]), each owned independently.  On error no output
 * is left allocated.
 * In the default batch mode (RAKS_BATCH_COHORT) the queries run as cohorts:
 * up to 32 queries at a time share one level loop on the device, each with
 * its central and marginal keywords as columns of one query-tagged
 * node x keyword hitting-level matrix (64 columns); one frontier scan and one
 * expansion per level serve all of them, so an arc is read once for every
 * query that expands its source node (Section 4.2.1's shared frontier, taken
 * from keywords to queries).  Both runs of a query advance together (the
 * marginal search does not depend on the central graphs, Section 4.2.3); its
 * RPG check starts once its central graphs are recovered and replays the
 * levels in between, so every decision is the one of the two sequential
 * runs.  A finished query frees its slot and columns and the next waiting
 * one is admitted at the next level boundary.  Queries with a per-query
 * alpha, more than 16 keywords, an empty keyword or max_level above 125 run
 * on the single-query path instead.
 * In RAKS_BATCH_LANES mode each lane runs whole single queries, taking the
 * next one when its previous one is done. */
int raks_query_batch(raks_ctx* ctx, const raks_query_desc* qs, int32_t n, raks_results** outs);

#define RAKS_BATCH_COHORT 0   /* queries share level loops (default) */
#define RAKS_BATCH_LANES 1    /* independent single-query runs on the lanes */
/* Selects how raks_query_batch and serving run queries.  RAKS_EINVAL for an
 * unknown mode, RAKS_ESTATE while serving runs. */
int raks_set_batch_mode(raks_ctx* ctx, int32_t mode);

/* Tuning of the cohort path (chosen per workload by the package's autotuner).
 *   expand_wg_per_cu: workgroups per compute unit of the expansion launch
 *     (0 = 8);
 *   expand_tile: arcs per tile of the expansion (each tile's entries and
 *     owner map live in LDS);
 *   admit_below: a batch admits waiting queries only while at most this many
 *     queries of the cohort are still exploring (32 admits whenever a query
 *     fits; 0 admits in waves, so a group starts level-aligned and shares more
 *     frontier nodes).  Serving always admits as soon as a query fits.
 * RAKS_EINVAL for values out of range, RAKS_ESTATE while serving runs. */
typedef struct {
    int32_t expand_wg_per_cu;
    int32_t admit_below;
    int32_t expand_tile;    /* examined arcs per expansion tile: 512, 1024 or 2048 (0 = 1024) */
    int32_t cohort_cols;    /* columns of the cohort: 16, 32 or 64 (0 = 64); a narrower cohort
                             * holds fewer queries at once and keeps its per-node reached masks
                             * in 2 or 4 bytes instead of 8 */
} raks_tuning;
int raks_set_tuning(raks_ctx* ctx, const raks_tuning* t);

/* Serving (continuous batching).  In RAKS_BATCH_COHORT mode one engine thread
 * runs the level loop: a submitted query joins the running cohort at the next
 * level boundary as soon as a slot, |C|+|M| columns and the device memory of
 * its post-processing state (a lane's recovery buffers; admission waits
 * while the allocation does not fit) are free, so queries that arrive while
 * others are on the GPU share their levels; finished queries are completed by
 * worker threads on their lanes' streams.  In RAKS_BATCH_LANES mode a worker
 * thread per lane runs submitted queries in arrival order as lanes become
 * free.  Results are those raks_query gives.  While serving runs,
 * raks_query / raks_query_batch / raks_load_graph / raks_set_alpha /
 * raks_set_batch_mode return RAKS_ESTATE. */
typedef struct {
    int32_t lanes;      /* lanes mode: 0 = as many as half of the free device memory holds, at most 8 */
    int32_t queue_cap;  /* queries submitted and not finished allowed (cohort mode) or waiting
                         * (lanes mode), 0 = unbounded */
} raks_serve_opts;
/* Starts serving (opts may be NULL).  RAKS_ESTATE without a graph or when
 * serving already runs. */
int raks_serve_start(raks_ctx* ctx, const raks_serve_opts* opts);

/* Queues a query (its arrays are copied) and returns its ticket.  RAKS_EAGAIN
 * when the queue is full; the query is validated when it runs, so invalid
 * queries fail at raks_poll / raks_wait. */
int raks_submit(raks_ctx* ctx, const raks_query_desc* q, uint64_t* ticket);

/* Takes the results of a finished query: RAKS_EAGAIN while it still runs
 * (the ticket stays valid), the query's own error code if it failed, and
 * RAKS_EINVAL for an unknown or already taken ticket.  *out is owned by the
 * caller (raks_results_free). */
int raks_poll(raks_ctx* ctx, uint64_t ticket, raks_results** out);

/* As raks_poll, but blocks until the query has finished. */
int raks_wait(raks_ctx* ctx, uint64_t ticket, raks_results** out);

/* Stops serving after every submitted query has run; results not taken are
 * freed.  Also done by raks_destroy. */
int raks_serve_stop(raks_ctx* ctx);

/* Frees results (NULL-safe). */
void raks_results_free(raks_results* r);

/* Per-kernel device time, accumulated while timing is enabled
 * (raks_set_timing).  kernel ids: 0 expansion (Algorithm 1), 1 frontier
 * scan, 2 identification/control step with Frontier Enqueue, 3 recovery,
 * 4 other. */
typedef struct {
    int64_t launches;
    double ms;               /* summed event-measured duration */
    double bytes;            /* algorithmic bytes moved (expansion only) */
} raks_kernel_timing;

/* Enables per-launch event timing for the kernel ids whose bit is set in
 * `mask` (bit k = kernel id k; 0 disables, 31 records all); a non-zero mask
 * resets the accumulators.  Each timed launch is bracketed by two events on
 * its lane's stream.  RAKS_EINVAL for mask outside 0..31. */
int raks_set_timing(raks_ctx* ctx, int32_t mask);
int raks_get_timing(raks_ctx* ctx, int32_t kernel, raks_kernel_timing* out);

/* Message of the last failing call on this thread ("" if none). */
const char* raks_last_error(void);

/* Library version string. */
const char* raks_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RAKS_H */
