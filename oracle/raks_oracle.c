/*
 * raks_oracle.c -- reference implementation of RAKS radial-pattern keyword
 * search ("Efficient Radial Pattern Keyword Search on Knowledge Graphs in
 * Parallel", Yang & Tung).
 *
 * TEST INFRASTRUCTURE.  Plain, single-threaded and deliberately literal: it
 * takes the paper's steps in the paper's order, with no blocking, fusion or
 * reordering beyond what the paper states.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the GPU library
 * shares no code with it.
 *
 * What it computes
 *   - activation levels (Section 3.1, Eqs. 1-3) in IEEE binary64, per arc
 *     (EDGE mode: label-frequency weights of Section 3.1) or per node (NODE
 *     mode: node weights min-max rescaled, the same Eqs. 1-3);
 *   - the exploration phase (Section 4.2, Algorithm 1) with the frontier flag
 *     array F, node-keyword matrix H and joining flag array CF;
 *   - result identification (Section 4.2.3): central nodes (Theorem
 *     "identifyCG"), termination after >= w central graphs, RPG check over the
 *     central-keyword nodes of each CG, the early termination of Theorem 4;
 *   - the recovering phase (Section 4.3, Algorithm 2, Lemma 1) for central
 *     graphs and for the marginal part of RPGs;
 *   - ranking by Eqs. 4-6.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes with its justification):
 *   R2  arcs are bi-directed; the reverse arc carries the same label and the
 *       label counts are taken on the bi-directed graph;
 *   R5  if all fine weights are equal the rescaled weight is 0;
 *   R6  "Rounding" is round-half-up, floor(v + 0.5) (Theorem 1's half-open
 *       intervals);
 *   R7  Eq. 1-3 evaluated as written: v = A - A*(alpha-x)/alpha, or
 *       v = A + A*(x-alpha)/(1-alpha), products and quotients left to right;
 *   R11 expansion happens only at levels below the level bound;
 *   R12 per level: enqueue, identify, test termination, expand;
 *   R13 CGs are ranked by (S^c, sum of central hitting levels, node id);
 *   R14 RPGs are ranked by (S^r, S^c, CG rank); S^r is kept as the integer
 *       gamma_num*S^c + (gamma_den-gamma_num)*S^m (gamma = num/den);
 *   R15 the marginal run blocks a node reached by all marginal keywords only
 *       when there are at least two marginal keywords;
 *   R17 a query keyword with no node ends its run with no results;
 *   R18 recovery keeps a visited set per (result, keyword) and applies the
 *       Lemma 1 test literally;
 *   R19 V_C = CG nodes whose hitting level for some central keyword is 0;
 *   R20 an RPG needs every marginal keyword to reach some node of V_C;
 *       S^m = max over marginal keywords of min over V_C of its hitting level;
 *   R30 the multiplicative combination of S^c and S^m (Section 3.3 allows
 *       one) is the integer S^c * S^m (without marginal keywords: S^c), and
 *       Theorem 4 becomes S^r(k-th) <= min S^c over CGs without RPG * S^m(k-th);
 *   R31 the re-ranking of ties (Section 3.3) orders RPGs of equal S^r by the
 *       sum of the activation levels of their arcs; every RPG whose S^r does
 *       not exceed the k-th one's is recovered before the top k are taken,
 *       and Theorem 4 must hold strictly, so that no later RPG of equal S^r
 *       can be missed.  The sum is reported for every result.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define INF_LEVEL 255

enum { MODE_EDGE = 0, MODE_NODE = 1 };
enum { END_NONE = 0, END_EXHAUSTED = 1, END_STOP = 2, END_LEVEL_BOUND = 3, END_EMPTY_KEYWORD = 4 };
enum { FLAG_NO_CG_BLOCK = 1, FLAG_NO_THM4 = 2, FLAG_NO_M_BLOCK = 4 };

typedef struct {
    int32_t n;
    int64_t A;
    const int64_t* row_ptr;
    const int32_t* col;
    const uint16_t* label;
    const uint8_t* node_weight;
    int32_t vocab;
    const int64_t* kw_ptr;
    const int32_t* kw_nodes;
} orc_graph;

typedef struct {
    int64_t levels, end_reason, frontier, e_arc, e_alg, gate_pass, h_writes;
} orc_run_stats;

/* ------------------------------------------------------------ helpers --- */

/* Position of arc (src -> dst, lab) in the row of src, or -1.  Rows are
 * sorted by (label, destination). */
static int64_t find_arc(const orc_graph* g, int32_t src, uint16_t lab, int32_t dst) {
    int64_t lo = g->row_ptr[src], hi = g->row_ptr[src + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->label[mid] < lab || (g->label[mid] == lab && g->col[mid] < dst)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < g->row_ptr[src + 1] && g->label[lo] == lab && g->col[lo] == dst) return lo;
    return -1;
}

/* Number of arcs out of x with label lab. */
static int64_t label_degree(const orc_graph* g, int32_t x, uint16_t lab) {
    int64_t lo = g->row_ptr[x], hi = g->row_ptr[x + 1];
    while (lo < hi) {          /* first arc with label >= lab */
        int64_t mid = lo + (hi - lo) / 2;
        if (g->label[mid] < lab) lo = mid + 1; else hi = mid;
    }
    int64_t first = lo;
    hi = g->row_ptr[x + 1];
    while (lo < hi) {          /* first arc with label > lab */
        int64_t mid = lo + (hi - lo) / 2;
        if (g->label[mid] <= lab) lo = mid + 1; else hi = mid;
    }
    return lo - first;
}

/* Input contract: CSR with monotone offsets, rows sorted strictly by
 * (label, destination), no self-loops, every arc has its reverse, keyword
 * lists sorted, unique and in range.  Returns 0 or a negative code. */
int orc_check_graph(const orc_graph* g) {
    if (g->n < 1 || g->A < 0 || g->row_ptr[0] != 0 || g->row_ptr[g->n] != g->A) return -1;
    for (int32_t v = 0; v < g->n; ++v) {
        if (g->row_ptr[v + 1] < g->row_ptr[v]) return -2;
        for (int64_t e = g->row_ptr[v]; e < g->row_ptr[v + 1]; ++e) {
            if (g->col[e] < 0 || g->col[e] >= g->n) return -3;
            if (g->col[e] == v) return -4;
            if (e > g->row_ptr[v]) {
                if (g->label[e] < g->label[e - 1]) return -5;
                if (g->label[e] == g->label[e - 1] && g->col[e] <= g->col[e - 1]) return -5;
            }
            if (find_arc(g, g->col[e], g->label[e], v) < 0) return -6;
        }
    }
    if (g->vocab < 0 || g->kw_ptr[0] != 0) return -7;
    for (int32_t t = 0; t < g->vocab; ++t) {
        if (g->kw_ptr[t + 1] < g->kw_ptr[t]) return -7;
        for (int64_t i = g->kw_ptr[t]; i < g->kw_ptr[t + 1]; ++i) {
            if (g->kw_nodes[i] < 0 || g->kw_nodes[i] >= g->n) return -8;
            if (i > g->kw_ptr[t] && g->kw_nodes[i] <= g->kw_nodes[i - 1]) return -8;
        }
    }
    return 0;
}

/* ---------------------------------------------- Section 3.1, Eqs. 1-3 --- */

/* Activation level of a rescaled fine-grained weight x in [0,1]. */
int orc_level_of(double x, double abar, double alpha) {
    double v;
    if (x <= alpha) {
        double reward = abar * (alpha - x) / alpha;            /* Eq. 1 */
        v = abar - reward;                                     /* Eq. 3, first case */
    } else {
        double penalty = abar * (x - alpha) / (1.0 - alpha);   /* Eq. 2 */
        v = abar + penalty;                                    /* Eq. 3, second case */
    }
    double r = floor(v + 0.5);                                 /* Rounding: half up */
    if (r < 0.0) r = 0.0;
    if (r > 254.0) r = 254.0;
    return (int)r;
}

/* Per-arc activation levels act[A]; in NODE mode also the per-node levels
 * act_node[n] (act[e] is then the level of the arc's destination).  The
 * fine weights, their extremes and the rescaled x are also returned when the
 * optional arrays are non-NULL (used by the bounds checks of Theorem 1). */
int orc_activation(const orc_graph* g, double abar, double alpha, int mode, uint8_t* act,
                   uint8_t* act_node, double* x_out, int64_t* c_out) {
    if (!(alpha > 0.0 && alpha < 1.0) || !(abar > 0.0)) return -1;
    if (mode == MODE_EDGE) {
        /* w_ij = log(|out-arcs of i with label l| + |in-arcs of j with label l|);
         * on the bi-directed graph the in-arcs of j with label l are the
         * reverses of its out-arcs with label l. */
        int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(g->A > 0 ? g->A : 1));
        if (!c) return -2;
        int64_t cmin = INT64_MAX, cmax = 0;
        for (int32_t i = 0; i < g->n; ++i) {
            for (int64_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                c[e] = label_degree(g, i, g->label[e]) + label_degree(g, g->col[e], g->label[e]);
                if (c[e] < cmin) cmin = c[e];
                if (c[e] > cmax) cmax = c[e];
            }
        }
        double wmin = log((double)cmin), wmax = log((double)cmax);
        for (int64_t e = 0; e < g->A; ++e) {
            double w = log((double)c[e]);
            double x = (cmax == cmin) ? 0.0 : (w - wmin) / (wmax - wmin);
            act[e] = (uint8_t)orc_level_of(x, abar, alpha);
            if (x_out) x_out[e] = x;
            if (c_out) c_out[e] = c[e];
        }
        free(c);
        return 0;
    }
    if (mode == MODE_NODE) {
        int wmin = 255, wmax = 0;
        for (int32_t v = 0; v < g->n; ++v) {
            if (g->node_weight[v] < wmin) wmin = g->node_weight[v];
            if (g->node_weight[v] > wmax) wmax = g->node_weight[v];
        }
        for (int32_t v = 0; v < g->n; ++v) {
            double x = (wmax == wmin) ? 0.0
                     : ((double)g->node_weight[v] - (double)wmin) / ((double)wmax - (double)wmin);
            act_node[v] = (uint8_t)orc_level_of(x, abar, alpha);
            if (x_out) x_out[v] = x;
        }
        for (int64_t e = 0; e < g->A; ++e) act[e] = act_node[g->col[e]];
        return 0;
    }
    return -1;
}

/* -------------------------------------- Section 4.2, exploration phase --- */

typedef struct {
    const orc_graph* g;
    const uint8_t* act;
    int32_t T;
    uint8_t* H;        /* node-keyword matrix, n x T, INF_LEVEL = not reached */
    uint8_t* F;        /* frontier flag array */
    uint8_t* CF;       /* joining flag array */
    int32_t* Q;        /* frontiers of the current level */
    int64_t nq;
    orc_run_stats st;
    uint64_t shuffle;  /* 0 = natural order; else seed of an order permutation */
    uint64_t rs;
} explore_t;

static uint64_t xs_next(uint64_t* s) {  /* xorshift64*, only for order shuffles */
    uint64_t x = *s;
    x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
    *s = x;
    return x * 0x2545F4914F6CDD1DULL;
}

static void shuffle_i64(int64_t* a, int64_t n, uint64_t* s) {
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)(xs_next(s) % (uint64_t)(i + 1));
        int64_t t = a[i]; a[i] = a[j]; a[j] = t;
    }
}

static int explore_init(explore_t* x, const orc_graph* g, const uint8_t* act, const int32_t* kws,
                        int32_t T, uint64_t shuffle) {
    memset(x, 0, sizeof(*x));
    x->g = g; x->act = act; x->T = T; x->shuffle = shuffle; x->rs = shuffle ? shuffle : 1;
    x->H = (uint8_t*)malloc((size_t)g->n * (size_t)(T > 0 ? T : 1));
    x->F = (uint8_t*)calloc((size_t)g->n, 1);
    x->CF = (uint8_t*)calloc((size_t)g->n, 1);
    x->Q = (int32_t*)malloc(sizeof(int32_t) * (size_t)g->n);
    if (!x->H || !x->F || !x->CF || !x->Q) return -1;
    memset(x->H, INF_LEVEL, (size_t)g->n * (size_t)T);
    int empty = 0;
    for (int32_t i = 0; i < T; ++i) {
        int32_t t = kws[i];
        if (g->kw_ptr[t + 1] == g->kw_ptr[t]) empty = 1;
        for (int64_t p = g->kw_ptr[t]; p < g->kw_ptr[t + 1]; ++p) {
            int32_t v = g->kw_nodes[p];
            x->H[(size_t)v * T + i] = 0;    /* keyword nodes start at distance 0 */
            x->F[v] = 1;                    /* and are the first frontiers */
        }
    }
    return empty;
}

static void explore_free(explore_t* x) { free(x->H); free(x->F); free(x->CF); free(x->Q); }

/* Frontier Enqueue (Section 4.2.2): extract F = 1 nodes, then clear F. */
static void enqueue(explore_t* x) {
    x->nq = 0;
    for (int32_t v = 0; v < x->g->n; ++v)
        if (x->F[v]) { x->Q[x->nq++] = v; x->F[v] = 0; }
    x->st.frontier += x->nq;
}

static int row_complete(const explore_t* x, int32_t v) {
    for (int32_t i = 0; i < x->T; ++i) if (x->H[(size_t)v * x->T + i] == INF_LEVEL) return 0;
    return 1;
}

/* Algorithm 1, Expansion Procedure, at Glevel l. */
static void expand(explore_t* x, int l, int use_cf) {
    const orc_graph* g = x->g;
    const int32_t T = x->T;
    int64_t* order = NULL;
    int64_t kw_order[64];
    int64_t* arc_order = NULL;
    if (x->shuffle) {
        order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(x->nq > 0 ? x->nq : 1));
        for (int64_t i = 0; i < x->nq; ++i) order[i] = i;
        shuffle_i64(order, x->nq, &x->rs);
    }
    for (int64_t qi = 0; qi < x->nq; ++qi) {
        int32_t f = x->Q[order ? order[qi] : qi];
        if (use_cf && x->CF[f]) continue;                      /* avoid repetitions / PTC */
        const int64_t r0 = g->row_ptr[f], r1 = g->row_ptr[f + 1], deg = r1 - r0;
        for (int32_t i = 0; i < T; ++i) kw_order[i] = i;
        if (x->shuffle) {
            shuffle_i64(kw_order, T, &x->rs);
            free(arc_order);
            arc_order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(deg > 0 ? deg : 1));
            for (int64_t k = 0; k < deg; ++k) arc_order[k] = r0 + k;
            shuffle_i64(arc_order, deg, &x->rs);
        }
        int active = 0;
        for (int32_t ii = 0; ii < T; ++ii) {
            const int32_t i = (int32_t)kw_order[ii];
            uint8_t sf = x->H[(size_t)f * T + i];              /* path score of f from t_i */
            if (sf > l) continue;                              /* not a frontier for t_i */
            active = 1;
            x->st.e_alg += deg;
            for (int64_t k = 0; k < deg; ++k) {
                const int64_t e = arc_order ? arc_order[k] : r0 + k;
                const int32_t nb = g->col[e];
                if (x->act[e] > l) { x->F[f] = 1; continue; }  /* f stays a frontier */
                uint8_t sn = x->H[(size_t)nb * T + i];
                if (sn != INF_LEVEL) continue;                 /* already reached by t_i */
                x->H[(size_t)nb * T + i] = (uint8_t)(l + 1);   /* expand f -> nb */
                x->F[nb] = 1;
                x->st.h_writes++;
            }
        }
        if (active) {
            x->st.e_arc += deg;
            for (int64_t e = r0; e < r1; ++e) if (x->act[e] <= l) x->st.gate_pass++;
        }
    }
    free(order);
    free(arc_order);
}

/* Exploration with no result identification (used by the checks of
 * Theorem "distGlevel"); block = 1 makes a node with a complete row stop
 * expanding, as the central and marginal runs do. */
int orc_explore(const orc_graph* g, const uint8_t* act, const int32_t* kws, int32_t T,
                int32_t block, int32_t max_level, uint64_t shuffle, uint8_t* H_out,
                orc_run_stats* st) {
    explore_t x;
    if (T < 1 || T > 64) return -1;
    if (explore_init(&x, g, act, kws, T, shuffle) < 0) { explore_free(&x); return -2; }
    for (int l = 0;; ++l) {
        enqueue(&x);
        x.st.levels = l + 1;
        if (x.nq == 0) { x.st.end_reason = END_EXHAUSTED; break; }
        if (block)
            for (int64_t qi = 0; qi < x.nq; ++qi)
                if (!x.CF[x.Q[qi]] && row_complete(&x, x.Q[qi])) x.CF[x.Q[qi]] = 1;
        if (l == max_level) { x.st.end_reason = END_LEVEL_BOUND; break; }
        expand(&x, l, block);
    }
    memcpy(H_out, x.H, (size_t)g->n * (size_t)T);
    if (st) *st = x.st;
    explore_free(&x);
    return 0;
}

/* ------------------------------------- Section 4.3, recovering phase --- */

typedef struct { int64_t* v; int64_t n, cap; } vec_t;

static int vec_push(vec_t* a, int64_t x) {
    if (a->n == a->cap) {
        int64_t nc = a->cap ? 2 * a->cap : 64;
        int64_t* nv = (int64_t*)realloc(a->v, sizeof(int64_t) * (size_t)nc);
        if (!nv) return -1;
        a->v = nv; a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static void sort_unique(vec_t* a) {
    if (a->n == 0) return;
    qsort(a->v, (size_t)a->n, sizeof(int64_t), cmp_i64);
    int64_t m = 1;
    for (int64_t i = 1; i < a->n; ++i) if (a->v[i] != a->v[m - 1]) a->v[m++] = a->v[i];
    a->n = m;
}

/* Algorithm 2 body for one keyword column: backward BFS from the start nodes
 * over in-arcs n -> q, recovering (n, e_nq) iff h_q = 1 + max(a_nq, h_n)
 * (Lemma 1), continuing from n unless h_n = 0.  Nodes and arcs (arc index
 * of n -> q in the CSR) are appended to the output vectors. */
static int recover_column(const orc_graph* g, const uint8_t* act, const uint8_t* H, int32_t T,
                          int32_t i, const int32_t* start, int64_t nstart, vec_t* nodes,
                          vec_t* arcs, int32_t* stamp, int32_t stamp_id, int32_t* queue) {
    int64_t qh = 0, qt = 0;
    for (int64_t s = 0; s < nstart; ++s) {
        if (stamp[start[s]] != stamp_id) { stamp[start[s]] = stamp_id; queue[qt++] = start[s]; }
        if (vec_push(nodes, start[s])) return -1;
    }
    while (qh < qt) {
        const int32_t q = queue[qh++];
        const int hq = H[(size_t)q * T + i];
        for (int64_t e = g->row_ptr[q]; e < g->row_ptr[q + 1]; ++e) {
            /* in-neighbour n of q: the arc n -> q is the reverse of q -> n */
            const int32_t n = g->col[e];
            const int64_t r = find_arc(g, n, g->label[e], q);
            if (r < 0) return -2;
            const int a = act[r];
            const int hn = H[(size_t)n * T + i];
            const int m = a > hn ? a : hn;
            if (hq == 1 + m) {
                if (vec_push(nodes, n) || vec_push(arcs, r)) return -1;
                if (hn != 0 && stamp[n] != stamp_id) { stamp[n] = stamp_id; queue[qt++] = n; }
            }
        }
    }
    return 0;
}

/* ---------------------------------------- Sections 3.3, 3.4 and 4.2.3 --- */

typedef struct {
    int32_t node;
    int32_t sc;      /* S^c, Eq. 4 (= max central hitting level, Theorem identifyCG) */
    int32_t sumh;    /* sum of central hitting levels: tie-break */
} cg_t;

static int cmp_cg(const void* a, const void* b) {
    const cg_t* x = (const cg_t*)a; const cg_t* y = (const cg_t*)b;
    if (x->sc != y->sc) return x->sc < y->sc ? -1 : 1;
    if (x->sumh != y->sumh) return x->sumh < y->sumh ? -1 : 1;
    return (x->node > y->node) - (x->node < y->node);
}

typedef struct { int64_t key; int32_t sc; int32_t rank; } rpg_key_t;

static int cmp_rpg(const void* a, const void* b) {
    const rpg_key_t* x = (const rpg_key_t*)a; const rpg_key_t* y = (const rpg_key_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->sc != y->sc) return x->sc < y->sc ? -1 : 1;
    return (x->rank > y->rank) - (x->rank < y->rank);
}

/* R31: (S^r, sum of arc levels, S^c, CG rank) */
typedef struct { int64_t key; int64_t wsum; int32_t sc; int32_t rank; int64_t t; int64_t sum; } rerank_t;

static int cmp_rerank(const void* a, const void* b) {
    const rerank_t* x = (const rerank_t*)a; const rerank_t* y = (const rerank_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->wsum != y->wsum) return x->wsum < y->wsum ? -1 : 1;
    if (x->sc != y->sc) return x->sc < y->sc ? -1 : 1;
    return (x->rank > y->rank) - (x->rank < y->rank);
}

typedef struct {
    const int32_t* central; int32_t n_central;
    const int32_t* marginal; int32_t n_marginal;
    int32_t k, w, gamma_num, gamma_den, max_level;
    int32_t score_mode;   /* 0: Eq. 6, 1: S^c * S^m (R30) */
    int32_t rerank;       /* 1: ties of S^r re-ranked by the sum of arc levels (R31) */
    int32_t flags;
    uint64_t shuffle;
} orc_query_t;

/* Output layout (int64 words):
 *   [0] status  [1] number of results  [2] number of CGs found
 *   [3..9]  run 1 stats  [10..16] run 2 stats   (levels, end, frontier,
 *                                                e_arc, e_alg, gate_pass, h_writes)
 *   per result: central, S^c, S^m, key, sum of arc levels, n_nodes, nodes...,
 *               n_arcs, (src, dst, label) per arc.
 * Nodes ascending; arcs ascending by CSR position (= by src, label, dst). */
#define HDR 17

static int emit(vec_t* out, int64_t x) { return vec_push(out, x); }

int orc_query(const orc_graph* g, const uint8_t* act, const orc_query_t* q, int64_t** out_buf,
              int64_t* out_len) {
    const int32_t n = g->n;
    const int C = q->n_central, M = q->n_marginal;
    const int64_t gn = q->gamma_num, gd = q->gamma_den;
    if (C < 1 || C > 64 || M < 0 || M > 64 || q->k < 1 || q->w < q->k || gd < 1 || gn < 0 ||
        gn > gd || q->max_level < 0 || q->max_level > 250)
        return -1;
    vec_t out = {0};
    for (int i = 0; i < HDR; ++i) emit(&out, 0);
    int64_t status = 0;
    int rc = 0;

    /* ---- run 1: central keywords -> top-w CGs ---- */
    explore_t x;
    int empty = explore_init(&x, g, act, q->central, C, q->shuffle);
    if (empty < 0) { explore_free(&x); free(out.v); return -2; }
    cg_t* cgs = (cg_t*)malloc(sizeof(cg_t) * (size_t)n);
    int64_t ncg = 0;
    if (empty) {
        x.st.end_reason = END_EMPTY_KEYWORD;
    } else {
        for (int l = 0;; ++l) {
            enqueue(&x);
            x.st.levels = l + 1;
            if (x.nq == 0) { x.st.end_reason = END_EXHAUSTED; break; }
            /* Result Identification (Theorem identifyCG) */
            for (int64_t qi = 0; qi < x.nq; ++qi) {
                const int32_t f = x.Q[qi];
                if (x.CF[f] || !row_complete(&x, f)) continue;
                x.CF[f] = 1;
                cg_t c = {f, 0, 0};
                for (int i = 0; i < C; ++i) {
                    int h = x.H[(size_t)f * C + i];
                    if (h > c.sc) c.sc = h;
                    c.sumh += h;
                }
                cgs[ncg++] = c;
            }
            if (ncg >= q->w) { x.st.end_reason = END_STOP; break; }
            if (l == q->max_level) { x.st.end_reason = END_LEVEL_BOUND; break; }
            expand(&x, l, !(q->flags & FLAG_NO_CG_BLOCK));
        }
    }
    if (x.st.end_reason == END_LEVEL_BOUND) status |= 1;
    qsort(cgs, (size_t)ncg, sizeof(cg_t), cmp_cg);
    const int64_t nsel = ncg < q->w ? ncg : q->w;
    uint8_t* Hc = x.H;
    x.H = NULL;
    orc_run_stats st1 = x.st;
    explore_free(&x);

    /* ---- recovering phase for the selected CGs (Algorithm 2) ---- */
    int32_t* stamp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    vec_t* cg_nodes = (vec_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(vec_t));
    vec_t* cg_arcs = (vec_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(vec_t));
    vec_t* vc = (vec_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(vec_t));
    for (int32_t v = 0; v < n; ++v) stamp[v] = -1;
    int32_t stamp_id = 0;
    for (int64_t r = 0; r < nsel && rc == 0; ++r) {
        const int32_t vc0 = cgs[r].node;
        for (int i = 0; i < C && rc == 0; ++i)
            rc = recover_column(g, act, Hc, C, i, &vc0, 1, &cg_nodes[r], &cg_arcs[r], stamp,
                                stamp_id++, queue);
        sort_unique(&cg_nodes[r]);
        sort_unique(&cg_arcs[r]);
        /* V_C: nodes of the CG containing a central keyword */
        for (int64_t k = 0; k < cg_nodes[r].n; ++k) {
            const int64_t v = cg_nodes[r].v[k];
            for (int i = 0; i < C; ++i)
                if (Hc[(size_t)v * C + i] == 0) { vec_push(&vc[r], v); break; }
        }
    }

    /* ---- run 2: marginal keywords -> RPGs ---- */
    int32_t* has_rpg = (int32_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int32_t));
    int32_t* sm = (int32_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int32_t));
    int64_t* key = (int64_t*)calloc((size_t)(nsel > 0 ? nsel : 1), sizeof(int64_t));
    uint8_t* dmin = (uint8_t*)calloc((size_t)(nsel > 0 ? nsel : 1) * (size_t)(M > 0 ? M : 1), 1);
    rpg_key_t* ranked = (rpg_key_t*)malloc(sizeof(rpg_key_t) * (size_t)(nsel > 0 ? nsel : 1));
    uint8_t* Hm = NULL;
    orc_run_stats st2;
    memset(&st2, 0, sizeof(st2));
    int64_t nres = 0;
    if (rc == 0 && M > 0 && nsel > 0) {
        explore_t y;
        int emptym = explore_init(&y, g, act, q->marginal, M, q->shuffle ? q->shuffle + 1 : 0);
        if (emptym < 0) rc = -2;
        else if (emptym) y.st.end_reason = END_EMPTY_KEYWORD;
        else {
            const int block = (M >= 2) && !(q->flags & FLAG_NO_M_BLOCK);
            int64_t nrpg = 0;
            for (int l = 0;; ++l) {
                enqueue(&y);
                y.st.levels = l + 1;
                if (y.nq == 0) { y.st.end_reason = END_EXHAUSTED; break; }
                /* PTC guard: stop expanding nodes reached by all marginal keywords */
                if (block)
                    for (int64_t qi = 0; qi < y.nq; ++qi)
                        if (!y.CF[y.Q[qi]] && row_complete(&y, y.Q[qi])) y.CF[y.Q[qi]] = 1;
                /* RPG identification: scan the rows of each CG's V_C */
                for (int64_t r = 0; r < nsel; ++r) {
                    if (has_rpg[r]) continue;
                    int all = 1, smax = 0;
                    for (int j = 0; j < M && all; ++j) {
                        int d = INF_LEVEL;
                        for (int64_t k = 0; k < vc[r].n; ++k) {
                            int h = y.H[(size_t)vc[r].v[k] * M + j];
                            if (h < d) d = h;
                        }
                        if (d == INF_LEVEL) all = 0;
                        dmin[r * M + j] = (uint8_t)d;
                        if (d > smax) smax = d;
                    }
                    if (!all) continue;
                    has_rpg[r] = 1;
                    sm[r] = smax;                                        /* Eq. 5 */
                    key[r] = q->score_mode ? (int64_t)cgs[r].sc * smax   /* R30 */
                                           : gn * cgs[r].sc + (gd - gn) * (int64_t)smax; /* Eq. 6, scaled by gamma_den */
                    ++nrpg;
                }
                if (nrpg == nsel) { y.st.end_reason = END_STOP; break; }
                if (nrpg >= q->k && !(q->flags & FLAG_NO_THM4)) {
                    /* Theorem 4 */
                    int64_t m = 0;
                    for (int64_t r = 0; r < nsel; ++r)
                        if (has_rpg[r]) { ranked[m].key = key[r]; ranked[m].sc = cgs[r].sc; ranked[m].rank = (int32_t)r; ++m; }
                    qsort(ranked, (size_t)m, sizeof(rpg_key_t), cmp_rpg);
                    const rpg_key_t kth = ranked[q->k - 1];
                    int64_t min_sc = INT64_MAX;
                    for (int64_t r = 0; r < nsel; ++r)
                        if (!has_rpg[r] && cgs[r].sc < min_sc) min_sc = cgs[r].sc;
                    const int64_t bound = q->score_mode ? min_sc * (int64_t)sm[kth.rank]
                                                        : gn * min_sc + (gd - gn) * (int64_t)sm[kth.rank];
                    if (q->rerank ? kth.key < bound : kth.key <= bound) {
                        y.st.end_reason = END_STOP;
                        break;
                    }
                }
                if (l == q->max_level) { y.st.end_reason = END_LEVEL_BOUND; break; }
                expand(&y, l, block);
            }
        }
        if (y.st.end_reason == END_LEVEL_BOUND) status |= 2;
        st2 = y.st;
        Hm = y.H;
        y.H = NULL;
        explore_free(&y);
    }

    /* ---- ranking and output ---- */
    int64_t m = 0;
    for (int64_t r = 0; r < nsel; ++r) {
        if (M == 0) { has_rpg[r] = 1; sm[r] = 0; key[r] = q->score_mode ? cgs[r].sc : gn * cgs[r].sc; }
        if (has_rpg[r]) { ranked[m].key = key[r]; ranked[m].sc = cgs[r].sc; ranked[m].rank = (int32_t)r; ++m; }
    }
    qsort(ranked, (size_t)m, sizeof(rpg_key_t), cmp_rpg);
    /* results to build: the top k, or with re-ranking every RPG whose key does
       not exceed the k-th one's (R31) */
    int64_t nbuild = m < q->k ? m : q->k;
    if (q->rerank && nbuild > 0)
        while (nbuild < m && ranked[nbuild].key <= ranked[q->k - 1].key) ++nbuild;
    vec_t* rnodes = (vec_t*)calloc((size_t)(nbuild > 0 ? nbuild : 1), sizeof(vec_t));
    vec_t* rarcs = (vec_t*)calloc((size_t)(nbuild > 0 ? nbuild : 1), sizeof(vec_t));
    rerank_t* order = (rerank_t*)malloc(sizeof(rerank_t) * (size_t)(nbuild > 0 ? nbuild : 1));
    for (int64_t t = 0; t < nbuild && rc == 0; ++t) {
        const int32_t r = ranked[t].rank;
        vec_t* nodes = &rnodes[t];
        vec_t* arcs = &rarcs[t];
        for (int64_t k = 0; k < cg_nodes[r].n; ++k) vec_push(nodes, cg_nodes[r].v[k]);
        for (int64_t k = 0; k < cg_arcs[r].n; ++k) vec_push(arcs, cg_arcs[r].v[k]);
        /* marginal part: SP(m_j, V_C) from the V_C nodes at distance D_j */
        int32_t* starts = (int32_t*)malloc(sizeof(int32_t) * (size_t)(vc[r].n > 0 ? vc[r].n : 1));
        for (int j = 0; j < M && rc == 0; ++j) {
            int64_t ns = 0;
            for (int64_t k = 0; k < vc[r].n; ++k)
                if (Hm[(size_t)vc[r].v[k] * M + j] == dmin[r * M + j]) starts[ns++] = (int32_t)vc[r].v[k];
            rc = recover_column(g, act, Hm, M, j, starts, ns, nodes, arcs, stamp, stamp_id++, queue);
        }
        free(starts);
        sort_unique(nodes);
        sort_unique(arcs);
        int64_t wsum = 0;
        for (int64_t k = 0; k < arcs->n; ++k) wsum += act[arcs->v[k]];
        order[t].key = ranked[t].key;
        order[t].wsum = q->rerank ? wsum : 0;
        order[t].sc = ranked[t].sc;
        order[t].rank = ranked[t].rank;
        order[t].t = t;
        order[t].sum = wsum;
    }
    if (q->rerank) qsort(order, (size_t)nbuild, sizeof(rerank_t), cmp_rerank);
    nres = nbuild < q->k ? nbuild : q->k;
    for (int64_t i = 0; i < nres && rc == 0; ++i) {
        const int64_t t = order[i].t;
        const int32_t r = ranked[t].rank;
        const vec_t* nodes = &rnodes[t];
        const vec_t* arcs = &rarcs[t];
        emit(&out, cgs[r].node); emit(&out, cgs[r].sc); emit(&out, sm[r]); emit(&out, key[r]);
        emit(&out, order[i].sum);
        emit(&out, nodes->n);
        for (int64_t k = 0; k < nodes->n; ++k) emit(&out, nodes->v[k]);
        emit(&out, arcs->n);
        for (int64_t k = 0; k < arcs->n; ++k) {
            const int64_t e = arcs->v[k];
            int32_t lo = 0, hi = n;   /* source row of arc e */
            while (hi - lo > 1) { int32_t mid = lo + (hi - lo) / 2; if (g->row_ptr[mid] <= e) lo = mid; else hi = mid; }
            emit(&out, lo); emit(&out, g->col[e]); emit(&out, g->label[e]);
        }
    }
    for (int64_t t = 0; t < nbuild; ++t) { free(rnodes[t].v); free(rarcs[t].v); }
    free(rnodes); free(rarcs); free(order);

    out.v[0] = status; out.v[1] = nres; out.v[2] = ncg;
    const orc_run_stats* sts[2] = {&st1, &st2};
    for (int s = 0; s < 2; ++s) {
        int64_t* d = out.v + 3 + 7 * s;
        d[0] = sts[s]->levels; d[1] = sts[s]->end_reason; d[2] = sts[s]->frontier;
        d[3] = sts[s]->e_arc; d[4] = sts[s]->e_alg; d[5] = sts[s]->gate_pass; d[6] = sts[s]->h_writes;
    }

    for (int64_t r = 0; r < nsel; ++r) { free(cg_nodes[r].v); free(cg_arcs[r].v); free(vc[r].v); }
    free(cg_nodes); free(cg_arcs); free(vc);
    free(has_rpg); free(sm); free(key); free(dmin); free(ranked);
    free(stamp); free(queue); free(cgs); free(Hc); free(Hm);
    if (rc) { free(out.v); return rc; }
    *out_buf = out.v;
    *out_len = out.n;
    return 0;
}

void orc_free(void* p) { free(p); }
