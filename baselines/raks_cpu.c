/*
 * raks_cpu.c -- the paper's multi-core CPU variant of RAKS ("Efficient Radial
 * Pattern Keyword Search on Knowledge Graphs in Parallel", Yang & Tung,
 * Section 4.2.4 "Scheduling"): OpenMP, one thread per frontier handling all
 * of its keywords (the coarse-grained CPU parallelism of Algorithm 1, line
 * 1), dynamic scheduling for load balance.
 *
 * A host baseline for the GPU library, not part of it: it shares no code
 * with the GPU path or with the plain reference implementation.  Its results
 * and work counters equal the reference's on every query (the writes of one
 * level all store the same value, Theorem "lockfree"; a compare-and-swap on
 * the H byte makes the count of written entries exact).  Activation levels
 * are an input of the query entry point; rcpu_activation computes them with
 * OpenMP (its own code: label runs counted per row, the destination's count
 * by a search of its row, Eqs. 1-3 once per distinct count).
 *
 * Output: the same int64 words as the reference implementation (status,
 * result count, CG count, two blocks of run counters, then per result:
 * central node, S^c, S^m, key, arc-level sum, nodes, arcs as triples).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NOT_REACHED 255

typedef struct {
    int32_t n;
    int64_t A;
    const int64_t* row_ptr;
    const int32_t* col;
    const uint16_t* label;
    int32_t vocab;
    const int64_t* kw_ptr;
    const int32_t* kw_nodes;
} rcpu_graph;

typedef struct {
    const int32_t* central;
    int32_t n_central;
    const int32_t* marginal;
    int32_t n_marginal;
    int32_t k, w, gamma_num, gamma_den, max_level;
    int32_t score_mode;   /* 0: gamma-weighted sum, 1: product S^c * S^m */
    int32_t rerank;       /* 1: equal keys re-ranked by the arcs' level sum */
} rcpu_query_t;

enum { E_NONE = 0, E_EXHAUSTED = 1, E_STOP = 2, E_BOUND = 3, E_EMPTY = 4 };

typedef struct { int64_t levels, end, frontier, e_arc, e_alg, gate, hw; } counters_t;

/* growable int64 list */
typedef struct { int64_t* p; int64_t n, cap; } list_t;

static void lpush(list_t* l, int64_t x) {
    if (l->n == l->cap) {
        l->cap = l->cap ? l->cap * 2 : 32;
        l->p = (int64_t*)realloc(l->p, sizeof(int64_t) * (size_t)l->cap);
    }
    l->p[l->n++] = x;
}

static int cmp64(const void* a, const void* b) {
    const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static void lsort_unique(list_t* l) {
    if (l->n < 2) return;
    qsort(l->p, (size_t)l->n, sizeof(int64_t), cmp64);
    int64_t w = 1;
    for (int64_t i = 1; i < l->n; ++i)
        if (l->p[i] != l->p[w - 1]) l->p[w++] = l->p[i];
    l->n = w;
}

/* ---------------------------------------------------------- one run --- */

typedef struct {
    const rcpu_graph* g;
    const uint8_t* act;
    int T;
    uint8_t* H;        /* n x T hitting levels */
    uint8_t* F;        /* frontier flags */
    uint8_t* CF;       /* joining flags */
    int32_t* Q;        /* frontiers of the level, node order */
    int64_t nq;
    int64_t* part;     /* per-thread counts for the ordered enqueue */
    counters_t c;
} run_t;

static int run_init(run_t* r, const rcpu_graph* g, const uint8_t* act, const int32_t* kws, int T) {
    memset(r, 0, sizeof(*r));
    r->g = g;
    r->act = act;
    r->T = T;
    const size_t n = (size_t)g->n;
    r->H = (uint8_t*)malloc(n * (size_t)T);
    r->F = (uint8_t*)calloc(n, 1);
    r->CF = (uint8_t*)calloc(n, 1);
    r->Q = (int32_t*)malloc(sizeof(int32_t) * n);
    r->part = (int64_t*)calloc((size_t)omp_get_max_threads() + 1, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)(n * (size_t)T); ++i) r->H[i] = NOT_REACHED;
    int empty = 0;
    for (int i = 0; i < T; ++i) {
        const int32_t t = kws[i];
        if (g->kw_ptr[t + 1] == g->kw_ptr[t]) empty = 1;
        for (int64_t p = g->kw_ptr[t]; p < g->kw_ptr[t + 1]; ++p) {
            r->H[(size_t)g->kw_nodes[p] * T + i] = 0;
            r->F[g->kw_nodes[p]] = 1;
        }
    }
    return empty;
}

static void run_free(run_t* r) { free(r->H); free(r->F); free(r->CF); free(r->Q); free(r->part); }

/* Frontier Enqueue in node order: each thread takes a contiguous range. */
static void run_enqueue(run_t* r) {
    const int32_t n = r->g->n;
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        nt = omp_get_num_threads();
        const int t = omp_get_thread_num();
        const int32_t lo = (int32_t)((int64_t)n * t / nt), hi = (int32_t)((int64_t)n * (t + 1) / nt);
        int64_t cnt = 0;
        for (int32_t v = lo; v < hi; ++v) cnt += r->F[v] != 0;
        r->part[t + 1] = cnt;
#pragma omp barrier
#pragma omp single
        {
            r->part[0] = 0;
            for (int i = 0; i < nt; ++i) r->part[i + 1] += r->part[i];
        }
        int64_t pos = r->part[t];
        for (int32_t v = lo; v < hi; ++v)
            if (r->F[v]) { r->Q[pos++] = v; r->F[v] = 0; }
    }
    r->nq = r->part[nt];
    r->c.frontier += r->nq;
}

static int complete(const run_t* r, int32_t v) {
    for (int i = 0; i < r->T; ++i)
        if (r->H[(size_t)v * r->T + i] == NOT_REACHED) return 0;
    return 1;
}

/* Algorithm 1 at Glevel l: one thread per frontier, all its keywords. */
static void run_expand(run_t* r, int l, int use_cf) {
    const rcpu_graph* g = r->g;
    const int T = r->T;
    int64_t e_arc = 0, e_alg = 0, gate = 0, hw = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : e_arc, e_alg, gate, hw)
    for (int64_t qi = 0; qi < r->nq; ++qi) {
        const int32_t f = r->Q[qi];
        if (use_cf && r->CF[f]) continue;
        const int64_t r0 = g->row_ptr[f], r1 = g->row_ptr[f + 1];
        int active = 0;
        for (int i = 0; i < T; ++i) {
            if (__atomic_load_n(&r->H[(size_t)f * T + i], __ATOMIC_RELAXED) > l) continue;
            active = 1;
            e_alg += r1 - r0;
            for (int64_t e = r0; e < r1; ++e) {
                if (r->act[e] > l) {                               /* f stays a frontier */
                    __atomic_store_n(&r->F[f], (uint8_t)1, __ATOMIC_RELAXED);
                    continue;
                }
                const int32_t nb = g->col[e];
                uint8_t* h = &r->H[(size_t)nb * T + i];
                uint8_t expect = NOT_REACHED;
                if (__atomic_load_n(h, __ATOMIC_RELAXED) != NOT_REACHED) continue;
                if (__atomic_compare_exchange_n(h, &expect, (uint8_t)(l + 1), 0, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED)) {
                    __atomic_store_n(&r->F[nb], (uint8_t)1, __ATOMIC_RELAXED);
                    ++hw;
                }
            }
        }
        if (active) {
            e_arc += r1 - r0;
            for (int64_t e = r0; e < r1; ++e) gate += r->act[e] <= l;
        }
    }
    r->c.e_arc += e_arc;
    r->c.e_alg += e_alg;
    r->c.gate += gate;
    r->c.hw += hw;
}

/* --------------------------------------------- activation (Eqs. 1-3) --- */

/* Level of a rescaled weight x in [0,1]: reward below alpha, penalty above,
 * rounded half up; IEEE binary64 in the order the equations are written. */
static int level_x(double x, double abar, double alpha) {
    double v;
    if (x <= alpha) v = abar - abar * (alpha - x) / alpha;
    else v = abar + abar * (x - alpha) / (1.0 - alpha);
    double r = floor(v + 0.5);
    if (r < 0.0) r = 0.0;
    if (r > 254.0) r = 254.0;
    return (int)r;
}

/* Arcs of row v with label lab (rows sorted by label, then destination). */
static int64_t label_run(const rcpu_graph* g, int32_t v, uint16_t lab) {
    int64_t lo = g->row_ptr[v], hi = g->row_ptr[v + 1];
    int64_t a = lo, b = hi;
    while (a < b) { const int64_t m = a + (b - a) / 2; if (g->label[m] < lab) a = m + 1; else b = m; }
    int64_t c = a, d = hi;
    while (c < d) { const int64_t m = c + (d - c) / 2; if (g->label[m] <= lab) c = m + 1; else d = m; }
    return c - a;
}

/* Per-arc levels act[A].  mode 0 (per arc): c = |arcs of the source with the
 * label| + |arcs of the destination with the label| (the in-arcs of the
 * destination are the reverses of its out-arcs), weight ln c min-max
 * rescaled; mode 1 (per node): the destination's node weight min-max
 * rescaled.  Returns 0, or -1 for bad arguments / -2 when memory runs out. */
int rcpu_activation(const rcpu_graph* g, const uint8_t* node_weight, double abar, double alpha,
                    int mode, int threads, uint8_t* act) {
    if (!(alpha > 0.0 && alpha < 1.0) || !(abar > 0.0)) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    const int64_t A = g->A;
    if (mode == 1) {
        int wmin = 255, wmax = 0;
        for (int32_t v = 0; v < g->n; ++v) {
            if (node_weight[v] < wmin) wmin = node_weight[v];
            if (node_weight[v] > wmax) wmax = node_weight[v];
        }
        uint8_t lut[256];
        for (int w = wmin; w <= wmax; ++w) {
            const double x = (wmax == wmin) ? 0.0 : ((double)w - (double)wmin) / ((double)wmax - (double)wmin);
            lut[w] = (uint8_t)level_x(x, abar, alpha);
        }
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < A; ++e) act[e] = lut[node_weight[g->col[e]]];
        return 0;
    }
    if (mode != 0) return -1;
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(A > 0 ? A : 1));
    if (!c) return -2;
    /* label runs of each row, then the destination's count of the same label */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t v = 0; v < g->n; ++v) {
        for (int64_t s = g->row_ptr[v]; s < g->row_ptr[v + 1];) {
            int64_t t = s + 1;
            while (t < g->row_ptr[v + 1] && g->label[t] == g->label[s]) ++t;
            for (int64_t e = s; e < t; ++e) c[e] = t - s;
            s = t;
        }
    }
    int64_t cmin = INT64_MAX, cmax = 0;
#pragma omp parallel for schedule(static) reduction(min : cmin) reduction(max : cmax)
    for (int64_t e = 0; e < A; ++e) {
        c[e] += label_run(g, g->col[e], g->label[e]);
        if (c[e] < cmin) cmin = c[e];
        if (c[e] > cmax) cmax = c[e];
    }
    if (A == 0) { free(c); return 0; }
    const int64_t span = cmax - cmin + 1;
    uint8_t* lut = (uint8_t*)malloc((size_t)span);
    if (!lut) { free(c); return -2; }
    const double wmin = log((double)cmin), wmax = log((double)cmax);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < span; ++k) {
        const double w = log((double)(cmin + k));
        const double x = (cmax == cmin) ? 0.0 : (w - wmin) / (wmax - wmin);
        lut[k] = (uint8_t)level_x(x, abar, alpha);
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < A; ++e) act[e] = lut[c[e] - cmin];
    free(lut);
    free(c);
    return 0;
}

/* Exploration alone (Algorithm 1, Sections 4.2.2-4.2.4) from the keywords'
 * node sets until the frontier is empty or the level bound: with `block`, a
 * node reached by every keyword stops expanding.  counters: levels, end
 * reason, frontier sum, e_arc, e_alg, gate passes, entries written. */
int rcpu_explore(const rcpu_graph* g, const uint8_t* act, const int32_t* kws, int32_t T,
                 int32_t block, int32_t max_level, int threads, int64_t* counters) {
    if (T < 1) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    run_t x;
    if (run_init(&x, g, act, kws, T)) { run_free(&x); return -1; }
    for (int l = 0;; ++l) {
        run_enqueue(&x);
        x.c.levels = l + 1;
        if (x.nq == 0) { x.c.end = E_EXHAUSTED; break; }
        if (block) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < x.nq; ++i)
                if (!x.CF[x.Q[i]] && complete(&x, x.Q[i])) x.CF[x.Q[i]] = 1;
        }
        if (l == max_level) { x.c.end = E_BOUND; break; }
        run_expand(&x, l, block);
    }
    const counters_t k = x.c;
    counters[0] = k.levels; counters[1] = k.end; counters[2] = k.frontier; counters[3] = k.e_arc;
    counters[4] = k.e_alg; counters[5] = k.gate; counters[6] = k.hw;
    run_free(&x);
    return 0;
}

/* ----------------------------------------------------------- recovery --- */

static int64_t arc_pos(const rcpu_graph* g, int32_t src, uint16_t lab, int32_t dst) {
    int64_t lo = g->row_ptr[src], hi = g->row_ptr[src + 1];
    while (lo < hi) {
        const int64_t m = lo + (hi - lo) / 2;
        if (g->label[m] < lab || (g->label[m] == lab && g->col[m] < dst)) lo = m + 1;
        else hi = m;
    }
    return (lo < g->row_ptr[src + 1] && g->label[lo] == lab && g->col[lo] == dst) ? lo : -1;
}

/* Algorithm 2 for one keyword column from the given start nodes: keeps the
 * in-arc n -> q when h_q = 1 + max(a, h_n) (Lemma 1) and continues from n
 * while h_n > 0.  stamp / queue are the calling thread's. */
static void recover(const rcpu_graph* g, const uint8_t* act, const uint8_t* H, int T, int col,
                    const int64_t* start, int64_t ns, list_t* nodes, list_t* arcs,
                    int32_t* stamp, int32_t id, int32_t* queue) {
    int64_t head = 0, tail = 0;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t v = (int32_t)start[s];
        lpush(nodes, v);
        if (stamp[v] != id) { stamp[v] = id; queue[tail++] = v; }
    }
    while (head < tail) {
        const int32_t q = queue[head++];
        const int hq = H[(size_t)q * T + col];
        for (int64_t e = g->row_ptr[q]; e < g->row_ptr[q + 1]; ++e) {
            const int32_t nb = g->col[e];
            const int64_t back = arc_pos(g, nb, g->label[e], q);
            const int a = act[back], hn = H[(size_t)nb * T + col];
            if (hq != 1 + (a > hn ? a : hn)) continue;
            lpush(nodes, nb);
            lpush(arcs, back);
            if (hn != 0 && stamp[nb] != id) { stamp[nb] = id; queue[tail++] = nb; }
        }
    }
}

/* ------------------------------------------------------------- query --- */

typedef struct { int32_t node, sc, sumh; } cg_t;

static int cg_less(const cg_t* a, const cg_t* b) {
    if (a->sc != b->sc) return a->sc < b->sc;
    if (a->sumh != b->sumh) return a->sumh < b->sumh;
    return a->node < b->node;
}

static int cmp_cg(const void* a, const void* b) {
    const cg_t* x = (const cg_t*)a;
    const cg_t* y = (const cg_t*)b;
    return cg_less(x, y) ? -1 : (cg_less(y, x) ? 1 : 0);
}

typedef struct { int64_t key, wsum; int32_t sc, rank; } ord_t;

static int cmp_ord(const void* a, const void* b) {
    const ord_t* x = (const ord_t*)a;
    const ord_t* y = (const ord_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->wsum != y->wsum) return x->wsum < y->wsum ? -1 : 1;
    if (x->sc != y->sc) return x->sc < y->sc ? -1 : 1;
    return (x->rank > y->rank) - (x->rank < y->rank);
}

int rcpu_query(const rcpu_graph* g, const uint8_t* act, const rcpu_query_t* q, int threads,
               int64_t** out_words, int64_t* out_len) {
    const int C = q->n_central, M = q->n_marginal;
    const int64_t gn = q->gamma_num, gd = q->gamma_den;
    if (C < 1 || M < 0 || q->k < 1 || q->w < q->k || gd < 1 || gn < 0 || gn > gd) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    const int32_t n = g->n;
    list_t out = {0};
    for (int i = 0; i < 17; ++i) lpush(&out, 0);
    int64_t status = 0;

    /* run 1: central keywords until w central graphs */
    run_t x;
    const int empty = run_init(&x, g, act, q->central, C);
    cg_t* cgs = (cg_t*)malloc(sizeof(cg_t) * (size_t)n);
    int64_t ncg = 0;
    if (empty) {
        x.c.end = E_EMPTY;
    } else {
        for (int l = 0;; ++l) {
            run_enqueue(&x);
            x.c.levels = l + 1;
            if (x.nq == 0) { x.c.end = E_EXHAUSTED; break; }
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < x.nq; ++i) {
                const int32_t f = x.Q[i];
                if (x.CF[f] || !complete(&x, f)) continue;
                x.CF[f] = 1;
                cg_t c = {f, 0, 0};
                for (int j = 0; j < C; ++j) {
                    const int h = x.H[(size_t)f * C + j];
                    c.sc = h > c.sc ? h : c.sc;
                    c.sumh += h;
                }
                int64_t slot;
#pragma omp atomic capture
                slot = ncg++;
                cgs[slot] = c;
            }
            if (ncg >= q->w) { x.c.end = E_STOP; break; }
            if (l == q->max_level) { x.c.end = E_BOUND; break; }
            run_expand(&x, l, 1);
        }
    }
    if (x.c.end == E_BOUND) status |= 1;
    qsort(cgs, (size_t)ncg, sizeof(cg_t), cmp_cg);
    const int64_t nsel = ncg < q->w ? ncg : q->w;
    const counters_t c1 = x.c;

    /* recovery of the selected CGs: one (CG, keyword) instance per task */
    const int nth = omp_get_max_threads();
    int32_t* stamps = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * (size_t)nth);
    int32_t* queues = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * (size_t)nth);
    for (int64_t i = 0; i < (int64_t)n * nth; ++i) stamps[i] = -1;
    list_t* inst_nodes = (list_t*)calloc((size_t)(nsel * C + 1), sizeof(list_t));
    list_t* inst_arcs = (list_t*)calloc((size_t)(nsel * C + 1), sizeof(list_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t it = 0; it < nsel * C; ++it) {
        const int t = omp_get_thread_num();
        const int64_t s = cgs[it / C].node;
        recover(g, act, x.H, C, (int)(it % C), &s, 1, &inst_nodes[it], &inst_arcs[it],
                stamps + (size_t)t * n, (int32_t)it, queues + (size_t)t * n);
    }
    list_t* cg_nodes = (list_t*)calloc((size_t)(nsel + 1), sizeof(list_t));
    list_t* cg_arcs = (list_t*)calloc((size_t)(nsel + 1), sizeof(list_t));
    list_t* vc = (list_t*)calloc((size_t)(nsel + 1), sizeof(list_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nsel; ++r) {
        for (int j = 0; j < C; ++j) {
            const list_t* a = &inst_nodes[r * C + j];
            const list_t* b = &inst_arcs[r * C + j];
            for (int64_t i = 0; i < a->n; ++i) lpush(&cg_nodes[r], a->p[i]);
            for (int64_t i = 0; i < b->n; ++i) lpush(&cg_arcs[r], b->p[i]);
        }
        lsort_unique(&cg_nodes[r]);
        lsort_unique(&cg_arcs[r]);
        for (int64_t i = 0; i < cg_nodes[r].n; ++i) {
            const int64_t v = cg_nodes[r].p[i];
            for (int j = 0; j < C; ++j)
                if (x.H[(size_t)v * C + j] == 0) { lpush(&vc[r], v); break; }
        }
    }
    for (int64_t i = 0; i < nsel * C; ++i) { free(inst_nodes[i].p); free(inst_arcs[i].p); }
    free(inst_nodes);
    free(inst_arcs);

    /* run 2: marginal keywords, RPG check over each CG's V_C, Theorem 4 */
    int32_t* has = (int32_t*)calloc((size_t)(nsel + 1), sizeof(int32_t));
    int32_t* sm = (int32_t*)calloc((size_t)(nsel + 1), sizeof(int32_t));
    int64_t* key = (int64_t*)calloc((size_t)(nsel + 1), sizeof(int64_t));
    uint8_t* dmin = (uint8_t*)calloc((size_t)(nsel + 1) * (size_t)(M > 0 ? M : 1), 1);
    ord_t* ord = (ord_t*)malloc(sizeof(ord_t) * (size_t)(nsel + 1));
    counters_t c2;
    memset(&c2, 0, sizeof(c2));
    run_t y;
    int have_y = 0;
    if (M > 0 && nsel > 0) {
        have_y = 1;
        const int emptym = run_init(&y, g, act, q->marginal, M);
        if (emptym) {
            y.c.end = E_EMPTY;
        } else {
            const int block = M >= 2;
            int64_t nrpg = 0;
            for (int l = 0;; ++l) {
                run_enqueue(&y);
                y.c.levels = l + 1;
                if (y.nq == 0) { y.c.end = E_EXHAUSTED; break; }
                if (block) {
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < y.nq; ++i)
                        if (!y.CF[y.Q[i]] && complete(&y, y.Q[i])) y.CF[y.Q[i]] = 1;
                }
                int64_t found = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : found)
                for (int64_t r = 0; r < nsel; ++r) {
                    if (has[r]) continue;
                    int all = 1, smax = 0;
                    for (int j = 0; j < M; ++j) {
                        int d = NOT_REACHED;
                        for (int64_t i = 0; i < vc[r].n; ++i) {
                            const int h = y.H[(size_t)vc[r].p[i] * M + j];
                            d = h < d ? h : d;
                        }
                        dmin[r * M + j] = (uint8_t)d;
                        if (d == NOT_REACHED) all = 0;
                        smax = d > smax ? d : smax;
                    }
                    if (!all) continue;
                    has[r] = 1;
                    sm[r] = smax;
                    key[r] = q->score_mode ? (int64_t)cgs[r].sc * smax : gn * cgs[r].sc + (gd - gn) * smax;
                    ++found;
                }
                nrpg += found;
                if (nrpg == nsel) { y.c.end = E_STOP; break; }
                if (nrpg >= q->k) {
                    int64_t m = 0, minsc = INT64_MAX;
                    for (int64_t r = 0; r < nsel; ++r) {
                        if (has[r]) { ord[m].key = key[r]; ord[m].wsum = 0; ord[m].sc = cgs[r].sc; ord[m].rank = (int32_t)r; ++m; }
                        else if (cgs[r].sc < minsc) minsc = cgs[r].sc;
                    }
                    qsort(ord, (size_t)m, sizeof(ord_t), cmp_ord);
                    const ord_t kth = ord[q->k - 1];
                    const int64_t bound = q->score_mode ? minsc * sm[kth.rank]
                                                        : gn * minsc + (gd - gn) * sm[kth.rank];
                    if (q->rerank ? kth.key < bound : kth.key <= bound) { y.c.end = E_STOP; break; }
                }
                if (l == q->max_level) { y.c.end = E_BOUND; break; }
                run_expand(&y, l, block);
            }
        }
        if (y.c.end == E_BOUND) status |= 2;
        c2 = y.c;
    }

    /* ranking, RPG recovery, output */
    int64_t m = 0;
    for (int64_t r = 0; r < nsel; ++r) {
        if (M == 0) { has[r] = 1; sm[r] = 0; key[r] = q->score_mode ? cgs[r].sc : gn * cgs[r].sc; }
        if (has[r]) { ord[m].key = key[r]; ord[m].wsum = 0; ord[m].sc = cgs[r].sc; ord[m].rank = (int32_t)r; ++m; }
    }
    qsort(ord, (size_t)m, sizeof(ord_t), cmp_ord);
    int64_t nb = m < q->k ? m : q->k;
    if (q->rerank && nb > 0)
        while (nb < m && ord[nb].key <= ord[q->k - 1].key) ++nb;
    list_t* rn = (list_t*)calloc((size_t)(nb + 1), sizeof(list_t));
    list_t* ra = (list_t*)calloc((size_t)(nb + 1), sizeof(list_t));
    int64_t* sums = (int64_t*)calloc((size_t)(nb + 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nb; ++t) {
        const int th = omp_get_thread_num();
        const int32_t r = ord[t].rank;
        for (int64_t i = 0; i < cg_nodes[r].n; ++i) lpush(&rn[t], cg_nodes[r].p[i]);
        for (int64_t i = 0; i < cg_arcs[r].n; ++i) lpush(&ra[t], cg_arcs[r].p[i]);
        int64_t* starts = (int64_t*)malloc(sizeof(int64_t) * (size_t)(vc[r].n + 1));
        for (int j = 0; j < M; ++j) {
            int64_t ns = 0;
            for (int64_t i = 0; i < vc[r].n; ++i)
                if (y.H[(size_t)vc[r].p[i] * M + j] == dmin[r * M + j]) starts[ns++] = vc[r].p[i];
            recover(g, act, y.H, M, j, starts, ns, &rn[t], &ra[t], stamps + (size_t)th * n,
                    (int32_t)(nsel * C + t * M + j), queues + (size_t)th * n);
        }
        free(starts);
        lsort_unique(&rn[t]);
        lsort_unique(&ra[t]);
        int64_t s = 0;
        for (int64_t i = 0; i < ra[t].n; ++i) s += act[ra[t].p[i]];
        sums[t] = s;
    }
    int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nb + 1));
    for (int64_t t = 0; t < nb; ++t) pick[t] = t;
    if (q->rerank) {
        ord_t* o2 = (ord_t*)malloc(sizeof(ord_t) * (size_t)(nb + 1));
        for (int64_t t = 0; t < nb; ++t) { o2[t] = ord[t]; o2[t].wsum = sums[t]; o2[t].rank = (int32_t)t; }
        /* rank field now indexes the built results; ties keep the CG order
           because results are built in (key, S^c, CG rank) order */
        qsort(o2, (size_t)nb, sizeof(ord_t), cmp_ord);
        for (int64_t t = 0; t < nb; ++t) pick[t] = o2[t].rank;
        free(o2);
    }
    const int64_t nres = nb < q->k ? nb : q->k;
    for (int64_t i = 0; i < nres; ++i) {
        const int64_t t = pick[i];
        const int32_t r = ord[t].rank;
        lpush(&out, cgs[r].node);
        lpush(&out, cgs[r].sc);
        lpush(&out, sm[r]);
        lpush(&out, key[r]);
        lpush(&out, sums[t]);
        lpush(&out, rn[t].n);
        for (int64_t k = 0; k < rn[t].n; ++k) lpush(&out, rn[t].p[k]);
        lpush(&out, ra[t].n);
        for (int64_t k = 0; k < ra[t].n; ++k) {
            const int64_t e = ra[t].p[k];
            int32_t lo = 0, hi = n;
            while (hi - lo > 1) { const int32_t mid = lo + (hi - lo) / 2; if (g->row_ptr[mid] <= e) lo = mid; else hi = mid; }
            lpush(&out, lo);
            lpush(&out, g->col[e]);
            lpush(&out, g->label[e]);
        }
    }
    out.p[0] = status;
    out.p[1] = nres;
    out.p[2] = ncg;
    const counters_t* cs[2] = {&c1, &c2};
    for (int s = 0; s < 2; ++s) {
        int64_t* d = out.p + 3 + 7 * s;
        d[0] = cs[s]->levels; d[1] = cs[s]->end; d[2] = cs[s]->frontier; d[3] = cs[s]->e_arc;
        d[4] = cs[s]->e_alg; d[5] = cs[s]->gate; d[6] = cs[s]->hw;
    }

    for (int64_t t = 0; t < nb; ++t) { free(rn[t].p); free(ra[t].p); }
    free(rn); free(ra); free(sums); free(pick);
    for (int64_t r = 0; r < nsel; ++r) { free(cg_nodes[r].p); free(cg_arcs[r].p); free(vc[r].p); }
    free(cg_nodes); free(cg_arcs); free(vc);
    free(has); free(sm); free(key); free(dmin); free(ord);
    free(stamps); free(queues); free(cgs);
    run_free(&x);
    if (have_y) run_free(&y);
    *out_words = out.p;
    *out_len = out.n;
    return 0;
}

void rcpu_free(void* p) { free(p); }
