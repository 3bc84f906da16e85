/*
 * synth.c -- seeded synthetic knowledge-graph generator.
 *
 * Builds the stand-in inputs for the paper's Wikidata dumps (Section 5.1,
 * Table 1): a bi-directed labelled graph in CSR form, a node weight per node,
 * and a keyword -> node inverted index.  It holds none of the search method's
 * arithmetic (no edge weights, activation levels, path scores or hitting
 * levels); both the reference implementation and the GPU library consume its
 * output unchanged.
 *
 * Recipe (all randomness from one xoshiro256** stream per stage, seeded with
 * splitmix64 from the user seed):
 *   1. degree weights x_u = floor(U^(-1/(alpha-1))), U uniform in (0,1],
 *      capped to [1, n-1]; a random permutation of x gives the target weights,
 *      so in- and out-degrees are both heavy-tailed (Chung-Lu sampling).
 *   2. optional planted hubs: a few nodes get a prescribed number of extra
 *      out-edges with Chung-Lu targets.
 *   3. remaining edges: source ~ x, target ~ permuted x, label uniform over
 *      n_labels.  Self-loops are rejected; duplicate (src,label,dst) triples
 *      are removed and redrawn until exactly n_edges distinct directed edges
 *      exist.
 *   4. node weight = min(255, floor(8*log2(1+in-degree)+0.5)) on the directed
 *      edges (log2 of in-degree quantised to uint8, 3 fractional bits).
 *   5. the graph is made bi-directed: every edge (u,l,v) also appears as
 *      (v,l,u) (Section 2 adds one reverse edge per edge); duplicates are
 *      merged.  Rows of the CSR are sorted by (label, destination).
 *   6. every node gets U{kw_min..kw_max} distinct keywords drawn from a
 *      truncated Zipf(s) law over the vocabulary.
 *   7. the average shortest hop count A-bar is estimated from sampled pairs as
 *      in Section 5.1 (abar_sources BFS roots x abar_targets reached targets),
 *      rounded to two decimals and returned as an integer x100.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define N_CHUNKS 256   /* fixed random-stream chunks: output independent of thread count */

/* ---------------------------------------------------------------- RNG --- */
/* xoshiro256** 1.0 and splitmix64, as published by Blackman and Vigna. */
typedef struct { uint64_t s[4]; } rng_t;

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t splitmix64(uint64_t* st) {
    uint64_t z = (*st += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t* r, uint64_t seed, uint64_t stream) {
    uint64_t st = seed ^ (0xa0761d6478bd642fULL * (stream + 1));
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&st);
}

static inline uint64_t rng_next(rng_t* r) {
    uint64_t* s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* uniform double in [0,1) with 53 random bits */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0,n) by 128-bit multiply (Lemire, without rejection;
 * the bias is below 2^-40 for every n used here) */
static inline uint64_t rng_below(rng_t* r, uint64_t n) {
    return (uint64_t)(((unsigned __int128)rng_next(r) * n) >> 64);
}

/* -------------------------------------------------------------- alias --- */
/* Walker/Vose alias table over non-negative weights. */
typedef struct { int64_t n; double* prob; int64_t* alias; } alias_t;

static int alias_build(alias_t* a, const double* w, int64_t n) {
    a->n = n;
    a->prob = (double*)malloc(sizeof(double) * (size_t)n);
    a->alias = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* small = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    int64_t* large = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* p = (double*)malloc(sizeof(double) * (size_t)n);
    if (!a->prob || !a->alias || !small || !large || !p) return -1;
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += w[i];
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        p[i] = w[i] * (double)n / sum;
        if (p[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = small[--ns], l = large[--nl];
        a->prob[s] = p[s];
        a->alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) { int64_t l = large[--nl]; a->prob[l] = 1.0; a->alias[l] = l; }
    while (ns > 0) { int64_t s = small[--ns]; a->prob[s] = 1.0; a->alias[s] = s; }
    free(small); free(large); free(p);
    return 0;
}

static inline int64_t alias_draw(const alias_t* a, rng_t* r) {
    int64_t i = (int64_t)rng_below(r, (uint64_t)a->n);
    return rng_unit(r) < a->prob[i] ? i : a->alias[i];
}

static void alias_free(alias_t* a) { free(a->prob); free(a->alias); }

/* --------------------------------------------------------- radix sort --- */
/* LSD radix sort of 64-bit keys, 8-bit digits; passes whose digit is
 * constant over all keys are skipped.  Parallel and stable: every thread
 * counts its contiguous slice, offsets are laid out digit-major then by
 * thread, and every thread scatters its slice in order, so the result does
 * not depend on the thread count. */
static int radix_sort_u64(uint64_t* keys, int64_t n, int key_bits) {
    if (n <= 1) return 0;
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    if (!tmp) return -1;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
    if (nt > 64) nt = 64;
#endif
    int64_t (*cnt)[256] = (int64_t(*)[256])calloc((size_t)nt, sizeof(int64_t[256]));
    if (!cnt) { free(tmp); return -1; }
    uint64_t* src = keys; uint64_t* dst = tmp;
    for (int shift = 0; shift < key_bits; shift += 8) {
        int trivial = 0;
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
            memset(cnt[t], 0, sizeof(cnt[t]));
            for (int64_t i = lo; i < hi; ++i) cnt[t][(src[i] >> shift) & 0xff]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t tot[256] = {0};
                for (int d = 0; d < 256; ++d)
                    for (int u = 0; u < nt; ++u) tot[d] += cnt[u][d];
                for (int d = 0; d < 256; ++d) if (tot[d] == n) trivial = 1;
                int64_t off = 0;
                for (int d = 0; d < 256; ++d)
                    for (int u = 0; u < nt; ++u) { int64_t c = cnt[u][d]; cnt[u][d] = off; off += c; }
            }
            if (!trivial)
                for (int64_t i = lo; i < hi; ++i) dst[cnt[t][(src[i] >> shift) & 0xff]++] = src[i];
        }
        if (trivial) continue;
        uint64_t* t = src; src = dst; dst = t;
    }
    if (src != keys) memcpy(keys, src, sizeof(uint64_t) * (size_t)n);
    free(cnt);
    free(tmp);
    return 0;
}

static int64_t unique_sorted_u64(uint64_t* k, int64_t n) {
    if (n == 0) return 0;
    int64_t m = 1;
    for (int64_t i = 1; i < n; ++i) if (k[i] != k[m - 1]) k[m++] = k[i];
    return m;
}

static int bits_for(uint64_t n) { /* bits needed for values 0..n-1 */
    int b = 1;
    while (b < 63 && ((uint64_t)1 << b) < n) ++b;
    return b;
}

/* ---------------------------------------------------------- interface --- */
typedef struct {
    int64_t n_nodes;
    int64_t n_edges;        /* distinct directed edges before the reverse edges */
    double pl_alpha;        /* power-law exponent of the degree weights (> 1) */
    int32_t n_labels;       /* 1..65536 */
    int32_t vocab;          /* number of distinct keywords */
    double zipf_s;          /* Zipf exponent of keyword popularity */
    int32_t kw_min, kw_max; /* keywords per node */
    int32_t n_hubs;         /* planted hubs, at most 8 */
    int64_t hub_deg[8];     /* extra out-edges of each hub */
    uint64_t seed;
    int32_t abar_sources, abar_targets;
} synth_params;

typedef struct {
    int64_t n_nodes, n_arcs, n_kw_entries, vocab, abar_x100, n_edges;
    int64_t* row_ptr;
    int32_t* col;
    uint16_t* label;
    uint8_t* node_weight;
    int64_t* kw_ptr;
    int32_t* kw_nodes;
    int64_t hubs[8];
} synth_graph;

void synth_free(synth_graph* g) {
    if (!g) return;
    free(g->row_ptr); free(g->col); free(g->label); free(g->node_weight);
    free(g->kw_ptr); free(g->kw_nodes);
    free(g);
}

static int64_t estimate_abar_x100(const synth_graph* g, const synth_params* p) {
    const int64_t n = g->n_nodes;
    const int S = p->abar_sources;
    /* roots first (sequential draws), then one BFS per root in parallel */
    int64_t* roots = (int64_t*)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    if (!roots) return -1;
    rng_t r; rng_seed(&r, p->seed, 7);
    int got = 0;
    for (int tries = 0; got < S && tries < 1000000; ++tries) {
        int64_t src = (int64_t)rng_below(&r, (uint64_t)n);
        if (g->row_ptr[src + 1] == g->row_ptr[src]) continue;
        roots[got++] = src;
    }
    int64_t hop_sum = 0, pairs = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : hop_sum, pairs)
    for (int s = 0; s < got; ++s) {
        int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        if (dist && queue) {
            for (int64_t i = 0; i < n; ++i) dist[i] = -1;
            int64_t qh = 0, qt = 0;
            dist[roots[s]] = 0; queue[qt++] = (int32_t)roots[s];
            while (qh < qt) {
                int32_t u = queue[qh++];
                for (int64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
                    int32_t v = g->col[e];
                    if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[qt++] = v; }
                }
            }
            rng_t rt; rng_seed(&rt, p->seed, 1000 + (uint64_t)s);
            if (qt > 1)
                for (int t = 0; t < p->abar_targets; ++t) {
                    int64_t idx = 1 + (int64_t)rng_below(&rt, (uint64_t)(qt - 1));
                    hop_sum += dist[queue[idx]];
                    ++pairs;
                }
        }
        free(dist); free(queue);
    }
    free(roots);
    if (pairs == 0) return -1;
    double mean = (double)hop_sum / (double)pairs;
    return (int64_t)floor(mean * 100.0 + 0.5);
}

/* Phase lines on stderr when SYNTH_PROGRESS is set (long generations). */
static void progress(const char* what, double t0) {
    const char* e = getenv("SYNTH_PROGRESS");
    if (e && *e && *e != '0') {
        fprintf(stderr, "[synth] %s (%.1f s)\n", what, omp_get_wtime() - t0);
        fflush(stderr);
    }
}

synth_graph* synth_generate(const synth_params* p) {
    const double t_start = omp_get_wtime();
    const int64_t n = p->n_nodes, E = p->n_edges;
    if (n < 2 || E < 1 || p->n_labels < 1 || p->n_labels > 65536 || p->vocab < 1 ||
        p->kw_min < 0 || p->kw_max < p->kw_min || p->kw_max > p->vocab || p->n_hubs < 0 ||
        p->n_hubs > 8 || p->pl_alpha <= 1.0 || n > ((int64_t)1 << 31) - 1)
        return NULL;
    const int nb = bits_for((uint64_t)n), lb = bits_for((uint64_t)p->n_labels);
    if (2 * nb + lb > 64) return NULL;
    int64_t hub_total = 0;
    for (int h = 0; h < p->n_hubs; ++h) hub_total += p->hub_deg[h];
    if (hub_total > E || (double)E > 0.5 * (double)n * (double)(n - 1) * p->n_labels) return NULL;

    synth_graph* g = (synth_graph*)calloc(1, sizeof(synth_graph));
    if (!g) return NULL;
    g->n_nodes = n; g->vocab = p->vocab; g->n_edges = E;

    /* 1. degree weights and Chung-Lu samplers */
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!w || !perm) goto fail;
    {
        rng_t r; rng_seed(&r, p->seed, 1);
        const double ex = -1.0 / (p->pl_alpha - 1.0);
        for (int64_t i = 0; i < n; ++i) {
            double u = 1.0 - rng_unit(&r);               /* (0,1] */
            double x = floor(pow(u, ex));
            if (x < 1.0) x = 1.0;
            if (x > (double)(n - 1)) x = (double)(n - 1);
            w[i] = x;
        }
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        for (int64_t i = n - 1; i > 0; --i) {
            int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
            int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }
    alias_t src_al, dst_al;
    if (alias_build(&src_al, w, n)) goto fail;
    {
        double* wt = (double*)malloc(sizeof(double) * (size_t)n);
        if (!wt) goto fail;
        for (int64_t i = 0; i < n; ++i) wt[i] = w[perm[i]];
        int rc = alias_build(&dst_al, wt, n);
        free(wt);
        if (rc) goto fail;
    }
    free(w); w = NULL;
    free(perm); perm = NULL;

    progress("degree weights", t_start);
    /* 2.-3. directed edges, deduplicated to exactly E */
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(2 * E));
    if (!keys) goto fail;
    {
        rng_t r; rng_seed(&r, p->seed, 2);
        const int sh_l = nb, sh_s = nb + lb;
        int64_t m = 0;
        for (int h = 0; h < p->n_hubs; ++h) {
            int64_t hub;
            for (;;) {   /* distinct hub ids */
                hub = (int64_t)rng_below(&r, (uint64_t)n);
                int dup = 0;
                for (int k = 0; k < h; ++k) if (g->hubs[k] == hub) dup = 1;
                if (!dup) break;
            }
            g->hubs[h] = hub;
            for (int64_t k = 0; k < p->hub_deg[h]; ++k) {
                int64_t t;
                do { t = alias_draw(&dst_al, &r); } while (t == hub);
                uint64_t l = rng_below(&r, (uint64_t)p->n_labels);
                keys[m++] = ((uint64_t)hub << sh_s) | (l << sh_l) | (uint64_t)t;
            }
        }
        for (int iter = 0; ; ++iter) {
            /* draw the missing E - m edges in N_CHUNKS independent streams */
            const int64_t need = E - m, base = m;
#pragma omp parallel for schedule(static)
            for (int c = 0; c < N_CHUNKS; ++c) {
                rng_t rc; rng_seed(&rc, p->seed, 100000 + (uint64_t)iter * N_CHUNKS + (uint64_t)c);
                const int64_t lo = need * c / N_CHUNKS, hi = need * (c + 1) / N_CHUNKS;
                for (int64_t i = lo; i < hi; ) {
                    int64_t s0 = alias_draw(&src_al, &rc), t0 = alias_draw(&dst_al, &rc);
                    if (s0 == t0) continue;
                    uint64_t l = rng_below(&rc, (uint64_t)p->n_labels);
                    keys[base + i] = ((uint64_t)s0 << sh_s) | (l << sh_l) | (uint64_t)t0;
                    ++i;
                }
            }
            m = E;
            if (radix_sort_u64(keys, m, 2 * nb + lb)) goto fail;
            m = unique_sorted_u64(keys, m);
            if (m == E || iter > 1000) break;
        }
        if (m != E) goto fail;
        alias_free(&src_al); alias_free(&dst_al);

        progress("directed edges", t_start);
        /* 4. node weights from directed in-degree */
        int64_t* indeg = (int64_t*)calloc((size_t)n, sizeof(int64_t));
        g->node_weight = (uint8_t*)malloc((size_t)n);
        if (!indeg || !g->node_weight) { free(indeg); goto fail; }
        const uint64_t nmask = ((uint64_t)1 << nb) - 1;
        for (int64_t i = 0; i < E; ++i) indeg[keys[i] & nmask]++;
        for (int64_t v = 0; v < n; ++v) {
            double q = floor(8.0 * log2(1.0 + (double)indeg[v]) + 0.5);
            g->node_weight[v] = (uint8_t)(q > 255.0 ? 255.0 : q);
        }
        free(indeg);

        /* 5. reverse edges, merge, CSR with rows sorted by (label, dst) */
        const uint64_t lmask = ((uint64_t)1 << lb) - 1;
        for (int64_t i = 0; i < E; ++i) {
            uint64_t k = keys[i];
            uint64_t s = k >> sh_s, l = (k >> sh_l) & lmask, t = k & nmask;
            keys[E + i] = (t << sh_s) | (l << sh_l) | s;
        }
        if (radix_sort_u64(keys, 2 * E, 2 * nb + lb)) goto fail;
        int64_t A = unique_sorted_u64(keys, 2 * E);
        g->n_arcs = A;
        g->row_ptr = (int64_t*)calloc((size_t)(n + 1), sizeof(int64_t));
        g->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(A > 0 ? A : 1));
        g->label = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)(A > 0 ? A : 1));
        if (!g->row_ptr || !g->col || !g->label) goto fail;
        for (int64_t i = 0; i < A; ++i) {
            uint64_t k = keys[i];
            g->row_ptr[(k >> sh_s) + 1]++;
            g->col[i] = (int32_t)(k & nmask);
            g->label[i] = (uint16_t)((k >> sh_l) & lmask);
        }
        for (int64_t v = 0; v < n; ++v) g->row_ptr[v + 1] += g->row_ptr[v];
    }
    free(keys); keys = NULL;
    progress("bi-directed CSR", t_start);

    /* 6. keywords per node, Zipf popularity */
    {
        double* zw = (double*)malloc(sizeof(double) * (size_t)p->vocab);
        if (!zw) goto fail;
        for (int32_t k = 0; k < p->vocab; ++k) zw[k] = pow((double)(k + 1), -p->zipf_s);
        alias_t za;
        int rc = alias_build(&za, zw, p->vocab);
        free(zw);
        if (rc) goto fail;
        rng_t r; rng_seed(&r, p->seed, 3);
        const int kmax = p->kw_max;
        int32_t* tags = (int32_t*)malloc(sizeof(int32_t) * (size_t)n * (size_t)(kmax > 0 ? kmax : 1));
        uint8_t* ntag = (uint8_t*)malloc((size_t)n);
        g->kw_ptr = (int64_t*)calloc((size_t)p->vocab + 1, sizeof(int64_t));
        if (!tags || !ntag || !g->kw_ptr) { free(tags); free(ntag); alias_free(&za); goto fail; }
        int64_t total = 0;
        for (int64_t v = 0; v < n; ++v) {
            int c = p->kw_min + (int)rng_below(&r, (uint64_t)(p->kw_max - p->kw_min + 1));
            ntag[v] = (uint8_t)c;
            for (int j = 0; j < c; ++j) {
                int32_t t;
                int dup;
                do {
                    t = (int32_t)alias_draw(&za, &r);
                    dup = 0;
                    for (int q = 0; q < j; ++q) if (tags[v * kmax + q] == t) dup = 1;
                } while (dup);
                tags[v * kmax + j] = t;
                g->kw_ptr[t + 1]++;
            }
            total += c;
        }
        alias_free(&za);
        for (int32_t k = 0; k < p->vocab; ++k) g->kw_ptr[k + 1] += g->kw_ptr[k];
        g->n_kw_entries = total;
        g->kw_nodes = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)p->vocab);
        if (!g->kw_nodes || !fill) { free(tags); free(ntag); free(fill); goto fail; }
        memcpy(fill, g->kw_ptr, sizeof(int64_t) * (size_t)p->vocab);
        for (int64_t v = 0; v < n; ++v)
            for (int j = 0; j < ntag[v]; ++j) g->kw_nodes[fill[tags[v * kmax + j]]++] = (int32_t)v;
        free(fill); free(tags); free(ntag);
    }

    progress("keywords", t_start);
    /* 7. A-bar from sampled pairs */
    g->abar_x100 = estimate_abar_x100(g, p);
    progress("average hop count", t_start);
    if (g->abar_x100 <= 0) goto fail;
    return g;

fail:
    free(w); free(perm);
    synth_free(g);
    return NULL;
}

void synth_sizes(const synth_graph* g, int64_t* out6) {
    out6[0] = g->n_nodes; out6[1] = g->n_arcs; out6[2] = g->n_kw_entries;
    out6[3] = g->vocab; out6[4] = g->abar_x100; out6[5] = g->n_edges;
}

void synth_copy(const synth_graph* g, int64_t* row_ptr, int32_t* col, uint16_t* label,
                uint8_t* node_weight, int64_t* kw_ptr, int32_t* kw_nodes, int64_t* hubs8) {
    memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * (size_t)(g->n_nodes + 1));
    memcpy(col, g->col, sizeof(int32_t) * (size_t)g->n_arcs);
    memcpy(label, g->label, sizeof(uint16_t) * (size_t)g->n_arcs);
    memcpy(node_weight, g->node_weight, (size_t)g->n_nodes);
    memcpy(kw_ptr, g->kw_ptr, sizeof(int64_t) * (size_t)(g->vocab + 1));
    memcpy(kw_nodes, g->kw_nodes, sizeof(int32_t) * (size_t)g->n_kw_entries);
    memcpy(hubs8, g->hubs, sizeof(int64_t) * 8);
}
