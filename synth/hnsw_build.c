/*
 * Deterministic HNSW construction for the two U-HNSW base graphs
 * (G1 under L1, G2 under L2; U-HNSW paper, Sec. 3.1), and for the extended
 * variant's G_0.5 under L0.5 (Sec. 4.5), and a graph for one fixed p (the
 * per-p HNSW baseline of Sec. 4.3). metric: 1 = L1, 2 = squared L2,
 * 3 = sum sqrt|a - b| (ranks like L0.5), 4 = sum |a - b|^mp for a given mp
 * (each term taken in double and rounded to float).
 *
 * The construction itself is the HNSW algorithm the paper builds on
 * (Sec. 2.2: incremental insertion, M neighbours per node, a dynamic
 * candidate list of size efConstruction, a layered graph). The paper does
 * not spell out its internals; this file uses the usual reading:
 *   - level of node v: floor(-ln(U_v) * mL), mL = 1/ln(M), with U_v in (0,1]
 *     drawn from splitmix64(seed ^ (v * golden)) -- a counter-based draw;
 *   - greedy descent above the node's level, efConstruction beam below;
 *   - neighbour choice by the diversity heuristic (keep candidate e unless a
 *     kept r has dist(e, r) < dist(q, e)), M per layer;
 *   - reverse links, and an over-full list (> M on upper layers, > 2M on
 *     layer 0) re-selected with the same heuristic.
 *
 * Determinism: nodes are inserted in id order, in batches. A batch first
 * searches the graph frozen at the batch start (parallel over members), then
 * applies links: each new node's own lists, then the reverse links grouped
 * by target node (parallel over targets, each target's requests in
 * ascending source id). The graph is therefore identical for any thread
 * count. Batch size grows with the graph (the number of nodes already in
 * it over 64, at least 1, at most batch_max; 1024 by default).
 *
 * Distances are FP32 in one fixed order (see dist_metric), independent of
 * the compiler. This file is an input generator: it shares no code with the
 * oracle or with the GPU library.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float d;
    int32_t id;
} pr_t;

static inline int pr_lt(pr_t a, pr_t b) { return a.d < b.d || (a.d == b.d && a.id < b.id); }

typedef struct {
    int64_t n;
    int d, metric, M, M0, efc;
    double mp; /* metric 4: the power */
    const float *base;
    int8_t *level;
    int max_level;
    int32_t entry;
    int32_t *adj0; /* n * M0 */
    uint8_t *cnt0; /* n */
    int64_t *upo;  /* n: row of layer 1 in uadj, -1 if level 0 */
    int32_t *uadj; /* nurows * M */
    uint8_t *ucnt; /* nurows */
    int64_t nurows;
} hb_t;

/* ---------------------------------------------------------------- distance */
/* One fixed FP32 order, so that any implementation following it gets the
 * same bits (a GPU construction of these graphs is compared edge for edge
 * with this builder): element j is accumulated by lane (j / 4) mod 16 of 16
 * lanes, each lane in ascending j from +0 (L2 by fused multiply-add), then
 * the lanes combine pairwise: for o = 8, 4, 2, 1, lane l < o takes
 * s_l + s_{l+o}. Compiled with -ffp-contract=off. */
#define HB_LANES 16
#define HB_V 4

static inline float term(int metric, double mp, float a, float b) {
    const float t = a - b;
    if (metric == 4) return (float)pow((double)fabsf(t), mp);
    return metric == 1 ? fabsf(t) : sqrtf(fabsf(t));
}

static float dist_metric(const float *a, const float *b, int d, int metric, double mp) {
    float s[HB_LANES];
    for (int l = 0; l < HB_LANES; l++) s[l] = 0.0f;
    for (int c = 0; c < d; c += HB_LANES * HB_V)
        for (int l = 0; l < HB_LANES; l++)
            for (int e = 0; e < HB_V; e++) {
                const int j = c + l * HB_V + e;
                if (j >= d) break;
                if (metric == 2) {
                    const float t = a[j] - b[j];
                    s[l] = fmaf(t, t, s[l]);
                } else {
                    s[l] = s[l] + term(metric, mp, a[j], b[j]);
                }
            }
    for (int o = HB_LANES / 2; o >= 1; o >>= 1)
        for (int l = 0; l < o; l++) s[l] = s[l] + s[l + o];
    return s[0];
}

static inline const float *vec(const hb_t *g, int32_t v) { return g->base + (int64_t)v * g->d; }

static inline float dist(const hb_t *g, const float *a, const float *b) {
    return dist_metric(a, b, g->d, g->metric, g->mp);
}

static inline int32_t *nbrs(const hb_t *g, int32_t v, int l, int *cnt) {
    if (l == 0) {
        *cnt = g->cnt0[v];
        return g->adj0 + (int64_t)v * g->M0;
    }
    int64_t r = g->upo[v] + (l - 1);
    *cnt = g->ucnt[r];
    return g->uadj + r * g->M;
}

static inline void set_cnt(hb_t *g, int32_t v, int l, int c) {
    if (l == 0)
        g->cnt0[v] = (uint8_t)c;
    else
        g->ucnt[g->upo[v] + (l - 1)] = (uint8_t)c;
}

/* ------------------------------------------------------------------- heaps */
typedef struct {
    pr_t *a;
    int n, cap;
} heap_t;

static void heap_reserve(heap_t *h, int cap) {
    if (cap > h->cap) {
        h->cap = cap * 2;
        h->a = (pr_t *)realloc(h->a, sizeof(pr_t) * (size_t)h->cap);
    }
}

/* min-heap when maxh == 0, max-heap when maxh == 1 */
static void heap_push(heap_t *h, pr_t x, int maxh) {
    heap_reserve(h, h->n + 1);
    int i = h->n++;
    while (i > 0) {
        int p = (i - 1) / 2;
        int up = maxh ? pr_lt(h->a[p], x) : pr_lt(x, h->a[p]);
        if (!up) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = x;
}

static pr_t heap_pop(heap_t *h, int maxh) {
    pr_t top = h->a[0];
    pr_t x = h->a[--h->n];
    int i = 0;
    for (;;) {
        int c = 2 * i + 1;
        if (c >= h->n) break;
        if (c + 1 < h->n) {
            int pick = maxh ? pr_lt(h->a[c], h->a[c + 1]) : pr_lt(h->a[c + 1], h->a[c]);
            if (pick) c++;
        }
        int down = maxh ? pr_lt(x, h->a[c]) : pr_lt(h->a[c], x);
        if (!down) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = x;
    return top;
}

static int pr_cmp(const void *x, const void *y) {
    pr_t a = *(const pr_t *)x, b = *(const pr_t *)y;
    return pr_lt(a, b) ? -1 : (pr_lt(b, a) ? 1 : 0);
}

/* ----------------------------------------------------------- workspace */
typedef struct {
    uint32_t *stamp;
    uint32_t cur;
    heap_t cand, res;
    pr_t *sorted;
    int sorted_cap;
    pr_t *tmp;
    int tmp_cap;
} ws_t;

static void ws_init(ws_t *w, int64_t n) {
    memset(w, 0, sizeof(*w));
    w->stamp = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
}

static void ws_free(ws_t *w) {
    free(w->stamp);
    free(w->cand.a);
    free(w->res.a);
    free(w->sorted);
    free(w->tmp);
}

static void ws_next(ws_t *w, int64_t n) {
    if (++w->cur == 0) {
        memset(w->stamp, 0, sizeof(uint32_t) * (size_t)n);
        w->cur = 1;
    }
}

/* Standard HNSW layer search from one entry point; returns count, results
 * ascending by (dist, id) in w->sorted. */
static int search_layer(const hb_t *g, ws_t *w, const float *q, int32_t ep, float dep, int ef, int l) {
    ws_next(w, g->n);
    w->cand.n = 0;
    w->res.n = 0;
    pr_t e0 = {dep, ep};
    w->stamp[ep] = w->cur;
    heap_push(&w->cand, e0, 0);
    heap_push(&w->res, e0, 1);
    while (w->cand.n > 0) {
        pr_t c = heap_pop(&w->cand, 0);
        if (w->res.n >= ef && pr_lt(w->res.a[0], c)) break;
        int cnt;
        const int32_t *nb = nbrs(g, c.id, l, &cnt);
        for (int i = 0; i < cnt; i++) {
            int32_t e = nb[i];
            if (w->stamp[e] == w->cur) continue;
            w->stamp[e] = w->cur;
            pr_t pe = {dist(g, q, vec(g, e)), e};
            if (w->res.n < ef || pr_lt(pe, w->res.a[0])) {
                heap_push(&w->cand, pe, 0);
                heap_push(&w->res, pe, 1);
                if (w->res.n > ef) heap_pop(&w->res, 1);
            }
        }
    }
    int nr = w->res.n;
    if (nr > w->sorted_cap) {
        w->sorted_cap = nr * 2;
        w->sorted = (pr_t *)realloc(w->sorted, sizeof(pr_t) * (size_t)w->sorted_cap);
    }
    memcpy(w->sorted, w->res.a, sizeof(pr_t) * (size_t)nr);
    qsort(w->sorted, (size_t)nr, sizeof(pr_t), pr_cmp);
    return nr;
}

/* Diversity heuristic over candidates sorted ascending by distance to the
 * base point: keep e unless some kept r has dist(e, r) < dist(base, e). */
static int heuristic(const hb_t *g, const pr_t *cand, int nc, int msel, int32_t *out) {
    int nout = 0;
    for (int i = 0; i < nc && nout < msel; i++) {
        const float *xe = vec(g, cand[i].id);
        int good = 1;
        for (int j = 0; j < nout; j++) {
            if (dist(g, xe, vec(g, out[j])) < cand[i].d) {
                good = 0;
                break;
            }
        }
        if (good) out[nout++] = cand[i].id;
    }
    return nout;
}

/* ----------------------------------------------------------- insertion */
typedef struct {
    int nl;        /* layers planned: 0..nl-1 */
    int32_t *ids;  /* nl * M */
    uint8_t *cnt;  /* nl */
} plan_t;

static void plan_node(const hb_t *g, ws_t *w, int32_t v, int lmax, int32_t ep, plan_t *pl) {
    const float *q = vec(g, v);
    int lv = g->level[v];
    int32_t cur = ep;
    float dcur = dist(g, q, vec(g, ep));
    for (int l = lmax; l > lv; l--) {
        int changed = 1;
        while (changed) {
            changed = 0;
            int cnt;
            const int32_t *nb = nbrs(g, cur, l, &cnt);
            for (int i = 0; i < cnt; i++) {
                float de = dist(g, q, vec(g, nb[i]));
                pr_t a = {de, nb[i]}, b = {dcur, cur};
                if (pr_lt(a, b)) {
                    cur = nb[i];
                    dcur = de;
                    changed = 1;
                }
            }
        }
    }
    int top = lv < lmax ? lv : lmax;
    pl->nl = top + 1;
    for (int l = top; l >= 0; l--) {
        int nr = search_layer(g, w, q, cur, dcur, g->efc, l);
        pl->cnt[l] = (uint8_t)heuristic(g, w->sorted, nr, g->M, pl->ids + (int64_t)l * g->M);
        cur = w->sorted[0].id;
        dcur = w->sorted[0].d;
    }
}

typedef struct {
    int32_t l, u, v;
} req_t;

static int req_cmp(const void *x, const void *y) {
    const req_t *a = (const req_t *)x, *b = (const req_t *)y;
    if (a->l != b->l) return a->l < b->l ? -1 : 1;
    if (a->u != b->u) return a->u < b->u ? -1 : 1;
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return 0;
}

static void add_link(hb_t *g, ws_t *w, int32_t u, int32_t v, int l) {
    int mmax = l ? g->M : g->M0;
    int cnt;
    int32_t *nb = nbrs(g, u, l, &cnt);
    if (cnt < mmax) {
        nb[cnt] = v;
        set_cnt(g, u, l, cnt + 1);
        return;
    }
    if (w->tmp_cap < cnt + 1) {
        w->tmp_cap = 2 * (cnt + 1);
        w->tmp = (pr_t *)realloc(w->tmp, sizeof(pr_t) * (size_t)w->tmp_cap);
    }
    const float *xu = vec(g, u);
    for (int i = 0; i < cnt; i++) {
        w->tmp[i].id = nb[i];
        w->tmp[i].d = dist(g, xu, vec(g, nb[i]));
    }
    w->tmp[cnt].id = v;
    w->tmp[cnt].d = dist(g, xu, vec(g, v));
    qsort(w->tmp, (size_t)cnt + 1, sizeof(pr_t), pr_cmp);
    int32_t keep[256];
    int nk = heuristic(g, w->tmp, cnt + 1, mmax, keep);
    memcpy(nb, keep, sizeof(int32_t) * (size_t)nk);
    set_cnt(g, u, l, nk);
}

static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

/* ----------------------------------------------------------- public API */
void *hb_build(const float *base, int64_t n, int d, int metric, double mp, int M, int efc, uint64_t seed,
               int nthreads, int verbose, int batch_max) {
    if (n < 1 || d < 1 || metric < 1 || metric > 4 || M < 2 || M > 127 || efc < 1 || batch_max < 1) return NULL;
    if (metric == 4 && !(mp > 0.0 && mp <= 2.0)) return NULL;
    hb_t *g = (hb_t *)calloc(1, sizeof(hb_t));
    g->n = n;
    g->d = d;
    g->metric = metric;
    g->mp = mp;
    g->M = M;
    g->M0 = 2 * M;
    g->efc = efc;
    g->base = base;
    g->level = (int8_t *)malloc((size_t)n);
    g->upo = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double ml = 1.0 / log((double)M);
    int64_t rows = 0;
    for (int64_t v = 0; v < n; v++) {
        uint64_t z = splitmix64(seed ^ ((uint64_t)v * 0x9E3779B97F4A7C15ULL));
        double u = ((double)(z >> 11) + 1.0) * (1.0 / 9007199254740992.0); /* (0, 1] */
        int lv = (int)floor(-log(u) * ml);
        if (lv > 30) lv = 30;
        g->level[v] = (int8_t)lv;
        g->upo[v] = lv ? rows : -1;
        rows += lv;
    }
    g->nurows = rows;
    g->adj0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)g->M0);
    g->cnt0 = (uint8_t *)calloc((size_t)n, 1);
    g->uadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rows ? rows : 1) * (size_t)M);
    g->ucnt = (uint8_t *)calloc((size_t)(rows ? rows : 1), 1);

    if (nthreads < 1) nthreads = omp_get_max_threads();
    ws_t *ws = (ws_t *)malloc(sizeof(ws_t) * (size_t)nthreads);
    for (int i = 0; i < nthreads; i++) ws_init(&ws[i], n);

    const int BMAX = batch_max;
    plan_t *plans = (plan_t *)calloc(BMAX, sizeof(plan_t));
    for (int i = 0; i < BMAX; i++) {
        plans[i].ids = (int32_t *)malloc(sizeof(int32_t) * 32 * (size_t)M);
        plans[i].cnt = (uint8_t *)malloc(32);
    }
    req_t *reqs = (req_t *)malloc(sizeof(req_t) * (size_t)BMAX * 32 * (size_t)M);

    g->entry = 0;
    g->max_level = g->level[0];
    int64_t done = 1;
    while (done < n) {
        int64_t b = done / 64;
        if (b < 1) b = 1;
        if (b > BMAX) b = BMAX;
        if (done + b > n) b = n - done;
        int lmax = g->max_level;
        int32_t ep = g->entry;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int64_t i = 0; i < b; i++) {
            plan_node(g, &ws[omp_get_thread_num()], (int32_t)(done + i), lmax, ep, &plans[i]);
        }
        /* new nodes' own lists */
        int64_t nreq = 0;
        for (int64_t i = 0; i < b; i++) {
            int32_t v = (int32_t)(done + i);
            for (int l = 0; l < plans[i].nl; l++) {
                int cnt;
                int32_t *nb = nbrs(g, v, l, &cnt);
                int c = plans[i].cnt[l];
                memcpy(nb, plans[i].ids + (int64_t)l * M, sizeof(int32_t) * (size_t)c);
                set_cnt(g, v, l, c);
                for (int j = 0; j < c; j++) {
                    reqs[nreq].l = l;
                    reqs[nreq].u = nb[j];
                    reqs[nreq].v = v;
                    nreq++;
                }
            }
        }
        qsort(reqs, (size_t)nreq, sizeof(req_t), req_cmp);
        /* group starts */
        int64_t *gs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nreq + 1));
        int64_t ng = 0;
        for (int64_t r = 0; r < nreq; r++)
            if (r == 0 || reqs[r].l != reqs[r - 1].l || reqs[r].u != reqs[r - 1].u) gs[ng++] = r;
        gs[ng] = nreq;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
        for (int64_t gi = 0; gi < ng; gi++) {
            ws_t *w = &ws[omp_get_thread_num()];
            for (int64_t r = gs[gi]; r < gs[gi + 1]; r++) add_link(g, w, reqs[r].u, reqs[r].v, reqs[r].l);
        }
        free(gs);
        for (int64_t i = 0; i < b; i++) {
            int32_t v = (int32_t)(done + i);
            if (g->level[v] > g->max_level) {
                g->max_level = g->level[v];
                g->entry = v;
            }
        }
        int64_t step = n / 10 > 0 ? n / 10 : 1;
        if (verbose && (done / step) != ((done + b) / step)) {
            fprintf(stderr, "[hnsw-build] L%d: %lld / %lld nodes\n", metric, (long long)(done + b), (long long)n);
            fflush(stderr);
        }
        done += b;
    }
    for (int i = 0; i < BMAX; i++) {
        free(plans[i].ids);
        free(plans[i].cnt);
    }
    free(plans);
    free(reqs);
    for (int i = 0; i < nthreads; i++) ws_free(&ws[i]);
    free(ws);
    return g;
}

int hb_max_level(void *h) { return ((hb_t *)h)->max_level; }
int32_t hb_entry(void *h) { return ((hb_t *)h)->entry; }

void hb_levels(void *h, int8_t *out) {
    hb_t *g = (hb_t *)h;
    memcpy(out, g->level, (size_t)g->n);
}

/* number of nodes present on layer l (level >= l) */
int64_t hb_layer_nodes(void *h, int l) {
    hb_t *g = (hb_t *)h;
    int64_t c = 0;
    for (int64_t v = 0; v < g->n; v++) c += g->level[v] >= l;
    return c;
}

int64_t hb_layer_edges(void *h, int l) {
    hb_t *g = (hb_t *)h;
    int64_t e = 0;
    for (int64_t v = 0; v < g->n; v++)
        if (g->level[v] >= l) {
            int cnt;
            nbrs(g, (int32_t)v, l, &cnt);
            e += cnt;
        }
    return e;
}

/* CSR of layer l: nodes (ascending ids; skipped when NULL), row_ptr, col. */
void hb_layer_csr(void *h, int l, int32_t *nodes, int64_t *row_ptr, int32_t *col) {
    hb_t *g = (hb_t *)h;
    int64_t r = 0, e = 0;
    row_ptr[0] = 0;
    for (int64_t v = 0; v < g->n; v++) {
        if (g->level[v] < l) continue;
        int cnt;
        const int32_t *nb = nbrs(g, (int32_t)v, l, &cnt);
        if (nodes) nodes[r] = (int32_t)v;
        memcpy(col + e, nb, sizeof(int32_t) * (size_t)cnt);
        e += cnt;
        row_ptr[++r] = e;
    }
}

void hb_free(void *h) {
    hb_t *g = (hb_t *)h;
    if (!g) return;
    free(g->level);
    free(g->upo);
    free(g->adj0);
    free(g->cnt0);
    free(g->uadj);
    free(g->ucnt);
    free(g);
}
