/*
 * CPU oracle for the U-HNSW query path -- TEST INFRASTRUCTURE ONLY (see
 * oracle.h). Compiled with -ffp-contract=off and without fast-math, so every
 * floating-point operation below happens exactly as written.
 *
 * Paper: Wang, Meng, Xu, "U-HNSW: An Efficient Graph-based Solution to ANNS
 * Under Universal L_p Metrics" (EDBT'27, arXiv 2605.02030).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ===================================================================== L_p
 * Sec. 1.1 / Sec. 2.1: a query is a tuple (q, p); distances are the L_p
 * (Minkowski) distance, d_p(x, q) = (sum_i |x_i - q_i|^p)^(1/p), for p in
 * [0.5, 2]. The paper never prints the formula; the Minkowski form is the one
 * its norm-equivalence argument (Sec. 3.1) refers to. Ranking uses the
 * un-rooted sum S_p, which is monotone in d_p. FP64 throughout.
 */
double orc_lp_sum(const float *x, const float *q, int d, double p) {
    double s = 0.0;
    for (int i = 0; i < d; i++) {
        double a = fabs((double)x[i] - (double)q[i]);
        s += pow(a, p);
    }
    return s;
}

double orc_lp_dist(const float *x, const float *q, int d, double p) { return pow(orc_lp_sum(x, q, d, p), 1.0 / p); }

/* ============================================================ brute force
 * Exact top-K under L_p (the set S* of the recall definition, Sec. 4.1.2),
 * ordered by (S_p, id): smaller id wins a tie.
 */
static int sid_less(double sa, int32_t ia, double sb, int32_t ib) { return sa < sb || (sa == sb && ia < ib); }

void orc_bruteforce(const float *base, int64_t n, int d, const float *qs, int64_t nq, const float *p, int K,
                    int32_t *ids, double *S, int nthreads) {
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t qi = 0; qi < nq; qi++) {
        int32_t *bi = ids + qi * K;
        double *bs = S + qi * K;
        int cnt = 0;
        const float *q = qs + qi * d;
        for (int64_t j = 0; j < n; j++) {
            double s = orc_lp_sum(base + j * d, q, d, (double)p[qi]);
            if (cnt == K && !sid_less(s, (int32_t)j, bs[K - 1], bi[K - 1])) continue;
            int pos = cnt < K ? cnt++ : K - 1;
            while (pos > 0 && sid_less(s, (int32_t)j, bs[pos - 1], bi[pos - 1])) {
                bs[pos] = bs[pos - 1];
                bi[pos] = bi[pos - 1];
                pos--;
            }
            bs[pos] = s;
            bi[pos] = (int32_t)j;
        }
        for (int r = cnt; r < K; r++) {
            bi[r] = -1;
            bs[r] = INFINITY;
        }
    }
}

/* ======================================================= storage formats
 * Precision form: the walk reads base vectors stored as bfloat16 or IEEE
 * binary16, each rounded to nearest-even from the FP32 value, and widened
 * exactly to FP32 before use.
 */
uint16_t orc_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if (isnan(f)) return (uint16_t)((u >> 16) | 0x0040);
    uint32_t hi = u >> 16, lo = u & 0xFFFFu;
    /* round the 16 dropped magnitude bits to nearest, ties to even */
    if (lo > 0x8000u || (lo == 0x8000u && (hi & 1u))) hi += 1;
    return (uint16_t)hi;
}

float orc_bf16_to_f32(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

uint16_t orc_to_f16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    if (isnan(f)) return sign | 0x7E00u;
    double a = fabs((double)f);
    if (isinf(f) || a >= 65520.0) return sign | 0x7C00u; /* 65520 ties to even -> 65536 -> inf */
    if (a == 0.0) return sign;
    int e;
    frexp(a, &e);
    int E = e - 1; /* a in [2^E, 2^(E+1)) */
    if (E < -14) E = -14;
    double quantum = ldexp(1.0, E - 10);
    double r = nearbyint(a / quantum) * quantum; /* round to nearest, ties to even */
    if (r == 0.0) return sign;
    frexp(r, &e);
    E = e - 1;
    if (E < -14) return sign | (uint16_t)(r / ldexp(1.0, -24)); /* subnormal */
    uint16_t ex = (uint16_t)(E + 15);
    uint16_t mant = (uint16_t)((r / ldexp(1.0, E) - 1.0) * 1024.0);
    return sign | (uint16_t)(ex << 10) | mant;
}

float orc_f16_to_f32(uint16_t h) {
    int ex = (h >> 10) & 0x1F, mant = h & 0x3FF;
    double s = (h & 0x8000u) ? -1.0 : 1.0, v;
    if (ex == 0)
        v = ldexp((double)mant, -24);
    else if (ex == 31)
        v = mant ? NAN : INFINITY;
    else
        v = ldexp(1.0 + mant / 1024.0, ex - 15);
    return (float)(s * v);
}

void orc_convert(const float *src, int64_t cnt, int storage, uint16_t *dst) {
    for (int64_t i = 0; i < cnt; i++) dst[i] = storage == ORC_BF16 ? orc_to_bf16(src[i]) : orc_to_f16(src[i]);
}

static float elem(const void *x, int storage, int64_t j) {
    if (storage == ORC_F32) return ((const float *)x)[j];
    uint16_t h = ((const uint16_t *)x)[j];
    return storage == ORC_BF16 ? orc_bf16_to_f32(h) : orc_f16_to_f32(h);
}

/* ====================================================== base distance
 * Base metrics of the candidate walk (Sec. 3.1: G1 under L1, G2 under L2;
 * Sec. 4.5's extended pair: G_0.5 under L0.5, G_1 under L1).
 * delta_1 = sum |x_j - q_j|, delta_2 = sum (x_j - q_j)^2 (squared L2, rank-
 * equivalent to L2), delta_0.5 = sum sqrt|x_j - q_j| (the L0.5 distance is
 * its square, so the two rank alike), and for a graph built for one p
 * (Sec. 4.3's per-p HNSW) delta_p = sum |x_j - q_j|^p (the L_p distance to
 * the power p; each term taken in FP64 and rounded once to FP32). Computed
 * in FP32 (the paper's kernels
 * are single precision, Sec. 2.1) in one fixed order, so that any
 * implementation that follows the same order gets the same bits:
 *   element j belongs to lane (j / v) mod g; each lane sums its elements in
 *   ascending j from +0 (L2 with a fused multiply-add; L0.5 adds the
 *   correctly rounded FP32 square root); lanes then combine pairwise, lane
 *   l < o taking s_l + s_{l+o}, for o = g/2, g/4, ..., 1.
 */
float orc_base_dist(const void *x, int storage, const float *q, int d, int metric, double mp, int g, int v) {
    float s[64];
    for (int l = 0; l < g; l++) s[l] = 0.0f;
    for (int j = 0; j < d; j++) {
        int lane = (j / v) % g;
        float diff = elem(x, storage, j) - q[j];
        if (metric == ORC_L1)
            s[lane] = s[lane] + fabsf(diff);
        else if (metric == ORC_L05)
            s[lane] = s[lane] + sqrtf(fabsf(diff));
        else if (metric == ORC_LP) /* |diff|^p in FP64, rounded once to FP32 */
            s[lane] = s[lane] + (float)pow((double)fabsf(diff), mp);
        else
            s[lane] = fmaf(diff, diff, s[lane]);
    }
    for (int o = g / 2; o >= 1; o /= 2)
        for (int l = 0; l < o; l++) s[l] = s[l] + s[l + o];
    return s[0];
}

static float base_key(const orc_data *D, int32_t id, const float *q, int metric, double mp, int g, int v) {
    size_t es = D->walk_storage == ORC_F32 ? 4 : 2;
    const char *row = (const char *)D->walk_base + (size_t)id * (size_t)D->d * es;
    return orc_base_dist(row, D->walk_storage, q, D->d, metric, mp, g, v);
}

/* ====================================================== KnnSearch
 * Candidate generation (Sec. 3.1) runs the standard HNSW KnnSearch on the
 * chosen graph; HNSW's search (Sec. 2.2) starts at a fixed entry point,
 * follows edges, and admits an unvisited node into the candidate list when
 * it beats the farthest member, the list being bounded by efSearch. The
 * reading taken here:
 *   - every comparison uses the key (delta, id), smaller id first;
 *   - descent: on layers L_max..1, move to the neighbour with the smallest
 *     key while that beats the current node (no visited set);
 *   - layer 0, batch-synchronous: W = sorted list of (key, id, expanded).
 *     Repeat: P = first w unexpanded entries of W (stop if none); mark them
 *     expanded; U = neighbours of P not yet visited (a set); mark U visited;
 *     W = the ef smallest keys of W u U (new entries unexpanded).
 *   - C = the first t entries of the final W.
 * With cache_slots > 0 the visited set is replaced by a lossy direct-mapped
 * cache (a forgotten id is seen again) and U is de-duplicated against itself
 * and against W; the result C is the same (a forgotten id is either in W or
 * worse than the worst of a full W), only n_b grows.
 */
typedef struct {
    float key;
    int32_t id;
    int expanded;
} went;

static int went_cmp(const void *a, const void *b) {
    const went *x = (const went *)a, *y = (const went *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int64_t layer_row(const orc_graph *G, int l, int32_t v) {
    if (l == 0) return v;
    int64_t lo = 0, hi = G->nnodes[l] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (G->nodes[l][mid] == v) return mid;
        if (G->nodes[l][mid] < v)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

static uint32_t cache_slot(int32_t id, int slots) {
    uint64_t h = (uint64_t)(uint32_t)id * 0x9E3779B97F4A7C15ULL;
    return (uint32_t)(h >> 40) & (uint32_t)(slots - 1);
}

int orc_knn_search(const orc_graph *G, const orc_data *D, const float *q, int metric, double mp, int ef, int t, int w,
                   int g, int v, int cache_slots, int32_t *c_ids, float *c_keys, orc_stats *st) {
    int n_b = 0, n_exp = 0;
    /* descent over the upper layers */
    int32_t cur = G->entry;
    float kcur = base_key(D, cur, q, metric, mp, g, v);
    n_b++;
    for (int l = G->max_level; l >= 1; l--) {
        for (;;) {
            int64_t r = layer_row(G, l, cur);
            int32_t best = -1;
            float kbest = 0.0f;
            for (int64_t e = G->row_ptr[l][r]; e < G->row_ptr[l][r + 1]; e++) {
                int32_t u = G->col[l][e];
                float ku = base_key(D, u, q, metric, mp, g, v);
                n_b++;
                if (best < 0 || ku < kbest || (ku == kbest && u < best)) {
                    best = u;
                    kbest = ku;
                }
            }
            if (best >= 0 && (kbest < kcur || (kbest == kcur && best < cur))) {
                cur = best;
                kcur = kbest;
            } else {
                break;
            }
        }
    }
    /* layer 0 */
    int32_t W0 = cur;
    int maxdeg = G->max_deg0;
    went *W = (went *)malloc(sizeof(went) * (size_t)(ef + w * maxdeg + 1));
    int32_t *U = (int32_t *)malloc(sizeof(int32_t) * (size_t)(w * maxdeg + 1));
    unsigned char *vis = NULL;
    int32_t *cache = NULL;
    if (cache_slots > 0) {
        cache = (int32_t *)malloc(sizeof(int32_t) * (size_t)cache_slots);
        for (int i = 0; i < cache_slots; i++) cache[i] = -1;
        cache[cache_slot(cur, cache_slots)] = cur;
    } else {
        vis = (unsigned char *)calloc((size_t)G->n, 1);
        vis[cur] = 1;
    }
    int nW = 1;
    W[0].key = kcur;
    W[0].id = cur;
    W[0].expanded = 0;
    for (;;) {
        int32_t P[64];
        int np = 0;
        for (int i = 0; i < nW && np < w; i++) {
            if (!W[i].expanded) {
                W[i].expanded = 1;
                P[np++] = W[i].id;
            }
        }
        if (np == 0) break;
        n_exp += np;
        int nU = 0;
        for (int a = 0; a < np; a++) {
            for (int64_t e = G->row_ptr[0][P[a]]; e < G->row_ptr[0][P[a] + 1]; e++) {
                int32_t u = G->col[0][e];
                if (cache) {
                    uint32_t s = cache_slot(u, cache_slots);
                    if (cache[s] == u) continue;
                    cache[s] = u;
                } else {
                    if (vis[u]) continue;
                    vis[u] = 1;
                }
                U[nU++] = u;
            }
        }
        if (cache) { /* de-duplicate U against itself and against W */
            int keep = 0;
            for (int i = 0; i < nU; i++) {
                int dup = 0;
                for (int j = 0; j < keep && !dup; j++) dup = U[j] == U[i];
                for (int j = 0; j < nW && !dup; j++) dup = W[j].id == U[i];
                if (!dup) U[keep++] = U[i];
            }
            nU = keep;
        }
        for (int i = 0; i < nU; i++) {
            W[nW].key = base_key(D, U[i], q, metric, mp, g, v);
            W[nW].id = U[i];
            W[nW].expanded = 0;
            nW++;
        }
        n_b += nU;
        qsort(W, (size_t)nW, sizeof(went), went_cmp);
        if (nW > ef) nW = ef;
    }
    int nc = nW < t ? nW : t;
    for (int i = 0; i < nc; i++) {
        c_ids[i] = W[i].id;
        c_keys[i] = W[i].key;
    }
    free(W);
    free(U);
    free(vis);
    free(cache);
    if (st) {
        st->n_b = n_b;
        st->n_exp = n_exp;
        st->nc = nc;
        st->entry0 = W0;
    }
    return nc;
}

/* ====================================================== verification
 * Candidate verification (Sec. 3.1 and Algorithm 1): R = first K points of
 * C; then for each next batch R' of kappa points of C (the last batch may be
 * short), R_new = the K points of R u R' with the smallest L_p distance; stop
 * and return R_new once |R_new n R| / K >= tau, else R = R_new. When C runs
 * out, the last R_new is returned. The ratio test is taken as the integer
 * test |R_new n R| >= m with m = ceil(tau*K) (see orc_m_of).
 * Keys are (S_p, id) in FP64. With early_abort a candidate's partial sum is
 * compared with the K-th S_p of R at the batch start; once strictly greater
 * the candidate cannot enter R_new and its sum is not finished (the sum of
 * non-negative terms only grows, so the result is unchanged).
 */
int orc_m_of(double tau, int K) { return (int)ceil(tau * (double)K - 1e-9); }

typedef struct {
    double s;
    int32_t id;
    int from_new;
} rent;

static int rent_cmp(const void *a, const void *b) {
    const rent *x = (const rent *)a, *y = (const rent *)b;
    if (x->s < y->s) return -1;
    if (x->s > y->s) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static double lp_sum_abort(const float *x, const float *q, int d, double p, double thr, int *aborted) {
    double s = 0.0;
    *aborted = 0;
    for (int i = 0; i < d; i++) {
        double a = fabs((double)x[i] - (double)q[i]);
        s += pow(a, p);
        if (s > thr) {
            *aborted = 1;
            return s;
        }
    }
    return s;
}

int orc_verify(const orc_data *D, const float *q, float p, int K, const int32_t *C, int nC, int kappa, int m,
               int early_abort, int32_t *ids, double *S, double *dist, orc_stats *st) {
    int d = D->d;
    double pp = (double)p;
    rent *R = (rent *)malloc(sizeof(rent) * (size_t)(K + kappa));
    int nR = nC < K ? nC : K;
    for (int i = 0; i < nR; i++) {
        R[i].s = orc_lp_sum(D->base + (int64_t)C[i] * d, q, d, pp);
        R[i].id = C[i];
        R[i].from_new = 0;
    }
    qsort(R, (size_t)nR, sizeof(rent), rent_cmp);
    int pos = nR, batches = 0;
    while (pos < nC) {
        int nb = nC - pos < kappa ? nC - pos : kappa;
        double thr = R[nR - 1].s; /* K-th S_p of R at the batch start (R is full here) */
        int nn = nR;
        for (int i = 0; i < nb; i++) {
            int32_t c = C[pos + i];
            const float *x = D->base + (int64_t)c * d;
            int ab = 0;
            double s = early_abort ? lp_sum_abort(x, q, d, pp, thr, &ab) : orc_lp_sum(x, q, d, pp);
            if (ab) continue;
            R[nn].s = s;
            R[nn].id = c;
            R[nn].from_new = 1;
            nn++;
        }
        pos += nb;
        batches++;
        for (int i = 0; i < nR; i++) R[i].from_new = 0;
        qsort(R, (size_t)nn, sizeof(rent), rent_cmp);
        int inter = 0; /* |R_new n R|: members of the first K that came from R */
        for (int i = 0; i < nR; i++) inter += !R[i].from_new;
        if (inter >= m) break;
    }
    for (int i = 0; i < nR; i++) {
        ids[i] = R[i].id;
        S[i] = R[i].s;
        dist[i] = pow(R[i].s, 1.0 / pp);
    }
    free(R);
    if (st) {
        st->n_p = pos;
        st->batches = batches;
        st->nres = nR;
        st->m = m;
    }
    return nR;
}

/* ====================================================== one query
 * Algorithm 1 end to end: graph choice (Sec. 3.1: G1 when p <= 1.4, else
 * G2; the compare is taken in FP32), candidate generation with t candidates,
 * verification. Defaults: t = min(ef, 6K) (the paper pairs t = 300 with
 * K = 50), kappa = max(K, 2) (kappa = K by default and kappa > 1),
 * tau = 0.92. The extended variant (Sec. 4.5) runs the same steps with
 * G_0.5 in G1's place and G_1 in G2's, and a cutoff of 0.6 (the caller's
 * prm->cutoff). The per-p variant runs them on a graph built for one p
 * (Sec. 4.3's HNSW baseline): its walk ranks by that p's sum, so for a
 * query of the same p the verification only confirms C's first K.
 */
int orc_query(const orc_graph *g1, const orc_graph *g2, const orc_data *D, const float *q, float p, int K, int ef,
              const orc_params *prm, int32_t *ids, double *S, double *dist, int32_t *c_ids, float *c_keys,
              orc_stats *st) {
    orc_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    int use_g1 = p <= prm->cutoff;
    st->graph = use_g1 ? 1 : 2;
    int tp = prm->t_param > 0 ? prm->t_param : 6 * K;
    int t = ef < tp ? ef : tp;
    if (t < K) t = K < ef ? K : ef;
    int kappa = prm->kappa > 0 ? prm->kappa : (K > 2 ? K : 2);
    int m = orc_m_of(prm->tau, K);
    int32_t *ci = c_ids ? c_ids : (int32_t *)malloc(sizeof(int32_t) * (size_t)t);
    float *ck = c_keys ? c_keys : (float *)malloc(sizeof(float) * (size_t)t);
    int metric = prm->variant == ORC_VARIANT_EXT      ? (use_g1 ? ORC_L05 : ORC_L1)
                 : prm->variant == ORC_VARIANT_PGRAPH ? (use_g1 ? ORC_LP : ORC_L2)
                                                      : (use_g1 ? ORC_L1 : ORC_L2);
    int nc = orc_knn_search(use_g1 ? g1 : g2, D, q, metric, prm->walk_p, ef, t, prm->w, prm->g, prm->v,
                            prm->cache_slots, ci, ck, st);
    int nr = orc_verify(D, q, p, K, ci, nc, kappa, m, prm->early_abort, ids, S, dist, st);
    if (!c_ids) free(ci);
    if (!c_keys) free(ck);
    return nr;
}

void orc_query_batch(const orc_graph *g1, const orc_graph *g2, const orc_data *D, const float *qs, int64_t nq,
                     const float *p, const int32_t *k, const int32_t *ef, const orc_params *prm, int k_stride,
                     int64_t *ids, double *dist, double *S, int c_stride, int32_t *c_ids, float *c_keys,
                     orc_stats *stats, int nthreads) {
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < nq; i++) {
        int K = k[i];
        int32_t *ri = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
        double *rs = (double *)malloc(sizeof(double) * (size_t)K);
        double *rd = (double *)malloc(sizeof(double) * (size_t)K);
        int nr = orc_query(g1, g2, D, qs + i * D->d, p[i], K, ef[i], prm, ri, rs, rd,
                           c_ids ? c_ids + i * c_stride : NULL, c_keys ? c_keys + i * c_stride : NULL,
                           stats ? stats + i : NULL);
        for (int r = 0; r < k_stride; r++) {
            ids[i * k_stride + r] = r < nr ? ri[r] : -1;
            if (dist) dist[i * k_stride + r] = r < nr ? rd[r] : INFINITY;
            if (S) S[i * k_stride + r] = r < nr ? rs[r] : INFINITY;
        }
        free(ri);
        free(rs);
        free(rd);
    }
}
