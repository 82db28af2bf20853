/*
 * CPU oracle for the U-HNSW query path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C that states what the query path computes
 * (Wang, Meng, Xu, "U-HNSW: An Efficient Graph-based Solution to ANNS Under
 * Universal L_p Metrics", EDBT'27). Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code with the GPU
 * library (no common headers, helpers or tables) and includes nothing from
 * it.
 *
 * Parity status per function (what pins it is listed in the test suite):
 *   orc_lp_sum / orc_lp_dist ........ pinned (closed forms p=1,2,0.5,1.5;
 *                                      norm inequalities; library cdist)
 *   orc_bruteforce .................. pinned (library cdist top-K)
 *   orc_base_dist ................... pinned (exact on integer data, and for
 *                                      L0.5 on perfect-square differences;
 *                                      FP64 error bound; lane-order cases;
 *                                      L_p: p = 1 is L1 bit for bit, p = 0.5
 *                                      on perfect squares is L0.5, any p on
 *                                      differences in {0, 1} counts them)
 *   orc_to_bf16 / orc_to_f16 ........ pinned (numpy float16, torch bfloat16)
 *   orc_knn_search .................. pinned (ef = n on a connected graph is
 *                                      the exact base-metric top-t; lossy
 *                                      visited cache gives the same C)
 *   orc_verify ...................... pinned (tau > 1 with t = n equals brute
 *                                      force; prefix invariant; p = 1, 2 stop
 *                                      after one batch; abort on/off equal)
 *   HNSW graph quality .............. parity unpinned (no reference build)
 */
#ifndef UHNSW_ORACLE_H
#define UHNSW_ORACLE_H
#include <stdint.h>

#define ORC_MAX_LAYERS 32
#define ORC_F32 0
#define ORC_BF16 1
#define ORC_F16 2

/* base metrics of the walk: L1, squared L2, L0.5 as sum sqrt|x - q|, and
 * L_p for a fixed p (the metric parameter mp) as sum |x - q|^p, the walk of
 * an HNSW graph built for that p (the per-p HNSW of Sec. 4.3) */
#define ORC_L1 1
#define ORC_L2 2
#define ORC_L05 3
#define ORC_LP 4

/* index variants: the paper's default pair (G1 under L1, G2 under L2) and
 * the extended pair of Sec. 4.5 (G_0.5 under L0.5, G_1 under L1) */
#define ORC_VARIANT_STD 0
#define ORC_VARIANT_EXT 1
/* a graph built for one p (walk_p): g1 = G_p walked under L_p, g2 walked
 * under L2 (taken only when p > cutoff) */
#define ORC_VARIANT_PGRAPH 2

typedef struct {
    int64_t n;
    int max_level;
    int32_t entry;
    int max_deg0;                          /* largest layer-0 degree */
    int64_t nnodes[ORC_MAX_LAYERS];        /* layer 0: n */
    const int32_t *nodes[ORC_MAX_LAYERS];  /* layer >= 1: ascending ids; layer 0 unused */
    const int64_t *row_ptr[ORC_MAX_LAYERS];
    const int32_t *col[ORC_MAX_LAYERS];
} orc_graph;

typedef struct {
    int64_t n;
    int d;
    const float *base;      /* n*d FP32, row-major: used by verification */
    int walk_storage;       /* ORC_F32 / ORC_BF16 / ORC_F16 */
    const void *walk_base;  /* n*d elements of walk_storage (== base for FP32) */
} orc_data;

typedef struct {
    double tau;      /* early-termination threshold (default 0.92) */
    float cutoff;    /* G1 if p <= cutoff (default 1.4f) */
    int t_param;     /* 0 -> 6*K; t = min(ef, t_param) */
    int kappa;       /* 0 -> max(K, 2) */
    int w;           /* beam width, 1 = standard HNSW */
    int early_abort; /* partial-sum abort in verification */
    int g, v;        /* lane-group size and elements per lane-load of the base distance */
    int cache_slots; /* 0 = exact visited set; else lossy cache of this many slots (power of 2) */
    int variant;     /* ORC_VARIANT_STD: g1 = G1 (L1), g2 = G2 (L2); ORC_VARIANT_EXT: g1 = G_0.5
                        (L0.5), g2 = G_1 (L1); ORC_VARIANT_PGRAPH: g1 = G_p (L_walk_p), g2 (L2) */
    double walk_p;   /* ORC_VARIANT_PGRAPH: the p G_p was built for */
} orc_params;

typedef struct {
    int32_t graph;   /* 1 = g1, 2 = g2 */
    int32_t n_b;     /* base-metric distance evaluations (descent + layer 0) */
    int32_t n_exp;   /* layer-0 expansions */
    int32_t n_p;     /* L_p distance evaluations */
    int32_t batches; /* verification batches taken */
    int32_t nc;      /* |C| */
    int32_t nres;    /* results returned */
    int32_t m;       /* intersection count needed to stop */
    int32_t entry0;  /* layer-0 start node (end of the descent) */
} orc_stats;

double orc_lp_sum(const float *x, const float *q, int d, double p);
double orc_lp_dist(const float *x, const float *q, int d, double p);
void orc_bruteforce(const float *base, int64_t n, int d, const float *qs, int64_t nq, const float *p, int K,
                    int32_t *ids, double *S, int nthreads);

uint16_t orc_to_bf16(float f);
uint16_t orc_to_f16(float f);
float orc_bf16_to_f32(uint16_t h);
float orc_f16_to_f32(uint16_t h);
void orc_convert(const float *src, int64_t cnt, int storage, uint16_t *dst);

float orc_base_dist(const void *x, int storage, const float *q, int d, int metric, double mp, int g, int v);

int orc_m_of(double tau, int K);

int orc_knn_search(const orc_graph *G, const orc_data *D, const float *q, int metric, double mp, int ef, int t, int w,
                   int g, int v, int cache_slots, int32_t *c_ids, float *c_keys, orc_stats *st);

int orc_verify(const orc_data *D, const float *q, float p, int K, const int32_t *C, int nC, int kappa, int m,
               int early_abort, int32_t *ids, double *S, double *dist, orc_stats *st);

int orc_query(const orc_graph *g1, const orc_graph *g2, const orc_data *D, const float *q, float p, int K, int ef,
              const orc_params *prm, int32_t *ids, double *S, double *dist, int32_t *c_ids, float *c_keys,
              orc_stats *st);

void orc_query_batch(const orc_graph *g1, const orc_graph *g2, const orc_data *D, const float *qs, int64_t nq,
                     const float *p, const int32_t *k, const int32_t *ef, const orc_params *prm, int k_stride,
                     int64_t *ids, double *dist, double *S, int c_stride, int32_t *c_ids, float *c_keys,
                     orc_stats *stats, int nthreads);
#endif
