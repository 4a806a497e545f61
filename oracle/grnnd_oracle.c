/*
 * grnnd_oracle.c -- plain, slow CPU reference for GRNND graph construction
 * (Li, Chang, Li, Miyazaki, "GRNND: A GPU-Parallel Relative NN-Descent
 * Algorithm for Efficient Approximate Nearest Neighbor Graph Construction").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker that the GPU library is
 * compared against. It shares no code, header, table or constant with the GPU
 * path. Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the library itself never does.
 *
 * Arithmetic: every distance is accumulated in FP64 over the FP32 inputs and
 * rounded once to FP32; that FP32 value is the key that is stored and compared
 * (the paper fixes no precision; its vectors are float).
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes of the repository):
 *   - keys are squared L2 distances (the square root of Alg. 5 is monotone and
 *     is dropped) or, for the inner-product metric, the negated inner product;
 *   - "(key, id)" order is lexicographic on (FP32 key, int32 id); a tie on the
 *     key is broken by the smaller id, both for "closer" and for sorting;
 *   - the prune test is strict: d(n_i, n_j) < max(d(v,n_i), d(v,n_j)) (Eq. 2);
 *   - "random neighbour pairs" (Alg. 4): candidates arrive in a hash order;
 *     each arriving candidate is paired with every candidate still alive, in
 *     arrival order; a pair that meets Eq. 2 redirects the farther one to the
 *     closer one's list and marks it dead (bottom); a dead arriving candidate
 *     stops its own scan;
 *   - the write pool of x after a round is the first R, by (key, id), of the
 *     de-duplicated multiset of items sent to x (Alg. 6 run to completion
 *     gives this set for any insertion order);
 *   - reverse-edge sampling (Section 3.6): m = floor(rho * k) entries of N_v,
 *     chosen as the m smallest in a hash order (or, as an option, the m
 *     nearest), receive v;
 *   - the output graph is the pool after a last ascending, strict, no-redirect
 *     pass of Alg. 2's scan (so every kept pair meets Eq. 1).
 *
 * Randomness comes from one counter-based hash, h(seed,a,b,c) =
 * mix(mix(mix(mix(seed) ^ a) ^ b) ^ c), where mix is the SplitMix64 output
 * function (Steele, Lea & Flood, OOPSLA 2014): z = x + 0x9E3779B97F4A7C15,
 * z = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z = (z ^ z>>27) * 0x94D049BB133111EB,
 * return z ^ z>>31. Domain tags: 0x1000+round (update order), 0x2000+t1
 * (reverse sampling), 0x3000 (initial draws).
 *
 * Near-tie tags: when tau > 0 the oracle marks every output row whose content
 * could legitimately differ from an implementation whose FP32 distances carry
 * a relative error up to tau of their natural scale (sum of squares for L2,
 * sum of |products| for IP). A tagged row is exempt from exact comparison.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_L2 = 0, ORC_IP = 1 };
enum { ORC_DISORDERED = 0, ORC_ASCENDING = 1, ORC_DESCENDING = 2 };
enum { ORC_MAXR = 256 };

/* ------------------------------------------------------------------ threads */
void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* --------------------------------------------------------------------- hash */
uint64_t orc_mix(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_hash(uint64_t seed, uint64_t a, uint64_t b, uint64_t c) {
    return orc_mix(orc_mix(orc_mix(orc_mix(seed) ^ a) ^ b) ^ c);
}

/* Order key for "hash order": high 32 bits of h, then the id. */
static uint64_t hash_order_key(uint64_t h, int32_t id) {
    return ((h >> 32) << 32) | (uint64_t)(uint32_t)id;
}

/* ----------------------------------------------------------------- distance */
/* Exact-ish distance in FP64 plus its error scale (see header). */
static double dist64(const float *x, const float *y, int32_t d, int32_t metric,
                     double *scale) {
    double s = 0.0, sc = 0.0;
    if (metric == ORC_L2) {
        for (int32_t k = 0; k < d; ++k) {
            double t = (double)x[k] - (double)y[k];
            s += t * t;
        }
        sc = s;
    } else {
        for (int32_t k = 0; k < d; ++k) {
            double p = (double)x[k] * (double)y[k];
            s += p;
            sc += fabs(p);
        }
        s = -s;
    }
    if (scale) *scale = sc;
    return s;
}

float orc_dist(const float *X, int32_t d, int32_t metric, int64_t a, int64_t b) {
    return (float)dist64(X + a * (int64_t)d, X + b * (int64_t)d, d, metric, NULL);
}

double orc_dist_exact(const float *X, int32_t d, int32_t metric, int64_t a, int64_t b) {
    return dist64(X + a * (int64_t)d, X + b * (int64_t)d, d, metric, NULL);
}

/* (key, id) strict order */
static int kid_less(float ka, int32_t ia, float kb, int32_t ib) {
    return (ka < kb) || (ka == kb && ia < ib);
}

/* ---------------------------------------------------------------- candidate */
typedef struct {
    int32_t id;
    float key;
    uint64_t ord; /* arrival sort key */
} cand_t;

static int cmp_cand_ord(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    return (x->ord < y->ord) ? -1 : (x->ord > y->ord) ? 1 : 0;
}

static int cmp_cand_kid_asc(const void *a, const void *b) {
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (kid_less(x->key, x->id, y->key, y->id)) return -1;
    if (kid_less(y->key, y->id, x->key, x->id)) return 1;
    return 0;
}

static int cmp_cand_kid_desc(const void *a, const void *b) {
    return -cmp_cand_kid_asc(a, b);
}

/*
 * One vertex's update (Alg. 4 body, Eq. 2), reading only its row of the read
 * pool. Emits exactly one item per valid candidate:
 *   survivor u            -> (dest = v,     cand = u,   key = key_u,   es = 0)
 *   u redirected to close -> (dest = close, cand = u,   key = d(u,close), es = scale)
 * Returns the number of items written. *near_tie is set when a prune decision
 * is within tau of its threshold; *ncmp counts the distance comparisons made.
 */
int32_t orc_scan_vertex(const float *X, int32_t d, int32_t metric, int32_t R,
                        const int32_t *row_ids, const float *row_keys, int64_t v,
                        uint64_t seed, uint32_t round, int32_t order, double tau,
                        int32_t *it_dest, int32_t *it_cand, float *it_key,
                        double *it_es, int32_t *near_tie, int64_t *ncmp) {
    cand_t c[ORC_MAXR];
    int K = 0;
    if (R > ORC_MAXR) abort(); /* the Python wrapper refuses such widths */
    for (int i = 0; i < R; ++i) {
        if (row_ids[i] < 0) continue;
        c[K].id = row_ids[i];
        c[K].key = row_keys[i];
        c[K].ord = 0;
        ++K;
    }
    /* arrival order (Section 3.3: disordered; Section 4.3: ascending/descending) */
    if (order == ORC_DISORDERED) {
        for (int i = 0; i < K; ++i)
            c[i].ord = hash_order_key(
                orc_hash(seed, 0x1000ULL + round, (uint64_t)v, (uint64_t)c[i].id), c[i].id);
        qsort(c, K, sizeof(cand_t), cmp_cand_ord);
    } else if (order == ORC_ASCENDING) {
        qsort(c, K, sizeof(cand_t), cmp_cand_kid_asc);
    } else {
        qsort(c, K, sizeof(cand_t), cmp_cand_kid_desc);
    }

    int alive[ORC_MAXR], na = 0;
    int dead[ORC_MAXR];
    memset(dead, 0, sizeof(dead));
    int nit = 0;
    const float *xs = X;
    for (int t = 0; t < K; ++t) {
        int u_dead = 0;
        for (int a = 0; a < na; ++a) {
            int w = alive[a];
            if (dead[w]) continue;
            double sc;
            double de = dist64(xs + (int64_t)c[t].id * d, xs + (int64_t)c[w].id * d, d,
                               metric, &sc);
            float d32 = (float)de;
            float thr = c[t].key > c[w].key ? c[t].key : c[w].key;
            if (ncmp) ++*ncmp;
            if (tau > 0.0 && fabs(de - (double)thr) < tau * sc && near_tie) *near_tie = 1;
            if (d32 < thr) {
                if (kid_less(c[w].key, c[w].id, c[t].key, c[t].id)) {
                    /* u is the farther one: redirect u to w's list, u dies */
                    it_dest[nit] = c[w].id; it_cand[nit] = c[t].id;
                    it_key[nit] = d32; it_es[nit] = sc; ++nit;
                    u_dead = 1;
                    break;
                }
                /* w is the farther one: redirect w to u's list, w dies */
                it_dest[nit] = c[t].id; it_cand[nit] = c[w].id;
                it_key[nit] = d32; it_es[nit] = sc; ++nit;
                dead[w] = 1;
            }
        }
        if (u_dead) dead[t] = 1;
        else alive[na++] = t;
    }
    for (int a = 0; a < na; ++a) {
        int u = alive[a];
        if (dead[u]) continue;
        it_dest[nit] = (int32_t)v; it_cand[nit] = c[u].id;
        it_key[nit] = c[u].key; it_es[nit] = 0.0; ++nit;
    }
    return nit;
}

/* -------------------------------------------------------------------- merge */
typedef struct {
    int32_t dest, cand;
    float key;
    double es;
} item_t;

static int cmp_item_dck(const void *a, const void *b) {
    const item_t *x = (const item_t *)a, *y = (const item_t *)b;
    if (x->dest != y->dest) return x->dest < y->dest ? -1 : 1;
    if (x->cand != y->cand) return x->cand < y->cand ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return 0;
}

static int cmp_item_kc(const void *a, const void *b) {
    const item_t *x = (const item_t *)a, *y = (const item_t *)b;
    if (kid_less(x->key, x->cand, y->key, y->cand)) return -1;
    if (kid_less(y->key, y->cand, x->key, x->cand)) return 1;
    return 0;
}

/*
 * pool_out[x] = first R by (key, cand) of the items sent to x, after dropping
 * cand == x and keeping one item (the smallest key) per cand. Rows are sorted
 * and padded with (-1, +inf). Alg. 6 semantics (dedupe, append, replace the
 * farthest if closer), taken to completion.
 */
void orc_merge(int64_t n, int32_t R, int64_t m, const int32_t *dest,
               const int32_t *cand, const float *key, const double *es,
               int32_t *out_ids, float *out_keys, double tau, uint8_t *tag) {
    for (int64_t i = 0; i < n * (int64_t)R; ++i) {
        out_ids[i] = -1;
        out_keys[i] = INFINITY;
    }
    if (m <= 0) return;
    item_t *it = (item_t *)malloc((size_t)m * sizeof(item_t));
    item_t *lst = (item_t *)malloc((size_t)m * sizeof(item_t));
    for (int64_t i = 0; i < m; ++i) {
        it[i].dest = dest[i];
        it[i].cand = cand[i];
        it[i].key = key[i];
        it[i].es = es ? es[i] : 0.0;
    }
    qsort(it, (size_t)m, sizeof(item_t), cmp_item_dck);
    int64_t i = 0;
    while (i < m) {
        int32_t x = it[i].dest;
        int64_t j = i;
        while (j < m && it[j].dest == x) ++j;
        int64_t nl = 0;
        for (int64_t p = i; p < j; ++p) {
            if (it[p].cand == x) continue;
            if (nl > 0 && lst[nl - 1].cand == it[p].cand) {
                if (it[p].es > lst[nl - 1].es) lst[nl - 1].es = it[p].es;
                continue; /* same cand, larger-or-equal key: keep the first */
            }
            lst[nl++] = it[p];
        }
        qsort(lst, (size_t)nl, sizeof(item_t), cmp_item_kc);
        int64_t keep = nl < R ? nl : R;
        for (int64_t p = 0; p < keep; ++p) {
            out_ids[(int64_t)x * R + p] = lst[p].cand;
            out_keys[(int64_t)x * R + p] = lst[p].key;
        }
        if (tag && tau > 0.0) {
            for (int64_t p = 0; p + 1 < nl && p < R; ++p) {
                double gap = fabs((double)lst[p + 1].key - (double)lst[p].key);
                if (gap < tau * (lst[p].es + lst[p + 1].es)) tag[x] = 1;
            }
        }
        i = j;
    }
    free(lst);
    free(it);
}

/* ------------------------------------------------------------------- init */
/*
 * Initial pools (Alg. 3): for each v draw ids
 * h(seed, 0x3000, v, j) mod n for j = 0, 1, ..., skipping v and repeats,
 * until min(S, n-1) distinct ids are held; keys are their distances to v.
 */
void orc_init(const float *X, int64_t n, int32_t d, int32_t metric, int32_t R,
              int32_t S, uint64_t seed, int32_t *out_ids, float *out_keys,
              double tau, uint8_t *tag) {
    int32_t want = S < n - 1 ? S : (int32_t)(n - 1);
    int64_t m = n * (int64_t)want;
    int32_t *dst = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    int32_t *cnd = (int32_t *)malloc((size_t)m * sizeof(int32_t));
    float *ky = (float *)malloc((size_t)m * sizeof(float));
    double *es = (double *)malloc((size_t)m * sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t v = 0; v < n; ++v) {
        int32_t got = 0;
        int32_t *ids = cnd + v * want;
        for (uint64_t j = 0; got < want; ++j) {
            int64_t id = (int64_t)(orc_hash(seed, 0x3000ULL, (uint64_t)v, j) % (uint64_t)n);
            if (id == v) continue;
            int dup = 0;
            for (int32_t q = 0; q < got; ++q)
                if (ids[q] == id) { dup = 1; break; }
            if (dup) continue;
            ids[got++] = (int32_t)id;
        }
        for (int32_t q = 0; q < want; ++q) {
            double sc;
            double de = dist64(X + v * (int64_t)d, X + (int64_t)ids[q] * d, d, metric, &sc);
            dst[v * want + q] = (int32_t)v;
            ky[v * want + q] = (float)de;
            es[v * want + q] = sc;
        }
    }
    orc_merge(n, R, m, dst, cnd, ky, es, out_ids, out_keys, tau, tag);
    free(dst); free(cnd); free(ky); free(es);
}

/* ---------------------------------------------------------- update round */
/* stats (int64[8]): 0 tile pairs sum K(K-1)/2, 1 comparisons made,
 * 2 redirects, 3 survivors, 4 items, 5 near-tie vertices */
void orc_update_round(const float *X, int64_t n, int32_t d, int32_t metric,
                      int32_t R, const int32_t *in_ids, const float *in_keys,
                      uint64_t seed, uint32_t round, int32_t order,
                      int32_t *out_ids, float *out_keys, double tau,
                      uint8_t *tag, int64_t *stats) {
    int64_t cap = n * (int64_t)R;
    int32_t *dst = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    int32_t *cnd = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *ky = (float *)malloc((size_t)cap * sizeof(float));
    double *es = (double *)malloc((size_t)cap * sizeof(double));
    int32_t *nit = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *near = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    int64_t ncmp = 0, npairs = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : ncmp, npairs)
    for (int64_t v = 0; v < n; ++v) {
        int64_t nc = 0;
        nit[v] = orc_scan_vertex(X, d, metric, R, in_ids + v * R, in_keys + v * R, v,
                                 seed, round, order, tau, dst + v * R, cnd + v * R,
                                 ky + v * R, es + v * R, &near[v], &nc);
        ncmp += nc;
        npairs += (int64_t)nit[v] * (nit[v] - 1) / 2;
    }
    /* compact */
    int64_t m = 0, nred = 0, nsurv = 0, nnear = 0;
    for (int64_t v = 0; v < n; ++v) {
        for (int32_t q = 0; q < nit[v]; ++q) {
            int64_t s = v * R + q;
            if (dst[s] == v) ++nsurv; else ++nred;
            dst[m] = dst[s]; cnd[m] = cnd[s]; ky[m] = ky[s]; es[m] = es[s];
            ++m;
        }
    }
    orc_merge(n, R, m, dst, cnd, ky, es, out_ids, out_keys, tau, tag);
    for (int64_t v = 0; v < n; ++v) {
        if (!near[v]) continue;
        ++nnear;
        if (!tag) continue;
        tag[v] = 1;
        for (int32_t q = 0; q < R; ++q)
            if (in_ids[v * R + q] >= 0) tag[in_ids[v * R + q]] = 1;
    }
    if (stats) {
        stats[0] += npairs; stats[1] += ncmp; stats[2] += nred;
        stats[3] += nsurv; stats[4] += m; stats[5] += nnear;
    }
    free(dst); free(cnd); free(ky); free(es); free(nit); free(near);
}

/* --------------------------------------------------------- reverse round */
/*
 * REVERSE_EDGE_SAMPLING (Alg. 3 after each outer iteration but the last;
 * Section 3.6): every v with k valid entries sends itself to m = floor(rho*k)
 * of them; every pool row is re-sent to its owner; the write pool is then
 * merged as in an update round. Section 3.6 calls the chosen entries the
 * "top" rho k neighbours. Two readings, selected by `mode`:
 *   ORC_REV_HASH    (0) the m smallest in hash order -- the pool order of the
 *                       paper's design is the random order disordered
 *                       propagation leaves behind, which a canonical pool
 *                       replaces by this hash order;
 *   ORC_REV_NEAREST (1) the m nearest, i.e. the first m by (key, id).
 */
enum { ORC_REV_HASH = 0, ORC_REV_NEAREST = 1 };

void orc_reverse_round(int64_t n, int32_t R, const int32_t *in_ids,
                       const float *in_keys, uint64_t seed, uint32_t t1, float rho,
                       int32_t mode, int32_t *out_ids, float *out_keys) {
    int64_t cap = n * (int64_t)R * 2;
    int32_t *dst = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    int32_t *cnd = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *ky = (float *)malloc((size_t)cap * sizeof(float));
    int64_t m = 0;
    cand_t c[ORC_MAXR];
    if (R > ORC_MAXR) abort();
    for (int64_t v = 0; v < n; ++v) {
        int K = 0;
        for (int i = 0; i < R; ++i) {
            int32_t id = in_ids[v * R + i];
            if (id < 0) continue;
            c[K].id = id;
            c[K].key = in_keys[v * R + i];
            c[K].ord = hash_order_key(
                orc_hash(seed, 0x2000ULL + t1, (uint64_t)v, (uint64_t)id), id);
            dst[m] = (int32_t)v; cnd[m] = id; ky[m] = c[K].key; ++m;
            ++K;
        }
        int ms = (int)floor((double)rho * (double)K);
        if (mode == ORC_REV_NEAREST)
            qsort(c, K, sizeof(cand_t), cmp_cand_kid_asc);
        else
            qsort(c, K, sizeof(cand_t), cmp_cand_ord);
        for (int i = 0; i < ms; ++i) {
            dst[m] = c[i].id; cnd[m] = (int32_t)v; ky[m] = c[i].key; ++m;
        }
    }
    orc_merge(n, R, m, dst, cnd, ky, NULL, out_ids, out_keys, 0.0, NULL);
    free(dst); free(cnd); free(ky);
}

/* -------------------------------------------------------------- finalize */
/*
 * Output graph: Alg. 2's scan over each pool row in ascending (key, id) with
 * the strict test of Eq. 1 and no redirection; the survivors, ascending,
 * padded with -1. Runs the same per-vertex scan as an update round in
 * ascending order; in that order the arriving candidate is always the
 * farther one, so only it can be dropped.
 */
void orc_finalize(const float *X, int64_t n, int32_t d, int32_t metric, int32_t R,
                  const int32_t *in_ids, const float *in_keys, int32_t *out_adj,
                  float *out_keys, double tau, uint8_t *tag, int64_t *stats) {
    int64_t npairs = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : npairs)
    for (int64_t v = 0; v < n; ++v) {
        int32_t dst[ORC_MAXR], cnd[ORC_MAXR];
        float ky[ORC_MAXR];
        double es[ORC_MAXR];
        int32_t near = 0;
        int32_t k = orc_scan_vertex(X, d, metric, R, in_ids + v * R, in_keys + v * R, v,
                                    0, 0, ORC_ASCENDING, tau, dst, cnd, ky, es, &near,
                                    NULL);
        npairs += (int64_t)k * (k - 1) / 2;
        int32_t o = 0;
        for (int32_t q = 0; q < k; ++q) {
            if (dst[q] != v) continue;
            out_adj[v * R + o] = cnd[q];
            if (out_keys) out_keys[v * R + o] = ky[q];
            ++o;
        }
        for (; o < R; ++o) {
            out_adj[v * R + o] = -1;
            if (out_keys) out_keys[v * R + o] = INFINITY;
        }
        if (tag && near) tag[v] = 1;
    }
    if (stats) stats[0] += npairs;
}

/* ----------------------------------------------------------------- build */
/* Alg. 3: init; T1 outer iterations of T2 update rounds, with reverse-edge
 * sampling after every outer iteration but the last; then the output pass. */
void orc_build(const float *X, int64_t n, int32_t d, int32_t metric, int32_t R,
               int32_t S, int32_t T1, int32_t T2, float rho, int32_t order,
               int32_t reverse_mode, uint64_t seed, int32_t *out_adj, float *out_keys,
               int64_t *stats) {
    int64_t cap = n * (int64_t)R;
    int32_t *ia = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *ka = (float *)malloc((size_t)cap * sizeof(float));
    int32_t *ib = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *kb = (float *)malloc((size_t)cap * sizeof(float));
    orc_init(X, n, d, metric, R, S, seed, ia, ka, 0.0, NULL);
    if (stats) stats[6] += n * (int64_t)(S < n - 1 ? S : n - 1);
    for (int32_t t1 = 1; t1 <= T1; ++t1) {
        for (int32_t t2 = 1; t2 <= T2; ++t2) {
            uint32_t round = (uint32_t)((t1 - 1) * T2 + (t2 - 1));
            orc_update_round(X, n, d, metric, R, ia, ka, seed, round, order, ib, kb, 0.0,
                             NULL, stats);
            int32_t *ti = ia; ia = ib; ib = ti;
            float *tk = ka; ka = kb; kb = tk;
        }
        if (t1 != T1) {
            orc_reverse_round(n, R, ia, ka, seed, (uint32_t)t1, rho, reverse_mode, ib, kb);
            int32_t *ti = ia; ia = ib; ib = ti;
            float *tk = ka; ka = kb; kb = tk;
        }
    }
    int64_t fst[8] = {0};
    orc_finalize(X, n, d, metric, R, ia, ka, out_adj, out_keys, 0.0, NULL, fst);
    if (stats) stats[7] += fst[0];
    free(ia); free(ka); free(ib); free(kb);
}

/* ------------------------------------------ sequential RNN-Descent */
/*
 * The sequential, in-place RNN-Descent of Alg. 1 with the update of Alg. 2,
 * kept as a second CPU reference graph (it is the CPU method the GPU design
 * starts from, not the GPU method). Vertices are updated one after another in
 * id order in each of the T1 x T2 passes. Alg. 2: N_v sorted by (key, id),
 * v and repeated ids dropped, the first R kept; the closest is accepted; each
 * further candidate n is compared with the accepted n' in order, and the
 * first n' with d(n, n') <= d(v, n) excludes it: n is appended to N_{n'} at
 * once (later vertices of the same pass see it); otherwise n is accepted.
 * N_v becomes the accepted list. Readings where the paper is silent: the
 * initial lists are the same hash draws as orc_init's; ADD_REVERSE_EDGES
 * appends v to N_n for every n in N_v, all taken from the lists as they stand
 * before any is changed; a list may grow past R between updates and is cut
 * by its next update; the output is the lists after the last pass, sorted,
 * de-duplicated, cut to R and passed through the same output pass as
 * orc_build (ascending, strict, no redirection).
 */
typedef struct {
    cand_t *e;
    int32_t len, cap;
} clist_t;

static void clist_push(clist_t *l, int32_t id, float key) {
    if (l->len == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 16;
        l->e = (cand_t *)realloc(l->e, (size_t)l->cap * sizeof(cand_t));
    }
    l->e[l->len].id = id;
    l->e[l->len].key = key;
    l->e[l->len].ord = 0;
    l->len++;
}

/* sort by (key, id), drop self and repeated ids (the first, closest, stays),
 * keep the first R */
static void clist_canon(clist_t *l, int64_t v, int32_t R) {
    qsort(l->e, (size_t)l->len, sizeof(cand_t), cmp_cand_kid_asc);
    int32_t o = 0;
    for (int32_t i = 0; i < l->len && o < R; ++i) {
        if (l->e[i].id == v) continue;
        int dup = 0;
        for (int32_t j = 0; j < o; ++j)
            if (l->e[j].id == l->e[i].id) { dup = 1; break; }
        if (!dup) l->e[o++] = l->e[i];
    }
    l->len = o;
}

void orc_rnn_descent_seq(const float *X, int64_t n, int32_t d, int32_t metric, int32_t R,
                         int32_t S, int32_t T1, int32_t T2, uint64_t seed, int32_t *out_adj,
                         float *out_keys) {
    int64_t cap = n * (int64_t)R;
    int32_t *ids = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    float *keys = (float *)malloc((size_t)cap * sizeof(float));
    orc_init(X, n, d, metric, R, S, seed, ids, keys, 0.0, NULL);
    clist_t *N = (clist_t *)calloc((size_t)n, sizeof(clist_t));
    for (int64_t v = 0; v < n; ++v)
        for (int32_t j = 0; j < R; ++j)
            if (ids[v * R + j] >= 0) clist_push(&N[v], ids[v * R + j], keys[v * R + j]);
    cand_t *acc = (cand_t *)malloc((size_t)R * sizeof(cand_t));
    cand_t *cur = (cand_t *)malloc((size_t)R * sizeof(cand_t));
    for (int32_t t1 = 1; t1 <= T1; ++t1) {
        for (int32_t t2 = 1; t2 <= T2; ++t2) {
            for (int64_t v = 0; v < n; ++v) {
                clist_canon(&N[v], v, R);
                int32_t k = N[v].len;
                memcpy(cur, N[v].e, (size_t)k * sizeof(cand_t));
                int32_t na = 0;
                for (int32_t i = 0; i < k; ++i) {
                    int keep = 1;
                    for (int32_t j = 0; j < na; ++j) {
                        double sc;
                        float dnn = (float)dist64(X + (int64_t)cur[i].id * d,
                                                  X + (int64_t)acc[j].id * d, d, metric, &sc);
                        if (dnn <= cur[i].key) {
                            keep = 0;
                            clist_push(&N[acc[j].id], cur[i].id, dnn);
                            break;
                        }
                    }
                    if (keep) acc[na++] = cur[i];
                }
                /* the accepted list replaces N_v; anything appended to N_v by
                 * this vertex's own redirections cannot occur (n' != v) */
                N[v].len = 0;
                for (int32_t j = 0; j < na; ++j) clist_push(&N[v], acc[j].id, acc[j].key);
            }
        }
        if (t1 != T1) {
            int32_t *sn = (int32_t *)malloc((size_t)n * sizeof(int32_t));
            int64_t tot = 0;
            for (int64_t v = 0; v < n; ++v) { sn[v] = N[v].len; tot += sn[v]; }
            int32_t *rid = (int32_t *)malloc((size_t)tot * sizeof(int32_t));
            float *rky = (float *)malloc((size_t)tot * sizeof(float));
            int64_t o = 0;
            for (int64_t v = 0; v < n; ++v)
                for (int32_t j = 0; j < sn[v]; ++j) {
                    rid[o] = N[v].e[j].id;
                    rky[o] = N[v].e[j].key;
                    ++o;
                }
            o = 0;
            for (int64_t v = 0; v < n; ++v)
                for (int32_t j = 0; j < sn[v]; ++j, ++o) clist_push(&N[rid[o]], (int32_t)v, rky[o]);
            free(sn); free(rid); free(rky);
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        clist_canon(&N[v], v, R);
        for (int32_t j = 0; j < R; ++j) {
            ids[v * R + j] = j < N[v].len ? N[v].e[j].id : -1;
            keys[v * R + j] = j < N[v].len ? N[v].e[j].key : INFINITY;
        }
        free(N[v].e);
    }
    orc_finalize(X, n, d, metric, R, ids, keys, out_adj, out_keys, 0.0, NULL, NULL);
    free(N); free(acc); free(cur); free(ids); free(keys);
}

/* ---------------------------------------------------------------- search */
/*
 * Best-first search with a candidate list of at most L entries ordered by
 * (key, id): start from `entry`; repeatedly expand the first unexpanded entry,
 * computing keys for its not-yet-visited neighbours and keeping the best L;
 * stop when every entry is expanded; return the first k (Section 4.1: one
 * search routine over every flat graph, parameterised by the list size).
 */
void orc_search(const float *X, int64_t n, int32_t d, int32_t metric,
                const int32_t *adj, int32_t R, int64_t entry, const float *Q,
                int64_t nq, int32_t k, int32_t L, int32_t *out_ids, float *out_keys) {
#pragma omp parallel
    {
        int32_t *stamp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        for (int64_t i = 0; i < n; ++i) stamp[i] = -1;
        float *lk = (float *)malloc((size_t)L * sizeof(float));
        int32_t *li = (int32_t *)malloc((size_t)L * sizeof(int32_t));
        uint8_t *le = (uint8_t *)malloc((size_t)L);
#pragma omp for schedule(dynamic, 16)
        for (int64_t qi = 0; qi < nq; ++qi) {
            const float *q = Q + qi * (int64_t)d;
            int32_t cnt = 0;
            int32_t stq = (int32_t)qi;
            stamp[entry] = stq;
            lk[0] = (float)dist64(q, X + entry * (int64_t)d, d, metric, NULL);
            li[0] = (int32_t)entry;
            le[0] = 0;
            cnt = 1;
            for (;;) {
                int32_t p = 0;
                while (p < cnt && le[p]) ++p;
                if (p == cnt) break;
                le[p] = 1;
                int32_t u = li[p];
                for (int32_t r = 0; r < R; ++r) {
                    int32_t nb = adj[(int64_t)u * R + r];
                    if (nb < 0) continue;
                    if (stamp[nb] == stq) continue;
                    stamp[nb] = stq;
                    float key = (float)dist64(q, X + (int64_t)nb * d, d, metric, NULL);
                    if (cnt == L && !kid_less(key, nb, lk[L - 1], li[L - 1])) continue;
                    int32_t pos = cnt < L ? cnt : L - 1;
                    while (pos > 0 && kid_less(key, nb, lk[pos - 1], li[pos - 1])) {
                        lk[pos] = lk[pos - 1]; li[pos] = li[pos - 1]; le[pos] = le[pos - 1];
                        --pos;
                    }
                    lk[pos] = key; li[pos] = nb; le[pos] = 0;
                    if (cnt < L) ++cnt;
                }
            }
            for (int32_t r = 0; r < k; ++r) {
                out_ids[qi * k + r] = r < cnt ? li[r] : -1;
                out_keys[qi * k + r] = r < cnt ? lk[r] : INFINITY;
            }
        }
        free(stamp); free(lk); free(li); free(le);
    }
}

/* Approximate medoid: the point nearest (L2, FP64) to the FP64 mean; ties by id. */
int64_t orc_medoid(const float *X, int64_t n, int32_t d) {
    double *mean = (double *)calloc((size_t)d, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < d; ++k) mean[k] += X[i * (int64_t)d + k];
    for (int32_t k = 0; k < d; ++k) mean[k] /= (double)n;
    int64_t best = 0;
    double bd = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < d; ++k) {
            double t = (double)X[i * (int64_t)d + k] - mean[k];
            s += t * t;
        }
        if (s < bd) { bd = s; best = i; }
    }
    free(mean);
    return best;
}
