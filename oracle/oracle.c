/* CPU oracle for the IMM hot path -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain C, deliberately simple.  Each function names the passage of the gIM paper (or of
 * the IMM / Philox papers) that it follows.  Build: gcc -O2 -fopenmp -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11, Sec. 5: the Philox round with multipliers
 * 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85).
 * One round maps (c0,c1,c2,c3) to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0));
 * the key is bumped between rounds.
 * ---------------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t draw_word(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                          int word) {
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word];
}

/* ------------------------------------------------------------------------------------
 * Threshold encodings.
 * IC (Sec. II-B; Alg. 3's test "p < p_uv"): an edge with probability p is live when a
 * uniform 32-bit draw x satisfies x < floor(p * 2^32); p = 1 saturates to "always".
 * ---------------------------------------------------------------------------------- */
uint32_t orc_ic_threshold(float p) {
    double t = floor((double)p * 4294967296.0);
    if (t >= 4294967296.0) return ORC_ALWAYS;
    return (uint32_t)t;
}

int orc_encode_ic(int64_t m, const float* p, uint32_t* thr) {
    for (int64_t e = 0; e < m; ++e) {
        if (!(p[e] >= 0.0f && p[e] <= 1.0f)) return -1;
        thr[e] = orc_ic_threshold(p[e]);
    }
    return 0;
}

/* LT (Sec. II-B Eq. 1 and Sec. III-G): a vertex picks at most one in-edge, edge j with
 * probability w_j / sum(w); a uniform draw is compared with consecutive prefix sums of the
 * in-weights and the first prefix above the draw wins.  Prefix sums are scaled to 2^32 in
 * exact integer arithmetic; the last one saturates so that the weights sum to one. */
int orc_encode_lt(int32_t n, const int64_t* in_off, const uint32_t* w, uint32_t* cum) {
    for (int32_t v = 0; v < n; ++v) {
        int64_t s = in_off[v], e = in_off[v + 1];
        if (e < s) return -1;
        uint64_t total = 0;
        for (int64_t j = s; j < e; ++j) {
            uint64_t wj = w ? (uint64_t)w[j] : 1u;
            if (wj == 0) return -2;
            total += wj;
        }
        uint64_t prefix = 0;
        for (int64_t j = s; j < e; ++j) {
            prefix += w ? (uint64_t)w[j] : 1u;
            if (j == e - 1) {
                cum[j] = ORC_ALWAYS;
            } else {
                unsigned __int128 num = (unsigned __int128)prefix << 32;
                cum[j] = (uint32_t)(num / total);
            }
        }
    }
    return 0;
}

/* randSelect(V) of Alg. 3: a uniform root by multiply-shift of one 32-bit draw. */
int32_t orc_root(uint64_t seed, uint32_t r, int32_t n) {
    uint32_t w0 = draw_word(seed, r, 0u, 0u, ORC_DOMAIN_ROOT, 0);
    return (int32_t)(((uint64_t)w0 * (uint64_t)(uint32_t)n) >> 32);
}

/* ------------------------------------------------------------------------------------
 * Random RR set under IC (Sec. II-E definition; Alg. 3; Sec. III-A "Parallel BFS").
 * The RR set of root v in a live-edge instance g is every vertex that reaches v in g.
 * A BFS from v over in-edges, testing each in-edge once with its own draw, enumerates
 * exactly that set.  The root is marked visited before the search starts so that it is
 * never enqueued twice.
 * ---------------------------------------------------------------------------------- */
int64_t orc_rr_ic(int32_t n, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* thr, uint64_t seed, uint32_t r, int32_t* out,
                  uint8_t* mark, int64_t* edges) {
    return orc_rr_ic_round(n, in_off, in_src, thr, seed, r, 0u, out, mark, edges);
}

/* The same search in the live-edge instance of round t (Sec. IV-H: one search per round
 * from the set's one root; round t's draws use counter word t, so the rounds' instances
 * are independent and round 0 is the plain one). */
int64_t orc_rr_ic_round(int32_t n, const int64_t* in_off, const int32_t* in_src,
                        const uint32_t* thr, uint64_t seed, uint32_t r, uint32_t t,
                        int32_t* out, uint8_t* mark, int64_t* edges) {
    int64_t size = 0, head = 0, examined = 0;
    int32_t root = orc_root(seed, r, n);
    out[size++] = root;
    mark[root] = 1;
    while (head < size) {
        int32_t u = out[head++];
        for (int64_t e = in_off[u]; e < in_off[u + 1]; ++e) {
            ++examined;
            uint32_t x = draw_word(seed, r, (uint32_t)(e >> 2), t, ORC_DOMAIN_IC, (int)(e & 3));
            int live = (thr[e] == ORC_ALWAYS) || (x < thr[e]);
            int32_t w = in_src[e];
            if (live && !mark[w]) {
                mark[w] = 1;
                out[size++] = w;
            }
        }
    }
    for (int64_t i = 0; i < size; ++i) mark[out[i]] = 0;
    if (edges) *edges = examined;
    return size;
}

/* Random RR set under LT (Sec. III-A: at most one live in-edge per vertex; Sec. III-G).
 * From the current vertex, one draw selects the first in-edge whose cumulative threshold
 * exceeds it; the walk continues from that in-neighbour and stops when the vertex has no
 * in-edge, no edge is selected, or the selected in-neighbour is already in the set. */
int64_t orc_rr_lt(int32_t n, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* cum, uint64_t seed, uint32_t r, int32_t* out,
                  uint8_t* mark, int64_t* edges) {
    return orc_rr_lt_round(n, in_off, in_src, cum, seed, r, 0u, out, mark, edges);
}

int64_t orc_rr_lt_round(int32_t n, const int64_t* in_off, const int32_t* in_src,
                        const uint32_t* cum, uint64_t seed, uint32_t r, uint32_t t,
                        int32_t* out, uint8_t* mark, int64_t* edges) {
    int64_t size = 0, examined = 0;
    int32_t v = orc_root(seed, r, n);
    out[size++] = v;
    mark[v] = 1;
    for (;;) {
        int64_t s = in_off[v], e = in_off[v + 1];
        if (e == s) break;
        examined += e - s;
        uint32_t x = draw_word(seed, r, (uint32_t)v, t, ORC_DOMAIN_LT, 0);
        int64_t pick = -1;
        for (int64_t j = s; j < e; ++j) {
            if (cum[j] == ORC_ALWAYS || x < cum[j]) {
                pick = j;
                break;
            }
        }
        if (pick < 0) break;
        int32_t u = in_src[pick];
        if (mark[u]) break;
        mark[u] = 1;
        out[size++] = u;
        v = u;
    }
    for (int64_t i = 0; i < size; ++i) mark[out[i]] = 0;
    if (edges) *edges = examined;
    return size;
}

/* ------------------------------------------------------------------------------------
 * RR-set collection R (Alg. 1 step 1; Alg. 6 concatenates sets into one array RR with
 * offsets).  Sets are kept in index order and each set sorted ascending.
 * ---------------------------------------------------------------------------------- */
struct orc_pool {
    int32_t n;
    int64_t m;
    const int64_t* in_off;
    const int32_t* in_src;
    const uint32_t* thr;
    int model;
    uint64_t seed;
    int64_t count, cap_sets;
    int64_t* off;       /* count + 1 */
    int64_t* edges;     /* per set */
    int32_t* ids;
    int64_t cap_ids;
};

orc_pool* orc_pool_new(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                       const uint32_t* thr_or_cum, int model, uint64_t seed) {
    if (n < 1 || m < 0 || (model != 0 && model != 1)) return NULL;
    orc_pool* p = (orc_pool*)calloc(1, sizeof(orc_pool));
    p->n = n; p->m = m; p->in_off = in_off; p->in_src = in_src; p->thr = thr_or_cum;
    p->model = model; p->seed = seed;
    p->cap_sets = 1024;
    p->off = (int64_t*)calloc((size_t)p->cap_sets + 1, sizeof(int64_t));
    p->edges = (int64_t*)calloc((size_t)p->cap_sets, sizeof(int64_t));
    p->cap_ids = 1 << 16;
    p->ids = (int32_t*)malloc((size_t)p->cap_ids * sizeof(int32_t));
    return p;
}

void orc_pool_free(orc_pool* p) {
    if (!p) return;
    free(p->off); free(p->edges); free(p->ids); free(p);
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int orc_pool_extend(orc_pool* p, int64_t upto, int nthreads) {
    if (upto <= p->count) return 0;
    if (upto > 0xFFFFFFFFll) return -1;     /* set index must fit the 32-bit counter word */
    if (upto > p->cap_sets) {
        int64_t cap = p->cap_sets;
        while (cap < upto) cap *= 2;
        p->off = (int64_t*)realloc(p->off, (size_t)(cap + 1) * sizeof(int64_t));
        p->edges = (int64_t*)realloc(p->edges, (size_t)cap * sizeof(int64_t));
        p->cap_sets = cap;
    }
    if (nthreads < 1) nthreads = 1;
    const int64_t chunk = 1 << 15;
    int32_t** sets = (int32_t**)malloc(sizeof(int32_t*) * (size_t)chunk);
    int64_t* sizes = (int64_t*)malloc(sizeof(int64_t) * (size_t)chunk);
    for (int64_t base = p->count; base < upto; base += chunk) {
        int64_t cnt = upto - base < chunk ? upto - base : chunk;
        #pragma omp parallel num_threads(nthreads)
        {
            int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)p->n);
            uint8_t* mark = (uint8_t*)calloc((size_t)p->n, 1);
            #pragma omp for schedule(dynamic, 64)
            for (int64_t j = 0; j < cnt; ++j) {
                int64_t ex = 0, sz;
                uint32_t r = (uint32_t)(base + j);
                if (p->model == 0)
                    sz = orc_rr_ic(p->n, p->in_off, p->in_src, p->thr, p->seed, r, out, mark, &ex);
                else
                    sz = orc_rr_lt(p->n, p->in_off, p->in_src, p->thr, p->seed, r, out, mark, &ex);
                qsort(out, (size_t)sz, sizeof(int32_t), cmp_i32);
                sets[j] = (int32_t*)malloc(sizeof(int32_t) * (size_t)sz);
                memcpy(sets[j], out, sizeof(int32_t) * (size_t)sz);
                sizes[j] = sz;
                p->edges[base + j] = ex;
            }
            free(out);
            free(mark);
        }
        for (int64_t j = 0; j < cnt; ++j) {
            int64_t at = p->off[base + j];
            if (at + sizes[j] > p->cap_ids) {
                int64_t cap = p->cap_ids;
                while (cap < at + sizes[j]) cap *= 2;
                p->ids = (int32_t*)realloc(p->ids, (size_t)cap * sizeof(int32_t));
                p->cap_ids = cap;
            }
            memcpy(p->ids + at, sets[j], sizeof(int32_t) * (size_t)sizes[j]);
            p->off[base + j + 1] = at + sizes[j];
            free(sets[j]);
        }
        p->count = base + cnt;
    }
    free(sets);
    free(sizes);
    return 0;
}

int64_t orc_pool_count(const orc_pool* p) { return p->count; }

int64_t orc_pool_total(const orc_pool* p, int64_t first, int64_t count) {
    if (first < 0 || count < 0 || first + count > p->count) return -1;
    return p->off[first + count] - p->off[first];
}

int64_t orc_pool_edges(const orc_pool* p, int64_t first, int64_t count) {
    if (first < 0 || count < 0 || first + count > p->count) return -1;
    int64_t s = 0;
    for (int64_t r = first; r < first + count; ++r) s += p->edges[r];
    return s;
}

int orc_pool_export(const orc_pool* p, int64_t first, int64_t count, int64_t* off,
                    int32_t* ids) {
    if (first < 0 || count < 0 || first + count > p->count) return -1;
    int64_t base = p->off[first];
    for (int64_t i = 0; i <= count; ++i) off[i] = p->off[first + i] - base;
    if (ids) memcpy(ids, p->ids + base, sizeof(int32_t) * (size_t)(p->off[first + count] - base));
    return 0;
}

/* Occur[] of Sec. III-B: how many sets of the range contain each vertex. */
int orc_pool_hist(const orc_pool* p, int64_t first, int64_t count, uint32_t* hist) {
    if (first < 0 || count < 0 || first + count > p->count) return -1;
    memset(hist, 0, sizeof(uint32_t) * (size_t)p->n);
    for (int64_t i = p->off[first]; i < p->off[first + count]; ++i) hist[p->ids[i]]++;
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Greedy maximum coverage (Alg. 1 lines 6-10; counters as Occur of Sec. III-H, covered
 * flags as in Alg. 7).  Round i takes the vertex outside S that lies in the most sets not
 * yet covered -- the smallest id among equals -- then removes every set containing it.
 * ---------------------------------------------------------------------------------- */
int orc_greedy_sets(int32_t n, int64_t nsets, const int64_t* off, const int32_t* ids,
                    int32_t k, int32_t* seeds, int64_t* covered) {
    if (k < 0 || k > n) return -1;
    int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    uint8_t* chosen = (uint8_t*)calloc((size_t)n, 1);
    uint8_t* done = (uint8_t*)calloc((size_t)(nsets > 0 ? nsets : 1), 1);
    for (int64_t i = off[0]; i < off[nsets]; ++i) cnt[ids[i]]++;
    int64_t ncov = 0;
    for (int32_t round = 0; round < k; ++round) {
        int32_t best = -1;
        for (int32_t v = 0; v < n; ++v) {
            if (chosen[v]) continue;
            if (best < 0 || cnt[v] > cnt[best]) best = v;
        }
        chosen[best] = 1;
        seeds[round] = best;
        for (int64_t r = 0; r < nsets; ++r) {
            if (done[r]) continue;
            int hit = 0;
            for (int64_t i = off[r]; i < off[r + 1]; ++i)
                if (ids[i] == best) { hit = 1; break; }
            if (!hit) continue;
            done[r] = 1;
            ++ncov;
            for (int64_t i = off[r]; i < off[r + 1]; ++i) cnt[ids[i]]--;
        }
    }
    free(cnt); free(chosen); free(done);
    if (covered) *covered = ncov;
    return 0;
}

int orc_pool_greedy(const orc_pool* p, int64_t first, int64_t count, int32_t k,
                    int32_t* seeds, int64_t* covered) {
    if (first < 0 || count < 0 || first + count > p->count) return -1;
    return orc_greedy_sets(p->n, count, p->off + first, p->ids, k, seeds, covered);
}

/* ------------------------------------------------------------------------------------
 * IMM sample sizes (Tang et al. 2015; the paper defers f(n, eps, k) of Alg. 2 and the
 * final theta = lambda* / LB to that work).  Natural logarithms throughout except log2 n
 * in the loop bound and in ln(log2 n).  ln C(n,k) is the ascending sum of
 * ln(n-i) - ln(i+1), so that it is reproducible without lgamma.
 * ---------------------------------------------------------------------------------- */
static double ln_of(double x) {
    volatile double v = x;      /* keep every logarithm a run-time libm call */
    return log(v);
}

static const double ORC_E = 2.718281828459045;

double orc_log_binom(int64_t n, int64_t k) {
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += ln_of((double)(n - i)) - ln_of((double)(i + 1));
    return s;
}

double orc_ell_adjusted(int64_t n, double ell) {
    return ell * (1.0 + ln_of(2.0) / ln_of((double)n));
}

double orc_lambda_prime(int64_t n, int64_t k, double eps, double ell_adj) {
    double ep = sqrt(2.0) * eps;
    double lnC = orc_log_binom(n, k);
    volatile double l2 = log2((double)n);
    return (2.0 + 2.0 / 3.0 * ep) * (lnC + ell_adj * ln_of((double)n) + ln_of(l2)) *
           (double)n / (ep * ep);
}

double orc_lambda_star(int64_t n, int64_t k, double eps, double ell_adj) {
    double lnC = orc_log_binom(n, k);
    double a = sqrt(ell_adj * ln_of((double)n) + ln_of(2.0));
    double b = sqrt((1.0 - 1.0 / ORC_E) * (lnC + ell_adj * ln_of((double)n) + ln_of(2.0)));
    return 2.0 * (double)n * ((1.0 - 1.0 / ORC_E) * a + b) * ((1.0 - 1.0 / ORC_E) * a + b) /
           (eps * eps);
}

/* Loop bound of Alg. 2, log2(n) - 1, read as floor(log2 n) - 1. */
int32_t orc_imax(int64_t n) {
    int32_t bits = 0;
    while (((int64_t)1 << bits) <= n) ++bits;   /* bit length of n */
    return bits - 2;
}

/* Alg. 2 (LB estimation) followed by Alg. 1 (sample theta = lambda* / LB sets, then greedy).
 * Sets generated during estimation are reused for the final sample unless fresh_final is
 * set, in which case the final sets are indices [|R_est|, |R_est| + theta). */
int orc_imm_solve(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                  const float* ic_p, const uint32_t* lt_w, int model, uint64_t seed,
                  int32_t k, double eps, double ell, int fresh_final, int nthreads,
                  int32_t* seeds, int64_t* info_i, double* info_d) {
    if (n < 2 || m < 0 || k < 1 || k > n || !(eps > 0.0 && eps < 1.0) || !(ell > 0.0))
        return -1;
    uint32_t* thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    int rc = (model == 0) ? (ic_p ? orc_encode_ic(m, ic_p, thr) : -1)
                          : orc_encode_lt(n, in_off, lt_w, thr);
    if (rc != 0) { free(thr); return -2; }
    orc_pool* pool = orc_pool_new(n, m, in_off, in_src, thr, model, seed);

    double L = orc_ell_adjusted(n, ell);
    double ep = sqrt(2.0) * eps;
    double lamP = orc_lambda_prime(n, k, eps, L);
    double lamS = orc_lambda_star(n, k, eps, L);
    int32_t imax = orc_imax(n);
    double LB = 1.0;
    int64_t cov = 0, phases = 0;
    for (int32_t i = 1; i <= imax; ++i) {
        double x = (double)n / (double)((int64_t)1 << i);
        int64_t th = (int64_t)ceil(lamP / x);
        if (orc_pool_extend(pool, th > pool->count ? th : pool->count, nthreads) != 0) {
            rc = -3; goto out;
        }
        int64_t R = pool->count;
        orc_pool_greedy(pool, 0, R, k, seeds, &cov);
        ++phases;
        if ((double)n * (double)cov / (double)R >= (1.0 + ep) * x) {
            LB = (double)n * (double)cov / (double)R / (1.0 + ep);
            break;
        }
    }
    {
        int64_t theta = (int64_t)ceil(lamS / LB);
        int64_t first = fresh_final ? pool->count : 0;
        int64_t upto = fresh_final ? pool->count + theta
                                   : (theta > pool->count ? theta : pool->count);
        if (orc_pool_extend(pool, upto, nthreads) != 0) { rc = -3; goto out; }
        int64_t R = upto - first;
        orc_pool_greedy(pool, first, R, k, seeds, &cov);
        ++phases;
        info_i[0] = theta;
        info_i[1] = pool->count;
        info_i[2] = cov;
        info_i[3] = phases;
        info_i[4] = orc_pool_edges(pool, 0, pool->count);
        info_i[5] = orc_pool_total(pool, 0, pool->count);
        info_d[0] = LB;
        info_d[1] = (double)n * (double)cov / (double)R;
        info_d[2] = lamP;
        info_d[3] = lamS;
    }
out:
    orc_pool_free(pool);
    free(thr);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Multi-round influence maximisation (gIM Sec. IV-H, Table 3: the CR-NAIMM algorithm of
 * Sun et al., KDD'18).  Influence spreads in T rounds, each an independent diffusion from
 * that round's seed set S_t (|S_t| <= k); the objective is the expected number of nodes
 * activated in at least one round.  A random multi-round RR set draws one root and runs
 * one reverse search per round t from it, in round t's own live-edge instance; its
 * elements are (node, round) pairs, stored as t * n + u.  A seed collection S (elements
 * (u, t) with at most k per round) covers the set when it shares an element with it, and
 * n times the covered fraction estimates the objective, as Eq. 3 does for one round.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t n, rounds;
    const int64_t* in_off;
    const int32_t* in_src;
    const uint32_t* thr;
    int model;
    uint64_t seed;
    int64_t count;
    int64_t* off;       /* count + 1 */
    int32_t* ids;       /* elements t * n + u, sorted per set */
    int64_t cap_sets, cap_ids, edges;
} orc_mr_pool;

/* Sets [count, upto) of a multi-round pool: set r is the union over t of
 * {t * n + u : u in RR_t(r)}. */
static int mr_extend(orc_mr_pool* p, int64_t upto) {
    if (upto <= p->count) return 0;
    if (upto > 0xFFFFFFFFll) return -1;
    if (upto > p->cap_sets) {
        while (p->cap_sets < upto) p->cap_sets *= 2;
        p->off = (int64_t*)realloc(p->off, (size_t)(p->cap_sets + 1) * sizeof(int64_t));
    }
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)p->n);
    uint8_t* mark = (uint8_t*)calloc((size_t)p->n, 1);
    for (int64_t r = p->count; r < upto; ++r) {
        int64_t at = p->off[r];
        for (int32_t t = 0; t < p->rounds; ++t) {
            int64_t ex = 0, sz;
            if (p->model == 0)
                sz = orc_rr_ic_round(p->n, p->in_off, p->in_src, p->thr, p->seed, (uint32_t)r,
                                     (uint32_t)t, out, mark, &ex);
            else
                sz = orc_rr_lt_round(p->n, p->in_off, p->in_src, p->thr, p->seed, (uint32_t)r,
                                     (uint32_t)t, out, mark, &ex);
            p->edges += ex;
            qsort(out, (size_t)sz, sizeof(int32_t), cmp_i32);
            if (at + sz > p->cap_ids) {
                while (p->cap_ids < at + sz) p->cap_ids *= 2;
                p->ids = (int32_t*)realloc(p->ids, (size_t)p->cap_ids * sizeof(int32_t));
            }
            for (int64_t i = 0; i < sz; ++i) p->ids[at + i] = t * p->n + out[i];
            at += sz;
        }
        p->off[r + 1] = at;
        p->count = r + 1;
    }
    free(out);
    free(mark);
    return 0;
}

/* Greedy over a partition matroid (CR-Greedy of Sun et al.): the ground set is
 * n_elem = parts * part_size elements, element e belonging to part e / part_size, and at
 * most k elements may be taken per part.  Each of the parts * k steps takes, among the
 * elements not yet taken whose part still has room, one contained in the most uncovered
 * sets (the smallest element among equals), then removes the sets it covers.  With one
 * part this is orc_greedy_sets. */
int orc_greedy_partition(int32_t part_size, int32_t parts, int64_t nsets, const int64_t* off,
                         const int32_t* ids, int32_t k, int32_t* seeds, int64_t* covered) {
    if (part_size < 1 || parts < 1 || k < 1 || k > part_size) return -1;
    const int64_t n_elem = (int64_t)part_size * parts;
    int64_t* cnt = (int64_t*)calloc((size_t)n_elem, sizeof(int64_t));
    uint8_t* chosen = (uint8_t*)calloc((size_t)n_elem, 1);
    int32_t* taken = (int32_t*)calloc((size_t)parts, sizeof(int32_t));
    uint8_t* done = (uint8_t*)calloc((size_t)(nsets > 0 ? nsets : 1), 1);
    for (int64_t i = off[0]; i < off[nsets]; ++i) cnt[ids[i]]++;
    int64_t ncov = 0;
    for (int32_t step = 0; step < parts * k; ++step) {
        int64_t best = -1;
        for (int64_t e = 0; e < n_elem; ++e) {
            if (chosen[e] || taken[e / part_size] >= k) continue;
            if (best < 0 || cnt[e] > cnt[best]) best = e;
        }
        chosen[best] = 1;
        taken[best / part_size]++;
        seeds[step] = (int32_t)best;
        for (int64_t r = 0; r < nsets; ++r) {
            if (done[r]) continue;
            int hit = 0;
            for (int64_t i = off[r]; i < off[r + 1]; ++i)
                if (ids[i] == best) { hit = 1; break; }
            if (!hit) continue;
            done[r] = 1;
            ++ncov;
            for (int64_t i = off[r]; i < off[r + 1]; ++i) cnt[ids[i]]--;
        }
    }
    free(cnt); free(chosen); free(taken); free(done);
    if (covered) *covered = ncov;
    return 0;
}

/* Sample sizes of the multi-round problem, read from IMM's (Tang et al.) with the two
 * quantities its proofs take from the problem: the union bound runs over the
 * C(n,k)^T feasible seed collections (ln C(n,k) becomes T ln C(n,k)), and the greedy's
 * approximation ratio is 1 - 1/e for one round but 1/2 for a partition matroid of T >= 2
 * parts.  With T = 1 both are IMM's own. */
double orc_mr_ratio(int32_t rounds) { return rounds == 1 ? 1.0 - 1.0 / ORC_E : 0.5; }

double orc_mr_lambda_prime(int64_t n, int64_t k, int32_t rounds, double eps, double ell_adj) {
    double ep = sqrt(2.0) * eps;
    double lnC = (double)rounds * orc_log_binom(n, k);
    volatile double l2 = log2((double)n);
    return (2.0 + 2.0 / 3.0 * ep) * (lnC + ell_adj * ln_of((double)n) + ln_of(l2)) *
           (double)n / (ep * ep);
}

double orc_mr_lambda_star(int64_t n, int64_t k, int32_t rounds, double eps, double ell_adj) {
    double g = orc_mr_ratio(rounds);
    double lnC = (double)rounds * orc_log_binom(n, k);
    double a = sqrt(ell_adj * ln_of((double)n) + ln_of(2.0));
    double b = sqrt(g * (lnC + ell_adj * ln_of((double)n) + ln_of(2.0)));
    return 2.0 * (double)n * (g * a + b) * (g * a + b) / (eps * eps);
}

/* CR-NAIMM: IMM's estimation loop (gIM Alg. 2) and final sample (Alg. 1) over multi-round
 * RR sets, with the partition-matroid greedy.  seeds: int32[rounds * k], elements
 * t * n + u in selection order.  info_i / info_d as orc_imm_solve. */
int orc_mrim_solve(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                   const float* ic_p, const uint32_t* lt_w, int model, uint64_t seed,
                   int32_t k, int32_t rounds, double eps, double ell,
                   int32_t* seeds, int64_t* info_i, double* info_d) {
    if (n < 2 || m < 0 || k < 1 || k > n || rounds < 1 || rounds > 32 ||
        (int64_t)n * rounds > 0x7FFFFFFFll || !(eps > 0.0 && eps < 1.0) || !(ell > 0.0))
        return -1;
    uint32_t* thr = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    int rc = (model == 0) ? (ic_p ? orc_encode_ic(m, ic_p, thr) : -1)
                          : orc_encode_lt(n, in_off, lt_w, thr);
    if (rc != 0) { free(thr); return -2; }
    orc_mr_pool P = {n, rounds, in_off, in_src, thr, model, seed, 0, NULL, NULL, 1024, 1 << 16, 0};
    P.off = (int64_t*)calloc((size_t)P.cap_sets + 1, sizeof(int64_t));
    P.ids = (int32_t*)malloc((size_t)P.cap_ids * sizeof(int32_t));

    double L = orc_ell_adjusted(n, ell);
    double ep = sqrt(2.0) * eps;
    double lamP = orc_mr_lambda_prime(n, k, rounds, eps, L);
    double lamS = orc_mr_lambda_star(n, k, rounds, eps, L);
    int32_t imax = orc_imax(n);
    double LB = 1.0;
    int64_t cov = 0, phases = 0;
    for (int32_t i = 1; i <= imax; ++i) {
        double x = (double)n / (double)((int64_t)1 << i);
        int64_t th = (int64_t)ceil(lamP / x);
        if (mr_extend(&P, th > P.count ? th : P.count) != 0) { rc = -3; goto out; }
        orc_greedy_partition(n, rounds, P.count, P.off, P.ids, k, seeds, &cov);
        ++phases;
        if ((double)n * (double)cov / (double)P.count >= (1.0 + ep) * x) {
            LB = (double)n * (double)cov / (double)P.count / (1.0 + ep);
            break;
        }
    }
    {
        int64_t theta = (int64_t)ceil(lamS / LB);
        int64_t upto = theta > P.count ? theta : P.count;
        if (mr_extend(&P, upto) != 0) { rc = -3; goto out; }
        orc_greedy_partition(n, rounds, upto, P.off, P.ids, k, seeds, &cov);
        ++phases;
        info_i[0] = theta;
        info_i[1] = P.count;
        info_i[2] = cov;
        info_i[3] = phases;
        info_i[4] = P.edges;
        info_i[5] = P.off[P.count];
        info_d[0] = LB;
        info_d[1] = (double)n * (double)cov / (double)upto;
        info_d[2] = lamP;
        info_d[3] = lamS;
    }
out:
    free(P.off);
    free(P.ids);
    free(thr);
    return rc;
}

/* Multi-round RR sets [0, count) of (graph, model, seed, rounds), for tests: off[count+1]
 * and ids (elements t * n + u, sorted per set); ids == NULL returns the member total in
 * *total only. */
int orc_mr_sets(int32_t n, const int64_t* in_off, const int32_t* in_src, const uint32_t* thr,
                int model, uint64_t seed, int32_t rounds, int64_t count, int64_t* off,
                int32_t* ids, int64_t* total, int64_t* edges) {
    if (n < 1 || rounds < 1 || count < 0) return -1;
    orc_mr_pool P = {n, rounds, in_off, in_src, thr, model, seed, 0, NULL, NULL, 1024, 1 << 16, 0};
    P.off = (int64_t*)calloc((size_t)P.cap_sets + 1, sizeof(int64_t));
    P.ids = (int32_t*)malloc((size_t)P.cap_ids * sizeof(int32_t));
    int rc = mr_extend(&P, count);
    if (rc == 0) {
        if (total) *total = P.off[count];
        if (edges) *edges = P.edges;
        if (off) memcpy(off, P.off, sizeof(int64_t) * (size_t)(count + 1));
        if (ids) memcpy(ids, P.ids, sizeof(int32_t) * (size_t)P.off[count]);
    }
    free(P.off);
    free(P.ids);
    return rc;
}

/* ------------------------------------------------------------------------------------
 * Forward Monte-Carlo influence spread (gIM Sec. II-C, the estimator of Kempe et al.):
 * simulation j draws an instance graph (IC: each edge kept with its probability; LT: each
 * vertex keeps at most one in-edge, edge e with its normalised weight) and counts the
 * vertices reachable from the seeds in it; E[I(S)] is the mean over simulations.  For
 * seeds of several rounds (Sec. IV-H) round t draws its own instance and the count is of
 * the vertices reached in at least one round.
 *
 * Draws (a contract of their own, independent of the RR sets' draws):
 *   IC edge e in simulation j, round t: word 0 of Philox(j, e, t, FWD_IC = 4); the edge
 *     is kept iff the word < thr[e] or thr[e] is ORC_ALWAYS (the IC encoding above);
 *   LT vertex v in simulation j, round t: word 0 of Philox(j, v, t, FWD_LT = 5); v keeps
 *     the first in-edge e whose cumulative threshold cum[e] exceeds the word (or is
 *     ORC_ALWAYS), none if there is no such edge (the LT encoding above).
 * The reachable set is found by a plain breadth-first search over out-edges, built here
 * from the in-edge lists.
 * ---------------------------------------------------------------------------------- */
#define ORC_DOMAIN_FWD_IC 4u
#define ORC_DOMAIN_FWD_LT 5u

/* LT: the in-edge vertex v keeps in instance (j, t), or -1. */
static int64_t fwd_lt_pick(const int64_t* in_off, const uint32_t* cum, uint64_t seed, uint32_t j,
                           uint32_t t, int32_t v) {
    uint32_t x = draw_word(seed, j, (uint32_t)v, t, ORC_DOMAIN_FWD_LT, 0);
    for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e)
        if (cum[e] == ORC_ALWAYS || x < cum[e]) return e;
    return -1;
}

int orc_spread_mc(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* thr_or_cum, int model, uint64_t seed, int32_t rounds,
                  const int32_t* elems, int32_t nelem, int64_t sims, int nthreads,
                  int64_t* per_sim, int64_t* total) {
    if (n < 1 || m < 0 || rounds < 1 || nelem < 0 || sims < 0 || sims > 0xFFFFFFFFll ||
        m > 0xFFFFFFFFll || (int64_t)n * rounds > 0x7FFFFFFFll)
        return -1;
    for (int32_t i = 0; i < nelem; ++i)
        if (elems[i] < 0 || (int64_t)elems[i] >= (int64_t)n * rounds) return -1;
    /* out-edge lists: out_off by counting sources, then each in-edge (u -> v, e) placed */
    int64_t* out_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* out_dst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t* out_eid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) out_off[in_src[e] + 1]++;
    for (int32_t u = 0; u < n; ++u) out_off[u + 1] += out_off[u];
    for (int32_t v = 0; v < n; ++v)
        for (int64_t e = in_off[v]; e < in_off[v + 1]; ++e) {
            int32_t u = in_src[e];
            int64_t at = out_off[u] + fill[u]++;
            out_dst[at] = v;
            out_eid[at] = e;
        }
    free(fill);
    int64_t sum = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(+ : sum)
    {
        uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);     /* this round's search */
        uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);     /* any round of this simulation */
        int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
        int32_t* reached = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 16)
        for (int64_t js = 0; js < sims; ++js) {
            const uint32_t j = (uint32_t)js;
            int64_t count = 0;
            for (int32_t t = 0; t < rounds; ++t) {
                int64_t size = 0, head = 0;
                for (int32_t i = 0; i < nelem; ++i) {
                    if (elems[i] / n != t) continue;
                    int32_t s = elems[i] % n;
                    if (!mark[s]) {
                        mark[s] = 1;
                        queue[size++] = s;
                    }
                }
                while (head < size) {
                    int32_t u = queue[head++];
                    for (int64_t a = out_off[u]; a < out_off[u + 1]; ++a) {
                        int32_t v = out_dst[a];
                        if (mark[v]) continue;
                        int64_t e = out_eid[a];
                        int live;
                        if (model == 0) {
                            uint32_t x = draw_word(seed, j, (uint32_t)e, (uint32_t)t, ORC_DOMAIN_FWD_IC, 0);
                            live = thr_or_cum[e] == ORC_ALWAYS || x < thr_or_cum[e];
                        } else {
                            live = fwd_lt_pick(in_off, thr_or_cum, seed, j, (uint32_t)t, v) == e;
                        }
                        if (live) {
                            mark[v] = 1;
                            queue[size++] = v;
                        }
                    }
                }
                for (int64_t i = 0; i < size; ++i) {
                    int32_t v = queue[i];
                    mark[v] = 0;
                    if (!seen[v]) {
                        seen[v] = 1;
                        reached[count++] = v;
                    }
                }
            }
            for (int64_t i = 0; i < count; ++i) seen[reached[i]] = 0;
            if (per_sim) per_sim[js] = count;
            sum += count;
        }
        free(mark);
        free(seen);
        free(queue);
        free(reached);
    }
    free(out_off);
    free(out_dst);
    free(out_eid);
    if (total) *total = sum;
    return 0;
}
