/* CPU oracle for the IMM hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct C implementation of what the GPU path computes, used
 * only by the test suite, the smoke check and the CPU-baseline leg of the benchmark.  It
 * shares no code with the GPU library: it has its own Philox generator, its own threshold
 * encoders, its own reverse BFS / reverse walk, its own greedy max-cover and its own IMM
 * driver.  The product path never calls into it.
 *
 * Paper: Shahrouz, Salehkaleybar, Hashemi, "gIM: GPU Accelerated RIS-based Influence
 * Maximization Algorithm", IEEE TPDS (arXiv 2009.07325).  IMM sample-size formulas:
 * Tang, Shi, Xiao, SIGMOD 2015.  Philox4x32-10: Salmon, Moraes, Dror, Shaw, SC'11.
 *
 * Random-number contract (shared by definition, not by code, with the GPU library):
 *   key     = (seed mod 2^32, seed >> 32)
 *   counter = (r, g, t, domain), domain ROOT=1, IC=2, LT=3, t = the round (0 for plain
 *             IMM; 0 .. T-1 for the T rounds of a multi-round set)
 *   root of RR set r : w0 of Philox(r, 0, 0, ROOT), root = (w0 * n) >> 32
 *   IC edge e of set r: word (e & 3) of Philox(r, e >> 2, t, IC)
 *   LT vertex v of set r: w0 of Philox(r, v, t, LT)
 *
 * Every function returns 0 on success and a negative value on invalid input.
 */
#ifndef IMM_ORACLE_H
#define IMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_DOMAIN_ROOT 1u
#define ORC_DOMAIN_IC 2u
#define ORC_DOMAIN_LT 3u
#define ORC_ALWAYS 0xFFFFFFFFu

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* IC threshold of a float32 probability: floor(p * 2^32), saturating to ORC_ALWAYS at
 * p = 1.  Edge live iff draw < t or t == ORC_ALWAYS. */
uint32_t orc_ic_threshold(float p);
int orc_encode_ic(int64_t m, const float* p, uint32_t* thr);

/* LT cumulative thresholds per in-list: cum_j = floor(S_j * 2^32 / T) with S_j the
 * prefix sum of raw integer weights and T their total; the last entry is ORC_ALWAYS.
 * w == NULL means unit weights (weighted-cascade LT). */
int orc_encode_lt(int32_t n, const int64_t* in_off, const uint32_t* w, uint32_t* cum);

int32_t orc_root(uint64_t seed, uint32_t r, int32_t n);

/* One RR set.  out (capacity n) receives the members in discovery order, mark (n bytes,
 * all zero) is restored to zero on return.  Returns the set size; *edges receives the
 * number of in-edges examined (sum of in-degrees of the members). */
int64_t orc_rr_ic(int32_t n, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* thr, uint64_t seed, uint32_t r, int32_t* out,
                  uint8_t* mark, int64_t* edges);
int64_t orc_rr_lt(int32_t n, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* cum, uint64_t seed, uint32_t r, int32_t* out,
                  uint8_t* mark, int64_t* edges);

/* The same with the round word t of the counter (multi-round IM, gIM Sec. IV-H): the
 * live-edge instance of round t of set r; t = 0 is the plain set. */
int64_t orc_rr_ic_round(int32_t n, const int64_t* in_off, const int32_t* in_src,
                        const uint32_t* thr, uint64_t seed, uint32_t r, uint32_t t,
                        int32_t* out, uint8_t* mark, int64_t* edges);
int64_t orc_rr_lt_round(int32_t n, const int64_t* in_off, const int32_t* in_src,
                        const uint32_t* cum, uint64_t seed, uint32_t r, uint32_t t,
                        int32_t* out, uint8_t* mark, int64_t* edges);

/* A growable collection of RR sets with indices [0, count), each stored sorted. */
typedef struct orc_pool orc_pool;
orc_pool* orc_pool_new(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                       const uint32_t* thr_or_cum, int model /*0 IC, 1 LT*/, uint64_t seed);
void orc_pool_free(orc_pool* p);
int orc_pool_extend(orc_pool* p, int64_t upto, int nthreads);
int64_t orc_pool_count(const orc_pool* p);
int64_t orc_pool_total(const orc_pool* p, int64_t first, int64_t count);
int64_t orc_pool_edges(const orc_pool* p, int64_t first, int64_t count);
int orc_pool_export(const orc_pool* p, int64_t first, int64_t count, int64_t* off,
                    int32_t* ids);
int orc_pool_hist(const orc_pool* p, int64_t first, int64_t count, uint32_t* hist);

/* Greedy max coverage over explicit sets (offsets off[0..nsets], ids), k rounds. */
int orc_greedy_sets(int32_t n, int64_t nsets, const int64_t* off, const int32_t* ids,
                    int32_t k, int32_t* seeds, int64_t* covered);
int orc_pool_greedy(const orc_pool* p, int64_t first, int64_t count, int32_t k,
                    int32_t* seeds, int64_t* covered);

/* IMM sample-size quantities (Tang et al. 2015), all in IEEE double. */
double orc_log_binom(int64_t n, int64_t k);
double orc_lambda_prime(int64_t n, int64_t k, double eps, double ell_adj);
double orc_lambda_star(int64_t n, int64_t k, double eps, double ell_adj);
double orc_ell_adjusted(int64_t n, double ell);
int32_t orc_imax(int64_t n);

/* Full IMM solve.  info_i: [theta, num_rr, covered, phases, edges_examined, pool_ids]
 * info_d: [lb, spread_est, lambda_prime, lambda_star]. */
int orc_imm_solve(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                  const float* ic_p, const uint32_t* lt_w, int model, uint64_t seed,
                  int32_t k, double eps, double ell, int fresh_final, int nthreads,
                  int32_t* seeds, int64_t* info_i, double* info_d);

/* Multi-round IM (gIM Sec. IV-H; CR-NAIMM of Sun et al., KDD'18).  Elements of a
 * multi-round RR set are (u, t) pairs stored as t * n + u. */
int orc_mr_sets(int32_t n, const int64_t* in_off, const int32_t* in_src, const uint32_t* thr,
                int model, uint64_t seed, int32_t rounds, int64_t count, int64_t* off,
                int32_t* ids, int64_t* total, int64_t* edges);
/* Greedy under a partition matroid: parts of part_size elements, at most k per part. */
int orc_greedy_partition(int32_t part_size, int32_t parts, int64_t nsets, const int64_t* off,
                         const int32_t* ids, int32_t k, int32_t* seeds, int64_t* covered);
double orc_mr_ratio(int32_t rounds);
double orc_mr_lambda_prime(int64_t n, int64_t k, int32_t rounds, double eps, double ell_adj);
double orc_mr_lambda_star(int64_t n, int64_t k, int32_t rounds, double eps, double ell_adj);
/* seeds: int32[rounds * k]; info_i / info_d as orc_imm_solve. */
int orc_mrim_solve(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                   const float* ic_p, const uint32_t* lt_w, int model, uint64_t seed,
                   int32_t k, int32_t rounds, double eps, double ell,
                   int32_t* seeds, int64_t* info_i, double* info_d);

/* Forward Monte-Carlo influence spread (gIM Sec. II-C): over simulations j in [0, sims),
 * the number of vertices reached from the seed elements (t * n + u: vertex u seeds round
 * t) in at least one round's instance graph.  IC edge e kept iff word 0 of Philox(j, e, t,
 * 4) < thr[e] (or thr[e] saturated); LT vertex v keeps the first in-edge e with word 0 of
 * Philox(j, v, t, 5) < cum[e] (or cum[e] saturated).  per_sim (sims entries, or NULL)
 * receives each simulation's count, *total their sum. */
int orc_spread_mc(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                  const uint32_t* thr_or_cum, int model, uint64_t seed, int32_t rounds,
                  const int32_t* elems, int32_t nelem, int64_t sims, int nthreads,
                  int64_t* per_sim, int64_t* total);

#ifdef __cplusplus
}
#endif
#endif
