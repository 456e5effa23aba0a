/* imm.h -- C ABI of libimm: IMM influence maximisation on AMD Instinct MI355X (gfx950).
 *
 * The library generates random reverse-reachable (RR) sets on the GPU, keeps them
 * resident in HBM, selects seeds by greedy maximum coverage on the GPU, and drives IMM's
 * lower-bound / sample-size loop from the host.
 *
 * Method: S. Shahrouz, S. Salehkaleybar, M. Hashemi, "gIM: GPU Accelerated RIS-based
 * Influence Maximization Algorithm" (IEEE TPDS; arXiv 2009.07325).  Passages are cited as
 * "gIM Sec./Alg./Eq.".  Sample sizes follow IMM (Tang, Shi, Xiao, SIGMOD 2015), which gIM
 * Alg. 2 defers to.
 *
 * Conventions
 *  - Every function returns an imm_status; nothing is thrown across the ABI.  After a
 *    non-OK status, imm_last_error() returns a thread-local description.
 *  - Input arrays may be host or device pointers (the library copies them with
 *    hipMemcpyDefault).  Output arrays named *_out are HOST pointers, owned by the caller.
 *  - Graphs and pools are opaque, device-resident and owned by the library; each create
 *    is paired with its destroy.  Calls on one object are not thread-safe; calls on
 *    distinct objects are.
 *  - `stream` arguments are hipStream_t values (NULL = the default stream).  Functions
 *    that return host results synchronise that stream before returning.
 *
 * Random-number contract (what makes results reproducible bit for bit): Philox4x32-10
 * (Salmon et al., SC'11) with key (seed mod 2^32, seed >> 32) and counter
 * (r, g, t, domain), t the round (0 except in multi-round sets, below):
 *    root of RR set r     : word 0 of counter (r, 0, 0, 1); root = (word * n) >> 32
 *    IC test of in-edge e : word (e & 3) of counter (r, e >> 2, t, 2)
 *    LT draw at vertex v  : word 0 of counter (r, v, t, 3)
 * so RR set r is a pure function of (graph, model, seed, r), whatever the launch shape.
 */
#ifndef IMM_H
#define IMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IMM_OK = 0,
    IMM_EINVAL = 1,      /* an argument is out of range or inconsistent */
    IMM_ENOMEM = 2,      /* device or host allocation failed */
    IMM_ECAPACITY = 3,   /* a count exceeds what the format holds (e.g. RR index >= 2^32) */
    IMM_EDEVICE = 4,     /* a HIP runtime call failed */
    IMM_ENOTIMPL = 5,    /* the requested feature is not built */
    IMM_EBUSY = 6,
    IMM_ECANCELLED = 7
} imm_status;

/* Diffusion models, gIM Sec. II-B: independent cascade and linear threshold. */
typedef enum { IMM_IC = 0, IMM_LT = 1 } imm_model;

typedef struct imm_graph imm_graph;
typedef struct imm_pool imm_pool;

/* imm_graph_create flag: also build the LT encoding (lt_w may then be NULL, meaning unit
 * raw weights, i.e. weighted-cascade LT with p(u,v) = 1/indeg(v)). */
#define IMM_GRAPH_LT 0x1u

typedef struct {
    uint64_t seed;          /* Philox key of the RR pool */
    int32_t fresh_final;    /* 0: the final sample reuses the estimation sets (IMM);
                               1: the final theta sets are fresh indices after them */
    int32_t reserved;
    void* stream;           /* hipStream_t or NULL */
} imm_options;

typedef struct {
    int64_t theta;          /* ceil(lambda* / LB) */
    int64_t num_rr;         /* RR sets generated (pool size after the solve) */
    int64_t covered;        /* sets covered by the returned seeds, in the final sample */
    int64_t edges_examined; /* in-edges examined while generating, sum of member indegrees
                               (imm_solve_pool: the pool's running total) */
    int64_t pool_ids;       /* total members over all generated sets (same convention) */
    int32_t phases;         /* greedy selections run (estimation phases + final) */
    int32_t heavy_redrawn;  /* IC sets of this solve's launches that outgrew a bounded heavy
                               member list and were drawn again in a full one (huge graphs) */
    double lb;              /* lower bound LB of OPT from gIM Alg. 2 (1.0 if no phase passes) */
    double spread_est;      /* n * covered / |final sample|, the estimate of gIM Eq. 3 */
    double lambda_prime;
    double lambda_star;
    double t_generate_s;    /* wall time in RR generation (device-synchronised) */
    double t_select_s;      /* wall time in seed selection */
    double t_total_s;
    double t_rr_kernel_s;   /* summed duration of the light RR-generation launches (IC: one
                               wave per set; LT: the walk kernel), HIP events on the stream */
    int64_t rr_kernel_launches;
    double t_rr_heavy_s;    /* same for the heavy launches (IC: one workgroup per set with
                               hub-heavy work; LT: walks too long for the on-chip list) */
    int64_t rr_heavy_launches;
    int64_t edges_heavy;    /* part of edges_examined in sets finished by the heavy launches */
} imm_info;

/* Selects the HIP device used by subsequent calls from this thread. */
imm_status imm_init(int32_t device);

/* Thread-local message for the last non-OK status ("" if none). */
const char* imm_last_error(void);

/* Device memory that objects release is kept by the library for reuse (at most 64 GiB per
 * device; it is also given back automatically when an allocation fails), and so are small
 * pinned host buffers (up to 1 MiB each: read-back of counters, coverage and seeds).  This
 * returns all of both to the HIP runtime.  Thread-safe. */
imm_status imm_release_cached_memory(void);

/* Upload a directed graph G = (V, E), gIM Sec. II-A, as the CSR of its transpose
 * (in-edges), and encode edge probabilities into 32-bit thresholds on the device.
 *   n        vertices, n >= 2
 *   m        edges, m >= 0
 *   in_off   int64[n+1], in_off[0] = 0, non-decreasing, in_off[n] = m
 *   in_src   int32[m], in_src[e] in [0, n): source u of in-edge e = (u, v) of vertex v
 *   ic_p     float32[m] IC probabilities p_uv in [0, 1], or NULL (no IC support);
 *            edge e is live when its draw x < floor(p * 2^32) (p = 1: always), the
 *            comparison "p < p_uv" of gIM Alg. 3
 *   lt_w     uint32[m] raw LT weights >= 1, normalised per vertex to sum 1 (gIM Sec.
 *            II-B, Eq. 1), or NULL for unit weights; used only with IMM_GRAPH_LT
 *   flags    IMM_GRAPH_LT or 0
 * Arrays may be host or device memory; they are copied and may be freed after return.
 * Errors: IMM_EINVAL for malformed arrays (checked on the device), IMM_ENOMEM. */
imm_status imm_graph_create(int32_t n, int64_t m, const int64_t* in_off, const int32_t* in_src,
                            const float* ic_p, const uint32_t* lt_w, uint32_t flags,
                            imm_graph** out);
imm_status imm_graph_destroy(imm_graph* g);
imm_status imm_graph_info(const imm_graph* g, int32_t* n, int64_t* m, int32_t* has_ic,
                          int32_t* has_lt);

/* Copy the device-side encodings back (for verification): thr uint32[m] (IC thresholds,
 * NULL to skip) and cum uint32[m] (LT cumulative thresholds, NULL to skip). */
imm_status imm_graph_export_encoding(const imm_graph* g, uint32_t* thr_out, uint32_t* cum_out);

/* An RR pool: the RR sets of (graph, model, seed) with indices [0, size), kept in HBM
 * (gIM Alg. 6 keeps all sets in one array RR with offsets).  Errors: IMM_EINVAL when the
 * graph lacks the model's encoding. */
imm_status imm_pool_create(const imm_graph* g, imm_model model, uint64_t seed, imm_pool** out);
imm_status imm_pool_destroy(imm_pool* p);
/* Number of sets, total members, and total in-edges examined so far. */
imm_status imm_pool_size(const imm_pool* p, int64_t* num_sets, int64_t* num_ids,
                         int64_t* edges_examined);

/* Ensure RR sets [0, upto) exist, generating only the missing indices (gIM Alg. 3-6 for
 * IC; Sec. III-G for LT).  Set r is every vertex that reaches its random root in the
 * live-edge instance drawn for r (gIM Sec. II-E), whatever order it was generated in.
 * Also maintains the pool's occurrence counts (Occur, gIM Sec. III-B).
 * Errors: IMM_ECAPACITY if upto >= 2^32; IMM_ENOMEM. */
imm_status imm_generate_rr(imm_pool* p, int64_t upto, void* stream);

/* Canonical export of sets [first, first+count) (each the random RR set of gIM Sec. II-C:
 * the vertices that reach the set's root in its live-edge instance): off_out
 * int64[count+1] (off_out[0] = 0) and ids_out int32[ids_cap] with each set's members sorted
 * ascending.  If ids_cap is too
 * small (or ids_out is NULL) only off_out and *ids_needed are written and IMM_ECAPACITY is
 * returned (ids_out == NULL returns IMM_OK). */
imm_status imm_rr_export(const imm_pool* p, int64_t first, int64_t count, int64_t* off_out,
                         int32_t* ids_out, int64_t ids_cap, int64_t* ids_needed);

/* Occurrence counts over sets [first, first+count): hist_out uint32[n], hist_out[v] =
 * number of those sets containing v (gIM Sec. III-B "Occur"). */
imm_status imm_rr_histogram(const imm_pool* p, int64_t first, int64_t count,
                            uint32_t* hist_out);

/* Greedy maximum coverage over sets [first, first+count), gIM Alg. 1 lines 6-10 with the
 * max reduction of Sec. III-H and the cover/decrement of Alg. 7: k rounds, each taking the
 * vertex outside S contained in the most uncovered sets (smallest id among ties) and
 * removing the sets it covers.  seeds_out int32[k] in selection order; *covered_out = sets
 * covered.  Requires 1 <= k <= n.  Runs on the device; synchronises `stream`. */
imm_status imm_select_seeds(imm_pool* p, int64_t first, int64_t count, int32_t k,
                            int32_t* seeds_out, int64_t* covered_out, void* stream);

/* ---- selection without allocation ----------------------------------------------------
 * For callers that cannot allocate (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the selection of imm_select_seeds, with identical
 * results, whose whole workspace (counters, inverted index, covered flags, argmax keys,
 * launch descriptor and grid barrier) lives in a static device array of
 * IMM_NOALLOC_SCRATCH_BYTES that each device holds from the library's load until the
 * process ends.  Calls no hipMalloc, hipFree or pinned-host allocation; the seeds and the
 * covered count are copied straight into the caller's (pageable) host memory.
 *   p, first, count, k   as imm_select_seeds (multi-round pools: k per round)
 *   seeds_out            int32[k x rounds], host, required
 *   covered_out          int64, host, or NULL
 * The workspace needs about 20.2 n + 4 count + 4 (ids held by the pool) + 12 k bytes,
 * plus 4 n when the range is not the pool's whole prefix, plus about 100 KiB
 * (imm_select_noalloc_bytes reports the exact figure); larger requests return
 * IMM_ECAPACITY before anything runs.  All calls on one device share its array: calls
 * that overlap on one device (other host threads, other streams) race and must not be
 * issued.  imm_init(device) looks the array up for that device; otherwise the first call
 * on a device does.  Synchronises `stream`. */
#define IMM_NOALLOC_SCRATCH_BYTES (64LL * 1024 * 1024)
imm_status imm_select_seeds_noalloc(const imm_pool* p, int64_t first, int64_t count, int32_t k,
                                    int32_t* seeds_out, int64_t* covered_out, void* stream);
/* Bytes of workspace imm_select_seeds_noalloc needs for these arguments (-1 for a NULL
 * pool or a negative count). */
int64_t imm_select_noalloc_bytes(const imm_pool* p, int64_t first, int64_t count, int32_t k);

/* IMM on graph g (gIM Alg. 2 then Alg. 1): estimate LB, sample theta = lambda* / LB RR sets,
 * select k seeds.  0 < eps < 1, ell > 0, 1 <= k <= n.  seeds_out int32[k].  The result is
 * a pure function of (g, model, opt->seed, k, eps, ell, opt->fresh_final). */
imm_status imm_solve(const imm_graph* g, int32_t k, double eps, double ell, imm_model model,
                     const imm_options* opt, int32_t* seeds_out, imm_info* info);

/* IMM against an existing pool (same graph/model/seed): consumes the pool's prefix and
 * extends it only where needed, so repeated queries share RR sets.  Identical results to
 * imm_solve with the pool's seed. */
imm_status imm_solve_pool(imm_pool* p, int32_t k, double eps, double ell, int32_t fresh_final,
                          void* stream, int32_t* seeds_out, imm_info* info);

/* ---- autotuning ---------------------------------------------------------------------
 * Times the generation of RR sets [0, pilot_sets) of (g, model, seed) under candidate
 * launch configurations and keeps the fastest for pools created on g with that model
 * afterwards (imm_pool_create, imm_solve, servers; not batches).  The knobs, tuned one
 * group at a time from the library defaults: IC light-wave budget of 4-edge groups
 * {1024 .. 16384} x threads per heavy set {128, 256}; the on-chip list capacity (frontier
 * capacity) of an IC light set {256, 512, 1024} or an LT walk {64, 128, 256}; the RR
 * indices a wave takes per work-counter fetch (queue depth) {4, 8, 16, 32}.  RR sets, and
 * therefore every result, are identical under all configurations (gIM Sec. III-F sizes its
 * blocks for the same purpose).  The IMM_LIGHT_BUDGET / IMM_HEAVY_BLOCK / IMM_LIGHT_CAP /
 * IMM_LT_LDS_CAP / IMM_FETCH environment variables still override.  Not thread-safe with
 * other calls on g. */
typedef struct {
    int64_t light_budget;
    int32_t heavy_block;
    int32_t candidates;           /* configurations timed */
    double best_sets_per_s;       /* pilot generation rate of the chosen configuration */
    double default_sets_per_s;    /* ... of the library defaults */
    int32_t light_cap;            /* chosen IC light-set list capacity */
    int32_t lt_cap;               /* chosen LT walk list capacity */
    int32_t fetch;                /* chosen RR indices per fetch */
    int32_t reserved;
} imm_tune_info;

imm_status imm_autotune(imm_graph* g, imm_model model, uint64_t seed, int64_t pilot_sets,
                        imm_tune_info* out);

/* ---- batched solves (many independent instances in shared launches) ---------------------
 * Solves every item as imm_solve(graph, k, eps, ell, model, {seed, fresh_final}) would, with
 * bit-identical seeds and info counters (theta, LB, covered, phases, num_rr).  The
 * instances advance together: each step generates the RR sets of every unfinished instance
 * in one launch per model and runs all their greedy selections in one cooperative launch
 * (gIM Sec. I motivates solving IM many times; the batch keeps the whole device busy with
 * instances that alone would fill a fraction of it).  The caller owns the items and their
 * seeds_out arrays (int32[k] each, host memory).  Graphs must be on the current device.
 * Arguments are validated before any work (IMM_EINVAL names the item).  On a device or
 * memory error the call returns it and sets status of every unfinished item.
 * info.t_total_s is the time from the call's start to the item's completion. */
typedef struct {
    const imm_graph* graph;
    int32_t k;
    imm_model model;
    double eps, ell;
    uint64_t seed;          /* Philox key of the instance's RR pool */
    int32_t fresh_final;
    imm_status status;      /* out */
    int32_t* seeds_out;     /* out: int32[k] in selection order */
    imm_info info;          /* out */
} imm_batch_item;

/* Whole-batch figures (stats may be NULL): ticks (generation + selection steps), wall
 * time in generation and selection, and the summed durations of the generation launches
 * (HIP events), as in imm_info. */
typedef struct {
    int64_t ticks;
    int64_t rr_sets;            /* RR sets generated over all items */
    int64_t edges_examined;
    int64_t edges_heavy;
    double t_generate_s, t_select_s, t_total_s;
    double t_rr_kernel_s;
    int64_t rr_kernel_launches;
    double t_rr_heavy_s;
    int64_t rr_heavy_launches;
    int64_t graph_ticks;        /* ticks whose selection half (per-item setup kernels and the
                                   greedy launch) ran as one captured HIP graph: with
                                   IMM_BATCH_GRAPH=1 (off by default, slower on the R-MAT
                                   mix: capture costs more than the launches it saves) */
} imm_batch_stats;

imm_status imm_batch_solve(imm_batch_item* items, int32_t count, void* stream,
                           imm_batch_stats* stats);

/* ---- serving (continuous batching over one resident graph) -----------------------------
 * A server keeps the graph and one RR pool per model (IC with seed_ic, LT with seed_lt;
 * a model is served when the graph has its encoding) resident in HBM.  Queries are
 * admitted while fewer than max_active are in flight and the estimated device memory stays
 * within hbm_budget_bytes; every scheduler tick extends each pool once, to the largest
 * demand among the active queries (RR sets are shared), and runs the greedy selections of
 * all active queries in one device launch.  A query's result equals imm_solve on the same
 * graph with the pool's seed, whatever else is in flight (gIM Sec. I and IV-H motivate
 * solving IM many times on one graph).  Thread-safe: submit/poll/wait from any thread. */
typedef struct imm_server imm_server;
typedef struct {
    int64_t submitted, completed, rejected, active, queued, ticks;
    double p50_latency_s, p99_latency_s, mean_latency_s, max_latency_s;
    double throughput_qps;     /* completed / (last completion - first submission) */
    int64_t pool_sets_ic, pool_sets_lt;
    int64_t device_bytes;      /* pools + selection workspaces */
    int64_t pool_resets;       /* pools emptied to give their memory to other queries (no
                                  active query read them; their sets are drawn again,
                                  identically, when needed) */
} imm_server_stats;

imm_status imm_server_create(const imm_graph* g, uint64_t seed_ic, uint64_t seed_lt,
                             int64_t hbm_budget_bytes, int32_t max_active, imm_server** out);
/* Queue one query; *ticket identifies it.  IMM_EINVAL for bad arguments (as imm_solve),
 * IMM_ECAPACITY when it can never fit the memory budget. */
imm_status imm_server_submit(imm_server* s, int32_t k, double eps, double ell, imm_model model,
                             int32_t fresh_final, uint64_t* ticket);
/* Non-blocking: *done = 1 and results written when the query has finished. */
imm_status imm_server_poll(imm_server* s, uint64_t ticket, int32_t* seeds_out, imm_info* info,
                           int32_t* done);
/* Blocks until the query finishes (IMM_EBUSY after timeout_s; timeout_s <= 0 waits
 * indefinitely).  info->t_total_s is the latency from submission to completion. */
imm_status imm_server_wait(imm_server* s, uint64_t ticket, double timeout_s, int32_t* seeds_out,
                           imm_info* info);
imm_status imm_server_stats_get(imm_server* s, imm_server_stats* out);
/* Stops the worker (queries still pending are dropped) and frees everything. */
imm_status imm_server_destroy(imm_server* s);

/* ---- multi-round influence maximisation (gIM Sec. IV-H, Table 3) -----------------------
 * Influence spreads in `rounds` independent rounds, round t starting from seed set S_t
 * (|S_t| <= k); the objective is the expected number of vertices active in at least one
 * round (CR-NAIMM, Sun et al., KDD'18, which gIM accelerates).  A multi-round RR set draws
 * one root (the root draw of the plain set) and runs one reverse search per round t from
 * it, in round t's live-edge instance: the edge draws use counter (r, g, t, domain) (t = 0
 * is the plain set).  Its elements are (vertex u, round t) pairs, numbered t * n + u.
 *
 * imm_mr_pool_create makes a pool of such sets (1 <= rounds <= 32, rounds * n < 2^31;
 * rounds = 1 is an ordinary pool).  On it, imm_generate_rr, imm_pool_size, imm_rr_export
 * (elements t * n + u, sorted per set) and imm_rr_histogram (hist_out uint32[rounds * n],
 * entry t * n + u) work as on plain pools; imm_select_seeds takes k as the seeds per round
 * and returns rounds * k elements in selection order: each step takes, among the elements
 * not chosen whose round holds fewer than k chosen, the one in the most uncovered sets
 * (smallest element among equals), the greedy of a partition matroid; imm_solve_pool runs
 * CR-NAIMM on it.  Errors as for plain pools. */
imm_status imm_mr_pool_create(const imm_graph* g, imm_model model, uint64_t seed, int32_t rounds,
                              imm_pool** out);

/* CR-NAIMM: IMM's estimation loop and final sample (gIM Alg. 2 and 1) over multi-round RR
 * sets, with the multi-round sample sizes (ln C(n,k) taken `rounds` times in the union
 * bound; greedy ratio 1/2 of a partition matroid instead of 1 - 1/e when rounds > 1).
 * seeds_out int32[rounds * k]: elements t * n + u in selection order (vertex u seeds round
 * t).  opt->fresh_final must be 0 when rounds > 1 (IMM_EINVAL).  The result is a pure
 * function of (g, model, opt->seed, k, rounds, eps, ell); rounds = 1 is imm_solve. */
imm_status imm_mrim_solve(const imm_graph* g, int32_t k, int32_t rounds, double eps, double ell,
                          imm_model model, const imm_options* opt, int32_t* seeds_out,
                          imm_info* info);
double imm_mr_lambda_prime(int64_t n, int64_t k, int32_t rounds, double eps, double ell);
double imm_mr_lambda_star(int64_t n, int64_t k, int32_t rounds, double eps, double ell);

/* ---- forward Monte-Carlo influence spread (gIM Sec. II-C) ----------------------------
 * Scores a seed set by simulation: E[I(S)] is the expected number of vertices reachable
 * from S in an instance graph (IC: each edge kept with its probability; LT: each vertex
 * keeps at most one in-edge, chosen with its normalised weight), which gIM uses to compare
 * solution quality.  Simulation j in [0, sims) of round t draws with its own contract,
 * independent of the RR sets':
 *    IC edge e (in-edge numbering) kept  : word 0 of Philox(j, e, t, 4) < thr[e], or thr[e]
 *                                          saturated
 *    LT vertex v keeps in-edge e          : the first e of v's in-list whose cumulative
 *                                          threshold exceeds word 0 of Philox(j, v, t, 5)
 * seeds (host or device, nseeds entries) are elements t * n + u (vertex u seeds round t;
 * rounds = 1: plain vertex ids); a simulation counts the vertices reached in at least one
 * round (the multi-round objective of Sec. IV-H).  Outputs (each may be NULL):
 * per_sim_out uint32[sims] (host) each simulation's count, *total_out their exact sum,
 * *mean_out the mean, *stderr_out the sample standard deviation / sqrt(sims).  The counts
 * are a pure function of (g, model, seed, seeds, rounds, j).  The first call on a graph
 * builds its out-edge lists (m x 8 B + (n + 1) x 8 B, kept until the graph is destroyed).
 * Errors: IMM_EINVAL (model not encoded, rounds outside [1, 32], sims outside [0, 2^32),
 * a seed element outside [0, rounds * n)), IMM_ENOMEM. */
imm_status imm_spread_mc(const imm_graph* g, imm_model model, int32_t rounds, const int32_t* seeds,
                         int32_t nseeds, int64_t sims, uint64_t seed, uint32_t* per_sim_out,
                         int64_t* total_out, double* mean_out, double* stderr_out, void* stream);

/* Measured peak of the IC generation roofline: Philox4x32-10 draws per second (in 1e9) of a
 * loop that only draws and ballots the four words against a threshold, as the IC kernels
 * do per 4 in-edges (8 waves per SIMD, two independent draws per lane, draws_per_lane in
 * [2, 2^24]).  Synchronises the device's null stream.  Errors: IMM_EINVAL, IMM_EDEVICE. */
imm_status imm_philox_rate(int64_t draws_per_lane, double* gphilox_s);

/* IMM sample-size quantities, exposed for verification (IEEE double, no FMA contraction):
 * ln C(n,k); lambda' of the LB loop; lambda* of the final sample; ell' = ell(1+ln2/ln n). */
double imm_log_binom(int64_t n, int64_t k);
double imm_lambda_prime(int64_t n, int64_t k, double eps, double ell);
double imm_lambda_star(int64_t n, int64_t k, double eps, double ell);

#ifdef __cplusplus
}
#endif
#endif /* IMM_H */
