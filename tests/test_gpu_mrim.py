"""GPU parity of multi-round influence maximisation (gIM Sec. IV-H, Table 3: CR-NAIMM).

A multi-round RR set is the union over rounds t of round t's reverse search from one root,
its elements (u, t) numbered t * n + u; the greedy is a partition matroid (at most k seeds
per round).  Every result of the HIP path -- sets, element counts, edges examined, the
partition greedy's seeds and coverage, and the whole CR-NAIMM solve (theta, LB bit for
bit) -- is compared with the oracle's.
"""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu


def _mr_pool(imm, g, model, seed, rounds, count, ic_p=None, lt_w=None, chunks=None):
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=lt_w,
                               lt=(model == imm.IMM_LT))
    pool = imm.Pool.create_mr(gg, model, seed, rounds)
    for upto in (chunks or [count]):
        imm.imm_generate_rr(pool.handle, upto)
    return gg, pool


@pytest.mark.parametrize("model,rounds", [(0, 5), (0, 2), (1, 5), (1, 3)])
def test_mr_sets_match_oracle(imm_gpu, model, rounds):
    imm = imm_gpu
    if model == imm.IMM_IC:
        g = graphs.rmat(13, 10 << 13, seed=71)
        ic_p, lt_w = graphs.weighted_cascade(g), None
    else:
        g = graphs.rmat(13, 10 << 13, seed=72)
        ic_p, lt_w = None, graphs.lt_uniform_weights(g, seed=73)
    count = 6000
    seed = 0x5EED0900 + model * 16 + rounds
    _, pool = _mr_pool(imm, g, model, seed, rounds, count, ic_p=ic_p, lt_w=lt_w,
                       chunks=[1, 333, 4000, count])
    off_g, ids_g = imm.imm_rr_export(pool.handle, 0, count)
    off_o, ids_o, edges_o = oracle.mr_sets(g, model, seed, rounds, count, ic_p=ic_p, lt_w=lt_w)
    assert np.array_equal(off_g, off_o), "multi-round set sizes differ"
    assert np.array_equal(ids_g, ids_o), "multi-round set elements differ"
    hist_g = imm.imm_rr_histogram(pool.handle, 0, count, g.n * rounds)
    hist_o = np.bincount(ids_o, minlength=g.n * rounds).astype(np.uint32)
    assert np.array_equal(hist_g, hist_o)
    n_sets, n_ids, edges = imm.imm_pool_size(pool.handle)
    assert (n_sets, n_ids, edges) == (count, len(ids_o), edges_o)


def test_mr_round_zero_is_the_plain_set(imm_gpu):
    """Round 0 of a multi-round set draws exactly the plain RR set of the same index."""
    imm = imm_gpu
    w = configs.c1()
    g = w.graph
    count, rounds = 3000, 4
    _, pool = _mr_pool(imm, g, imm.IMM_IC, w.seed, rounds, count, ic_p=w.ic_p)
    off_m, ids_m = imm.imm_rr_export(pool.handle, 0, count)
    ref = oracle.Pool(g, oracle.IC, w.seed, ic_p=w.ic_p)
    ref.extend(count)
    off_p, ids_p = ref.export()
    for r in range(0, count, 97):
        elems = ids_m[off_m[r]:off_m[r + 1]]
        assert np.array_equal(elems[elems < g.n], ids_p[off_p[r]:off_p[r + 1]])


@pytest.mark.parametrize("first,count,k", [(0, 5000, 1), (0, 5000, 10), (700, 3000, 40)])
def test_mr_select_matches_partition_greedy(imm_gpu, first, count, k):
    imm = imm_gpu
    g = graphs.rmat(12, 12 << 12, seed=81)
    ic_p = graphs.weighted_cascade(g)
    rounds, seed = 5, 0x5EED0A01
    _, pool = _mr_pool(imm, g, imm.IMM_IC, seed, rounds, first + count, ic_p=ic_p)
    seeds_g, cov_g = imm.imm_select_seeds(pool.handle, first, count, k, rounds=rounds)
    off, ids, _ = oracle.mr_sets(g, oracle.IC, seed, rounds, first + count, ic_p=ic_p)
    off_r = off[first:first + count + 1] - off[first]
    ids_r = ids[off[first]:off[first + count]]
    seeds_o, cov_o = oracle.greedy_partition(g.n, rounds, off_r, ids_r, k)
    assert np.array_equal(seeds_g, seeds_o)
    assert cov_g == cov_o
    # the constraint itself: at most k per round
    assert np.bincount(seeds_g // g.n, minlength=rounds).max() <= k


def test_mr_select_parts_fill_early(imm_gpu):
    """Few vertices (n = 40) and k close to n: parts fill while others still offer the
    largest counts, so the full-part exclusion decides most steps."""
    imm = imm_gpu
    g = graphs.erdos_renyi(40, 300, seed=82)
    ic_p = np.full(g.m, 0.3, dtype=np.float32)
    rounds, seed, count, k = 3, 0x5EED0A02, 4000, 30
    _, pool = _mr_pool(imm, g, imm.IMM_IC, seed, rounds, count, ic_p=ic_p)
    seeds_g, cov_g = imm.imm_select_seeds(pool.handle, 0, count, k, rounds=rounds)
    off, ids, _ = oracle.mr_sets(g, oracle.IC, seed, rounds, count, ic_p=ic_p)
    seeds_o, cov_o = oracle.greedy_partition(g.n, rounds, off, ids, k)
    assert np.array_equal(seeds_g, seeds_o)
    assert cov_g == cov_o


def _mrim_both(imm, g, model, k, rounds, eps, seed, ic_p=None, lt_w=None):
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=lt_w,
                               lt=(model == imm.IMM_LT))
    seeds, info = imm.imm_mrim_solve(gg.handle, k, rounds, eps, 1.0, model, seed)
    ref = oracle.mrim_solve(g, model, k, rounds, eps, 1.0, seed, ic_p=ic_p, lt_w=lt_w)
    assert np.array_equal(seeds, ref["seeds"]), (seeds[:12], ref["seeds"][:12])
    assert info["theta"] == ref["theta"]
    assert info["num_rr"] == ref["num_rr"]
    assert info["covered"] == ref["covered"]
    assert info["lb"] == ref["lb"]
    assert info["lambda_prime"] == ref["lambda_prime"]
    assert info["lambda_star"] == ref["lambda_star"]
    assert info["spread_est"] == ref["spread_est"]
    assert info["edges_examined"] == ref["edges"]
    assert info["pool_ids"] == ref["pool_ids"]
    return seeds, info


def test_mrim_solve_table3_config_ic(imm_gpu):
    """k = 10, T = 5, eps = 0.1 (the setting of gIM Table 3) on a weighted-cascade R-MAT."""
    imm = imm_gpu
    g = graphs.rmat(12, 8 << 12, seed=91)
    _mrim_both(imm, g, imm.IMM_IC, 10, 5, 0.1, 0x5EED0B01, ic_p=graphs.weighted_cascade(g))


def test_mrim_solve_lt(imm_gpu):
    imm = imm_gpu
    g = graphs.rmat(11, 8 << 11, seed=92)
    _mrim_both(imm, g, imm.IMM_LT, 5, 3, 0.2, 0x5EED0B02, lt_w=graphs.lt_uniform_weights(g, 93))


def test_mrim_one_round_is_imm(imm_gpu):
    imm = imm_gpu
    w = configs.c1()
    gg = imm.Graph.from_arrays(w.graph.n, w.graph.in_off, w.graph.in_src, ic_p=w.ic_p)
    s1, i1 = imm.imm_mrim_solve(gg.handle, w.k, 1, w.eps, w.ell, imm.IMM_IC, w.seed)
    s0, i0 = imm.imm_solve(gg.handle, w.k, w.eps, w.ell, imm.IMM_IC, w.seed)
    assert np.array_equal(s1, s0)
    assert (i1["theta"], i1["lb"], i1["covered"]) == (i0["theta"], i0["lb"], i0["covered"])

