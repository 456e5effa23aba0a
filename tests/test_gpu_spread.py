"""GPU parity of the forward Monte-Carlo spread (gIM Sec. II-C): every simulation's count
of reached vertices equals the oracle's, for IC (weighted cascade and per-edge
probabilities), LT, several rounds, and the seeds a solve returns."""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu


def _both(imm, g, model, seeds, sims, seed, ic_p=None, lt_w=None, rounds=1):
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=lt_w,
                               lt=(model == imm.IMM_LT))
    got = imm.imm_spread_mc(gg.handle, model, seeds, sims, seed, rounds=rounds, per_sim=True)
    tot, per = oracle.spread_mc(g, model, seeds, sims, seed, ic_p=ic_p, lt_w=lt_w, rounds=rounds,
                                per_sim=True)
    assert np.array_equal(got["per_sim"].astype(np.int64), per)
    assert got["total"] == tot
    assert got["mean"] == tot / sims
    return got


def test_spread_ic_wc_rmat(imm_gpu):
    g = graphs.rmat(14, 10 << 14, seed=101)
    seeds = np.arange(0, g.n, 331, dtype=np.int32)
    _both(imm_gpu, g, imm_gpu.IMM_IC, seeds, 3000, 0x5EED0C01, ic_p=graphs.weighted_cascade(g))


def test_spread_ic_per_edge_probabilities(imm_gpu):
    g = graphs.erdos_renyi(5000, 40_000, seed=102)
    rng = np.random.default_rng(103)
    p = (rng.random(g.m) * 0.3).astype(np.float32)
    p[::13] = 1.0
    p[::17] = 0.0
    _both(imm_gpu, g, imm_gpu.IMM_IC, [7, 1234, 4999], 2000, 0x5EED0C02, ic_p=p)


@pytest.mark.parametrize("unit", [False, True])
def test_spread_lt(imm_gpu, unit):
    g = graphs.rmat(13, 12 << 13, seed=104)
    w = None if unit else graphs.lt_uniform_weights(g, seed=105)
    seeds = np.arange(3, g.n, 257, dtype=np.int32)
    _both(imm_gpu, g, imm_gpu.IMM_LT, seeds, 2000, 0x5EED0C03, lt_w=w)


@pytest.mark.parametrize("model", [0, 1])
def test_spread_multi_round(imm_gpu, model):
    g = graphs.rmat(12, 8 << 12, seed=106)
    ic_p = graphs.weighted_cascade(g) if model == 0 else None
    rng = np.random.default_rng(107)
    rounds = 4
    el = np.unique(rng.integers(0, g.n * rounds, size=40)).astype(np.int32)
    _both(imm_gpu, g, model, el, 1500, 0x5EED0C04, ic_p=ic_p, rounds=rounds)


def test_spread_of_solve_seeds_c1(imm_gpu):
    """The seeds of the 1000-vertex ER solve, scored by 20000 simulations; the mean agrees
    with the solve's own RIS estimate (gIM Eq. 3) within the sampling error."""
    imm = imm_gpu
    w = configs.c1()
    g = w.graph
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=w.ic_p)
    seeds, info = imm.imm_solve(gg.handle, w.k, w.eps, w.ell, imm.IMM_IC, w.seed)
    got = _both(imm, g, imm.IMM_IC, seeds, 20_000, 0x5EED5EED, ic_p=w.ic_p)
    f = info["covered"] / info["num_rr"]
    sd_ris = g.n * np.sqrt(f * (1 - f) / info["num_rr"])
    assert abs(got["mean"] - info["spread_est"]) < 5 * np.hypot(got["stderr"], sd_ris)


def test_spread_edge_cases(imm_gpu):
    imm = imm_gpu
    g = graphs.erdos_renyi(100, 400, seed=108)
    p = graphs.weighted_cascade(g)
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    assert imm.imm_spread_mc(gg.handle, imm.IMM_IC, [], 50, 1)["total"] == 0
    assert imm.imm_spread_mc(gg.handle, imm.IMM_IC, [3], 0, 1)["total"] == 0
    with pytest.raises(imm.ImmError):
        imm.imm_spread_mc(gg.handle, imm.IMM_IC, [100], 5, 1)
    with pytest.raises(imm.ImmError):
        imm.imm_spread_mc(gg.handle, imm.IMM_LT, [3], 5, 1)
