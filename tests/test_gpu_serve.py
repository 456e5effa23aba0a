"""Served queries: each result is the same alone and in the mix.

A server over one resident graph (IC and WC-LT pools) answers a stream of queries with
different k, eps and model, admitted while others are in flight.  Every answer must equal
imm_solve on the same graph with the pool's seed (bit-exact seeds, theta, LB, covered),
and a sample is also checked against the CPU oracle.
"""
import numpy as np
import pytest

import oracle
from synth import graphs

pytestmark = pytest.mark.gpu

SEED_IC, SEED_LT = 0x5EED0005, 0x5EED0006


@pytest.fixture(scope="module")
def served_graph(imm_gpu):
    g = graphs.rmat(12, 10 << 12, seed=81)
    p = graphs.trivalency(g, seed=82)
    p[::3] = graphs.weighted_cascade(g)[::3]
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p, lt_w=None, lt=True)
    return g, p, gg


def _queries(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        out.append(dict(k=int(rng.integers(1, 40)), eps=float(rng.choice([0.5, 0.3, 0.2])),
                        model=int(rng.integers(0, 2))))
    return out


def _alone(imm, gg, q):
    seed = SEED_IC if q["model"] == imm.IMM_IC else SEED_LT
    return imm.imm_solve(gg.handle, q["k"], q["eps"], 1.0, q["model"], seed)


@pytest.mark.parametrize("max_active", [1, 4, 16])
def test_served_results_equal_solo_solves(imm_gpu, served_graph, max_active):
    _served_equal_solo(imm_gpu, served_graph, max_active, qseed=max_active)


def test_served_hot_sets_one_launch_each(imm_gpu, served_graph, monkeypatch):
    """With a hot set available (forced small here: 256 of 4096 vertices), the selections
    of a tick run one launch each with their hot sets instead of one launch of several
    instances; every answer still equals the solo solve."""
    monkeypatch.setenv("IMM_SELECT_HOT", "256")
    _served_equal_solo(imm_gpu, served_graph, 16, qseed=99)


def _served_equal_solo(imm_gpu, served_graph, max_active, qseed):
    g, p, gg = served_graph
    imm = imm_gpu
    qs = _queries(14, seed=qseed)
    srv = imm.imm_server_create(gg.handle, SEED_IC, SEED_LT, 8 << 30, max_active)
    try:
        tickets = [imm.imm_server_submit(srv, q["k"], q["eps"], 1.0, q["model"]) for q in qs[:8]]
        # wait for one, then submit the rest while the others are in flight
        imm.imm_server_wait(srv, tickets[0], qs[0]["k"], timeout_s=60)
        tickets += [imm.imm_server_submit(srv, q["k"], q["eps"], 1.0, q["model"]) for q in qs[8:]]
        results = [imm.imm_server_wait(srv, t, q["k"], timeout_s=60) for t, q in zip(tickets, qs)]
        stats = imm.imm_server_stats_get(srv)
    finally:
        imm.imm_server_destroy(srv)
    assert stats["completed"] == len(qs) and stats["rejected"] == 0
    assert 0 < stats["p50_latency_s"] <= stats["p99_latency_s"] <= stats["max_latency_s"]
    for q, (seeds, info) in zip(qs, results):
        s_alone, i_alone = _alone(imm, gg, q)
        assert np.array_equal(seeds, s_alone), q
        for key in ("theta", "covered", "phases", "num_rr"):
            assert info[key] == i_alone[key], (q, key)
        assert info["lb"] == i_alone["lb"]


def test_served_results_match_oracle(imm_gpu, served_graph):
    g, p, gg = served_graph
    imm = imm_gpu
    qs = [dict(k=5, eps=0.5, model=0), dict(k=12, eps=0.3, model=1), dict(k=3, eps=0.4, model=0)]
    srv = imm.imm_server_create(gg.handle, SEED_IC, SEED_LT, 8 << 30, 3)
    try:
        tickets = [imm.imm_server_submit(srv, q["k"], q["eps"], 1.0, q["model"]) for q in qs]
        results = [imm.imm_server_wait(srv, t, q["k"], timeout_s=60) for t, q in zip(tickets, qs)]
    finally:
        imm.imm_server_destroy(srv)
    for q, (seeds, info) in zip(qs, results):
        if q["model"] == 0:
            ref = oracle.imm_solve(g, oracle.IC, q["k"], q["eps"], 1.0, SEED_IC, ic_p=p)
        else:
            ref = oracle.imm_solve(g, oracle.LT, q["k"], q["eps"], 1.0, SEED_LT, lt_w=None)
        assert np.array_equal(seeds, ref["seeds"]), q
        assert info["theta"] == ref["theta"] and info["covered"] == ref["covered"]


def test_server_rejects_queries_beyond_budget(imm_gpu, served_graph):
    g, p, gg = served_graph
    imm = imm_gpu
    srv = imm.imm_server_create(gg.handle, SEED_IC, SEED_LT, 1 << 16, 2)
    try:
        with pytest.raises(imm.ImmError) as e:
            imm.imm_server_submit(srv, 10, 0.1, 1.0, imm.IMM_IC)
        assert e.value.status == 3      # IMM_ECAPACITY
        with pytest.raises(imm.ImmError):
            imm.imm_server_submit(srv, 0, 0.1, 1.0, imm.IMM_IC)   # k out of range
    finally:
        imm.imm_server_destroy(srv)


def test_server_rejects_query_whose_pool_would_outgrow_budget(imm_gpu):
    """Every edge live on a dense random graph: each RR set is the giant component (about
    5000 members).  Under a 256 MiB budget, k = 2 with eps = 0.5 needs a few hundred sets
    and is served; eps = 0.05 needs ~10^4 sets in its first estimation phase alone, so it is
    rejected with IMM_ECAPACITY once the pool's mean set size is known, before the pool
    grows.  The server keeps serving: later queries complete and equal solo solves."""
    imm = imm_gpu
    g = graphs.erdos_renyi(5000, 50_000, seed=8)
    p = np.ones(g.m, dtype=np.float32)
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    srv = imm.imm_server_create(gg.handle, SEED_IC, SEED_LT, 256 << 20, 4)
    try:
        t_small = imm.imm_server_submit(srv, 2, 0.5, 1.0, imm.IMM_IC)
        t_big = imm.imm_server_submit(srv, 2, 0.05, 1.0, imm.IMM_IC)
        small = imm.imm_server_wait(srv, t_small, 2, timeout_s=60)
        with pytest.raises(imm.ImmError) as e:
            imm.imm_server_wait(srv, t_big, 2, timeout_s=60)
        assert e.value.status == 3      # IMM_ECAPACITY
        t_after = imm.imm_server_submit(srv, 3, 0.5, 1.0, imm.IMM_IC)
        after = imm.imm_server_wait(srv, t_after, 3, timeout_s=60)
        stats = imm.imm_server_stats_get(srv)
    finally:
        imm.imm_server_destroy(srv)
    assert stats["rejected"] == 1 and stats["completed"] == 2
    for (seeds, info), k in ((small, 2), (after, 3)):
        s_alone, i_alone = imm.imm_solve(gg.handle, k, 0.5, 1.0, imm.IMM_IC, SEED_IC)
        assert np.array_equal(seeds, s_alone)
        assert info["theta"] == i_alone["theta"] and info["covered"] == i_alone["covered"]


def test_served_results_equal_solo_after_pool_resets(imm_gpu, served_graph, monkeypatch):
    """A pool that no active query reads may be emptied to give its memory to others; its
    sets are drawn again, identically, when a later query needs them.  With
    IMM_SERVE_FRUGAL=1 the server empties every such pool after each tick, so queries of
    one model that follow queries of the other redraw their pool: every answer must still
    equal the solo solve."""
    g, p, gg = served_graph
    imm = imm_gpu
    monkeypatch.setenv("IMM_SERVE_FRUGAL", "1")
    qs = [dict(k=8, eps=0.3, model=0), dict(k=5, eps=0.5, model=1), dict(k=20, eps=0.2, model=0),
          dict(k=12, eps=0.3, model=1), dict(k=3, eps=0.5, model=0)]
    srv = imm.imm_server_create(gg.handle, SEED_IC, SEED_LT, 8 << 30, 1)
    try:
        results = []
        for q in qs:                        # one at a time: the other model's pool is idle
            t = imm.imm_server_submit(srv, q["k"], q["eps"], 1.0, q["model"])
            results.append(imm.imm_server_wait(srv, t, q["k"], timeout_s=60))
        stats = imm.imm_server_stats_get(srv)
    finally:
        imm.imm_server_destroy(srv)
    assert stats["completed"] == len(qs) and stats["pool_resets"] >= 3
    for q, (seeds, info) in zip(qs, results):
        s_alone, i_alone = _alone(imm, gg, q)
        assert np.array_equal(seeds, s_alone), q
        for key in ("theta", "covered", "phases", "num_rr"):
            assert info[key] == i_alone[key], (q, key)
        assert info["lb"] == i_alone["lb"]
