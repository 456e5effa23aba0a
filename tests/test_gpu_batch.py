"""Batched solves: every instance's result in the batch equals its solo solve and the oracle.

imm_batch_solve advances many independent IMM instances together (shared generation and
selection launches).  Each instance must come out bit-identical to imm_solve on the same
(graph, model, seed, k, eps, ell, fresh_final): seeds, theta, LB, covered, phases, num_rr.
The mix covers IC and LT, sets that overflow the light path (heavy launches), id buffers
that overflow their first size estimate (capacity retries), fresh final samples, and the
smallest instances of the 256-instance R-MAT mix.
"""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu

KEYS = ("theta", "covered", "phases", "num_rr", "lb", "lambda_prime", "lambda_star")


def _chain(n):
    """Directed path 0 -> 1 -> ... -> n-1: every LT walk runs back to vertex 0."""
    src = np.arange(n - 1, dtype=np.int32)
    dst = np.arange(1, n, dtype=np.int32)
    return graphs.from_edges(n, src, dst)


@pytest.fixture(scope="module")
def mix(imm_gpu):
    imm = imm_gpu
    out = []

    def add(g, ic_p, lt, model, k, eps, seed, fresh=False, ell=1.0):
        gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=None, lt=lt)
        out.append(dict(g=g, ic_p=ic_p, gg=gg, graph=gg, k=k, eps=eps, ell=ell, model=model,
                        seed=seed, fresh_final=fresh))

    c1 = configs.c1()
    add(c1.graph, c1.ic_p, False, imm.IMM_IC, 10, 0.5, c1.seed)
    er = graphs.erdos_renyi(5000, 40_000, seed=7)
    add(er, np.ones(er.m, np.float32), False, imm.IMM_IC, 3, 0.5, 0x5EED0101)   # heavy sets
    r12 = graphs.rmat(12, 10 << 12, seed=81)
    add(r12, graphs.weighted_cascade(r12), True, imm.IMM_IC, 20, 0.3, 0x5EED0102, fresh=True)
    add(r12, None, True, imm.IMM_LT, 15, 0.4, 0x5EED0103)
    ch = _chain(3000)
    add(ch, None, True, imm.IMM_LT, 2, 0.5, 0x5EED0104)                        # long walks
    r13 = graphs.rmat(13, 12 << 13, seed=82)
    add(r13, graphs.trivalency(r13, seed=83), False, imm.IMM_IC, 40, 0.2, 0x5EED0105, ell=1.5)
    add(r13, graphs.trivalency(r13, seed=83), False, imm.IMM_IC, 1, 0.5, 0x5EED0106)
    return out


def _solo(imm, it):
    return imm.imm_solve(it["gg"].handle, it["k"], it["eps"], it["ell"], it["model"],
                         it["seed"], fresh_final=it["fresh_final"])


def test_batch_equals_solo_solves(imm_gpu, mix):
    imm = imm_gpu
    res = imm.imm_batch_solve(mix)
    assert len(res) == len(mix)
    for it, (seeds, info) in zip(mix, res):
        s_alone, i_alone = _solo(imm, it)
        tag = (it["g"].n, it["model"], it["k"], it["eps"])
        assert np.array_equal(seeds, s_alone), tag
        for key in KEYS:
            assert info[key] == i_alone[key], (tag, key)
        assert info["edges_examined"] == i_alone["edges_examined"], tag
        assert info["pool_ids"] == i_alone["pool_ids"], tag


def test_batch_order_does_not_matter(imm_gpu, mix):
    imm = imm_gpu
    fwd = imm.imm_batch_solve(mix)
    rev = imm.imm_batch_solve(mix[::-1])[::-1]
    for (s1, i1), (s2, i2) in zip(fwd, rev):
        assert np.array_equal(s1, s2)
        assert all(i1[k] == i2[k] for k in KEYS)


def test_batch_matches_oracle(imm_gpu, mix):
    imm = imm_gpu
    res = imm.imm_batch_solve(mix)
    for it, (seeds, info) in zip(mix, res):
        if it["g"].n > 5000:
            continue
        model = oracle.IC if it["model"] == imm.IMM_IC else oracle.LT
        ref = oracle.imm_solve(it["g"], model, it["k"], it["eps"], it["ell"], it["seed"],
                               ic_p=it["ic_p"], lt_w=None, fresh_final=it["fresh_final"])
        assert np.array_equal(seeds, ref["seeds"]), (it["g"].n, it["k"])
        assert info["theta"] == ref["theta"] and info["covered"] == ref["covered"]
        assert info["lb"] == ref["lb"]


def test_batch_smallest_mix_instances_match_oracle(imm_gpu):
    """The three smallest instances of the 256-instance R-MAT mix, batched, against the
    oracle (each also against its solo solve)."""
    imm = imm_gpu
    specs = {s.index: s for s in configs.c4_specs()}
    ws = [configs.c4_instance(specs[i]) for i in (229, 250, 168)]
    ggs = [imm.Graph.from_arrays(w.graph.n, w.graph.in_off, w.graph.in_src, ic_p=w.ic_p)
           for w in ws]
    items = [dict(graph=gg, k=w.k, eps=w.eps, ell=w.ell, model=imm.IMM_IC, seed=w.seed)
             for w, gg in zip(ws, ggs)]
    res = imm.imm_batch_solve(items)
    for w, gg, (seeds, info) in zip(ws, ggs, res):
        ref = oracle.imm_solve(w.graph, oracle.IC, w.k, w.eps, w.ell, w.seed, ic_p=w.ic_p)
        assert np.array_equal(seeds, ref["seeds"]), w.name
        assert info["theta"] == ref["theta"] and info["covered"] == ref["covered"], w.name
        s_alone, i_alone = imm.imm_solve(gg.handle, w.k, w.eps, w.ell, imm.IMM_IC, w.seed)
        assert np.array_equal(seeds, s_alone) and i_alone["num_rr"] == info["num_rr"]


def test_batch_validates_before_work(imm_gpu, mix):
    imm = imm_gpu
    assert imm.imm_batch_solve([]) == []
    bad = [dict(mix[0]), dict(mix[1])]
    bad[1]["k"] = 0
    with pytest.raises(imm.ImmError) as e:
        imm.imm_batch_solve(bad)
    assert e.value.status == 1 and "item 1" in str(e.value)
    bad = [dict(mix[0])]
    bad[0]["eps"] = 1.5
    with pytest.raises(imm.ImmError):
        imm.imm_batch_solve(bad)
    # C1's graph has no LT encoding
    bad = [dict(mix[0])]
    bad[0]["model"] = imm.IMM_LT
    with pytest.raises(imm.ImmError):
        imm.imm_batch_solve(bad)


def test_batch_graph_ticks_equal_direct_ticks(imm_gpu, mix, monkeypatch):
    """With IMM_BATCH_GRAPH=1 the selection half of every tick runs as one captured graph;
    the results equal those of the same batch without capture (the default), and the
    captured path was the one taken."""
    imm = imm_gpu
    monkeypatch.setenv("IMM_BATCH_GRAPH", "1")
    st_g = {}
    res_g = imm.imm_batch_solve(mix, stats=st_g)
    assert st_g["graph_ticks"] == st_g["ticks"] > 0
    monkeypatch.setenv("IMM_BATCH_GRAPH", "0")
    st_d = {}
    res_d = imm.imm_batch_solve(mix, stats=st_d)
    assert st_d["graph_ticks"] == 0
    for (s1, i1), (s2, i2) in zip(res_g, res_d):
        assert np.array_equal(s1, s2)
        assert all(i1[k] == i2[k] for k in KEYS)

