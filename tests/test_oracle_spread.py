"""Pins of the oracle's forward Monte-Carlo spread (gIM Sec. II-C, the estimator of Kempe et
al. that RIS replaces): each simulation counts the vertices reachable from the seeds in one
instance graph.

Checked against: closed forms (every edge live: descendants in networkx; every edge dead:
the seeds), instance graphs materialised from the published Philox draws and searched with
networkx (IC and LT), exact expected spread by enumeration of every instance of an 11-edge
graph (IC, LT and two rounds), gIM Eq. 3 (n Pr[S meets a random RR set] estimates the same
quantity from the oracle's own RR sets), and thread-count determinism.
"""
import itertools
import math

import networkx as nx
import numpy as np
import pytest

import oracle
from synth import configs, graphs

ALWAYS = 0xFFFFFFFF


def nx_graph(g, keep=None):
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    dst = g.dst()
    for e in range(g.m):
        if keep is None or keep[e]:
            G.add_edge(int(g.in_src[e]), int(dst[e]))
    return G


def reach(G, S):
    out = set(S)
    for s in S:
        out |= nx.descendants(G, s)
    return out


def word(seed, c0, c1, c2, c3):
    return int(oracle.philox([c0, c1, c2, c3], [seed & 0xFFFFFFFF, seed >> 32])[0])


def test_all_live_reaches_descendants():
    g = graphs.erdos_renyi(300, 900, seed=3)
    p = np.ones(g.m, dtype=np.float32)
    G = nx_graph(g)
    S = [5, 17, 250]
    total, per = oracle.spread_mc(g, oracle.IC, S, 40, 0x11, ic_p=p, per_sim=True)
    assert (per == len(reach(G, S))).all()
    # two rounds, every edge live in both: the union of the rounds' reaches
    el = [5, 300 + 42, 300 + 17]
    _, per2 = oracle.spread_mc(g, oracle.IC, el, 10, 0x12, ic_p=p, rounds=2, per_sim=True)
    assert (per2 == len(reach(G, [5]) | reach(G, [42, 17]))).all()


def test_all_dead_reaches_seeds_only():
    g = graphs.erdos_renyi(200, 1500, seed=4)
    p = np.zeros(g.m, dtype=np.float32)
    _, per = oracle.spread_mc(g, oracle.IC, [1, 2, 3, 190], 25, 0x13, ic_p=p, per_sim=True)
    assert (per == 4).all()
    # rounds: distinct vertices over the rounds
    _, per = oracle.spread_mc(g, oracle.IC, [1, 200 + 1, 200 + 7, 400 + 9], 25, 0x14, ic_p=p,
                              rounds=3, per_sim=True)
    assert (per == 3).all()


def test_ic_simulations_equal_reach_in_materialised_instances():
    g = graphs.erdos_renyi(400, 2400, seed=5)
    rng = np.random.default_rng(6)
    p = rng.random(g.m).astype(np.float32) * 0.5
    p[::9] = 1.0
    thr = oracle.encode_ic(p)
    seed, S, sims = 0xC0FFEE, [3, 77, 391], 12
    _, per = oracle.spread_mc(g, oracle.IC, S, sims, seed, ic_p=p, per_sim=True)
    for j in range(sims):
        keep = [thr[e] == ALWAYS or word(seed, j, e, 0, 4) < thr[e] for e in range(g.m)]
        assert per[j] == len(reach(nx_graph(g, keep), S)), j
    # round t of a multi-round simulation draws with t in the third counter word
    el = [3, 400 + 77]
    _, per2 = oracle.spread_mc(g, oracle.IC, el, 4, seed, ic_p=p, rounds=2, per_sim=True)
    for j in range(4):
        k0 = [thr[e] == ALWAYS or word(seed, j, e, 0, 4) < thr[e] for e in range(g.m)]
        k1 = [thr[e] == ALWAYS or word(seed, j, e, 1, 4) < thr[e] for e in range(g.m)]
        assert per2[j] == len(reach(nx_graph(g, k0), [3]) | reach(nx_graph(g, k1), [77]))


def test_lt_simulations_equal_reach_in_materialised_instances():
    g = graphs.erdos_renyi(300, 1800, seed=7)
    w = graphs.lt_uniform_weights(g, seed=8)
    cum = oracle.encode_lt(g.in_off, w)
    seed, S, sims = 0xD00D, [0, 150, 299], 10
    _, per = oracle.spread_mc(g, oracle.LT, S, sims, seed, lt_w=w, per_sim=True)
    for j in range(sims):
        keep = np.zeros(g.m, dtype=bool)
        for v in range(g.n):
            x = word(seed, j, v, 0, 5)
            for e in range(int(g.in_off[v]), int(g.in_off[v + 1])):
                if cum[e] == ALWAYS or x < cum[e]:
                    keep[e] = True
                    break
        assert per[j] == len(reach(nx_graph(g, keep), S)), j


# ---- exact expected spread by enumeration of every instance graph ---------------------------
def _tiny_graph():
    edges = [(0, 1), (1, 2), (2, 0), (3, 2), (4, 3), (5, 4), (6, 5), (0, 7), (7, 6), (2, 5),
             (1, 6)]
    return graphs.from_edges(8, [a for a, _ in edges], [b for _, b in edges])


TINY_P = np.array([0.3, 0.8, 0.5, 0.25, 0.6, 0.9, 0.4, 0.7, 0.2, 0.55, 0.35], dtype=np.float32)


def _ic_instances(g, thr):
    q = [1.0 if t == ALWAYS else t / 2 ** 32 for t in thr.tolist()]
    for mask in range(1 << g.m):
        pr = 1.0
        keep = []
        for e in range(g.m):
            keep.append(bool(mask >> e & 1))
            pr *= q[e] if keep[-1] else 1.0 - q[e]
        if pr > 0:
            yield pr, keep


def _z_ok(total, sims, exact, var_bound):
    mean = total / sims
    return abs(mean - exact) < 5 * math.sqrt(var_bound / sims) + 1e-9


def test_ic_mean_matches_exact_expected_spread():
    g = _tiny_graph()
    thr = oracle.encode_ic(TINY_P)
    inst = [(pr, nx_graph(g, keep)) for pr, keep in _ic_instances(g, thr)]
    sims = 200_000
    for S in ([0], [3], [0, 4], [2, 6], [1, 5, 7]):
        exact = sum(pr * len(reach(G, S)) for pr, G in inst)
        total = oracle.spread_mc(g, oracle.IC, S, sims, 0xA11CE, ic_p=TINY_P)
        assert _z_ok(total, sims, exact, g.n ** 2 / 4), (S, total / sims, exact)


def test_lt_mean_matches_exact_expected_spread():
    g = _tiny_graph()
    w = np.array([3, 1, 2, 5, 1, 4, 2, 2, 7, 1, 3], dtype=np.uint32)
    cum = oracle.encode_lt(g.in_off, w)
    choices = []                        # per vertex: (probability, kept in-edge or None)
    for v in range(g.n):
        opts, prev = [], 0
        for e in range(int(g.in_off[v]), int(g.in_off[v + 1])):
            c = 2 ** 32 if cum[e] == ALWAYS else int(cum[e])
            opts.append(((c - prev) / 2 ** 32, e))
            prev = c
        if prev < 2 ** 32:
            opts.append(((2 ** 32 - prev) / 2 ** 32, None))
        choices.append(opts)
    inst = []
    for combo in itertools.product(*choices):
        pr = math.prod(q for q, _ in combo)
        keep = np.zeros(g.m, dtype=bool)
        for _, e in combo:
            if e is not None:
                keep[e] = True
        inst.append((pr, nx_graph(g, keep)))
    sims = 200_000
    for S in ([0], [5], [1, 3], [6, 7]):
        exact = sum(pr * len(reach(G, S)) for pr, G in inst)
        total = oracle.spread_mc(g, oracle.LT, S, sims, 0xB0B, lt_w=w)
        assert _z_ok(total, sims, exact, g.n ** 2 / 4), (S, total / sims, exact)


def test_two_round_mean_matches_exact_expected_spread():
    """Rounds are independent instances: a vertex stays inactive with the product over the
    rounds of its probability of not being reached."""
    g = _tiny_graph()
    thr = oracle.encode_ic(TINY_P)
    inst = [(pr, nx_graph(g, keep)) for pr, keep in _ic_instances(g, thr)]

    def p_reached(S):
        out = np.zeros(g.n)
        for pr, G in inst:
            for v in reach(G, S):
                out[v] += pr
        return out
    sims = 200_000
    for coll in ([[0], [3]], [[4], [4]], [[1, 6], [5]], [[], [7]]):
        miss = np.ones(g.n)
        for S in coll:
            miss *= 1.0 - p_reached(S)
        exact = float((1.0 - miss).sum())
        el = [t * g.n + u for t, S in enumerate(coll) for u in S]
        total = oracle.spread_mc(g, oracle.IC, el, sims, 0xCAB, ic_p=TINY_P, rounds=2)
        assert _z_ok(total, sims, exact, g.n ** 2 / 4), (coll, total / sims, exact)


def test_forward_mean_agrees_with_ris_estimate_on_c1():
    """gIM Eq. 3: n Pr[S meets a random RR set] and the forward mean estimate the same
    E[I(S)]; the two independent estimates agree within their sampling error."""
    w = configs.c1()
    g = w.graph
    ref = oracle.imm_solve(g, oracle.IC, w.k, w.eps, w.ell, w.seed, ic_p=w.ic_p)
    S = ref["seeds"]
    sims = 20_000
    total, per = oracle.spread_mc(g, oracle.IC, S, sims, 0x5EED5EED, ic_p=w.ic_p, per_sim=True)
    mean, sd_mc = total / sims, per.std() / math.sqrt(sims)
    f = ref["covered"] / ref["num_rr"]
    sd_ris = g.n * math.sqrt(f * (1 - f) / ref["num_rr"])
    assert abs(mean - ref["spread_est"]) < 5 * math.hypot(sd_mc, sd_ris), (mean, ref["spread_est"])


def test_thread_count_does_not_change_counts():
    g = graphs.rmat(12, 40_000, seed=9)
    p = graphs.weighted_cascade(g)
    S = list(range(0, 4096, 97))
    outs = [oracle.spread_mc(g, oracle.IC, S, 300, 0x77, ic_p=p, threads=t, per_sim=True)
            for t in (1, 3, 8)]
    for tot, per in outs[1:]:
        assert tot == outs[0][0] and np.array_equal(per, outs[0][1])


def test_rejects_out_of_range_seed_elements():
    g = _tiny_graph()
    with pytest.raises(ValueError):
        oracle.spread_mc(g, oracle.IC, [8], 5, 1, ic_p=TINY_P)
    with pytest.raises(ValueError):
        oracle.spread_mc(g, oracle.IC, [16], 5, 1, ic_p=TINY_P, rounds=2)
