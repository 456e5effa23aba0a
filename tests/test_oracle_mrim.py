"""Pins of the oracle's multi-round IM (gIM Sec. IV-H, Table 3: CR-NAIMM of Sun et al.).

A multi-round RR set draws one root and runs one reverse search per round t from it, each
in round t's own live-edge instance (counter word t); its elements are (u, t) pairs stored
as t * n + u.  Seeds are chosen by the greedy of a partition matroid (at most k per
round).  Each test checks the oracle against something it does not compute itself:
plain IMM (one round is exactly IMM), networkx reachability in materialised worlds, exact
enumeration of live-edge worlds, a literal recount greedy, brute-force optima, mpmath.
"""
import itertools
import math

import mpmath
import networkx as nx
import numpy as np
import pytest

import oracle
from synth import configs, graphs
from test_oracle_pins import (_ic_world_probs, _mp_quantities, _reach_matrix, _tiny_graph,
                              nx_graph, philox_word)

ALWAYS = 0xFFFFFFFF
TINY_P = np.array([0.3, 0.8, 0.5, 0.25, 0.6, 0.9, 0.4, 0.7, 0.2, 0.55, 0.35], dtype=np.float32)


# ---- one round is plain IMM -----------------------------------------------------------------
@pytest.mark.parametrize("case", ["c1", "lt", "tiny"])
def test_one_round_is_plain_imm(case):
    if case == "c1":
        w = configs.c1()
        g, model, kw, k, eps, seed = w.graph, oracle.IC, dict(ic_p=w.ic_p), w.k, w.eps, w.seed
    elif case == "lt":
        g = graphs.rmat(11, 8 << 11, seed=71)
        model, kw, k, eps, seed = oracle.LT, dict(lt_w=graphs.lt_uniform_weights(g, seed=72)), 8, 0.3, 77
    else:
        g, model, kw, k, eps, seed = _tiny_graph(), oracle.IC, dict(ic_p=TINY_P), 2, 0.3, 5
    a = oracle.mrim_solve(g, model, k, 1, eps, 1.0, seed, **kw)
    b = oracle.imm_solve(g, model, k, eps, 1.0, seed, **kw)
    assert a["seeds"].tolist() == b["seeds"].tolist()
    for key in ("theta", "num_rr", "covered", "phases", "edges", "pool_ids", "lb", "spread_est",
                "lambda_prime", "lambda_star"):
        assert a[key] == b[key], key


# ---- each round's slice is reverse reachability in that round's world -------------------------
@pytest.mark.parametrize("model", [oracle.IC, oracle.LT])
def test_round_slices_are_reverse_reach_in_round_worlds(model):
    g = graphs.erdos_renyi(300, 1500, seed=73)
    seed, rounds = 0x5EED0F01, 4
    if model == oracle.IC:
        p = graphs.trivalency(g, seed=74) * np.float32(5)
        thr, kw = oracle.encode_ic(p), dict(ic_p=p)
    else:
        w = graphs.lt_uniform_weights(g, seed=75)
        thr, kw = oracle.encode_lt(g.in_off, w), dict(lt_w=w)
    off, ids, _ = oracle.mr_sets(g, model, seed, rounds, 60, **kw)
    dst = g.dst().tolist()
    src = g.in_src.tolist()
    for r in range(60):
        elems = ids[off[r]:off[r + 1]]
        root = oracle.root(seed, r, g.n)
        for t in range(rounds):
            got = sorted((elems[(elems // g.n) == t] - t * g.n).tolist())
            # the live-edge instance of round t, drawn edge by edge from the counter
            W = nx.DiGraph()
            W.add_nodes_from(range(g.n))
            if model == oracle.IC:
                for e in range(g.m):
                    x = philox_word(seed, r, e >> 2, t, 2, e & 3)
                    if thr[e] == ALWAYS or x < thr[e]:
                        W.add_edge(src[e], dst[e])
                want = sorted({root} | nx.ancestors(W, root))
            else:
                # LT: every vertex keeps the first in-edge above its draw; the walk from the
                # root follows the kept edges until it repeats a vertex
                want, v, seen = [], root, set()
                while v not in seen:
                    seen.add(v)
                    s0, e0 = int(g.in_off[v]), int(g.in_off[v + 1])
                    if s0 == e0:
                        break
                    x = philox_word(seed, r, v, t, 3, 0)
                    j = next(j for j in range(s0, e0) if thr[j] == ALWAYS or x < thr[j])
                    v = src[j]
                want = sorted(seen)
            assert got == want, (r, t)
            assert root in got


# ---- exact membership and the multi-round Eq. 3 by enumeration ---------------------------------
def test_membership_and_multi_round_estimator_by_enumeration():
    g = _tiny_graph()
    thr = oracle.encode_ic(TINY_P)
    n, rounds = g.n, 2
    worlds = [(pr, _reach_matrix(n, live)) for pr, live in _ic_world_probs(g, thr)]
    reach_p = np.zeros((n, n))           # reach_p[u, v] = Pr[u reaches v] in one round
    for pr, reach in worlds:
        for u in range(n):
            for v in range(n):
                if reach[u] >> v & 1:
                    reach_p[u, v] += pr

    def reached(S):                      # Pr[S reaches v] in one round, for every v
        out = np.zeros(n)
        for pr, reach in worlds:
            acc = 0
            for u in S:
                acc |= reach[u]
            for v in range(n):
                if acc >> v & 1:
                    out[v] += pr
        return out
    count = 200_000
    off, ids, _ = oracle.mr_sets(g, oracle.IC, 0x5EED0F02, rounds, count, ic_p=TINY_P)
    # Pr[(u, t) in R] = (1/n) sum_v Pr[u reaches v], the same for every round
    hist = np.bincount(ids, minlength=n * rounds)
    member = reach_p.sum(axis=1) / n
    for t in range(rounds):
        for u in range(n):
            q = member[u]
            z = (hist[t * n + u] - count * q) / math.sqrt(count * q * (1 - q) + 1e-12)
            assert abs(z) < 5, (u, t, z)
    # n Pr[S meets R] = E[# nodes active in some round] = sum_v 1 - prod_t (1 - Pr[S_t ~> v])
    collections = [[[0], [3]], [[2], []], [[4], [4]], [[1, 6], [5]], [[], [7]]]
    sets = [ids[off[r]:off[r + 1]] for r in range(count)]
    for coll in collections:
        elems = {t * n + u for t, S in enumerate(coll) for u in S}
        # rounds are independent instances: a node stays inactive with the product of its
        # per-round probabilities of not being reached
        miss = np.ones(n)
        for S in coll:
            miss *= 1.0 - reached(S)
        exact = float((1.0 - miss).sum())
        hits = sum(1 for s in sets if elems.intersection(s.tolist()))
        q = hits / count
        est = n * q
        sd = n * math.sqrt(q * (1 - q) / count) + 1e-9
        assert abs(est - exact) < 5 * sd, (coll, est, exact)


# ---- the partition-matroid greedy ---------------------------------------------------------------
def _recount_greedy(part, parts, sets, k):
    """The greedy read literally: each step recounts, for every element whose part has
    room, the uncovered sets containing it, and takes the best (smallest element on ties)."""
    chosen, taken, covered = [], [0] * parts, [False] * len(sets)
    for _ in range(parts * k):
        best, best_c = None, -1
        for e in range(part * parts):
            if e in chosen or taken[e // part] >= k:
                continue
            c = sum(1 for i, s in enumerate(sets) if not covered[i] and e in s)
            if c > best_c:
                best, best_c = e, c
        chosen.append(best)
        taken[best // part] += 1
        for i, s in enumerate(sets):
            if best in s:
                covered[i] = True
    return chosen, sum(covered)


def _to_csr(sets):
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in sets])
    ids = np.array([e for s in sets for e in sorted(s)], dtype=np.int32)
    return off, ids


def test_partition_greedy_against_recount_and_optimum():
    rng = np.random.default_rng(76)
    for trial in range(60):
        part, parts, k = int(rng.integers(2, 6)), int(rng.integers(1, 4)), int(rng.integers(1, 3))
        k = min(k, part)
        sets = [set(rng.choice(part * parts, int(rng.integers(1, min(4, part * parts) + 1)),
                               replace=False).tolist())
                for _ in range(int(rng.integers(1, 25)))]
        off, ids = _to_csr(sets)
        seeds, cov = oracle.greedy_partition(part, parts, off, ids, k)
        want, want_cov = _recount_greedy(part, parts, sets, k)
        assert seeds.tolist() == want and cov == want_cov
        if parts == 1:
            s1, c1 = oracle.greedy_sets(part, off, ids, k)
            assert s1.tolist() == seeds.tolist() and c1 == cov
        # 1/2 of the best feasible collection (Fisher, Nemhauser, Wolsey 1978)
        opt = 0
        per_part = [list(itertools.combinations(range(t * part, (t + 1) * part), k))
                    for t in range(parts)]
        for combo in itertools.product(*per_part):
            S = set(itertools.chain(*combo))
            opt = max(opt, sum(1 for s in sets if S & s))
        assert cov >= 0.5 * opt


# ---- sample sizes ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,rounds,eps", [(1000, 10, 5, 0.1), (1 << 20, 10, 5, 0.1),
                                            (75_879, 10, 5, 0.1), (5000, 3, 2, 0.4)])
def test_mr_sample_sizes_against_mpmath(n, k, rounds, eps):
    mpmath.mp.dps = 60
    n_ = mpmath.mpf(n)
    ellp = 1 + mpmath.log(2) / mpmath.log(n_)
    lnc = rounds * mpmath.log(mpmath.binomial(n, k))
    ep = mpmath.sqrt(2) * eps
    lam1 = (2 + 2 * ep / 3) * (lnc + ellp * mpmath.log(n_) + mpmath.log(mpmath.log(n_, 2))) * n_ / ep ** 2
    gam = mpmath.mpf(1) / 2
    a = mpmath.sqrt(ellp * mpmath.log(n_) + mpmath.log(2))
    b = mpmath.sqrt(gam * (lnc + ellp * mpmath.log(n_) + mpmath.log(2)))
    lam2 = 2 * n_ * (gam * a + b) ** 2 / mpmath.mpf(eps) ** 2
    assert abs(oracle.mr_lambda_prime(n, k, rounds, eps, 1.0) / float(lam1) - 1) < 1e-12
    assert abs(oracle.mr_lambda_star(n, k, rounds, eps, 1.0) / float(lam2) - 1) < 1e-12


def test_mr_sample_sizes_reduce_to_imm_and_grow_with_rounds():
    for n, k, eps in [(1000, 10, 0.5), (1 << 20, 50, 0.1), (4, 2, 0.3)]:
        _, lam1, lam2 = _mp_quantities(n, k, eps, 1.0)
        assert oracle.mr_lambda_prime(n, k, 1, eps, 1.0) == oracle.lambda_prime(n, k, eps, 1.0)
        assert oracle.mr_lambda_star(n, k, 1, eps, 1.0) == oracle.lambda_star(n, k, eps, 1.0)
        assert abs(oracle.mr_lambda_star(n, k, 1, eps, 1.0) / float(lam2) - 1) < 1e-12
        ls = [oracle.mr_lambda_star(n, k, t, eps, 1.0) for t in (2, 3, 5, 8)]
        assert all(x < y for x, y in zip(ls, ls[1:]))


# ---- end-to-end guarantee on a tiny graph --------------------------------------------------------
def test_mrim_meets_half_guarantee_on_tiny_graph():
    g = _tiny_graph()
    thr = oracle.encode_ic(TINY_P)
    n, rounds, k, eps = g.n, 2, 1, 0.3
    reach_p = np.zeros((n, n))
    for pr, live in _ic_world_probs(g, thr):
        reach = _reach_matrix(n, live)
        for u in range(n):
            for v in range(n):
                if reach[u] >> v & 1:
                    reach_p[u, v] += pr

    def objective(coll):          # E[# nodes active in at least one round]
        tot = 0.0
        for v in range(n):
            miss = 1.0
            for S in coll:
                miss *= np.prod([1.0 - reach_p[u, v] for u in S])
            tot += 1.0 - miss
        return tot

    opt = max(objective([[a], [b]]) for a in range(n) for b in range(n))
    fails = 0
    for s in range(60):
        res = oracle.mrim_solve(g, oracle.IC, k, rounds, eps, 1.0, 3000 + s, ic_p=TINY_P)
        coll = [[int(e) % n for e in res["seeds"] if int(e) // n == t] for t in range(rounds)]
        assert all(len(S) == k for S in coll)
        if objective(coll) < (0.5 - eps) * opt:
            fails += 1
    assert fails <= 60 / n + 3
