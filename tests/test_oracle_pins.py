"""Pins of the CPU oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself: published
known-answer vectors, an independent library (rocRAND, networkx, mpmath), closed forms,
brute-force enumeration of live-edge worlds, exhaustive search, or invariants.  A plausible
mistake in the oracle (wrong edge direction, unmarked root, wrong tie-break, a dropped term
in a sample-size formula, an off-by-one in a threshold) makes at least one of them fail.
"""
import itertools
import math
import os
import subprocess
import tempfile

import mpmath
import networkx as nx
import numpy as np
import pytest

import oracle
from conftest import ROOT
from synth import configs, graphs

GOLDEN = os.path.join(ROOT, "tests", "golden")
ALWAYS = 0xFFFFFFFF


def nx_graph(g):
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    dst = g.dst()
    G.add_edges_from(zip(g.in_src.tolist(), dst.tolist()))
    return G


def philox_word(seed, c0, c1, c2, c3, word):
    return int(oracle.philox([c0, c1, c2, c3], [seed & 0xFFFFFFFF, seed >> 32])[word])


# ---- P10: Philox -----------------------------------------------------------------------
def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        assert oracle.philox(v[0:4], v[4:6]).tolist() == v[6:10]


def _rocrand_probe():
    exe = os.path.join(tempfile.gettempdir(), f"imm_rocrand_philox_{os.getuid()}")
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox.cpp")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        r = subprocess.run(["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", src, "-o", exe],
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("cannot build the rocRAND probe: " + r.stderr[-300:])
    return exe


def test_philox_matches_rocrand_on_random_counters():
    exe = _rocrand_probe()
    rng = np.random.default_rng(10)
    rows = rng.integers(0, 1 << 32, size=(4000, 6), dtype=np.uint64)
    rows[:10, 2] = 0
    rows[:10, 3] = [1, 2, 3, 1, 2, 3, 1, 2, 3, 2]       # the contract's domain words
    inp = "\n".join(" ".join(str(int(x)) for x in r) for r in rows)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(x) for x in l.split()] for l in out.strip().splitlines()])
    ref = np.array([oracle.philox(r[:4], r[4:]) for r in rows])
    assert np.array_equal(got, ref)


def test_root_sampler_is_multiply_shift_and_uniform():
    seed, n = 0x1234_5678_9ABC, 64
    roots = np.array([oracle.root(seed, r, n) for r in range(64_000)])
    for r in range(50):
        w = philox_word(seed, r, 0, 0, 1, 0)
        assert roots[r] == (w * n) >> 32
    counts = np.bincount(roots, minlength=n)
    chi2 = ((counts - 1000.0) ** 2 / 1000.0).sum()
    assert chi2 < 130.0          # 63 dof: mean 63, sd ~11


# ---- P12: encoders --------------------------------------------------------------------------
def test_encoding_spot_values():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "encoding_spot_values.txt"))
            if l.strip() and not l.startswith("#")]
    for kind, d, j, val in rows:
        d, val = int(d), int(val)
        if kind == "ic_wc":
            assert oracle.lib().orc_ic_threshold(np.float32(1.0) / np.float32(d)) == val
        else:
            g = graphs.from_edges(d + 1, list(range(1, d + 1)), [0] * d)
            cum = oracle.encode_lt(g.in_off, None)
            assert int(cum[int(j) - 1]) == val


def test_ic_encoding_closed_form():
    rng = np.random.default_rng(1)
    p = rng.random(50_000).astype(np.float32)
    p[:4] = [0.0, 1.0, np.float32(1) - np.float32(2 ** -24), np.float32(2 ** -33)]
    thr = oracle.encode_ic(p)
    # exact: p * 2^32 as a rational, floor, saturate at 2^32
    exact = [min(math.floor(float(x) * 2 ** 32), ALWAYS) for x in p]
    assert thr.tolist() == exact
    assert thr[1] == ALWAYS and thr[2] == 0xFFFFFF00 and thr[3] == 0
    assert (thr[4:] < ALWAYS).all()
    with pytest.raises(ValueError):
        oracle.encode_ic(np.array([1.5], dtype=np.float32))


def test_lt_encoding_exact_rationals():
    g = graphs.rmat(9, 3000, seed=3)
    w = graphs.lt_uniform_weights(g, seed=4)
    cum = oracle.encode_lt(g.in_off, w)
    for v in range(g.n):
        s, e = int(g.in_off[v]), int(g.in_off[v + 1])
        if s == e:
            continue
        ws = [int(x) for x in w[s:e]]
        T = sum(ws)
        pref = np.cumsum(ws)
        for j in range(e - s - 1):
            assert int(cum[s + j]) == (int(pref[j]) << 32) // T
        assert int(cum[e - 1]) == ALWAYS
        assert all(cum[s + j] <= cum[s + j + 1] for j in range(e - s - 1))


# ---- P1 / P2 / P3 / P9: RR sets ---------------------------------------------------------
def test_p1_all_live_rr_set_is_root_plus_ancestors():
    for g in (graphs.erdos_renyi(300, 900, seed=5), graphs.rmat(8, 700, seed=6)):
        thr = oracle.encode_ic(np.ones(g.m, dtype=np.float32))
        G = nx_graph(g)
        for r in range(300):
            s, edges = oracle.rr_set(g, oracle.IC, thr, 77, r)
            root = oracle.root(77, r, g.n)
            assert s[0] == root
            assert set(s.tolist()) == nx.ancestors(G, root) | {root}
            assert len(set(s.tolist())) == len(s)
            assert edges == int(g.in_degree()[s].sum())


def test_p2_all_dead_sets_are_roots_and_greedy_takes_most_frequent():
    g = graphs.erdos_renyi(50, 400, seed=7)
    p = np.zeros(g.m, dtype=np.float32)
    pool = oracle.Pool(g, oracle.IC, 5, ic_p=p)
    pool.extend(3000)
    off, ids = pool.export()
    assert np.array_equal(off, np.arange(3001))
    roots = [oracle.root(5, r, g.n) for r in range(3000)]
    assert ids.tolist() == roots
    h = pool.hist()
    assert np.array_equal(h, np.bincount(roots, minlength=g.n))
    seeds, cov = pool.greedy(8)
    order = sorted(range(g.n), key=lambda v: (-int(h[v]), v))[:8]
    assert seeds.tolist() == order
    assert cov == sum(h[v] for v in order)


def _ic_world_set(g, thr, seed, r):
    """Materialise the live-edge instance of set r, then reverse reachability (networkx)."""
    dst = g.dst()
    live = []
    for e in range(g.m):
        x = philox_word(seed, r, e >> 2, 0, 2, e & 3)
        if thr[e] == ALWAYS or x < thr[e]:
            live.append((int(g.in_src[e]), int(dst[e])))
    W = nx.DiGraph()
    W.add_nodes_from(range(g.n))
    W.add_edges_from(live)
    root = oracle.root(seed, r, g.n)
    return nx.ancestors(W, root) | {root}


def test_p3_ic_set_equals_reverse_reach_in_materialised_world():
    g = graphs.erdos_renyi(120, 700, seed=8)
    rng = np.random.default_rng(9)
    p = (rng.random(g.m) * 0.6).astype(np.float32)
    thr = oracle.encode_ic(p)
    seed = 0xC0FFEE
    sizes = []
    for r in range(0, 4000, 40):
        s, _ = oracle.rr_set(g, oracle.IC, thr, seed, r)
        assert set(s.tolist()) == _ic_world_set(g, thr, seed, r), r
        sizes.append(len(s))
    assert max(sizes) > 5    # the sample includes non-trivial sets


def _lt_world_pick(g, cum, seed, r, v):
    s, e = int(g.in_off[v]), int(g.in_off[v + 1])
    if s == e:
        return None
    x = philox_word(seed, r, v, 0, 3, 0)
    for j in range(s, e):
        if cum[j] == ALWAYS or x < cum[j]:
            return int(g.in_src[j])
    return None


def test_p3_lt_set_equals_reverse_reach_in_materialised_world():
    g = graphs.rmat(7, 600, seed=10)
    w = graphs.lt_uniform_weights(g, seed=11)
    cum = oracle.encode_lt(g.in_off, w)
    seed = 31337
    for r in range(300):
        W = nx.DiGraph()
        W.add_nodes_from(range(g.n))
        for v in range(g.n):
            u = _lt_world_pick(g, cum, seed, r, v)
            if u is not None:
                W.add_edge(u, v)
        root = oracle.root(seed, r, g.n)
        s, edges = oracle.rr_set(g, oracle.LT, cum, seed, r)
        assert set(s.tolist()) == nx.ancestors(W, root) | {root}
        assert edges == int(g.in_degree()[s].sum())


def test_p6_lt_functional_graph_follows_unique_in_edge():
    n = 40
    rng = np.random.default_rng(12)
    parent = rng.integers(0, n, n)
    for v in range(n):
        if parent[v] == v:
            parent[v] = (v + 1) % n
    g = graphs.from_edges(n, parent.tolist(), list(range(n)))
    cum = oracle.encode_lt(g.in_off, None)
    for r in range(200):
        s, _ = oracle.rr_set(g, oracle.LT, cum, 3, r)
        v = oracle.root(3, r, n)
        walk = [v]
        while parent[walk[-1]] not in walk:
            walk.append(int(parent[walk[-1]]))
        assert s.tolist() == walk


def test_p9_invariants_on_c1():
    w = configs.c1()
    pool = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
    pool.extend(2000)
    off, ids = pool.export()
    G = nx_graph(w.graph)
    deg = w.graph.in_degree()
    assert (np.diff(off) >= 1).all()
    for r in range(0, 2000, 97):
        s = ids[off[r]:off[r + 1]]
        root = oracle.root(w.seed, r, w.graph.n)
        assert root in s
        assert (np.diff(s) > 0).all()                     # sorted, no duplicates
        assert set(s.tolist()) <= nx.ancestors(G, root) | {root}
    assert pool.hist().sum() == len(ids) == pool.total()
    assert pool.edges() == int(deg[ids].sum())


def test_p13_thread_count_does_not_change_results():
    w = configs.c1()
    outs = []
    for t in (1, 2, 5):
        pool = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
        pool.extend(1500, threads=t)
        pool.extend(4000, threads=t)
        outs.append(pool.export())
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    a = oracle.imm_solve(w.graph, 0, 5, 0.5, 1.0, w.seed, ic_p=w.ic_p, threads=1)
    b = oracle.imm_solve(w.graph, 0, 5, 0.5, 1.0, w.seed, ic_p=w.ic_p, threads=7)
    assert np.array_equal(a["seeds"], b["seeds"]) and a["theta"] == b["theta"]


# ---- P4 / P5: exact probabilities by enumeration of live-edge worlds ---------------------
def _tiny_graph():
    edges = [(0, 1), (1, 2), (2, 0), (3, 2), (4, 3), (5, 4), (6, 5), (0, 7), (7, 6), (2, 5),
             (1, 6)]
    return graphs.from_edges(8, [a for a, _ in edges], [b for _, b in edges])


def _ic_world_probs(g, thr):
    """Yield (probability, edge list) for every live-edge world (effective probabilities)."""
    q = [1.0 if t == ALWAYS else t / 2 ** 32 for t in thr.tolist()]
    dst = g.dst().tolist()
    src = g.in_src.tolist()
    for mask in range(1 << g.m):
        pr = 1.0
        live = []
        for e in range(g.m):
            if mask >> e & 1:
                pr *= q[e]
                live.append((src[e], dst[e]))
            else:
                pr *= 1.0 - q[e]
        if pr > 0:
            yield pr, live


def _reach_matrix(n, live):
    reach = [1 << v for v in range(n)]          # reach[u]: vertices u reaches
    changed = True
    while changed:
        changed = False
        for a, b in live:
            nr = reach[a] | reach[b]
            if nr != reach[a]:
                reach[a] = nr
                changed = True
    return reach


def test_p4_p5_ic_membership_and_ris_estimator_by_enumeration():
    g = _tiny_graph()
    p = np.array([0.3, 0.8, 0.5, 0.25, 0.6, 0.9, 0.4, 0.7, 0.2, 0.55, 0.35], dtype=np.float32)
    thr = oracle.encode_ic(p)
    n = g.n
    member = np.zeros(n)                 # Pr[u in RR] = (1/n) sum_v Pr[u reaches v]
    sets = [[0], [3], [0, 4], [2, 6], [1, 5, 7]]
    spread = np.zeros(len(sets))         # E[I(S)] by forward reachability
    for pr, live in _ic_world_probs(g, thr):
        reach = _reach_matrix(n, live)
        for u in range(n):
            member[u] += pr * bin(reach[u]).count("1") / n
        for i, S in enumerate(sets):
            acc = 0
            for u in S:
                acc |= reach[u]
            spread[i] += pr * bin(acc).count("1")
    theta = 200_000
    pool = oracle.Pool(g, oracle.IC, 0xBEEF, ic_p=p)
    pool.extend(theta)
    h = pool.hist().astype(float)
    z = (h / theta - member) / np.sqrt(member * (1 - member) / theta + 1e-300)
    assert np.abs(z).max() < 5.0, z
    # expected set size equals the sum of membership probabilities
    off, ids = pool.export()
    assert abs(len(ids) / theta - member.sum()) < 5 * np.sqrt(n * n / theta)
    # Eq. 3: E[I(S)] = n Pr[S meets RR]
    for i, S in enumerate(sets):
        hit = 0
        for r in range(theta):
            s = ids[off[r]:off[r + 1]]
            if np.intersect1d(s, S).size:
                hit += 1
        f = hit / theta
        est = n * f
        sd = n * math.sqrt(max(f * (1 - f), 1e-12) / theta)
        assert abs(est - spread[i]) < 5 * sd + 1e-9, (S, est, spread[i])


def test_p4_lt_membership_by_enumeration():
    g = _tiny_graph()
    w = np.array([3, 1, 2, 5, 1, 4, 2, 2, 7, 1, 3], dtype=np.uint32)
    cum = oracle.encode_lt(g.in_off, w)
    n = g.n
    choices = []                       # per vertex: list of (prob, chosen source or None)
    for v in range(n):
        s, e = int(g.in_off[v]), int(g.in_off[v + 1])
        opts, prev = [], 0
        for j in range(s, e):
            c = 2 ** 32 if cum[j] == ALWAYS else int(cum[j])
            opts.append(((c - prev) / 2 ** 32, int(g.in_src[j])))
            prev = c
        if prev < 2 ** 32:
            opts.append(((2 ** 32 - prev) / 2 ** 32, None))
        choices.append(opts)
    member = np.zeros(n)
    for combo in itertools.product(*choices):
        pr = 1.0
        live = []
        for v, (q, u) in enumerate(combo):
            pr *= q
            if u is not None:
                live.append((u, v))
        reach = _reach_matrix(n, live)
        for u in range(n):
            member[u] += pr * bin(reach[u]).count("1") / n
    theta = 200_000
    pool = oracle.Pool(g, oracle.LT, 0xFACE, lt_w=w)
    pool.extend(theta)
    h = pool.hist().astype(float)
    z = (h / theta - member) / np.sqrt(member * (1 - member) / theta + 1e-300)
    assert np.abs(z).max() < 5.0, z


# ---- P7: greedy --------------------------------------------------------------------------
def _recount_greedy(n, sets, k):
    """Alg. 1 lines 6-10 taken literally: recount membership over the remaining sets."""
    remaining = [set(s) for s in sets]
    chosen = []
    covered = 0
    for _ in range(k):
        counts = [0] * n
        for s in remaining:
            for v in s:
                counts[v] += 1
        best = max((v for v in range(n) if v not in chosen), key=lambda v: (counts[v], -v))
        chosen.append(best)
        keep = [s for s in remaining if best not in s]
        covered += len(remaining) - len(keep)
        remaining = keep
    return chosen, covered


def test_p7_greedy_against_recount_and_exhaustive_optimum():
    rng = np.random.default_rng(13)
    for trial in range(40):
        n = int(rng.integers(3, 16))
        nsets = int(rng.integers(1, 40))
        sets = [sorted(set(rng.integers(0, n, int(rng.integers(1, 5))).tolist()))
                for _ in range(nsets)]
        off = np.cumsum([0] + [len(s) for s in sets])
        ids = np.array([v for s in sets for v in s], dtype=np.int32)
        for k in (1, 2, 3):
            if k > n:
                continue
            seeds, cov = oracle.greedy_sets(n, off, ids, k)
            exp_seeds, exp_cov = _recount_greedy(n, sets, k)
            assert seeds.tolist() == exp_seeds and cov == exp_cov
            opt = max(sum(1 for s in sets if set(s) & set(c))
                      for c in itertools.combinations(range(n), k))
            if k == 1:
                assert cov == opt
            assert cov >= (1 - 1 / math.e) * opt - 1e-9
            assert len(set(seeds.tolist())) == k


def test_greedy_excludes_chosen_vertices_when_all_gains_are_zero():
    sets = [[2], [2], [2]]
    seeds, cov = oracle.greedy_sets(5, np.array([0, 1, 2, 3]), np.array([2, 2, 2], np.int32), 4)
    assert seeds.tolist() == [2, 0, 1, 3] and cov == 3


# ---- P8 / P14: sample-size formulas -----------------------------------------------------------
def _mp_quantities(n, k, eps, ell):
    mpmath.mp.dps = 60
    n_, k_ = mpmath.mpf(n), k
    ellp = ell * (1 + mpmath.log(2) / mpmath.log(n_))
    lnc = mpmath.log(mpmath.binomial(n, k_))
    ep = mpmath.sqrt(2) * eps
    lam1 = (2 + 2 * ep / 3) * (lnc + ellp * mpmath.log(n_) + mpmath.log(mpmath.log(n_, 2))) * n_ / ep ** 2
    e = mpmath.e
    a = mpmath.sqrt(ellp * mpmath.log(n_) + mpmath.log(2))
    b = mpmath.sqrt((1 - 1 / e) * (lnc + ellp * mpmath.log(n_) + mpmath.log(2)))
    lam2 = 2 * n_ * ((1 - 1 / e) * a + b) ** 2 / mpmath.mpf(eps) ** 2
    return lnc, lam1, lam2


@pytest.mark.parametrize("n,k,eps,ell", [
    (1000, 10, 0.5, 1.0), (1 << 20, 50, 0.1, 1.0), (1 << 22, 100, 0.1, 1.0),
    (1 << 24, 200, 0.05, 1.0), (75_879, 50, 0.05, 1.0), (4, 2, 0.3, 2.0)])
def test_p8_sample_sizes_against_mpmath(n, k, eps, ell):
    lnc, lam1, lam2 = _mp_quantities(n, k, eps, ell)
    assert abs(oracle.log_binom(n, k) - float(lnc)) <= 1e-9 * max(1.0, abs(float(lnc)))
    assert abs(oracle.lambda_prime(n, k, eps, ell) / float(lam1) - 1) < 1e-12
    assert abs(oracle.lambda_star(n, k, eps, ell) / float(lam2) - 1) < 1e-12
    assert oracle.imax(n) == int(mpmath.floor(mpmath.log(n, 2))) - 1


def test_p8_reference_magnitudes():
    assert round(oracle.lambda_prime(1000, 10, 0.5, 1.0) / 1e5, 3) == 3.155
    assert round(oracle.lambda_star(1000, 10, 0.5, 1.0) / 1e5, 3) == 5.238
    assert round(oracle.lambda_star(1 << 24, 200, 0.05, 1.0) / 1e13, 3) == 2.401


def test_p14_monotonicity():
    n = 1 << 16
    for k in (1, 10, 100):
        ls = [oracle.lambda_star(n, k, e, 1.0) for e in (0.05, 0.1, 0.2, 0.5)]
        assert all(a > b for a, b in zip(ls, ls[1:]))
    ks = [oracle.lambda_star(n, k, 0.1, 1.0) for k in (1, 2, 10, 100, 1000)]
    assert all(a < b for a, b in zip(ks, ks[1:]))


def test_imax_small_n():
    assert [oracle.imax(n) for n in (2, 3, 4, 7, 8, 1000, 1024, 1025)] == [0, 0, 1, 1, 2, 8, 9, 9]


# ---- the IMM driver: loop structure re-derived independently --------------------------------
def test_imm_driver_phase_structure_c1():
    """Re-run gIM Alg. 2 / Alg. 1 from mpmath sample sizes and the (pinned) greedy, and check
    the oracle driver's theta, LB and set count."""
    w = configs.c1()
    n, k, eps, ell = w.graph.n, w.k, w.eps, w.ell
    _, lam1, lam2 = _mp_quantities(n, k, eps, ell)
    pool = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
    ep = math.sqrt(2) * eps
    lb, used, phases = 1.0, 0, 0
    for i in range(1, int(mpmath.floor(mpmath.log(n, 2))) - 1 + 1):
        x = n / 2 ** i
        used = max(used, int(mpmath.ceil(lam1 / x)))
        pool.extend(used)
        _, cov = pool.greedy(k, 0, used)
        phases += 1
        if n * cov / used >= (1 + ep) * x:
            lb = n * cov / used / (1 + ep)
            break
    theta = int(mpmath.ceil(lam2 / lb))
    ref = oracle.imm_solve(w.graph, oracle.IC, k, eps, ell, w.seed, ic_p=w.ic_p)
    assert abs(ref["lb"] / lb - 1) < 1e-12
    assert ref["theta"] == theta
    assert ref["num_rr"] == max(used, theta)
    assert ref["phases"] == phases + 1


def _fresh_final_case(g, ic_p, k, eps, ell, seed):
    """gIM Alg. 2 then Alg. 1 with a fresh final sample, re-derived from mpmath sample sizes
    and the pinned pool / greedy: returns the expected (seeds, covered, theta, num_rr,
    phases, lb, spread_est) and the result greedy would give on the reuse reading."""
    n = g.n
    _, lam1, lam2 = _mp_quantities(n, k, eps, ell)
    pool = oracle.Pool(g, oracle.IC, seed, ic_p=ic_p)
    ep = math.sqrt(2) * eps
    lb, used, phases = 1.0, 0, 0
    for i in range(1, int(mpmath.floor(mpmath.log(n, 2))) - 1 + 1):
        x = n / 2 ** i
        used = max(used, int(mpmath.ceil(lam1 / x)))
        pool.extend(used)
        _, cov = pool.greedy(k, 0, used)
        phases += 1
        if n * cov / used >= (1 + ep) * x:
            lb = n * cov / used / (1 + ep)
            break
    theta = int(mpmath.ceil(lam2 / lb))
    # the final sample: fresh indices [|R_est|, |R_est| + theta), selected on their own
    pool.extend(used + theta)
    off, ids = pool.export(used, theta)
    seeds, cov = oracle.greedy_sets(n, off, ids, k)
    off0, ids0 = pool.export(0, used + theta)
    reuse = oracle.greedy_sets(n, off0, ids0, k)
    return dict(seeds=seeds, covered=cov, theta=theta, num_rr=used + theta, phases=phases + 1,
                lb=lb, spread_est=n * cov / theta), reuse


@pytest.mark.parametrize("case", ["c1", "tiny"])
def test_imm_driver_fresh_final_sample(case):
    """fresh_final = 1 (the corrected IMM of Chen, CSoNet'18; reading of gIM Alg. 1): the
    final theta sets are indices [|R_est|, |R_est| + theta), disjoint from the estimation
    sets, and greedy runs on exactly those.  The driver's seeds, covered count, set count
    and estimate must equal the re-derivation; the reuse reading ([0, upto)) must not."""
    if case == "c1":
        w = configs.c1()
        g, p, k, eps, ell, seed = w.graph, w.ic_p, w.k, w.eps, w.ell, w.seed
    else:
        g = _tiny_graph()
        p = np.array([0.3, 0.8, 0.5, 0.25, 0.6, 0.9, 0.4, 0.7, 0.2, 0.55, 0.35], dtype=np.float32)
        k, eps, ell, seed = 2, 0.3, 1.0, 0x5EED00F1
    exp, reuse = _fresh_final_case(g, p, k, eps, ell, seed)
    got = oracle.imm_solve(g, oracle.IC, k, eps, ell, seed, ic_p=p, fresh_final=True)
    assert got["seeds"].tolist() == exp["seeds"].tolist()
    assert got["covered"] == exp["covered"]
    assert got["theta"] == exp["theta"]
    assert got["num_rr"] == exp["num_rr"]
    assert got["phases"] == exp["phases"]
    assert abs(got["lb"] / exp["lb"] - 1) < 1e-12
    assert got["spread_est"] == exp["spread_est"]
    # the test tells the readings apart: the reuse range gives another answer
    assert (reuse[0].tolist(), reuse[1]) != (exp["seeds"].tolist(), exp["covered"])
    plain = oracle.imm_solve(g, oracle.IC, k, eps, ell, seed, ic_p=p, fresh_final=False)
    assert plain["num_rr"] == max(exp["num_rr"] - exp["theta"], exp["theta"])


# ---- P11: end-to-end approximation guarantee on a tiny graph ----------------------------------
def test_p11_imm_meets_guarantee_on_tiny_graph():
    g = _tiny_graph()
    p = np.array([0.3, 0.8, 0.5, 0.25, 0.6, 0.9, 0.4, 0.7, 0.2, 0.55, 0.35], dtype=np.float32)
    thr = oracle.encode_ic(p)
    n, k, eps = g.n, 2, 0.3
    worlds = [(pr, _reach_matrix(n, live)) for pr, live in _ic_world_probs(g, thr)]

    def spread(S):
        tot = 0.0
        for pr, reach in worlds:
            acc = 0
            for u in S:
                acc |= reach[u]
            tot += pr * bin(acc).count("1")
        return tot

    opt = max(spread(c) for c in itertools.combinations(range(n), k))
    fails = 0
    for s in range(100):
        res = oracle.imm_solve(g, oracle.IC, k, eps, 1.0, 1000 + s, ic_p=p)
        if spread(res["seeds"].tolist()) < (1 - 1 / math.e - eps) * opt:
            fails += 1
    assert fails <= 100 / n + 3
