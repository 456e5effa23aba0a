"""GPU parity: every result of the HIP path equals the CPU oracle's, bit for bit.

Integer results (thresholds, RR sets, occurrence counts, seeds, covered counts, edge counts)
and the double-precision IMM quantities (lambda', lambda*, LB, theta) are compared exactly:
under the shared Philox contract there is exactly one correct answer.
"""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu


def _gpu_graph(imm, g, ic_p=None, lt_w=None, lt=False):
    return imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=lt_w, lt=lt)


def _compare_pool(imm, g, model, seed, count, ic_p=None, lt_w=None, chunks=None):
    gg = _gpu_graph(imm, g, ic_p=ic_p, lt_w=lt_w, lt=(model == imm.IMM_LT))
    pool = imm.Pool.create(gg, model, seed)
    for upto in (chunks or [count]):
        imm.imm_generate_rr(pool.handle, upto)
    off_g, ids_g = imm.imm_rr_export(pool.handle, 0, count)
    ref = oracle.Pool(g, model, seed, ic_p=ic_p, lt_w=lt_w)
    ref.extend(count)
    off_o, ids_o = ref.export()
    assert np.array_equal(off_g, off_o), "set sizes differ"
    assert np.array_equal(ids_g, ids_o), "set members differ"
    hist_g = imm.imm_rr_histogram(pool.handle, 0, count, g.n)
    assert np.array_equal(hist_g, ref.hist())
    n_sets, n_ids, edges = imm.imm_pool_size(pool.handle)
    assert n_sets == count and n_ids == ref.total() and edges == ref.edges()
    return pool, ref


def test_ic_encoding_matches_oracle(imm_gpu):
    g = graphs.erdos_renyi(3000, 40_000, seed=11)
    rng = np.random.default_rng(5)
    p = rng.random(g.m).astype(np.float32)
    p[::7] = 0.0
    p[::11] = 1.0
    p[::13] = np.float32(1.0) - np.float32(2.0 ** -24)
    p[::17] = np.float32(2.0 ** -40)
    gg = _gpu_graph(imm_gpu, g, ic_p=p)
    thr, _ = imm_gpu.imm_graph_export_encoding(gg.handle, ic=True)
    assert np.array_equal(thr, oracle.encode_ic(p))


def test_wc_encoding_full_size_c2(imm_gpu):
    w = configs.c2()
    gg = _gpu_graph(imm_gpu, w.graph, ic_p=w.ic_p)
    thr, _ = imm_gpu.imm_graph_export_encoding(gg.handle, ic=True)
    assert np.array_equal(thr, oracle.encode_ic(w.ic_p))


@pytest.mark.parametrize("unit", [False, True])
def test_lt_encoding_matches_oracle(imm_gpu, unit):
    g = graphs.rmat(12, 60_000, seed=21)
    w = None if unit else graphs.lt_uniform_weights(g, seed=22)
    gg = _gpu_graph(imm_gpu, g, lt_w=w, lt=True)
    _, cum = imm_gpu.imm_graph_export_encoding(gg.handle, ic=False, lt=True)
    assert np.array_equal(cum, oracle.encode_lt(g.in_off, w))


def test_rr_sets_ic_c1(imm_gpu):
    w = configs.c1()
    _compare_pool(imm_gpu, w.graph, imm_gpu.IMM_IC, w.seed, 6000, ic_p=w.ic_p)


def test_rr_sets_ic_rmat_wc_chunked(imm_gpu):
    g = graphs.rmat(15, 16 << 15, seed=31)
    p = graphs.weighted_cascade(g)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 0xABCDEF0123, 30_000, ic_p=p,
                  chunks=[1, 777, 10_000, 30_000])


def test_rr_sets_ic_per_edge_thresholds(imm_gpu):
    g = graphs.rmat(13, 12 << 13, seed=41)
    p = graphs.trivalency(g, seed=42)
    p[::5] = np.float32(0.5)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 99, 20_000, ic_p=p)


@pytest.mark.parametrize("block,budget", [("256", None), ("1024", None), ("256", "16")])
def test_rr_sets_ic_bounded_heavy_lists(imm_gpu, monkeypatch, block, budget):
    """Heavy member lists bounded to 1024 entries (as on huge graphs, where full lists would
    leave too few slots): a set that outgrows its list is dropped and drawn again from its
    root in a full list.  Sets, histogram and in-edges examined must equal the oracle's
    (p = 0.12 on a random graph: ~600 of 2000 sets exceed 1024 members, a few dozen fall
    between 64 and 1024), and a solve must report sets drawn again."""
    monkeypatch.setenv("IMM_HEAVY_LIST", "1024")
    monkeypatch.setenv("IMM_HEAVY_BLOCK", block)
    if budget:
        monkeypatch.setenv("IMM_LIGHT_BUDGET", budget)
    g = graphs.erdos_renyi(5000, 50_000, seed=51)
    p = np.full(g.m, 0.12, dtype=np.float32)
    _, ref = _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 0x5EED0601, 2000, ic_p=p, chunks=[300, 2000])
    sizes = np.diff(ref.export()[0])
    assert (sizes > 1024).sum() > 500 and ((sizes > 64) & (sizes <= 1024)).sum() > 10
    _, info, _ = _solve_both(imm_gpu, g, imm_gpu.IMM_IC, 5, 0.5, 1.0, 0x5EED0602,
                             ic_p=np.full(g.m, 0.15, dtype=np.float32))
    assert info["heavy_redrawn"] > 0


@pytest.mark.parametrize("budget", ["2", "16"])
def test_rr_sets_ic_handoff(imm_gpu, monkeypatch, budget):
    """A light budget of a few 4-edge groups: almost every set with more than one level is
    abandoned by the light kernel at a level boundary and resumed by the heavy kernel
    from there (handoff).  Sets, histogram and in-edges examined must equal the oracle's,
    in chunked launches and with per-edge thresholds."""
    monkeypatch.setenv("IMM_LIGHT_BUDGET", budget)
    g = graphs.rmat(13, 12 << 13, seed=43)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 0x5EED0401, 6000, ic_p=graphs.weighted_cascade(g),
                  chunks=[100, 2500, 6000])
    p = graphs.trivalency(g, seed=44)
    p[::5] = np.float32(0.5)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 0x5EED0402, 8000, ic_p=p)
    w = configs.c1()
    _, info, _ = _solve_both(imm_gpu, w.graph, imm_gpu.IMM_IC, w.k, w.eps, w.ell, w.seed,
                             ic_p=w.ic_p)
    assert info["rr_heavy_launches"] > 0 and info["edges_heavy"] > 0


def _wide_handoff_graph():
    """Hub 0 has 300 in-neighbours 1..300; each of those has in-edges from 301 and 302;
    every other vertex (and 301, 302) has an in-edge from the hub.  A root outside 1..302
    reaches the hub at level 1 and its 300 in-neighbours at level 2, so a light budget of
    100 4-edge groups abandons the set with 300 unexpanded members (more than the heavy
    kernel's 256-entry record ring), whose expansion finds only two new members."""
    n, hub, wide = 1000, 0, 300
    src, dst = [], []
    for u in range(1, wide + 1):
        src.append(u); dst.append(hub)
        src.extend([wide + 1, wide + 2]); dst.extend([u, u])
    for v in range(wide + 1, n):
        src.append(hub); dst.append(v)
    return graphs.from_edges(n, src, dst)


@pytest.mark.parametrize("block", ["64", "256"])
def test_rr_sets_ic_handoff_wide_level(imm_gpu, monkeypatch, block):
    """Handoff of a set whose unexpanded members outnumber the heavy kernel's record ring:
    every member the heavy kernel expands must use its own vertex record.  Single pools
    (all edges live; every edge live with probability 0.97) and a batch of two instances
    must equal the oracle."""
    imm = imm_gpu
    monkeypatch.setenv("IMM_LIGHT_BUDGET", "100")
    monkeypatch.setenv("IMM_HEAVY_BLOCK", block)
    g = _wide_handoff_graph()
    p1 = np.ones(g.m, dtype=np.float32)
    p2 = np.full(g.m, 0.97, dtype=np.float32)
    for p, seed in ((p1, 0x5EED0501), (p2, 0x5EED0502)):
        pool, ref = _compare_pool(imm, g, imm.IMM_IC, seed, 3000, ic_p=p, chunks=[700, 3000])
        off, _ = ref.export()
        assert (np.diff(off) > 256).sum() > 1000
    gg1 = _gpu_graph(imm, g, ic_p=p1)
    gg2 = _gpu_graph(imm, g, ic_p=p2)
    items = [dict(graph=gg1, k=5, eps=0.5, ell=1.0, model=imm.IMM_IC, seed=0x5EED0503),
             dict(graph=gg2, k=3, eps=0.4, ell=1.0, model=imm.IMM_IC, seed=0x5EED0504)]
    stats = {}
    res = imm.imm_batch_solve(items, stats=stats)
    assert stats["rr_heavy_launches"] > 0
    for (seeds, info), it, p in zip(res, items, (p1, p2)):
        ref = oracle.imm_solve(g, oracle.IC, it["k"], it["eps"], 1.0, it["seed"], ic_p=p)
        assert np.array_equal(seeds, ref["seeds"])
        assert info["theta"] == ref["theta"] and info["covered"] == ref["covered"]
        assert info["num_rr"] == ref["num_rr"] and info["lb"] == ref["lb"]


def test_rr_sets_ic_big_sets(imm_gpu):
    """p = 1 everywhere on a dense ER graph: RR(r) = all ancestors of the root, thousands
    of vertices, beyond the on-chip member list, so the HBM big-set path runs."""
    g = graphs.erdos_renyi(5000, 50_000, seed=51)
    p = np.ones(g.m, dtype=np.float32)
    pool, ref = _compare_pool(imm_gpu, g, imm_gpu.IMM_IC, 7, 300, ic_p=p)
    off, _ = ref.export()
    assert np.diff(off).max() > 2048


@pytest.mark.parametrize("unit", [False, True])
def test_rr_sets_lt(imm_gpu, unit):
    g = graphs.rmat(14, 16 << 14, seed=61)
    w = None if unit else graphs.lt_uniform_weights(g, seed=62)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_LT, 0x5EED0003, 40_000, lt_w=w,
                  chunks=[5, 40_000])


def test_rr_sets_lt_long_walks(imm_gpu):
    """A functional graph (one in-edge per vertex, a long cycle plus hubs) gives long walks
    and exercises the search over long in-lists."""
    n = 6000
    src = list(range(1, n)) + [0]
    dst = list(range(0, n - 1)) + [n - 1]
    rng = np.random.default_rng(3)
    hubs = rng.integers(0, n, 200)
    for h in hubs:          # vertex h gets many in-edges -> long in-lists
        for u in rng.choice(n, 300, replace=False):
            if u != h and u != (h + 1) % n:
                src.append(int(u)); dst.append(int(h))
    g = graphs.from_edges(n, src, dst)
    w = graphs.lt_uniform_weights(g, seed=64)
    _compare_pool(imm_gpu, g, imm_gpu.IMM_LT, 1234, 3000, lt_w=w)


@pytest.mark.parametrize("lds_cap,ext_cap", [(4, 16), (1, 0), (32, 1)])
def test_rr_sets_lt_extension_lists(imm_gpu, monkeypatch, lds_cap, ext_cap):
    """First-pass walks past the LDS list continue in the group's extension list in HBM,
    and walks past both are redrawn by the HBM-list kernel; small list capacities force
    both paths on ordinary walks (the defaults hold 256 + 1024 members)."""
    monkeypatch.setenv("IMM_LT_LDS_CAP", str(lds_cap))
    monkeypatch.setenv("IMM_LT_EXT_CAP", str(ext_cap))
    g = graphs.rmat(14, 16 << 14, seed=61)
    w = graphs.lt_uniform_weights(g, seed=62)
    _, ref = _compare_pool(imm_gpu, g, imm_gpu.IMM_LT, 0x5EED0013, 20_000, lt_w=w,
                           chunks=[3, 20_000])
    sizes = np.diff(ref.export()[0])
    assert (sizes > lds_cap).sum() > 100 and (sizes > lds_cap + ext_cap).sum() > 10


@pytest.mark.parametrize("first,count,k", [(0, 5000, 10), (1000, 3000, 25), (0, 5000, 1000)])
def test_select_matches_oracle(imm_gpu, first, count, k):
    w = configs.c1()
    gg = _gpu_graph(imm_gpu, w.graph, ic_p=w.ic_p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, w.seed)
    imm_gpu.imm_generate_rr(pool.handle, first + count)
    seeds_g, cov_g = imm_gpu.imm_select_seeds(pool.handle, first, count, k)
    ref = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
    ref.extend(first + count)
    seeds_o, cov_o = ref.greedy(k, first, count)
    assert np.array_equal(seeds_g, seeds_o)
    assert cov_g == cov_o
    assert len(set(seeds_g.tolist())) == k


@pytest.mark.parametrize("bucketed", ["0", "1"])
def test_select_index_builds_match_oracle(imm_gpu, monkeypatch, bucketed):
    """Both inverted-index builds: per-entry atomics (IMM_INV_BUCKETED=0, the form graphs
    of more than 2^25 vertices take) and vertex buckets (the default), on growing prefixes
    (index segments) of one pool, each selection against the oracle's greedy."""
    monkeypatch.setenv("IMM_INV_BUCKETED", bucketed)
    g = graphs.rmat(14, 12 << 14, seed=92)
    ic_p = graphs.weighted_cascade(g)
    gg = _gpu_graph(imm_gpu, g, ic_p=ic_p)
    seed = 0x5EED0302
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=ic_p)
    for end in (3000, 7000, 12000):
        imm_gpu.imm_generate_rr(pool.handle, end)
        ref.extend(end)
        seeds_g, cov_g = imm_gpu.imm_select_seeds(pool.handle, 0, end, 20)
        seeds_o, cov_o = ref.greedy(20, 0, end)
        assert np.array_equal(seeds_g, seeds_o), end
        assert cov_g == cov_o, end


def test_select_growing_prefixes_match_oracle(imm_gpu):
    """Selections over longer and longer prefixes of one pool read the inverted index as
    segments (one per batch of new sets, more segments than a solve makes); every
    selection must equal the oracle's greedy and a fresh pool's single-segment one."""
    g = graphs.rmat(12, 12 << 12, seed=91)
    ic_p = graphs.weighted_cascade(g)
    gg = _gpu_graph(imm_gpu, g, ic_p=ic_p)
    seed = 0x5EED0301
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=ic_p)
    ends = [500, 700, 1000, 1600, 2600, 4000] + [4000 + 300 * i for i in range(1, 14)]
    for end in ends:
        imm_gpu.imm_generate_rr(pool.handle, end)
        seeds_g, cov_g = imm_gpu.imm_select_seeds(pool.handle, 0, end, 15)
        ref.extend(end)
        seeds_o, cov_o = ref.greedy(15, 0, end)
        assert np.array_equal(seeds_g, seeds_o), end
        assert cov_g == cov_o, end
    fresh = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    imm_gpu.imm_generate_rr(fresh.handle, ends[-1])
    seeds_f, cov_f = imm_gpu.imm_select_seeds(fresh.handle, 0, ends[-1], 15)
    assert np.array_equal(seeds_f, seeds_g) and cov_f == cov_g


def _solve_both(imm, g, model, k, eps, ell, seed, ic_p=None, lt_w=None, fresh=False):
    gg = _gpu_graph(imm, g, ic_p=ic_p, lt_w=lt_w, lt=(model == imm.IMM_LT))
    seeds_g, info = imm.imm_solve(gg.handle, k, eps, ell, model, seed, fresh_final=fresh)
    ref = oracle.imm_solve(g, model, k, eps, ell, seed, ic_p=ic_p, lt_w=lt_w, fresh_final=fresh)
    assert np.array_equal(seeds_g, ref["seeds"])
    for key in ("theta", "num_rr", "covered", "phases"):
        assert info[key] == ref[key], key
    assert info["edges_examined"] == ref["edges"]
    assert info["pool_ids"] == ref["pool_ids"]
    assert info["lb"] == ref["lb"]
    assert info["spread_est"] == ref["spread_est"]
    assert info["lambda_prime"] == ref["lambda_prime"]
    assert info["lambda_star"] == ref["lambda_star"]
    return seeds_g, info, ref


def test_solve_c1_matches_oracle(imm_gpu):
    w = configs.c1()
    _solve_both(imm_gpu, w.graph, imm_gpu.IMM_IC, w.k, w.eps, w.ell, w.seed, ic_p=w.ic_p)


def test_solve_c1_fresh_final_matches_oracle(imm_gpu):
    w = configs.c1()
    _solve_both(imm_gpu, w.graph, imm_gpu.IMM_IC, w.k, w.eps, w.ell, w.seed, ic_p=w.ic_p,
                fresh=True)


def test_solve_lt_small_matches_oracle(imm_gpu):
    g = graphs.rmat(12, 16 << 12, seed=71)
    w = graphs.lt_uniform_weights(g, seed=72)
    _solve_both(imm_gpu, g, imm_gpu.IMM_LT, 20, 0.3, 1.0, 0x5EED0003, lt_w=w)


def test_solve_pool_prefix_reuse(imm_gpu):
    """Queries against one shared pool return what independent solves return."""
    w = configs.c1()
    gg = _gpu_graph(imm_gpu, w.graph, ic_p=w.ic_p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, w.seed)
    for k, eps in [(10, 0.5), (5, 0.3), (20, 0.5), (10, 0.5)]:
        s_pool, i_pool = imm_gpu.imm_solve_pool(pool.handle, k, eps, 1.0)
        s_alone, i_alone = imm_gpu.imm_solve(gg.handle, k, eps, 1.0, imm_gpu.IMM_IC, w.seed)
        assert np.array_equal(s_pool, s_alone)
        assert i_pool["theta"] == i_alone["theta"] and i_pool["covered"] == i_alone["covered"]


def test_solve_after_cache_release_matches(imm_gpu):
    """Releasing the cached device blocks and pinned host buffers between solves changes
    nothing: the next solve allocates afresh and returns the same seeds and coverage."""
    w = configs.c1()
    gg = _gpu_graph(imm_gpu, w.graph, ic_p=w.ic_p)
    s1, i1 = imm_gpu.imm_solve(gg.handle, w.k, w.eps, w.ell, imm_gpu.IMM_IC, w.seed)
    imm_gpu.imm_release_cached_memory()
    s2, i2 = imm_gpu.imm_solve(gg.handle, w.k, w.eps, w.ell, imm_gpu.IMM_IC, w.seed)
    imm_gpu.imm_release_cached_memory()
    assert np.array_equal(s1, s2)
    assert i1["theta"] == i2["theta"] and i1["covered"] == i2["covered"]
