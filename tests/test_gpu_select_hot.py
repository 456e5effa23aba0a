"""Greedy selection in hot mode against the oracle.

A single-instance selection keeps exact counts only for its most frequent vertices (the
hot set: every vertex whose initial count exceeds a threshold C chosen so that at most T
vertices do) while the best hot count exceeds C, since no other count can then be larger;
the first round where it does not, every count is recounted exactly and the selection
continues over all vertices.  T is forced small here (IMM_SELECT_HOT) so that small pools
run both the hot rounds and the recount; which of the two a case reaches is derived from
the oracle's own counts and gains (the recount happens in the first round whose gain is at
most C), and every selection is compared with the oracle's greedy (gIM Alg. 1, Alg. 7)."""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu


def _threshold(h0: np.ndarray, T: int):
    """The hot threshold C of the selection: the smallest c in [0, 4094] with at most T
    counts above it (None: no hot set)."""
    h0 = np.asarray(h0, dtype=np.int64)
    above = np.array([(h0 > c).sum() for c in range(4095)])
    ok = np.nonzero(above <= T)[0]
    return int(ok[0]) if len(ok) else None


def _gains(ref, k: int, first: int, count: int) -> np.ndarray:
    """Per-round gains of the oracle's greedy (greedy is prefix-consistent in k)."""
    cov = [0] + [ref.greedy(j, first, count)[1] for j in range(1, k + 1)]
    return np.diff(np.asarray(cov, dtype=np.int64))


def _recount_round(ref, T, k, first, count):
    C = _threshold(ref.hist(first, count), T)
    if C is None:
        return None, None
    g = _gains(ref, k, first, count)
    late = np.nonzero(g <= C)[0]
    return C, (int(late[0]) if len(late) else None)


@pytest.mark.parametrize("T,k,first,count", [(8, 60, 0, 6000), (64, 60, 0, 6000),
                                             (256, 60, 0, 6000), (16, 40, 1000, 3000)])
def test_hot_mode_with_recount_c1(imm_gpu, monkeypatch, T, k, first, count):
    """Flat (Erdos-Renyi) graph: the hot set stops sufficing after a few rounds."""
    monkeypatch.setenv("IMM_SELECT_HOT", str(T))
    w = configs.c1()
    gg = imm_gpu.Graph.from_arrays(w.graph.n, w.graph.in_off, w.graph.in_src, ic_p=w.ic_p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, w.seed)
    imm_gpu.imm_generate_rr(pool.handle, first + count)
    ref = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
    ref.extend(first + count)
    C, late = _recount_round(ref, T, k, first, count)
    assert C is not None and late is not None and late >= 1   # hot rounds, then the recount
    seeds, cov = imm_gpu.imm_select_seeds(pool.handle, first, count, k)
    seeds_o, cov_o = ref.greedy(k, first, count)
    assert np.array_equal(seeds, seeds_o) and cov == cov_o
    seeds_n, cov_n = imm_gpu.imm_select_seeds_noalloc(pool.handle, first, count, k)
    assert np.array_equal(seeds_n, seeds_o) and cov_n == cov_o


@pytest.mark.parametrize("T", [None, 4096, 64])
def test_hot_mode_skewed_rmat(imm_gpu, monkeypatch, T):
    """R-MAT (skewed): with the default hot set (16384 of 65536 vertices) every round stays
    in hot mode; a small one ends in the recount."""
    if T is None:
        monkeypatch.delenv("IMM_SELECT_HOT", raising=False)
    else:
        monkeypatch.setenv("IMM_SELECT_HOT", str(T))
    g = graphs.rmat(16, 16 << 16, seed=93)
    p = graphs.weighted_cascade(g)
    seed, count, k = 0x5EED0404, 20_000, 30
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    imm_gpu.imm_generate_rr(pool.handle, count)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=p)
    ref.extend(count)
    C, late = _recount_round(ref, 16384 if T is None else T, k, 0, count)
    assert C is not None
    if T is None:
        assert late is None                       # hot mode throughout
    seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, count, k)
    seeds_o, cov_o = ref.greedy(k, 0, count)
    assert np.array_equal(seeds, seeds_o) and cov == cov_o


def test_hot_mode_growing_prefixes(imm_gpu, monkeypatch):
    """Selections over longer prefixes of one pool (inverted index kept as segments) in hot
    mode, each against the oracle."""
    monkeypatch.setenv("IMM_SELECT_HOT", "128")
    g = graphs.rmat(12, 12 << 12, seed=91)
    p = graphs.weighted_cascade(g)
    seed = 0x5EED0301
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=p)
    for end in (500, 1000, 2600, 4000, 5200):
        imm_gpu.imm_generate_rr(pool.handle, end)
        ref.extend(end)
        seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, end, 25)
        seeds_o, cov_o = ref.greedy(25, 0, end)
        assert np.array_equal(seeds, seeds_o) and cov == cov_o, end


@pytest.mark.parametrize("T", [32, 512])
def test_hot_mode_multi_round_partition(imm_gpu, monkeypatch, T):
    """Multi-round pool (partition matroid over rounds) in hot mode."""
    monkeypatch.setenv("IMM_SELECT_HOT", str(T))
    g = graphs.rmat(12, 40_000, seed=71)
    p = graphs.weighted_cascade(g)
    rounds, k, count, seed = 3, 8, 3000, 0x5EED7102
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    pool = imm_gpu.Pool.create_mr(gg, imm_gpu.IMM_IC, seed, rounds)
    imm_gpu.imm_generate_rr(pool.handle, count)
    seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, count, k, rounds=rounds)
    off, ids, _ = oracle.mr_sets(g, oracle.IC, seed, rounds, count, ic_p=p)
    seeds_o, cov_o = oracle.greedy_partition(g.n, rounds, off, ids, k)
    assert np.array_equal(seeds, seeds_o) and cov == cov_o


@pytest.mark.parametrize("dense", ["1", "300"])
@pytest.mark.parametrize("T", [None, 64])
def test_dense_rounds_match_oracle(imm_gpu, monkeypatch, dense, T):
    """Dense rounds: each block counts its decrements of hot vertices per hot position in
    LDS, stores the counts as its row of a grid-wide table, and the next argmax subtracts the
    column sums from the hot counters.  Forced for every hot round (gain >= 1) or for the
    rounds with a large gain only, with the default hot set (hot mode throughout) and a small
    one (dense rounds, then the recount); against the oracle's greedy and the selection with
    dense rounds off."""
    if T is None:
        monkeypatch.delenv("IMM_SELECT_HOT", raising=False)
    else:
        monkeypatch.setenv("IMM_SELECT_HOT", str(T))
    g = graphs.rmat(16, 16 << 16, seed=93)
    p = graphs.weighted_cascade(g)
    seed, count, k = 0x5EED0404, 20_000, 30
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    imm_gpu.imm_generate_rr(pool.handle, count)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=p)
    ref.extend(count)
    gains = _gains(ref, k, 0, count)
    assert (gains >= int(dense)).sum() >= 2           # some rounds are dense
    monkeypatch.setenv("IMM_SELECT_DENSE", dense)
    seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, count, k)
    seeds_o, cov_o = ref.greedy(k, 0, count)
    assert np.array_equal(seeds, seeds_o) and cov == cov_o
    monkeypatch.setenv("IMM_SELECT_DENSE", "0")
    seeds_0, cov_0 = imm_gpu.imm_select_seeds(pool.handle, 0, count, k)
    assert np.array_equal(seeds_0, seeds_o) and cov_0 == cov_o


def test_dense_rounds_growing_prefixes(imm_gpu, monkeypatch):
    """Dense rounds over longer prefixes of one pool (index segments), each against the
    oracle."""
    monkeypatch.setenv("IMM_SELECT_HOT", "128")
    monkeypatch.setenv("IMM_SELECT_DENSE", "1")
    g = graphs.rmat(12, 12 << 12, seed=91)
    p = graphs.weighted_cascade(g)
    seed = 0x5EED0301
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, seed)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=p)
    for end in (500, 1000, 2600, 4000, 5200):
        imm_gpu.imm_generate_rr(pool.handle, end)
        ref.extend(end)
        seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, end, 25)
        seeds_o, cov_o = ref.greedy(25, 0, end)
        assert np.array_equal(seeds, seeds_o) and cov == cov_o, end
