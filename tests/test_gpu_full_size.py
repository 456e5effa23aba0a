"""GPU parity on the code paths that full-size workloads take.

* Selection over 2^22 vertices: 1024 argmax tiles of 4096 counters, so each block of the
  cooperative launch loads a group of four tiles of one instance (gIM Sec. III-H's max
  reduction, Alg. 7's cover step), against the oracle's greedy (gIM Alg. 1).
* A batch whose instances have more than 256 argmax tiles in total, so blocks reduce
  tiles of two different instances in one round.
* Whole IMM solves at full size (R-MAT scale 20 / WC IC / k = 50 and R-MAT scale 22 /
  LT / k = 100, both eps = 0.1) against results the oracle alone produced
  (tests/golden/make_full_size.py).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from conftest import ROOT
from synth import configs, graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _select_both(imm, g, ic_p, seed, count, k):
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p)
    pool = imm.Pool.create(gg, imm.IMM_IC, seed)
    imm.imm_generate_rr(pool.handle, count)
    seeds_g, cov_g = imm.imm_select_seeds(pool.handle, 0, count, k)
    ref = oracle.Pool(g, oracle.IC, seed, ic_p=ic_p)
    ref.extend(count)
    off, ids = ref.export()
    seeds_o, cov_o = oracle.greedy_sets(g.n, off, ids, k)
    assert np.array_equal(seeds_g, seeds_o), (seeds_g[:8], seeds_o[:8])
    assert cov_g == cov_o
    return seeds_o, ref


@pytest.fixture(scope="module")
def big_sparse():
    g = graphs.rmat(22, 1 << 22, seed=0xB16)
    return g


@pytest.mark.parametrize("k", [1, 20])
def test_select_grouped_argmax_tiles_wc(imm_gpu, big_sparse, k):
    """R-MAT with 2^22 vertices and average in-degree 1, weighted cascade: hubs sit at
    random ids across all tiles."""
    g = big_sparse
    _select_both(imm_gpu, g, graphs.weighted_cascade(g), 0x5EED0701, 200_000, k)


@pytest.mark.parametrize("k", [1, 20])
def test_select_grouped_argmax_tiles_ties(imm_gpu, big_sparse, k):
    """Every edge dead: each set is its root, so the counts are root multiplicities (0, 1,
    2, ... over 2^22 vertices) and almost every round is decided by the smallest-id rule
    among equal counts held in different tiles and blocks."""
    g = big_sparse
    p = np.zeros(g.m, dtype=np.float32)
    seeds, ref = _select_both(imm_gpu, g, p, 0x5EED0702, 300_000, k)
    h = ref.hist()
    top = h[seeds]
    assert (np.diff(top.astype(np.int64)) <= 0).all()
    if k > 1:
        assert (h[seeds[-1]] == h).sum() > 1      # the last round was a tie


def test_batch_more_than_256_tiles_matches_oracle(imm_gpu):
    """65 instances of 12,289..16,384 vertices (four argmax tiles each, 260 in total):
    some blocks of the cooperative selection reduce tiles of two instances per round."""
    imm = imm_gpu
    rng = np.random.default_rng(0x7135)
    items, refs = [], []
    for i in range(65):
        n = int(rng.integers(12_289, 16_385))
        g = graphs.rmat(14, 4 * n, seed=2000 + i, n=n)
        p = graphs.weighted_cascade(g)
        gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=p)
        k, eps = int(rng.integers(2, 16)), float(rng.choice([0.5, 0.4]))
        seed = 0x5EED2000 + i
        items.append(dict(graph=gg, k=k, eps=eps, ell=1.0, model=imm.IMM_IC, seed=seed))
        refs.append((g, p, k, eps, seed))
    tiles = sum((it["graph"].n + 4095) // 4096 for it in items)
    assert tiles > 256
    res = imm.imm_batch_solve(items)
    for (seeds, info), (g, p, k, eps, seed) in zip(res, refs):
        ref = oracle.imm_solve(g, oracle.IC, k, eps, 1.0, seed, ic_p=p)
        assert np.array_equal(seeds, ref["seeds"]), seed
        for key in ("theta", "covered", "num_rr", "phases"):
            assert info[key] == ref[key], (seed, key)
        assert info["lb"] == ref["lb"]


def _input_digest(w):
    h = hashlib.sha256()
    for a in (w.graph.in_off, w.graph.in_src, w.ic_p, w.lt_w):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_solve_matches_oracle_golden(imm_gpu, name):
    imm = imm_gpu
    gold = json.load(open(os.path.join(GOLDEN, f"full_size_{name}.json")))
    w = {"c2": configs.c2, "c3": configs.c3}[name]()
    assert _input_digest(w) == gold["input_sha256"], "synthetic inputs differ from the golden's"
    model = imm.IMM_IC if w.model == "IC" else imm.IMM_LT
    gg = imm.Graph.from_arrays(w.graph.n, w.graph.in_off, w.graph.in_src, ic_p=w.ic_p,
                               lt_w=w.lt_w, lt=(w.model == "LT"))
    seeds, info = imm.imm_solve(gg.handle, w.k, w.eps, w.ell, model, w.seed)
    assert seeds.tolist() == gold["seeds"]
    for key in ("theta", "num_rr", "covered", "phases", "edges_examined", "pool_ids"):
        assert info[key] == gold[key], key
    assert info["lb"] == float.fromhex(gold["lb_hex"])
    assert info["spread_est"] == float.fromhex(gold["spread_est_hex"])
    assert info["lambda_prime"] == float.fromhex(gold["lambda_prime_hex"])
    assert info["lambda_star"] == float.fromhex(gold["lambda_star_hex"])
