"""The no-allocation selection entry point (imm_select_seeds_noalloc) against the ordinary
one (imm_select_seeds), through the C ABI: identical seeds and covered counts on two calls
in a row, the second on a smaller input (the static scratch keeps the first call's
contents), on plain IC, LT and multi-round pools; oversized requests are refused before
anything runs.  The ordinary entry point is itself pinned to the oracle's greedy by the
selection parity tests; the first case here is also compared with the oracle directly."""
import numpy as np
import pytest

import oracle
from synth import configs, graphs

pytestmark = pytest.mark.gpu


def _pool(imm, g, model, seed, count, ic_p=None, lt_w=None, rounds=1):
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=ic_p, lt_w=lt_w,
                               lt=(model == imm.IMM_LT))
    if rounds > 1:
        pool = imm.Pool.create_mr(gg, model, seed, rounds)
    else:
        pool = imm.Pool.create(gg, model, seed)
    imm.imm_generate_rr(pool.handle, count)
    return gg, pool


def _same(imm, pool, first, count, k, rounds=1):
    ref = imm.imm_select_seeds(pool.handle, first, count, k, rounds=rounds)
    got = imm.imm_select_seeds_noalloc(pool.handle, first, count, k, rounds=rounds)
    assert np.array_equal(got[0], ref[0]), (first, count, k)
    assert got[1] == ref[1], (first, count, k)
    need = imm.imm_select_noalloc_bytes(pool.handle, first, count, k)
    assert 0 < need <= imm.IMM_NOALLOC_SCRATCH_BYTES
    return got


def test_noalloc_select_ic_matches_ordinary_and_oracle(imm_gpu):
    w = configs.c1()
    gg, pool = _pool(imm_gpu, w.graph, imm_gpu.IMM_IC, w.seed, 6000, ic_p=w.ic_p)
    seeds, cov = _same(imm_gpu, pool, 0, 6000, 25)            # whole prefix
    ref = oracle.Pool(w.graph, oracle.IC, w.seed, ic_p=w.ic_p)
    ref.extend(6000)
    seeds_o, cov_o = ref.greedy(25, 0, 6000)
    assert np.array_equal(seeds, seeds_o) and cov == cov_o
    # second call, smaller input: a sub-range (its own histogram) and fewer seeds
    _same(imm_gpu, pool, 1000, 2500, 7)
    _same(imm_gpu, pool, 0, 6000, 25)                         # and the first again


def test_noalloc_select_lt_and_multi_round(imm_gpu):
    g = graphs.rmat(12, 40_000, seed=71)
    lt_w = graphs.lt_uniform_weights(g, seed=72)
    gg, pool = _pool(imm_gpu, g, imm_gpu.IMM_LT, 0x5EED7101, 8000, lt_w=lt_w)
    _same(imm_gpu, pool, 0, 8000, 40)
    _same(imm_gpu, pool, 500, 3000, 3)
    ic_p = graphs.weighted_cascade(g)
    gg2, mr = _pool(imm_gpu, g, imm_gpu.IMM_IC, 0x5EED7102, 3000, ic_p=ic_p, rounds=3)
    _same(imm_gpu, mr, 0, 3000, 6, rounds=3)
    _same(imm_gpu, mr, 100, 1000, 2, rounds=3)


def test_noalloc_select_rejects_oversized_requests(imm_gpu):
    n = 1 << 22                           # 20 B per vertex alone exceed 64 MiB
    g = graphs.from_edges(n, np.array([0, 5], dtype=np.int64), np.array([1, 1], dtype=np.int64))
    gg = imm_gpu.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=np.full(g.m, 0.5, np.float32))
    pool = imm_gpu.Pool.create(gg, imm_gpu.IMM_IC, 7)
    imm_gpu.imm_generate_rr(pool.handle, 100)
    assert imm_gpu.imm_select_noalloc_bytes(pool.handle, 0, 100, 1) > imm_gpu.IMM_NOALLOC_SCRATCH_BYTES
    with pytest.raises(imm_gpu.ImmError) as e:
        imm_gpu.imm_select_seeds_noalloc(pool.handle, 0, 100, 1)
    assert e.value.status == 3                                 # IMM_ECAPACITY
    with pytest.raises(imm_gpu.ImmError) as e:
        imm_gpu.imm_select_seeds_noalloc(pool.handle, 50, 51, 1)   # beyond the pool
    assert e.value.status == 1                                 # IMM_EINVAL
    # the ordinary entry point still answers the same request
    seeds, cov = imm_gpu.imm_select_seeds(pool.handle, 0, 100, 1)
    assert cov >= 1 and 0 <= seeds[0] < n
