"""Autotuning: the chosen launch configuration changes speed, never results.

imm_autotune times pilot generation under candidate launch configurations (light-wave
budget x heavy block size, list capacity, fetch depth) and stores the fastest on the graph.  Every RR set is keyed by (seed, set, edge), so
pools and solves after tuning must be bit-identical to those before it.
"""
import numpy as np
import pytest

from synth import graphs

pytestmark = pytest.mark.gpu


def _sets(imm, gg, model, seed, count):
    p = imm.Pool.create(gg, model, seed)
    imm.imm_generate_rr(p.handle, count)
    return imm.imm_rr_export(p.handle, 0, count)


@pytest.mark.parametrize("kind", ["er_p1", "rmat_wc", "rmat_lt"])
def test_tuned_results_equal_default(imm_gpu, kind):
    imm = imm_gpu
    if kind == "er_p1":         # every set overflows the light path
        g = graphs.erdos_renyi(5000, 40_000, seed=7)
        gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=np.ones(g.m, np.float32))
        model, k, eps = imm.IMM_IC, 3, 0.5
    elif kind == "rmat_wc":
        g = graphs.rmat(14, 16 << 14, seed=91)
        gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=graphs.weighted_cascade(g))
        model, k, eps = imm.IMM_IC, 20, 0.3
    else:
        g = graphs.rmat(13, 12 << 13, seed=92)
        gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, lt=True)
        model, k, eps = imm.IMM_LT, 10, 0.3
    seed = 0x5EED0200
    before_sets = _sets(imm, gg, model, seed, 3000)
    before = imm.imm_solve(gg.handle, k, eps, 1.0, model, seed)
    info = imm.imm_autotune(gg.handle, model, seed, 2000)
    assert info["fetch"] in (4, 8, 16, 32)
    assert info["default_sets_per_s"] > 0
    # the chosen configuration was the fastest measured, the default among them
    assert info["best_sets_per_s"] >= info["default_sets_per_s"]
    if model == imm.IMM_IC:
        # defaults, 9 other budget x block pairs, 2 list capacities, 3 fetch depths
        assert info["candidates"] == 15
        assert info["light_budget"] in (1024, 2048, 4096, 8192, 16384)
        assert info["heavy_block"] in (128, 256)
        assert info["light_cap"] in (256, 512, 1024)
    else:
        assert info["candidates"] == 6          # defaults, 2 walk list capacities, 3 depths
        assert info["lt_cap"] in (64, 128, 256)
    after_sets = _sets(imm, gg, model, seed, 3000)
    for a, b in zip(before_sets, after_sets):
        assert np.array_equal(a, b)
    after = imm.imm_solve(gg.handle, k, eps, 1.0, model, seed)
    assert np.array_equal(before[0], after[0])
    for key in ("theta", "covered", "num_rr", "lb", "edges_examined", "pool_ids"):
        assert before[1][key] == after[1][key], key


def test_autotune_rejects_bad_arguments(imm_gpu):
    imm = imm_gpu
    g = graphs.erdos_renyi(100, 400, seed=3)
    gg = imm.Graph.from_arrays(g.n, g.in_off, g.in_src, ic_p=np.full(g.m, 0.1, np.float32))
    with pytest.raises(imm.ImmError):
        imm.imm_autotune(gg.handle, imm.IMM_LT, 1, 100)      # no LT encoding
    with pytest.raises(imm.ImmError):
        imm.imm_autotune(gg.handle, imm.IMM_IC, 1, 0)
