"""The five synthetic workloads (graphs, weights, queries and seeds).

C1  ER G(1000, 10000), WC IC, k=10, eps=0.5, ell=1            (small; oracle in seconds)
C2  R-MAT scale 20, 2^24 edges, WC IC, k=50, eps=0.1           (stand-in for higgs/pokec-sized
                                                                 social graphs of Table 1)
C3  R-MAT scale 22, 2^26 edges, LT uniform-normalised, k=100, eps=0.1
C4  256 R-MAT instances, n log-uniform in [1e4, 2e6], avg degree log-uniform in [4, 32],
    WC IC, k ~ U{5..100}, eps ~ U{0.5, 0.2, 0.1}
C5  R-MAT scale 24, 2^28 edges, trivalency IC / WC-LT, served query stream

Everything is seeded; the same call yields the same arrays on every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import graphs


@dataclass
class Workload:
    name: str
    graph: graphs.Graph
    model: str                     # "IC" or "LT"
    ic_p: np.ndarray | None        # float32[m] IC probabilities
    lt_w: np.ndarray | None        # uint32[m] raw LT weights (None = unit weights, i.e. WC-LT)
    k: int
    eps: float
    ell: float
    seed: int                      # RR-pool / Philox seed


def c1() -> Workload:
    g = graphs.erdos_renyi(1000, 10_000, seed=1)
    return Workload("C1-er1000-wc-ic", g, "IC", graphs.weighted_cascade(g), None,
                    k=10, eps=0.5, ell=1.0, seed=0x5EED0001)


def c2(scale: int = 20, edge_factor: int = 16) -> Workload:
    g = graphs.rmat(scale, edge_factor << scale, seed=2)
    return Workload(f"C2-rmat{scale}-wc-ic", g, "IC", graphs.weighted_cascade(g), None,
                    k=50, eps=0.1, ell=1.0, seed=0x5EED0002)


def c3(scale: int = 22, edge_factor: int = 16) -> Workload:
    g = graphs.rmat(scale, edge_factor << scale, seed=3)
    return Workload(f"C3-rmat{scale}-lt-uniform", g, "LT", None,
                    graphs.lt_uniform_weights(g, seed=33), k=100, eps=0.1, ell=1.0,
                    seed=0x5EED0003)


@dataclass
class InstanceSpec:
    index: int
    n: int
    m: int
    scale: int
    k: int
    eps: float
    graph_seed: int
    pool_seed: int


def c4_specs(count: int = 256, sampler_seed: int = 4) -> list[InstanceSpec]:
    rng = np.random.Generator(np.random.PCG64(sampler_seed))
    out = []
    for i in range(count):
        n = int(round(graphs.log_uniform(rng, 1e4, 2e6)))
        deg = 2.0 ** rng.uniform(2.0, 5.0)
        m = int(round(n * deg))
        k = int(rng.integers(5, 101))
        eps = float(rng.choice([0.5, 0.2, 0.1]))
        out.append(InstanceSpec(i, n, m, max(1, math.ceil(math.log2(n))), k, eps,
                                1000 + i, 0x5EED1000 + i))
    return out


def c4_instance(spec: InstanceSpec) -> Workload:
    g = graphs.rmat(spec.scale, spec.m, seed=spec.graph_seed, n=spec.n)
    return Workload(f"C4-inst{spec.index}", g, "IC", graphs.weighted_cascade(g), None,
                    k=spec.k, eps=spec.eps, ell=1.0, seed=spec.pool_seed)


def c5_graph(scale: int = 24, edge_factor: int = 16, progress=None) -> tuple[graphs.Graph, np.ndarray]:
    g = graphs.rmat(scale, edge_factor << scale, seed=5, progress=progress)
    return g, graphs.trivalency(g, seed=55)


C5_POOL_SEED_IC = 0x5EED0005
C5_POOL_SEED_LT = 0x5EED0006
