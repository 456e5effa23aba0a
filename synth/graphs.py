"""Seeded synthetic graphs and edge weights for the influence-maximisation workloads.

This module produces *inputs only*: vertex/edge structure in in-edge CSR form and the raw
per-edge weights that the diffusion models consume.  It holds none of the method's
arithmetic (no thresholds, no random draws of the diffusion process, no RR sets); both
the CPU oracle and the GPU library encode these raw weights themselves.

Graph families (all directed, no self-loops, no duplicate edges):
  * Erdos-Renyi G(n, m): m distinct ordered pairs drawn uniformly.
  * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM'04) with quadrant probabilities (a, b, c, d),
    vertex ids permuted by a seeded permutation (as Graph500 does) so that degree is not
    correlated with id.
Weights:
  * weighted cascade (WC): p(u,v) = 1/indeg(v) as float32 -- the scheme the paper uses for
    both IC and LT (Sec. IV-B, experiment setup).
  * trivalency: p drawn uniformly from {0.1, 0.01, 0.001} as float32.
  * LT raw integer weights in [1, 2^31], i.e. uniform on (0, 1] in 2^31 steps; the
    per-vertex normalisation to sum 1 is part of the LT encoding, done by each consumer.

Edge order inside each vertex's in-list is ascending source id.  That order matters: the
edge index e keys the IC random stream and the LT walk takes the first matching in-edge.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_libsynth.so")
_lib = None


def build_native(force: bool = False) -> str:
    """Compile the candidate-draw helper (plain C, OpenMP) next to this file."""
    src = os.path.join(_HERE, "_gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _native():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_native())
        i32, i64, u32, u64, p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_void_p)
        lib.synth_rmat_draw.argtypes = [i32, i64, u64, i64, i64, u32, u32, u32, p, p]
        lib.synth_er_draw.argtypes = [i64, u64, i64, i64, p, p]
        lib.synth_hash_keys.argtypes = [p, i64, u64, p]
        lib.synth_ba.argtypes = [i32, i32, u64, p, p, p]
        lib.synth_ba.restype = i64
        _lib = lib
    return _lib


@dataclass
class Graph:
    """In-edge CSR of a directed graph: in-edges of v are in_src[in_off[v]:in_off[v+1]]."""
    n: int
    in_off: np.ndarray            # int64[n+1]
    in_src: np.ndarray            # int32[m]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.in_off[-1])

    def in_degree(self) -> np.ndarray:
        return np.diff(self.in_off)

    def dst(self) -> np.ndarray:
        """Destination vertex of every edge (int32[m])."""
        return np.repeat(np.arange(self.n, dtype=np.int32), self.in_degree())


def _distinct(draw, m: int, batch: int, seed: int, progress=None) -> tuple[np.ndarray, np.ndarray]:
    """Draw candidate (src, dst) pairs with ``draw(first, count)`` until at least ``m``
    distinct non-loop pairs exist, then keep a seeded uniform subset of exactly ``m``
    (the m distinct pairs with the smallest seeded hash).  ``progress(msg)``, if given, is
    called after each step."""
    keys = np.zeros(0, dtype=np.int64)
    first = 0
    while True:
        s, d = draw(first, batch)
        first += batch
        if progress:
            progress(f"drew {first} candidate edges")
        keep = s != d
        k = s[keep].astype(np.int64) << 32 | d[keep].astype(np.int64)
        keys = np.unique(np.concatenate([keys, k]))
        if progress:
            progress(f"{len(keys)} distinct edges")
        if len(keys) >= m:
            break
        # deterministic growth: the next batch size depends only on counts so far
        batch = max(1024, int((m - len(keys)) * 1.5) + 1024)
    if len(keys) > m:
        h = np.empty(len(keys), dtype=np.uint64)
        _native().synth_hash_keys(keys.ctypes.data, len(keys), seed ^ 0xD15C, h.ctypes.data)
        sel = np.argpartition(h, m - 1)[:m]
        sel.sort()
        keys = keys[sel]
    return (keys >> 32).astype(np.int32), (keys & 0xFFFFFFFF).astype(np.int32)


def _to_in_csr(n: int, src: np.ndarray, dst: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    key = dst.astype(np.int64) * n + src.astype(np.int64)
    key.sort()
    d = (key // n).astype(np.int64)
    s = (key % n).astype(np.int32)
    counts = np.bincount(d, minlength=n)
    in_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=in_off[1:])
    return in_off, s


def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """Directed G(n, m): m distinct ordered pairs (u != v), uniform."""
    if n < 2 or m > n * (n - 1):
        raise ValueError("infeasible G(n, m)")
    def draw(first, count):
        src = np.empty(count, dtype=np.int32)
        dst = np.empty(count, dtype=np.int32)
        _native().synth_er_draw(n, seed, first, count, src.ctypes.data, dst.ctypes.data)
        return src, dst

    src, dst = _distinct(draw, m, int(m * 1.05) + 64, seed)
    in_off, in_src = _to_in_csr(n, src, dst)
    return Graph(n, in_off, in_src, name=f"er_n{n}_m{m}", meta=dict(kind="er", seed=seed))


def rmat(scale: int, m: int, seed: int, a=0.57, b=0.19, c=0.19, n: int | None = None,
         permute: bool = True, progress=None) -> Graph:
    """R-MAT graph on 2^scale vertex slots with exactly m distinct non-loop edges.

    If ``n`` is given (n <= 2^scale), candidate edges with an endpoint >= n are rejected,
    which yields an R-MAT-shaped graph on n vertices.
    """
    nslots = 1 << scale
    if n is None:
        n = nslots
    if not (2 <= n <= nslots) or m > n * (n - 1):
        raise ValueError("infeasible R-MAT parameters")
    # integer quadrant thresholds on a 32-bit uniform draw
    ta = min(int(a * 2**32), 2**32 - 1)
    tab = min(int((a + b) * 2**32), 2**32 - 1)
    tabc = min(int((a + b + c) * 2**32), 2**32 - 1)

    def draw(first, count):
        src = np.empty(count, dtype=np.int32)
        dst = np.empty(count, dtype=np.int32)
        _native().synth_rmat_draw(scale, n, seed, first, count, ta, tab, tabc,
                                  src.ctypes.data, dst.ctypes.data)
        return src, dst

    overdraw = 1.25 if n == nslots else 1.25 * (nslots / n) ** 2
    src, dst = _distinct(draw, m, int(m * min(overdraw, 64.0)) + 1024, seed, progress)
    if permute:
        perm = np.random.Generator(np.random.PCG64(seed)).permutation(n).astype(np.int32)
        src, dst = perm[src], perm[dst]
        if progress:
            progress("ids permuted")
    in_off, in_src = _to_in_csr(n, src, dst)
    if progress:
        progress("in-edge CSR built")
    return Graph(n, in_off, in_src, name=f"rmat_s{scale}_n{n}_m{m}",
                 meta=dict(kind="rmat", scale=scale, seed=seed, abcd=(a, b, c, 1 - a - b - c)))


def barabasi_albert(n: int, r: int, seed: int) -> Graph:
    """Barabasi-Albert graph (preferential attachment, r edges per new vertex, starting
    from a clique of r + 1), the density family of gIM Sec. IV-F; each undirected edge
    becomes two directed edges."""
    if r < 1 or n < r + 2:
        raise ValueError("infeasible Barabasi-Albert graph")
    r0 = r + 1
    mu = r0 * (r0 - 1) // 2 + (n - r0) * r
    src = np.empty(mu, dtype=np.int32)
    dst = np.empty(mu, dtype=np.int32)
    ends = np.empty(2 * mu, dtype=np.int32)
    got = _native().synth_ba(n, r, seed, src.ctypes.data, dst.ctypes.data, ends.ctypes.data)
    assert got == mu
    del ends
    in_off, in_src = _to_in_csr(n, np.concatenate([src, dst]), np.concatenate([dst, src]))
    return Graph(n, in_off, in_src, name=f"ba_n{n}_r{r}", meta=dict(kind="ba", r=r, seed=seed))


def weighted_cascade(g: Graph) -> np.ndarray:
    """WC probabilities p(u,v) = 1/indeg(v), computed as a float32 division."""
    deg = g.in_degree().astype(np.float32)
    dst = g.dst()
    return (np.float32(1.0) / deg[dst]).astype(np.float32)


def trivalency(g: Graph, seed: int) -> np.ndarray:
    """IC probabilities drawn uniformly from {0.1, 0.01, 0.001} (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.array([0.1, 0.01, 0.001], dtype=np.float32)
    return vals[rng.integers(0, 3, g.m)]


def lt_uniform_weights(g: Graph, seed: int) -> np.ndarray:
    """Raw LT weights, uniform on (0, 1] as integers in [1, 2^31] (uint32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = (rng.integers(0, 1 << 32, g.m, dtype=np.uint64) >> np.uint64(1)) + np.uint64(1)
    return w.astype(np.uint32)


def from_edges(n: int, src, dst, name: str = "edges") -> Graph:
    """In-edge CSR from an explicit edge list (for small hand-made test graphs)."""
    src = np.asarray(src, dtype=np.int32)
    dst = np.asarray(dst, dtype=np.int32)
    if len(src) and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("endpoint out of range")
    in_off, in_src = _to_in_csr(n, src, dst)
    return Graph(n, in_off, in_src, name=name, meta=dict(kind="explicit"))


def log_uniform(rng, lo: float, hi: float) -> float:
    return float(10 ** rng.uniform(math.log10(lo), math.log10(hi)))
