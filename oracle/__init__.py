"""Python access to the CPU oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain C implementation of the IMM hot path (RR-set generation under IC
and LT, occurrence histogram, greedy max coverage, IMM's LB/theta loop) written from the
gIM paper and the IMM paper.  Only the test suite, the smoke check and the benchmark's CPU
baseline may import this package; the GPU library never does, and this package never
imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

IC, LT = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, u64, dbl, p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p)
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_ic_threshold.argtypes = [ctypes.c_float]
        L.orc_ic_threshold.restype = u32
        L.orc_encode_ic.argtypes = [i64, p, p]
        L.orc_encode_lt.argtypes = [i32, p, p, p]
        L.orc_root.argtypes = [u64, u32, i32]
        L.orc_root.restype = i32
        for f in (L.orc_rr_ic, L.orc_rr_lt):
            f.argtypes = [i32, p, p, p, u64, u32, p, p, p]
            f.restype = i64
        L.orc_pool_new.argtypes = [i32, i64, p, p, p, ctypes.c_int, u64]
        L.orc_pool_new.restype = p
        L.orc_pool_free.argtypes = [p]
        L.orc_pool_extend.argtypes = [p, i64, ctypes.c_int]
        L.orc_pool_count.argtypes = [p]
        L.orc_pool_count.restype = i64
        for f in (L.orc_pool_total, L.orc_pool_edges):
            f.argtypes = [p, i64, i64]
            f.restype = i64
        L.orc_pool_export.argtypes = [p, i64, i64, p, p]
        L.orc_pool_hist.argtypes = [p, i64, i64, p]
        L.orc_greedy_sets.argtypes = [i32, i64, p, p, i32, p, p]
        L.orc_pool_greedy.argtypes = [p, i64, i64, i32, p, p]
        L.orc_log_binom.argtypes = [i64, i64]
        L.orc_log_binom.restype = dbl
        for f in (L.orc_lambda_prime, L.orc_lambda_star):
            f.argtypes = [i64, i64, dbl, dbl]
            f.restype = dbl
        L.orc_ell_adjusted.argtypes = [i64, dbl]
        L.orc_ell_adjusted.restype = dbl
        L.orc_imax.argtypes = [i64]
        L.orc_imax.restype = i32
        L.orc_imm_solve.argtypes = [i32, i64, p, p, p, p, ctypes.c_int, u64, i32, dbl, dbl,
                                    ctypes.c_int, ctypes.c_int, p, p, p]
        for f in (L.orc_rr_ic_round, L.orc_rr_lt_round):
            f.argtypes = [i32, p, p, p, u64, u32, u32, p, p, p]
            f.restype = i64
        L.orc_mr_sets.argtypes = [i32, p, p, p, ctypes.c_int, u64, i32, i64, p, p, p, p]
        L.orc_greedy_partition.argtypes = [i32, i32, i64, p, p, i32, p, p]
        L.orc_mr_ratio.argtypes = [i32]
        L.orc_mr_ratio.restype = dbl
        for f in (L.orc_mr_lambda_prime, L.orc_mr_lambda_star):
            f.argtypes = [i64, i64, i32, dbl, dbl]
            f.restype = dbl
        L.orc_mrim_solve.argtypes = [i32, i64, p, p, p, p, ctypes.c_int, u64, i32, i32, dbl,
                                     dbl, p, p, p]
        L.orc_spread_mc.argtypes = [i32, i64, p, p, p, ctypes.c_int, u64, i32, p, i32, i64,
                                    ctypes.c_int, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def default_threads() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def encode_ic(p: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.float32)
    thr = np.zeros(len(p), dtype=np.uint32)
    if lib().orc_encode_ic(len(p), _ptr(p), _ptr(thr)) != 0:
        raise ValueError("IC probabilities must lie in [0, 1]")
    return thr


def encode_lt(in_off: np.ndarray, w: np.ndarray | None) -> np.ndarray:
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    n = len(in_off) - 1
    cum = np.zeros(int(in_off[-1]), dtype=np.uint32)
    wa = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
    if lib().orc_encode_lt(n, _ptr(in_off), _ptr(wa), _ptr(cum)) != 0:
        raise ValueError("invalid LT weights")
    return cum


def root(seed: int, r: int, n: int) -> int:
    return lib().orc_root(seed, r, n)


class Pool:
    """RR sets [0, count) of one (graph, model, seed), each sorted ascending."""

    def __init__(self, graph, model: int, seed: int, ic_p=None, lt_w=None):
        self.n = graph.n
        self.in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
        self.in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
        self.model = model
        self.seed = seed
        if model == IC:
            self.thr = encode_ic(ic_p)
        else:
            self.thr = encode_lt(self.in_off, lt_w)
        self._p = lib().orc_pool_new(self.n, len(self.in_src), _ptr(self.in_off),
                                     _ptr(self.in_src), _ptr(self.thr), model, seed)
        if not self._p:
            raise ValueError("invalid pool arguments")

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_pool_free(self._p)
            self._p = None

    def extend(self, upto: int, threads: int | None = None) -> None:
        if lib().orc_pool_extend(self._p, upto, threads or default_threads()) != 0:
            raise ValueError("pool extension failed")

    @property
    def count(self) -> int:
        return lib().orc_pool_count(self._p)

    def total(self, first: int = 0, count: int | None = None) -> int:
        count = self.count - first if count is None else count
        return lib().orc_pool_total(self._p, first, count)

    def edges(self, first: int = 0, count: int | None = None) -> int:
        count = self.count - first if count is None else count
        return lib().orc_pool_edges(self._p, first, count)

    def export(self, first: int = 0, count: int | None = None):
        count = self.count - first if count is None else count
        off = np.zeros(count + 1, dtype=np.int64)
        lib().orc_pool_export(self._p, first, count, _ptr(off), None)
        ids = np.zeros(int(off[-1]), dtype=np.int32)
        lib().orc_pool_export(self._p, first, count, _ptr(off), _ptr(ids))
        return off, ids

    def hist(self, first: int = 0, count: int | None = None) -> np.ndarray:
        count = self.count - first if count is None else count
        h = np.zeros(self.n, dtype=np.uint32)
        lib().orc_pool_hist(self._p, first, count, _ptr(h))
        return h

    def greedy(self, k: int, first: int = 0, count: int | None = None):
        count = self.count - first if count is None else count
        seeds = np.zeros(k, dtype=np.int32)
        cov = np.zeros(1, dtype=np.int64)
        if lib().orc_pool_greedy(self._p, first, count, k, _ptr(seeds), _ptr(cov)) != 0:
            raise ValueError("invalid greedy arguments")
        return seeds, int(cov[0])


def rr_set(graph, model: int, thr: np.ndarray, seed: int, r: int):
    """One RR set (discovery order) and its edges-examined count."""
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    out = np.zeros(graph.n, dtype=np.int32)
    mark = np.zeros(graph.n, dtype=np.uint8)
    ex = np.zeros(1, dtype=np.int64)
    f = lib().orc_rr_ic if model == IC else lib().orc_rr_lt
    sz = f(graph.n, _ptr(in_off), _ptr(in_src), _ptr(thr), seed, r, _ptr(out), _ptr(mark),
           _ptr(ex))
    return out[:sz].copy(), int(ex[0])


def greedy_sets(n: int, off: np.ndarray, ids: np.ndarray, k: int):
    off = np.ascontiguousarray(off, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    seeds = np.zeros(k, dtype=np.int32)
    cov = np.zeros(1, dtype=np.int64)
    if lib().orc_greedy_sets(n, len(off) - 1, _ptr(off), _ptr(ids), k, _ptr(seeds),
                             _ptr(cov)) != 0:
        raise ValueError("invalid greedy arguments")
    return seeds, int(cov[0])


def log_binom(n: int, k: int) -> float:
    return lib().orc_log_binom(n, k)


def ell_adjusted(n: int, ell: float) -> float:
    return lib().orc_ell_adjusted(n, ell)


def lambda_prime(n: int, k: int, eps: float, ell: float) -> float:
    return lib().orc_lambda_prime(n, k, eps, ell_adjusted(n, ell))


def lambda_star(n: int, k: int, eps: float, ell: float) -> float:
    return lib().orc_lambda_star(n, k, eps, ell_adjusted(n, ell))


def imax(n: int) -> int:
    return lib().orc_imax(n)


def imm_solve(graph, model: int, k: int, eps: float, ell: float, seed: int, ic_p=None,
              lt_w=None, fresh_final: bool = False, threads: int | None = None) -> dict:
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    p = None if ic_p is None else np.ascontiguousarray(ic_p, dtype=np.float32)
    w = None if lt_w is None else np.ascontiguousarray(lt_w, dtype=np.uint32)
    seeds = np.zeros(k, dtype=np.int32)
    ii = np.zeros(6, dtype=np.int64)
    dd = np.zeros(4, dtype=np.float64)
    rc = lib().orc_imm_solve(graph.n, len(in_src), _ptr(in_off), _ptr(in_src), _ptr(p), _ptr(w),
                             model, seed, k, eps, ell, int(fresh_final),
                             threads or default_threads(), _ptr(seeds), _ptr(ii), _ptr(dd))
    if rc != 0:
        raise ValueError(f"oracle imm_solve failed ({rc})")
    return dict(seeds=seeds, theta=int(ii[0]), num_rr=int(ii[1]), covered=int(ii[2]),
                phases=int(ii[3]), edges=int(ii[4]), pool_ids=int(ii[5]), lb=float(dd[0]),
                spread_est=float(dd[1]), lambda_prime=float(dd[2]), lambda_star=float(dd[3]))


# ---- multi-round IM (gIM Sec. IV-H: CR-NAIMM) ----------------------------------------------
def rr_set_round(graph, model: int, thr: np.ndarray, seed: int, r: int, t: int):
    """Round t's RR set of multi-round set r (discovery order) and its edges examined."""
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    out = np.zeros(graph.n, dtype=np.int32)
    mark = np.zeros(graph.n, dtype=np.uint8)
    ex = np.zeros(1, dtype=np.int64)
    f = lib().orc_rr_ic_round if model == IC else lib().orc_rr_lt_round
    sz = f(graph.n, _ptr(in_off), _ptr(in_src), _ptr(thr), seed, r, t, _ptr(out), _ptr(mark),
           _ptr(ex))
    return out[:sz].copy(), int(ex[0])


def mr_sets(graph, model: int, seed: int, rounds: int, count: int, ic_p=None, lt_w=None):
    """Multi-round RR sets [0, count): offsets, elements t * n + u (sorted per set), and the
    in-edges examined."""
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    thr = encode_ic(ic_p) if model == IC else encode_lt(in_off, lt_w)
    off = np.zeros(count + 1, dtype=np.int64)
    tot = np.zeros(1, dtype=np.int64)
    ed = np.zeros(1, dtype=np.int64)
    L = lib()
    if L.orc_mr_sets(graph.n, _ptr(in_off), _ptr(in_src), _ptr(thr), model, seed, rounds, count,
                     None, None, _ptr(tot), None) != 0:
        raise ValueError("invalid multi-round set arguments")
    ids = np.zeros(int(tot[0]), dtype=np.int32)
    L.orc_mr_sets(graph.n, _ptr(in_off), _ptr(in_src), _ptr(thr), model, seed, rounds, count,
                  _ptr(off), _ptr(ids), None, _ptr(ed))
    return off, ids, int(ed[0])


def greedy_partition(part_size: int, parts: int, off: np.ndarray, ids: np.ndarray, k: int):
    off = np.ascontiguousarray(off, dtype=np.int64)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    seeds = np.zeros(parts * k, dtype=np.int32)
    cov = np.zeros(1, dtype=np.int64)
    if lib().orc_greedy_partition(part_size, parts, len(off) - 1, _ptr(off), _ptr(ids), k,
                                  _ptr(seeds), _ptr(cov)) != 0:
        raise ValueError("invalid greedy arguments")
    return seeds, int(cov[0])


def mr_lambda_prime(n: int, k: int, rounds: int, eps: float, ell: float) -> float:
    return lib().orc_mr_lambda_prime(n, k, rounds, eps, ell_adjusted(n, ell))


def mr_lambda_star(n: int, k: int, rounds: int, eps: float, ell: float) -> float:
    return lib().orc_mr_lambda_star(n, k, rounds, eps, ell_adjusted(n, ell))


def mrim_solve(graph, model: int, k: int, rounds: int, eps: float, ell: float, seed: int,
               ic_p=None, lt_w=None) -> dict:
    """CR-NAIMM: seeds are elements t * n + u (round t, vertex u) in selection order."""
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    p = None if ic_p is None else np.ascontiguousarray(ic_p, dtype=np.float32)
    w = None if lt_w is None else np.ascontiguousarray(lt_w, dtype=np.uint32)
    seeds = np.zeros(rounds * k, dtype=np.int32)
    ii = np.zeros(6, dtype=np.int64)
    dd = np.zeros(4, dtype=np.float64)
    rc = lib().orc_mrim_solve(graph.n, len(in_src), _ptr(in_off), _ptr(in_src), _ptr(p), _ptr(w),
                              model, seed, k, rounds, eps, ell, _ptr(seeds), _ptr(ii), _ptr(dd))
    if rc != 0:
        raise ValueError(f"oracle mrim_solve failed ({rc})")
    return dict(seeds=seeds, theta=int(ii[0]), num_rr=int(ii[1]), covered=int(ii[2]),
                phases=int(ii[3]), edges=int(ii[4]), pool_ids=int(ii[5]), lb=float(dd[0]),
                spread_est=float(dd[1]), lambda_prime=float(dd[2]), lambda_star=float(dd[3]))


# ---- forward Monte-Carlo spread (gIM Sec. II-C) -------------------------------------------
def spread_mc(graph, model: int, seeds, sims: int, seed: int, ic_p=None, lt_w=None,
              rounds: int = 1, threads: int | None = None, per_sim: bool = False):
    """Vertices reached from `seeds` (elements t * n + u when rounds > 1) summed over
    simulations [0, sims); with per_sim also each simulation's count."""
    in_off = np.ascontiguousarray(graph.in_off, dtype=np.int64)
    in_src = np.ascontiguousarray(graph.in_src, dtype=np.int32)
    thr = encode_ic(ic_p) if model == IC else encode_lt(in_off, lt_w)
    el = np.ascontiguousarray(seeds, dtype=np.int32)
    ps = np.zeros(max(sims, 1), dtype=np.int64) if per_sim else None
    tot = np.zeros(1, dtype=np.int64)
    rc = lib().orc_spread_mc(graph.n, len(in_src), _ptr(in_off), _ptr(in_src), _ptr(thr), model,
                             seed, rounds, _ptr(el), len(el), sims, threads or default_threads(),
                             _ptr(ps), _ptr(tot))
    if rc != 0:
        raise ValueError("invalid spread arguments")
    return (int(tot[0]), ps[:sims]) if per_sim else int(tot[0])
