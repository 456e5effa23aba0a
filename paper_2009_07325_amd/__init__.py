"""IMM influence maximisation on AMD Instinct MI355X: Python binding of libimm.

Thin ctypes marshalling over the C ABI in include/imm.h; every step of the computation
runs in the library's HIP kernels.  The binding keeps the ABI's function names.  Arrays
are numpy arrays (host) or objects exposing ``data_ptr()`` (e.g. torch CUDA tensors).

Loading fails loudly when libimm.so has not been built (``python -m
paper_2009_07325_amd.build``); there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimm.so")

IMM_IC, IMM_LT = 0, 1
IMM_GRAPH_LT = 0x1
IMM_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024   # as include/imm.h
STATUS = {0: "IMM_OK", 1: "IMM_EINVAL", 2: "IMM_ENOMEM", 3: "IMM_ECAPACITY", 4: "IMM_EDEVICE",
          5: "IMM_ENOTIMPL", 6: "IMM_EBUSY", 7: "IMM_ECANCELLED"}

# every entry point declared in include/imm.h
EXPORTS = ("imm_init", "imm_last_error", "imm_release_cached_memory", "imm_graph_create",
           "imm_graph_destroy",
           "imm_graph_info", "imm_graph_export_encoding", "imm_pool_create", "imm_pool_destroy",
           "imm_pool_size", "imm_generate_rr", "imm_rr_export", "imm_rr_histogram",
           "imm_select_seeds", "imm_solve", "imm_solve_pool", "imm_log_binom",
           "imm_lambda_prime", "imm_lambda_star", "imm_autotune", "imm_batch_solve",
           "imm_server_create",
           "imm_server_submit",
           "imm_server_poll", "imm_server_wait", "imm_server_stats_get", "imm_server_destroy",
           "imm_mr_pool_create", "imm_mrim_solve", "imm_mr_lambda_prime", "imm_mr_lambda_star",
           "imm_spread_mc", "imm_select_seeds_noalloc", "imm_select_noalloc_bytes",
           "imm_philox_rate")


class ImmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class ImmOptions(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("fresh_final", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class ImmInfo(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_int64), ("num_rr", ctypes.c_int64),
                ("covered", ctypes.c_int64), ("edges_examined", ctypes.c_int64),
                ("pool_ids", ctypes.c_int64), ("phases", ctypes.c_int32),
                ("heavy_redrawn", ctypes.c_int32), ("lb", ctypes.c_double),
                ("spread_est", ctypes.c_double), ("lambda_prime", ctypes.c_double),
                ("lambda_star", ctypes.c_double), ("t_generate_s", ctypes.c_double),
                ("t_select_s", ctypes.c_double), ("t_total_s", ctypes.c_double),
                ("t_rr_kernel_s", ctypes.c_double), ("rr_kernel_launches", ctypes.c_int64),
                ("t_rr_heavy_s", ctypes.c_double), ("rr_heavy_launches", ctypes.c_int64),
                ("edges_heavy", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class ImmTuneInfo(ctypes.Structure):
    _fields_ = [("light_budget", ctypes.c_int64), ("heavy_block", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("best_sets_per_s", ctypes.c_double),
                ("default_sets_per_s", ctypes.c_double), ("light_cap", ctypes.c_int32),
                ("lt_cap", ctypes.c_int32), ("fetch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ImmBatchItem(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_void_p), ("k", ctypes.c_int32), ("model", ctypes.c_int),
                ("eps", ctypes.c_double), ("ell", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("fresh_final", ctypes.c_int32), ("status", ctypes.c_int),
                ("seeds_out", ctypes.c_void_p), ("info", ImmInfo)]


class ImmBatchStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("rr_sets", ctypes.c_int64),
                ("edges_examined", ctypes.c_int64), ("edges_heavy", ctypes.c_int64),
                ("t_generate_s", ctypes.c_double), ("t_select_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("t_rr_kernel_s", ctypes.c_double),
                ("rr_kernel_launches", ctypes.c_int64), ("t_rr_heavy_s", ctypes.c_double),
                ("rr_heavy_launches", ctypes.c_int64), ("graph_ticks", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ImmServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("active", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("mean_latency_s", ctypes.c_double), ("max_latency_s", ctypes.c_double),
                ("throughput_qps", ctypes.c_double), ("pool_sets_ic", ctypes.c_int64),
                ("pool_sets_lt", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("pool_resets", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libimm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2009_07325_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u32, u64, dbl, p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p)
        pp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "imm_init": [i32],
            "imm_release_cached_memory": [],
            "imm_graph_create": [i32, i64, p, p, p, p, u32, pp],
            "imm_graph_destroy": [p],
            "imm_graph_info": [p, p, p, p, p],
            "imm_graph_export_encoding": [p, p, p],
            "imm_pool_create": [p, ctypes.c_int, u64, pp],
            "imm_pool_destroy": [p],
            "imm_pool_size": [p, p, p, p],
            "imm_generate_rr": [p, i64, p],
            "imm_rr_export": [p, i64, i64, p, p, i64, p],
            "imm_rr_histogram": [p, i64, i64, p],
            "imm_select_seeds": [p, i64, i64, i32, p, p, p],
            "imm_select_seeds_noalloc": [p, i64, i64, i32, p, p, p],
            "imm_philox_rate": [i64, ctypes.POINTER(ctypes.c_double)],
            "imm_solve": [p, i32, dbl, dbl, ctypes.c_int, ctypes.POINTER(ImmOptions), p,
                          ctypes.POINTER(ImmInfo)],
            "imm_solve_pool": [p, i32, dbl, dbl, i32, p, p, ctypes.POINTER(ImmInfo)],
            "imm_autotune": [p, ctypes.c_int, u64, i64, ctypes.POINTER(ImmTuneInfo)],
            "imm_batch_solve": [ctypes.POINTER(ImmBatchItem), i32, p,
                                ctypes.POINTER(ImmBatchStats)],
            "imm_server_create": [p, u64, u64, i64, i32, pp],
            "imm_server_submit": [p, i32, dbl, dbl, ctypes.c_int, i32, ctypes.POINTER(ctypes.c_uint64)],
            "imm_server_poll": [p, u64, p, ctypes.POINTER(ImmInfo), ctypes.POINTER(ctypes.c_int32)],
            "imm_server_wait": [p, u64, dbl, p, ctypes.POINTER(ImmInfo)],
            "imm_server_stats_get": [p, ctypes.POINTER(ImmServerStats)],
            "imm_server_destroy": [p],
            "imm_mr_pool_create": [p, ctypes.c_int, u64, i32, pp],
            "imm_mrim_solve": [p, i32, i32, dbl, dbl, ctypes.c_int, ctypes.POINTER(ImmOptions), p,
                               ctypes.POINTER(ImmInfo)],
            "imm_spread_mc": [p, ctypes.c_int, i32, p, i32, i64, u64, p,
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.imm_last_error.argtypes = []
        L.imm_last_error.restype = ctypes.c_char_p
        L.imm_select_noalloc_bytes.argtypes = [p, i64, i64, i32]
        L.imm_select_noalloc_bytes.restype = i64
        L.imm_log_binom.argtypes = [i64, i64]
        L.imm_log_binom.restype = dbl
        for name in ("imm_lambda_prime", "imm_lambda_star"):
            f = getattr(L, name)
            f.argtypes = [i64, i64, dbl, dbl]
            f.restype = dbl
        for name in ("imm_mr_lambda_prime", "imm_mr_lambda_star"):
            f = getattr(L, name)
            f.argtypes = [i64, i64, i32, dbl, dbl]
            f.restype = dbl
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise ImmError(status, lib().imm_last_error().decode(errors="replace"))


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


def _stream(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# ---- entry points (same names as the C ABI) ------------------------------------------
def imm_init(device: int = 0) -> None:
    _check(lib().imm_init(device))


def imm_last_error() -> str:
    return lib().imm_last_error().decode(errors="replace")


def imm_graph_create(n: int, in_off, in_src, ic_p=None, lt_w=None, flags: int = 0):
    """Returns an opaque graph handle (ctypes.c_void_p)."""
    def host(a, dt):
        if a is None or hasattr(a, "data_ptr"):
            return a
        return np.ascontiguousarray(a, dtype=dt)
    in_off = host(in_off, np.int64)
    in_src = host(in_src, np.int32)
    ic_p = host(ic_p, np.float32)
    lt_w = host(lt_w, np.uint32)
    m = int(in_src.numel() if hasattr(in_src, "numel") else len(in_src))
    out = ctypes.c_void_p()
    _check(lib().imm_graph_create(n, m, _ptr(in_off), _ptr(in_src), _ptr(ic_p), _ptr(lt_w),
                                  flags, ctypes.byref(out)))
    return out


def imm_graph_destroy(g) -> None:
    _check(lib().imm_graph_destroy(g))


def imm_graph_info(g) -> dict:
    n, m, ic, lt = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().imm_graph_info(g, ctypes.byref(n), ctypes.byref(m), ctypes.byref(ic),
                                ctypes.byref(lt)))
    return dict(n=n.value, m=m.value, has_ic=bool(ic.value), has_lt=bool(lt.value))


def imm_graph_export_encoding(g, ic: bool = True, lt: bool = False):
    info = imm_graph_info(g)
    thr = np.zeros(info["m"], dtype=np.uint32) if ic else None
    cum = np.zeros(info["m"], dtype=np.uint32) if lt else None
    _check(lib().imm_graph_export_encoding(g, _ptr(thr), _ptr(cum)))
    return thr, cum


def imm_pool_create(g, model: int, seed: int):
    out = ctypes.c_void_p()
    _check(lib().imm_pool_create(g, model, seed, ctypes.byref(out)))
    return out


def imm_pool_destroy(p) -> None:
    _check(lib().imm_pool_destroy(p))


def imm_pool_size(p) -> tuple[int, int, int]:
    a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().imm_pool_size(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def imm_generate_rr(p, upto: int, stream=None) -> None:
    _check(lib().imm_generate_rr(p, upto, _stream(stream)))


def imm_rr_export(p, first: int, count: int) -> tuple[np.ndarray, np.ndarray]:
    off = np.zeros(count + 1, dtype=np.int64)
    need = ctypes.c_int64()
    _check(lib().imm_rr_export(p, first, count, _ptr(off), None, 0, ctypes.byref(need)))
    ids = np.zeros(max(need.value, 1), dtype=np.int32)
    _check(lib().imm_rr_export(p, first, count, _ptr(off), _ptr(ids), len(ids),
                               ctypes.byref(need)))
    return off, ids[:need.value]


def imm_rr_histogram(p, first: int, count: int, n: int) -> np.ndarray:
    h = np.zeros(n, dtype=np.uint32)
    _check(lib().imm_rr_histogram(p, first, count, _ptr(h)))
    return h


def imm_release_cached_memory() -> None:
    _check(lib().imm_release_cached_memory())


def imm_select_seeds(p, first: int, count: int, k: int, stream=None,
                     rounds: int = 1) -> tuple[np.ndarray, int]:
    """k seeds per round; a multi-round pool of `rounds` rounds returns rounds * k elements."""
    seeds = np.zeros(k * rounds, dtype=np.int32)
    cov = ctypes.c_int64()
    _check(lib().imm_select_seeds(p, first, count, k, _ptr(seeds), ctypes.byref(cov),
                                  _stream(stream)))
    return seeds, cov.value


def imm_select_seeds_noalloc(p, first: int, count: int, k: int, stream=None,
                             rounds: int = 1) -> tuple[np.ndarray, int]:
    """imm_select_seeds with its workspace in the library's static device scratch."""
    seeds = np.zeros(k * rounds, dtype=np.int32)
    cov = ctypes.c_int64()
    _check(lib().imm_select_seeds_noalloc(p, first, count, k, _ptr(seeds), ctypes.byref(cov),
                                          _stream(stream)))
    return seeds, cov.value


def imm_philox_rate(draws_per_lane: int = 16384) -> float:
    """Measured Philox4x32-10 draws per second (1e9) of a draw-and-ballot loop."""
    out = ctypes.c_double()
    _check(lib().imm_philox_rate(draws_per_lane, ctypes.byref(out)))
    return out.value


def imm_select_noalloc_bytes(p, first: int, count: int, k: int) -> int:
    return int(lib().imm_select_noalloc_bytes(p, first, count, k))


def imm_solve(g, k: int, eps: float, ell: float, model: int, seed: int,
              fresh_final: bool = False, stream=None) -> tuple[np.ndarray, dict]:
    opt = ImmOptions(seed=seed, fresh_final=int(fresh_final), reserved=0,
                     stream=_stream(stream))
    seeds = np.zeros(k, dtype=np.int32)
    info = ImmInfo()
    _check(lib().imm_solve(g, k, eps, ell, model, ctypes.byref(opt), _ptr(seeds),
                           ctypes.byref(info)))
    return seeds, info.as_dict()


def imm_solve_pool(p, k: int, eps: float, ell: float, fresh_final: bool = False,
                   stream=None, rounds: int = 1) -> tuple[np.ndarray, dict]:
    seeds = np.zeros(k * rounds, dtype=np.int32)
    info = ImmInfo()
    _check(lib().imm_solve_pool(p, k, eps, ell, int(fresh_final), _stream(stream), _ptr(seeds),
                                ctypes.byref(info)))
    return seeds, info.as_dict()


def imm_mr_pool_create(g, model: int, seed: int, rounds: int):
    out = ctypes.c_void_p()
    _check(lib().imm_mr_pool_create(g, model, seed, rounds, ctypes.byref(out)))
    return out


def imm_mrim_solve(g, k: int, rounds: int, eps: float, ell: float, model: int, seed: int,
                   stream=None) -> tuple[np.ndarray, dict]:
    """Multi-round IM: rounds * k elements t * n + u in selection order."""
    opt = ImmOptions(seed=seed, fresh_final=0, reserved=0, stream=_stream(stream))
    seeds = np.zeros(k * rounds, dtype=np.int32)
    info = ImmInfo()
    _check(lib().imm_mrim_solve(g, k, rounds, eps, ell, model, ctypes.byref(opt), _ptr(seeds),
                                ctypes.byref(info)))
    return seeds, info.as_dict()


def imm_mr_lambda_prime(n: int, k: int, rounds: int, eps: float, ell: float) -> float:
    return lib().imm_mr_lambda_prime(n, k, rounds, eps, ell)


def imm_mr_lambda_star(n: int, k: int, rounds: int, eps: float, ell: float) -> float:
    return lib().imm_mr_lambda_star(n, k, rounds, eps, ell)


def imm_spread_mc(g, model: int, seeds, sims: int, seed: int, rounds: int = 1,
                  per_sim: bool = False, stream=None) -> dict:
    """Forward Monte-Carlo spread of `seeds` (elements t * n + u when rounds > 1): exact
    total of the per-simulation counts, mean and standard error (and the counts)."""
    el = np.ascontiguousarray(seeds, dtype=np.int32)
    ps = np.zeros(max(sims, 1), dtype=np.uint32) if per_sim else None
    tot, mean, se = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(lib().imm_spread_mc(g, model, rounds, _ptr(el), len(el), sims, seed, _ptr(ps),
                               ctypes.byref(tot), ctypes.byref(mean), ctypes.byref(se),
                               _stream(stream)))
    out = dict(total=tot.value, mean=mean.value, stderr=se.value)
    if per_sim:
        out["per_sim"] = ps[:sims]
    return out


def imm_autotune(g, model: int, seed: int, pilot_sets: int) -> dict:
    info = ImmTuneInfo()
    _check(lib().imm_autotune(g, model, seed, pilot_sets, ctypes.byref(info)))
    return info.as_dict()


def imm_batch_solve(items, stream=None, stats: dict | None = None) -> list[tuple[np.ndarray, dict]]:
    """items: sequence of dicts with graph, k, eps, model, seed and optionally ell (1.0) and
    fresh_final (False).  Returns (seeds, info) per item, in order; `stats`, if given, is
    filled with the whole-batch figures."""
    arr = (ImmBatchItem * len(items))()
    seeds = []
    for i, it in enumerate(items):
        s = np.zeros(int(it["k"]), dtype=np.int32)
        seeds.append(s)
        g = it["graph"]
        arr[i].graph = g.handle if isinstance(g, Graph) else g
        arr[i].k = int(it["k"])
        arr[i].model = int(it["model"])
        arr[i].eps = float(it["eps"])
        arr[i].ell = float(it.get("ell", 1.0))
        arr[i].seed = int(it["seed"])
        arr[i].fresh_final = int(bool(it.get("fresh_final", False)))
        arr[i].seeds_out = s.ctypes.data
    bs = ImmBatchStats()
    _check(lib().imm_batch_solve(arr, len(items), _stream(stream), ctypes.byref(bs)))
    if stats is not None:
        stats.update(bs.as_dict())
    return [(seeds[i], arr[i].info.as_dict()) for i in range(len(items))]


def imm_server_create(g, seed_ic: int, seed_lt: int, hbm_budget_bytes: int, max_active: int):
    out = ctypes.c_void_p()
    _check(lib().imm_server_create(g, seed_ic, seed_lt, hbm_budget_bytes, max_active,
                                   ctypes.byref(out)))
    return out


def imm_server_submit(srv, k: int, eps: float, ell: float, model: int,
                      fresh_final: bool = False) -> int:
    t = ctypes.c_uint64()
    _check(lib().imm_server_submit(srv, k, eps, ell, model, int(fresh_final), ctypes.byref(t)))
    return t.value


def imm_server_poll(srv, ticket: int, k: int):
    """(done, seeds, info) -- seeds/info are None until the query has finished."""
    seeds = np.zeros(k, dtype=np.int32)
    info = ImmInfo()
    done = ctypes.c_int32()
    _check(lib().imm_server_poll(srv, ticket, _ptr(seeds), ctypes.byref(info), ctypes.byref(done)))
    return (True, seeds, info.as_dict()) if done.value else (False, None, None)


def imm_server_wait(srv, ticket: int, k: int, timeout_s: float = 0.0):
    seeds = np.zeros(k, dtype=np.int32)
    info = ImmInfo()
    _check(lib().imm_server_wait(srv, ticket, timeout_s, _ptr(seeds), ctypes.byref(info)))
    return seeds, info.as_dict()


def imm_server_stats_get(srv) -> dict:
    st = ImmServerStats()
    _check(lib().imm_server_stats_get(srv, ctypes.byref(st)))
    return st.as_dict()


def imm_server_destroy(srv) -> None:
    _check(lib().imm_server_destroy(srv))


def imm_log_binom(n: int, k: int) -> float:
    return lib().imm_log_binom(n, k)


def imm_lambda_prime(n: int, k: int, eps: float, ell: float) -> float:
    return lib().imm_lambda_prime(n, k, eps, ell)


def imm_lambda_star(n: int, k: int, eps: float, ell: float) -> float:
    return lib().imm_lambda_star(n, k, eps, ell)


@dataclass
class Graph:
    """Owning wrapper of a device graph (destroyed with the object)."""
    handle: ctypes.c_void_p
    n: int
    m: int

    @classmethod
    def from_arrays(cls, n, in_off, in_src, ic_p=None, lt_w=None, lt: bool = False) -> "Graph":
        h = imm_graph_create(n, in_off, in_src, ic_p, lt_w, IMM_GRAPH_LT if lt else 0)
        return cls(h, n, int(len(in_src)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.imm_graph_destroy(self.handle)
            self.handle = None


@dataclass
class Pool:
    """Owning wrapper of a device RR pool."""
    handle: ctypes.c_void_p
    graph: Graph

    rounds: int = 1

    @classmethod
    def create(cls, graph: Graph, model: int, seed: int) -> "Pool":
        return cls(imm_pool_create(graph.handle, model, seed), graph)

    @classmethod
    def create_mr(cls, graph: Graph, model: int, seed: int, rounds: int) -> "Pool":
        """A multi-round pool: elements t * n + u over `rounds` rounds."""
        return cls(imm_mr_pool_create(graph.handle, model, seed, rounds), graph, rounds)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.imm_pool_destroy(self.handle)
            self.handle = None
