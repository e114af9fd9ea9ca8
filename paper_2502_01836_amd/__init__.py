"""LeaFi learned-filter leaf-scan k-NN on MI355X (gfx950).

Python face of libleafi (include/leafi.h).  Tensors must be CUDA (HIP)
tensors on the current device; the current torch stream is passed to the
library.  Nothing here computes: every call goes to the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import LeafiError, check, load, struct_dict
from ._lib import LEAFI_SEARCH_FILTER_TILE_LARGE as SEARCH_FILTER_TILE_LARGE
from ._lib import LEAFI_SEARCH_FILTER_TILE_SMALL as SEARCH_FILTER_TILE_SMALL
from ._lib import LEAFI_SEARCH_HOST_ROUNDS as SEARCH_HOST_ROUNDS
from ._lib import LEAFI_SEARCH_NO_GRAPH as SEARCH_NO_GRAPH

__all__ = ["Index", "Server", "TorchAllocator", "LeafiError", "load", "znorm", "mlp_infer", "mlp_sgd_step",
           "cnn_infer", "cnn_sgd_step",
           "version"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return load().leafi_version().decode()


class TorchAllocator:
    """Device memory for an index handle from torch's caching allocator
    (leafi_alloc_fn / leafi_free_fn).  `limit` (bytes, optional) makes it
    refuse any allocation that would take its live total above the limit."""

    def __init__(self, limit=None):
        torch = _torch()
        self.device = torch.cuda.current_device()
        self.limit = limit
        self.live = {}

        def alloc(ctx, nbytes, out):
            try:
                if self.limit is not None and sum(self.live.values()) + nbytes > self.limit:
                    return 1
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
            except Exception:
                return 1
            self.live[ptr] = int(nbytes)
            out[0] = ptr
            return 0

        def free(ctx, ptr):
            self.live.pop(ptr, None)
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch may already be gone
                pass

        # the ctypes callbacks must outlive every handle that uses them
        self.alloc_fn = _lib.ALLOC_FN(alloc)
        self.free_fn = _lib.FREE_FN(free)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())


class Index:
    """One index handle: leaf store, filters and calibration on the current device.

    allocator: "torch" (default: torch's caching allocator owns every device
    byte of the handle), "hip" (the library's own hipMalloc), or a
    TorchAllocator instance."""

    def __init__(self, allocator="torch"):
        lib = load()
        h = ctypes.c_void_p()
        if allocator == "torch":
            allocator = TorchAllocator()
        if allocator == "hip" or allocator is None:
            self._alloc = None
            check(lib.leafi_create(_lib.ALLOC_FN(), _lib.FREE_FN(), None, ctypes.byref(h)))
        else:
            self._alloc = allocator
            check(lib.leafi_create(allocator.alloc_fn, allocator.free_fn, None, ctypes.byref(h)))
        self._h = h
        self._m = None

    def close(self):
        if getattr(self, "_h", None):
            load().leafi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- build
    def build(self, series, leaf_capacity: int, n_segments: int = 16, split_rule: str = "median"):
        torch = _torch()
        n, m = series.shape
        o = _lib.BuildOpts(leaf_capacity, n_segments, {"median": 0, "midpoint": 1, "isax": 2}[split_rule], 0)
        check(load().leafi_build_index(self._h, _dev(series, torch.float32, "series"), n, m, ctypes.byref(o),
                                       _stream()))
        self._m = m
        return self

    def info(self) -> dict:
        i = _lib.Info()
        check(load().leafi_get_info(self._h, ctypes.byref(i)))
        return struct_dict(i)

    def leaves(self):
        inf = self.info()
        off = np.zeros(inf["n_leaves"] + 1, dtype=np.int64)
        mem = np.zeros(inf["n_series"], dtype=np.int64)
        check(load().leafi_export_leaves(self._h, off.ctypes.data_as(ctypes.c_void_p),
                                         mem.ctypes.data_as(ctypes.c_void_p)))
        return off, mem

    def boxes(self) -> np.ndarray:
        inf = self.info()
        b = np.zeros((inf["n_leaves"], inf["n_segments"], 4), dtype=np.float32)
        check(load().leafi_export_boxes(self._h, b.ctypes.data_as(ctypes.c_void_p)))
        return b

    # -------------------------------------------------------------- filters
    def train_filters(self, **kw) -> dict:
        """Algorithm 1 (leafi_train_filters); options are leafi_train_opts
        fields, with selection given as "size" (Algorithm 3) or "knapsack"
        (Equations 1-2) and arch as "mlp" or "cnn"."""
        o = _lib.TrainOpts()
        load().leafi_default_train_opts(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown training option {k}")
            if k == "selection" and isinstance(v, str):
                v = {"size": _lib.LEAFI_SELECT_SIZE, "knapsack": _lib.LEAFI_SELECT_KNAPSACK}[v]
            if k == "arch" and isinstance(v, str):
                v = {"mlp": _lib.LEAFI_FILTER_MLP, "cnn": _lib.LEAFI_FILTER_CNN}[v]
            setattr(o, k, v)
        r = _lib.TrainReport()
        check(load().leafi_train_filters(self._h, ctypes.byref(o), ctypes.byref(r), _stream()))
        return struct_dict(r)

    def examples(self):
        """The kept training set (train_filters(keep_examples=1)): raw queries
        [nq, m] (device), example queries [F, n_ex] int32 (host), targets
        [F, n_ex] (device) and the number of training examples per filter."""
        torch = _torch()
        nq, nex, ntr = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        lib = load()
        check(lib.leafi_get_examples(self._h, ctypes.byref(nq), ctypes.byref(nex), ctypes.byref(ntr), None, None,
                                     None, _stream()))
        inf = self.info()
        F, m = inf["n_filters"], inf["m"]
        q = torch.empty((nq.value, m), dtype=torch.float32, device="cuda")
        exq = np.zeros((F, nex.value), dtype=np.int32)
        y = torch.empty((F, nex.value), dtype=torch.float32, device="cuda")
        check(lib.leafi_get_examples(self._h, None, None, None, ctypes.c_void_p(q.data_ptr()),
                                     exq.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(y.data_ptr()), _stream()))
        return q, exq, y, ntr.value

    def train_trace(self):
        """Of the kept training run: (epochs run per filter [F] int32,
        validation MSE after each epoch [F, max_epochs], NaN past the end)."""
        me = ctypes.c_int32()
        lib = load()
        check(lib.leafi_get_train_trace(self._h, ctypes.byref(me), None, None))
        F = self.info()["n_filters"]
        ep = np.zeros(F, dtype=np.int32)
        tr = np.zeros((F, me.value), dtype=np.float32)
        check(lib.leafi_get_train_trace(self._h, None, ep.ctypes.data_as(ctypes.c_void_p),
                                        tr.ctypes.data_as(ctypes.c_void_p)))
        return ep, tr

    def set_filters(self, leaf_ids, weights, hidden: int):
        torch = _torch()
        ids = np.ascontiguousarray(leaf_ids, dtype=np.int32)
        check(load().leafi_set_filters(self._h, len(ids), hidden, ids.ctypes.data_as(ctypes.c_void_p),
                                       _dev(weights, torch.float32, "weights"), _stream()))

    def set_cnn_filters(self, leaf_ids, weights, channels: int):
        """Install CNN filters (LEAFI_FILTER_CNN packing) on the given leaves."""
        torch = _torch()
        ids = np.ascontiguousarray(leaf_ids, dtype=np.int32)
        check(load().leafi_set_cnn_filters(self._h, len(ids), channels, ids.ctypes.data_as(ctypes.c_void_p),
                                           _dev(weights, torch.float32, "weights"), _stream()))

    def get_filters(self):
        torch = _torch()
        inf = self.info()
        F, h, m = inf["n_filters"], inf["hidden"], inf["m"]
        ids = np.zeros(F, dtype=np.int32)
        P = 3 * h * h + 6 * h + 1 if inf["filter_arch"] == _lib.LEAFI_FILTER_CNN else h * m + 2 * h + 1
        w = torch.empty((F, P), dtype=torch.float32, device="cuda")
        check(load().leafi_get_filters(self._h, ids.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.c_void_p(w.data_ptr()) if F else None, _stream()))
        return ids, w

    # -------------------------------------------------------------- calibration
    def calibrate(self, calib, ks, targets, mapping: str = "step", corrected: bool = True):
        torch = _torch()
        ks_a = np.ascontiguousarray(ks, dtype=np.int32)
        t_a = np.ascontiguousarray(targets, dtype=np.float32)
        flags = {"step": _lib.LEAFI_CALIB_STEP, "steffen": _lib.LEAFI_CALIB_STEFFEN}[mapping]
        if not corrected:
            flags |= _lib.LEAFI_CALIB_NO_CORRECTION
        check(load().leafi_calibrate(self._h, _dev(calib, torch.float32, "calib"), calib.shape[0],
                                     ks_a.ctypes.data_as(ctypes.c_void_p), len(ks_a),
                                     t_a.ctypes.data_as(ctypes.c_void_p), len(t_a), flags, _stream()))

    def offsets(self) -> np.ndarray:
        inf = self.info()
        o = np.zeros((inf["n_calibrated"], inf["n_filters"]), dtype=np.float32)
        check(load().leafi_get_offsets(self._h, o.ctypes.data_as(ctypes.c_void_p)))
        return o

    def set_offsets(self, ks, targets, offsets):
        ks_a = np.ascontiguousarray(ks, dtype=np.int32)
        t_a = np.ascontiguousarray(targets, dtype=np.float32)
        o = np.ascontiguousarray(offsets, dtype=np.float32)
        check(load().leafi_set_offsets(self._h, ks_a.ctypes.data_as(ctypes.c_void_p), len(ks_a),
                                       t_a.ctypes.data_as(ctypes.c_void_p), len(t_a),
                                       o.ctypes.data_as(ctypes.c_void_p)))

    # -------------------------------------------------------------- search
    def search(self, queries, k=1, target=1.0, k_max=None, scan: str = "bf16", use_filters: bool = True,
               schedule=(1, 0), kprime: int = 0, with_stats: bool = False, out=None, flags: int = 0):
        torch = _torch()
        nq = queries.shape[0]
        dev = queries.device
        kt = k if isinstance(k, torch.Tensor) else torch.full((nq,), int(k), dtype=torch.int32, device=dev)
        tt = target if isinstance(target, torch.Tensor) else torch.full((nq,), float(target), dtype=torch.float32,
                                                                         device=dev)
        if k_max is None:
            k_max = int(k) if not isinstance(k, torch.Tensor) else int(kt.max().item()) if nq else 1
        o = _lib.SearchOpts()
        load().leafi_default_search_opts(ctypes.byref(o))
        o.k_max = k_max
        o.scan = {"bf16": _lib.LEAFI_SCAN_BF16, "fp32": _lib.LEAFI_SCAN_FP32}[scan]
        o.use_filters = 1 if use_filters else 0
        o.n_schedule = len(schedule)
        for i, s in enumerate(schedule):
            o.schedule[i] = s
        o.kprime = kprime
        o.flags = flags
        if out is None:
            ids = torch.empty((nq, k_max), dtype=torch.int64, device=dev)
            dists = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        else:
            ids, dists = out
        st = _lib.SearchStats()
        check(load().leafi_search_knn(self._h, _dev(queries, torch.float32, "queries"), nq,
                                      _dev(kt, torch.int32, "k"), _dev(tt, torch.float32, "target"),
                                      ctypes.byref(o), _dev(ids, torch.int64, "ids"),
                                      _dev(dists, torch.float32, "dists"),
                                      ctypes.byref(st) if with_stats else None, _stream()))
        if with_stats:
            return ids, dists, struct_dict(st)
        return ids, dists

    def search_noalloc(self, queries, k, target, out, k_max: int, use_filters: bool = True, schedule=(1, 0),
                       kprime: int = 0, flags: int = 0):
        """leafi_search_knn_noalloc: the planned batch search with every buffer
        carved from the library's fixed scratch area (nothing allocated).
        k [nq] int32, target [nq] fp32 and out = (ids, dists) are device
        tensors; results are written into out."""
        torch = _torch()
        nq = queries.shape[0]
        o = _lib.SearchOpts()
        load().leafi_default_search_opts(ctypes.byref(o))
        o.k_max = k_max
        o.use_filters = 1 if use_filters else 0
        o.n_schedule = len(schedule)
        for i, s_ in enumerate(schedule):
            o.schedule[i] = s_
        o.kprime = kprime
        o.flags = flags
        check(load().leafi_search_knn_noalloc(self._h, _dev(queries, torch.float32, "queries"), nq,
                                              _dev(k, torch.int32, "k"), _dev(target, torch.float32, "target"),
                                              ctypes.byref(o), _dev(out[0], torch.int64, "ids"),
                                              _dev(out[1], torch.float32, "dists"), _stream()))
        return out

    def searcher(self, queries, k, target, out, k_max: int, use_filters: bool = True, schedule=(1, 0),
                 kprime: int = 0, flags: int = 0, with_stats: bool = False):
        """A search bound to fixed device buffers (queries [nq, m] fp32, k [nq]
        int32, target [nq] fp32, out = (ids [nq, k_max] int64, dists [nq,
        k_max] fp32)): the arguments are marshalled once, so each call costs
        one library call.  The buffers' contents may change between calls.
        Returns a function of no arguments that returns the statistics dict
        (with_stats) or None."""
        torch = _torch()
        nq = queries.shape[0]
        o = _lib.SearchOpts()
        load().leafi_default_search_opts(ctypes.byref(o))
        o.k_max = k_max
        o.use_filters = 1 if use_filters else 0
        o.n_schedule = len(schedule)
        for i, s_ in enumerate(schedule):
            o.schedule[i] = s_
        o.kprime = kprime
        o.flags = flags
        st = _lib.SearchStats()
        args = (self._h, _dev(queries, torch.float32, "queries"), nq, _dev(k, torch.int32, "k"),
                _dev(target, torch.float32, "target"), ctypes.byref(o), _dev(out[0], torch.int64, "ids"),
                _dev(out[1], torch.float32, "dists"), ctypes.byref(st) if with_stats else None, _stream())
        fn = load().leafi_search_knn
        keep = (queries, k, target, out, o, st)  # the buffers stay alive with the closure

        def run():
            check(fn(*args))
            return struct_dict(keep[5]) if with_stats else None
        return run

    def autotune(self, queries, k=1, target=1.0, k_max=None, use_filters: bool = True, schedule=(1, 0),
                 kprime: int = 0, repeats: int = 5):
        """Time the BF16 scan's tile shapes on this sample batch and keep the
        fastest for later searches; returns the tuner's report."""
        torch = _torch()
        nq = queries.shape[0]
        dev = queries.device
        kt = k if isinstance(k, torch.Tensor) else torch.full((nq,), int(k), dtype=torch.int32, device=dev)
        tt = target if isinstance(target, torch.Tensor) else torch.full((nq,), float(target), dtype=torch.float32,
                                                                         device=dev)
        if k_max is None:
            k_max = int(k) if not isinstance(k, torch.Tensor) else int(kt.max().item())
        o = _lib.SearchOpts()
        load().leafi_default_search_opts(ctypes.byref(o))
        o.k_max = k_max
        o.use_filters = 1 if use_filters else 0
        o.n_schedule = len(schedule)
        for i, s_ in enumerate(schedule):
            o.schedule[i] = s_
        o.kprime = kprime
        rep = _lib.TuneReport()
        check(load().leafi_autotune(self._h, _dev(queries, torch.float32, "queries"), nq, _dev(kt, torch.int32, "k"),
                                    _dev(tt, torch.float32, "target"), ctypes.byref(o), repeats, ctypes.byref(rep),
                                    _stream()))
        n = rep.n_candidates
        return {"candidates": [{"chunk_rows": rep.chunk_rows[i], "queries_per_tile": rep.queries_per_tile[i],
                                "ms": rep.ms[i]} for i in range(n)],
                "chosen": {"chunk_rows": rep.chunk_rows[rep.chosen], "queries_per_tile": rep.queries_per_tile[rep.chosen],
                           "ms": rep.ms[rep.chosen]}}

    def set_tiling(self, chunk_rows: int = 1024, queries_per_tile: int = 32):
        check(load().leafi_set_tiling(self._h, chunk_rows, queries_per_tile))

    def graph_note(self) -> str:
        """Why planned batches stopped being captured into graphs ('' while they are)."""
        return (load().leafi_graph_note(self._h) or b"").decode()

    def set_plan_capacity(self, max_items: int = 0):
        """Item capacity of a planned batch's passes (0 = what 16 GiB of buffers hold)."""
        check(load().leafi_set_plan_capacity(self._h, int(max_items)))

    def lower_bounds(self, queries):
        torch = _torch()
        nq = queries.shape[0]
        lb = torch.empty((nq, self.info()["n_leaves"]), dtype=torch.float32, device=queries.device)
        check(load().leafi_lower_bounds(self._h, _dev(queries, torch.float32, "queries"), nq,
                                        _dev(lb, torch.float32, "lb"), _stream()))
        return lb

    def select_knapsack(self, queries, a: float = 2.0, t_filter: float = 0.0, t_series: float = 0.0,
                        hidden: int = 0, mem_budget: int = 8 << 30) -> dict:
        """Leaf selection as a knapsack (leafi_select_knapsack) over raw
        training queries (device [nq, m] fp32): the selected leaves (by
        benefit, largest first) and per leaf the benefit b, p_lb and the ideal
        filter rate p_f.  t_filter / t_series <= 0: measured on this GPU."""
        torch = _torch()
        nq = queries.shape[0]
        N = self.info()["n_leaves"]
        ids = np.zeros(N, dtype=np.int32)
        ns = ctypes.c_int32()
        b, pl, pf = (np.zeros(N, dtype=np.float64) for _ in range(3))
        check(load().leafi_select_knapsack(self._h, _dev(queries, torch.float32, "queries"), nq, a, t_filter, t_series,
                                           hidden, mem_budget, ids.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns),
                                           b.ctypes.data_as(ctypes.c_void_p), pl.ctypes.data_as(ctypes.c_void_p),
                                           pf.ctypes.data_as(ctypes.c_void_p), _stream()))
        return {"leaves": ids[:ns.value].copy(), "benefit": b, "p_lb": pl, "p_f": pf}

    def leaf_knn(self, queries, k: int):
        torch = _torch()
        nq = queries.shape[0]
        N = self.info()["n_leaves"]
        d = torch.empty((nq, N, k), dtype=torch.float32, device=queries.device)
        ids = torch.empty((nq, N, k), dtype=torch.int64, device=queries.device)
        check(load().leafi_leaf_knn(self._h, _dev(queries, torch.float32, "queries"), nq, k,
                                    _dev(d, torch.float32, "d"), _dev(ids, torch.int64, "ids"), _stream()))
        return d, ids


class Server:
    """Continuous-batching request server over a built (and calibrated) Index.

    The index must not be used by other calls while the server exists.
    Queries are host arrays (numpy fp32 [m] or [n, m]).
    """

    def __init__(self, index: Index, k_max: int = 1, max_slots: int = 1024, scan: str = "bf16",
                 use_filters: bool = True, schedule=(1, 0), queue_capacity: int = 1 << 20,
                 mem_budget: int = 4 << 30):
        lib = load()
        o = _lib.ServerOpts()
        lib.leafi_default_server_opts(ctypes.byref(o))
        o.max_slots = max_slots
        o.k_max = k_max
        o.scan = {"bf16": _lib.LEAFI_SCAN_BF16, "fp32": _lib.LEAFI_SCAN_FP32}[scan]
        o.use_filters = 1 if use_filters else 0
        o.n_schedule = len(schedule)
        for i, v in enumerate(schedule):
            o.schedule[i] = v
        o.queue_capacity = queue_capacity
        o.mem_budget = mem_budget
        h = ctypes.c_void_p()
        check(lib.leafi_server_create(index._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._index = index  # keeps the index alive
        self.k_max = k_max
        self.m = index.info()["m"]

    @property
    def slots(self) -> int:
        n = ctypes.c_int32()
        check(load().leafi_server_info(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            load().leafi_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, query, k: int = 1, target: float = 1.0) -> int:
        q = np.ascontiguousarray(query, dtype=np.float32)
        t = ctypes.c_uint64()
        check(load().leafi_server_submit(self._h, q.ctypes.data_as(ctypes.c_void_p), k, target, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """Returns None while running, else (ids [k_max], dists [k_max], latency_ms)."""
        ids = np.empty(self.k_max, dtype=np.int64)
        d = np.empty(self.k_max, dtype=np.float32)
        lat = ctypes.c_double()
        done = ctypes.c_int32()
        check(load().leafi_server_poll(self._h, ticket, ids.ctypes.data_as(ctypes.c_void_p),
                                       d.ctypes.data_as(ctypes.c_void_p), ctypes.byref(lat), ctypes.byref(done)))
        return (ids, d, lat.value) if done.value else None

    def replay(self, queries, arrival_s, ks, targets):
        q = np.ascontiguousarray(queries, dtype=np.float32)
        n = q.shape[0]
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        k = np.ascontiguousarray(np.broadcast_to(ks, (n,)), dtype=np.int32)
        t = np.ascontiguousarray(np.broadcast_to(targets, (n,)), dtype=np.float32)
        ids = np.empty((n, self.k_max), dtype=np.int64)
        d = np.empty((n, self.k_max), dtype=np.float32)
        lat = np.empty(n, dtype=np.float64)
        rep = _lib.ServerReport()
        P = ctypes.c_void_p
        check(load().leafi_server_replay(self._h, q.ctypes.data_as(P), n, arr.ctypes.data_as(P),
                                         k.ctypes.data_as(P), t.ctypes.data_as(P), ids.ctypes.data_as(P),
                                         d.ctypes.data_as(P), lat.ctypes.data_as(P), ctypes.byref(rep)))
        return ids, d, lat, struct_dict(rep)


def znorm(x):
    torch = _torch()
    out = torch.empty_like(x)
    n, m = x.shape
    check(load().leafi_znorm(_dev(x, torch.float32, "x"), n, m, _dev(out, torch.float32, "out"), _stream()))
    return out


def mlp_infer(weights, m: int, hidden: int, x):
    torch = _torch()
    F = weights.shape[0]
    nq = x.shape[0]
    out = torch.empty((nq, F), dtype=torch.float32, device=x.device)
    check(load().leafi_mlp_infer(_dev(weights, torch.float32, "weights"), F, m, hidden,
                                 _dev(x, torch.float32, "x"), nq, _dev(out, torch.float32, "out"), _stream()))
    return out


def mlp_sgd_step(weights, m: int, hidden: int, x, y, lr: float):
    """One SGD step per filter in place; x [F, B, m], y [F, B]; returns the batch losses."""
    torch = _torch()
    F, B, _ = x.shape
    loss = torch.empty((F,), dtype=torch.float32, device=x.device)
    check(load().leafi_mlp_sgd_step(_dev(weights, torch.float32, "weights"), F, m, hidden,
                                    _dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), B, lr,
                                    _dev(loss, torch.float32, "loss"), _stream()))
    return loss


def cnn_infer(weights, m: int, channels: int, x):
    """CNN filter predictions d^f [nq, F] for z-normalised x [nq, m]."""
    torch = _torch()
    F = weights.shape[0]
    nq = x.shape[0]
    out = torch.empty((nq, F), dtype=torch.float32, device=x.device)
    check(load().leafi_cnn_infer(_dev(weights, torch.float32, "weights"), F, m, channels,
                                 _dev(x, torch.float32, "x"), nq, _dev(out, torch.float32, "out"), _stream()))
    return out


def cnn_sgd_step(weights, m: int, channels: int, x, y, lr: float):
    """One SGD step per CNN filter in place; x [F, B, m], y [F, B]; returns the batch losses."""
    torch = _torch()
    F, B, _ = x.shape
    loss = torch.empty((F,), dtype=torch.float32, device=x.device)
    check(load().leafi_cnn_sgd_step(_dev(weights, torch.float32, "weights"), F, m, channels,
                                    _dev(x, torch.float32, "x"), _dev(y, torch.float32, "y"), B, lr,
                                    _dev(loss, torch.float32, "loss"), _stream()))
    return loss
