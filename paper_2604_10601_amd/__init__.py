"""Python binding of libgmatch (the gfx950 subgraph-matching engine).

Argument marshalling only: every step of a search runs in the HIP kernels
behind the C ABI declared in include/gmatch.h.  The shared library is built
in-tree by ``paper_2604_10601_amd/build.py`` (or ``__graft_entry__.build()``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmatch.so")

GM_OK, GM_ERR_ARG, GM_ERR_GRAPH, GM_ERR_QUERY, GM_ERR_ORDER = 0, -1, -2, -3, -4
GM_ERR_NOMEM, GM_ERR_DEVICE, GM_ERR_BUFFER, GM_ERR_STATE = -5, -6, -7, -8
GM_DONE, GM_CAPPED, GM_TIMEOUT = 0, 1, 2

ABI_FUNCTIONS = ("gm_create", "gm_destroy", "gm_load_graph", "gm_load_graph_device", "gm_load_query", "gm_set_order",
                 "gm_get_order", "gm_count", "gm_enumerate", "gm_count_batch", "gm_tune_batch",
                 "gm_get_options", "gm_serve_open", "gm_serve_submit", "gm_serve_poll", "gm_serve_stats",
                 "gm_serve_close", "gm_serve_request_bytes", "gm_order_features", "gm_candidate_orders",
                 "gm_model_create",
                 "gm_model_destroy", "gm_model_predict", "gm_model_train", "gm_model_get_params",
                 "gm_model_set_params", "gm_model_last_error", "gm_choose_order", "gm_set_symmetry_breaking", "gm_free_query",
                 "gm_candidate_sets", "gm_count_noalloc", "gm_set_split", "gm_get_split",
                 "gm_choose_plan", "gm_last_error")

ORDER_FEATURES = 192


class GmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gmatch error {status}: {message}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("tau", ctypes.c_int64),
        ("pool_row_limit", ctypes.c_int64),
        ("disable_stealing", ctypes.c_int32),
        ("steal_threshold", ctypes.c_int32),
        ("waves_per_cu", ctypes.c_int32),
        ("skip_symmetry_check", ctypes.c_int32),
        ("stack_layout", ctypes.c_int32),
        ("disable_label_index", ctypes.c_int32),
        ("batch_single_launch", ctypes.c_int32),
        ("batch_streams", ctypes.c_int32),
        ("pool_hub_cut", ctypes.c_int32),
        ("disable_hub_bitmaps", ctypes.c_int32),
        ("hub_bitmap_mib", ctypes.c_int32),
        ("candidate_graph", ctypes.c_int32),
        ("pool_roots_per_item", ctypes.c_int32),
        ("merge_ratio", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("kernel_ms", ctypes.c_double),
        ("launches", ctypes.c_int32),
        ("grid_waves", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("tasks", ctypes.c_uint64),
        ("scanned", ctypes.c_uint64),
        ("lookups", ctypes.c_uint64),
        ("probes", ctypes.c_uint64),
        ("groups", ctypes.c_uint64),
        ("steals", ctypes.c_uint64),
        ("bytes", ctypes.c_uint64),
        ("bytes_late", ctypes.c_uint64),
        ("reserved", ctypes.c_uint64 * 2),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Tuning(ctypes.Structure):  # gm_tuning
    _fields_ = [
        ("waves_per_cu", ctypes.c_int32),
        ("steal_threshold", ctypes.c_int32),
        ("stack_layout", ctypes.c_int32),
        ("batch_single_launch", ctypes.c_int32),
        ("batch_streams", ctypes.c_int32),
        ("trials", ctypes.c_int32),
        ("best_ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
        ("merge_ratio", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class _CResult(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64),
        ("outcome", ctypes.c_int32),
        ("pool_depth", ctypes.c_int32),
        ("search_ms", ctypes.c_double),
        ("pool_rows", ctypes.c_uint64),
        ("groups", ctypes.c_uint64),
        ("tasks", ctypes.c_uint64),
        ("lanes_active", ctypes.c_uint64),
        ("lanes_issued", ctypes.c_uint64),
        ("probes", ctypes.c_uint64),
        ("steals", ctypes.c_uint64),
        ("rows", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("grid_waves", ctypes.c_int32),
        ("candidate_rounds", ctypes.c_int32),
        ("kernel_tasks", ctypes.c_uint64),
        ("kernel_probes", ctypes.c_uint64),
        ("kernel_groups", ctypes.c_uint64),
        ("scanned", ctypes.c_uint64),
        ("kernel_scanned", ctypes.c_uint64),
        ("kernel_lookups", ctypes.c_uint64),
        ("candidate_ms", ctypes.c_double),
        ("candidate_edges", ctypes.c_uint64),
        ("kernel_bytes", ctypes.c_uint64),
        ("query_ms", ctypes.c_double),
        ("kernel_bytes_late", ctypes.c_uint64),
    ]


class ServeOptions(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("waves_per_cu", ctypes.c_int32),
        ("batch_streams", ctypes.c_int32),
        ("max_pending", ctypes.c_int64),
        ("memory_mib", ctypes.c_int64),
        ("reserved", ctypes.c_int32 * 4),
    ]


@dataclasses.dataclass
class Result:
    count: int
    outcome: int
    pool_depth: int
    search_ms: float
    pool_rows: int
    groups: int
    tasks: int
    lanes_active: int
    lanes_issued: int
    probes: int
    steals: int
    rows: int
    kernel_ms: float
    grid_waves: int
    kernel_tasks: int = 0
    kernel_probes: int = 0
    kernel_groups: int = 0
    scanned: int = 0
    kernel_scanned: int = 0
    kernel_lookups: int = 0
    matches: Optional[np.ndarray] = None
    candidate_rounds: int = 0
    candidate_ms: float = 0.0
    candidate_edges: int = 0
    kernel_bytes: int = 0
    kernel_bytes_late: int = 0
    query_ms: float = 0.0

    @property
    def idle_rate(self) -> float:
        return 1.0 - self.lanes_active / self.lanes_issued if self.lanes_issued else 0.0


class _CServeResult(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("qid", ctypes.c_int32),
        ("slot", ctypes.c_int32),
        ("submit_ms", ctypes.c_double),
        ("start_ms", ctypes.c_double),
        ("done_ms", ctypes.c_double),
        ("result", _CResult),
        ("status", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


@dataclasses.dataclass
class ServeResult:
    ticket: int
    qid: int
    slot: int
    submit_ms: float
    start_ms: float
    done_ms: float
    result: "Result"
    status: int = 0

    @property
    def latency_ms(self) -> float:
        return self.done_ms - self.submit_ms


_lib = None


def load_library():
    """Load libgmatch.so (raises if it has not been built).

    PyTorch for ROCm ships its own HIP and HSA runtimes, and two runtimes in one
    process cannot both own the GPU: whichever initialises second finds no
    device.  When torch is installed it is therefore imported first, so that
    libgmatch binds to the runtime torch has loaded and device buffers and
    streams can pass between the two.  Without torch the system runtime is used.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_10601_amd/build.py")
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime before libgmatch resolves its own)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.gm_create.argtypes = [i32, ctypes.POINTER(Options), ctypes.POINTER(p)]
    lib.gm_destroy.argtypes = [p]
    lib.gm_destroy.restype = None
    lib.gm_load_graph.argtypes = [p, i32, p, p, p]
    lib.gm_load_graph_device.argtypes = [p, i32, p, i32, p, p, p]
    lib.gm_load_query.argtypes = [p, i32, i32, p, p, ctypes.POINTER(i32)]
    lib.gm_set_order.argtypes = [p, i32, p]
    lib.gm_get_order.argtypes = [p, i32, p]
    lib.gm_count.argtypes = [p, i32, u64, dbl, ctypes.POINTER(_CResult)]
    lib.gm_enumerate.argtypes = [p, i32, p, u64, dbl, ctypes.POINTER(_CResult)]
    lib.gm_count_batch.argtypes = [p, i32, p, u64, dbl, p, ctypes.POINTER(BatchInfo)]
    lib.gm_count_noalloc.argtypes = [p, i32, u64, dbl, ctypes.POINTER(_CResult)]
    lib.gm_tune_batch.argtypes = [p, i32, p, u64, dbl, ctypes.POINTER(Tuning)]
    lib.gm_get_options.argtypes = [p, ctypes.POINTER(Options)]
    lib.gm_serve_open.argtypes = [p, ctypes.POINTER(ServeOptions), ctypes.POINTER(p)]
    lib.gm_serve_submit.argtypes = [p, i32, u64, dbl, ctypes.POINTER(u64)]
    lib.gm_serve_poll.argtypes = [p, p, i32, dbl, ctypes.POINTER(i32)]
    lib.gm_serve_stats.argtypes = [p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64)]
    lib.gm_serve_close.argtypes = [p]
    lib.gm_serve_request_bytes.argtypes = [p, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.gm_order_features.argtypes = [p, i32, p, p]
    lib.gm_candidate_orders.argtypes = [p, i32, i32, u64, p, ctypes.POINTER(i32)]
    lib.gm_model_create.argtypes = [i32, i32, i32, u64, ctypes.POINTER(p)]
    lib.gm_model_destroy.argtypes = [p]
    lib.gm_model_destroy.restype = None
    lib.gm_model_predict.argtypes = [p, p, i32, i32, p]
    lib.gm_model_train.argtypes = [p, p, p, i32, i32, i32, i32, ctypes.c_float, u64, ctypes.POINTER(ctypes.c_float)]
    lib.gm_model_get_params.argtypes = [p, p, p, p, p, p, p]
    lib.gm_model_set_params.argtypes = [p, p, p, p, p, p, p]
    lib.gm_model_last_error.argtypes = [p]
    lib.gm_model_last_error.restype = ctypes.c_char_p
    lib.gm_choose_order.argtypes = [p, p, i32, i32, u64, ctypes.c_float, ctypes.POINTER(i32), p]
    lib.gm_set_symmetry_breaking.argtypes = [p, i32, i32, ctypes.POINTER(u64)]
    lib.gm_set_split.argtypes = [p, i32, i32]
    lib.gm_get_split.argtypes = [p, i32, ctypes.POINTER(i32)]
    lib.gm_choose_plan.argtypes = [p, p, i32, i32, u64, p, i32, ctypes.c_float, u64, dbl, ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), p, ctypes.POINTER(dbl)]
    lib.gm_free_query.argtypes = [p, i32]
    lib.gm_candidate_sets.argtypes = [p, i32, p, ctypes.POINTER(u64), ctypes.POINTER(i32)]
    lib.gm_last_error.argtypes = [p]
    lib.gm_last_error.restype = ctypes.c_char_p
    for name in ("gm_create", "gm_load_graph", "gm_load_graph_device", "gm_load_query", "gm_set_order", "gm_get_order", "gm_count",
                 "gm_enumerate", "gm_count_batch", "gm_tune_batch", "gm_get_options", "gm_serve_open",
                 "gm_serve_submit", "gm_serve_poll", "gm_serve_stats", "gm_serve_close", "gm_serve_request_bytes",
                 "gm_order_features",
                 "gm_candidate_orders", "gm_model_create", "gm_model_predict", "gm_model_train",
                 "gm_model_get_params", "gm_model_set_params", "gm_choose_order", "gm_set_symmetry_breaking",
                 "gm_free_query", "gm_candidate_sets", "gm_count_noalloc", "gm_set_split", "gm_get_split",
                 "gm_choose_plan"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Engine:
    """One resident data graph on one GPU (device=-1: host-only checks and planning)."""

    def __init__(self, device: int = 0, tau: int = 0, pool_row_limit: int = 0, disable_stealing: bool = False,
                 steal_threshold: int = 0, waves_per_cu: int = 0, skip_symmetry_check: bool = False,
                 stack_layout: int = 0, disable_label_index: bool = False, batch_single_launch: bool = False,
                 batch_streams: int = 0, pool_hub_cut: int = 0, disable_hub_bitmaps: bool = False,
                 hub_bitmap_mib: int = 0, candidate_graph: bool = False, pool_roots_per_item: int = 0,
                 merge_ratio: int = 0):
        self._lib = load_library()
        opt = Options()
        opt.tau = tau
        opt.pool_row_limit = pool_row_limit
        opt.disable_stealing = int(disable_stealing)
        opt.steal_threshold = steal_threshold
        opt.waves_per_cu = waves_per_cu
        opt.skip_symmetry_check = int(skip_symmetry_check)
        opt.stack_layout = stack_layout
        opt.disable_label_index = int(disable_label_index)
        opt.batch_single_launch = int(batch_single_launch)
        opt.batch_streams = batch_streams
        opt.pool_hub_cut = pool_hub_cut
        opt.disable_hub_bitmaps = int(disable_hub_bitmaps)
        opt.hub_bitmap_mib = hub_bitmap_mib
        opt.candidate_graph = int(candidate_graph)
        opt.pool_roots_per_item = pool_roots_per_item
        opt.merge_ratio = merge_ratio
        h = ctypes.c_void_p()
        st = self._lib.gm_create(device, ctypes.byref(opt), ctypes.byref(h))
        if st != GM_OK:
            raise GmError(st, self._lib.gm_last_error(None).decode())
        self._h = h
        self._k = {}
        self._n = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st: int):
        if st != GM_OK:
            raise GmError(st, self._lib.gm_last_error(self._h).decode())

    def load_graph(self, row_ptr, col, labels) -> None:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        lb = np.ascontiguousarray(labels, dtype=np.int32)
        self._check(self._lib.gm_load_graph(self._h, rp.shape[0] - 1, _ptr(rp), _ptr(cl), _ptr(lb)))
        self._n = rp.shape[0] - 1

    def load_graph_device(self, n: int, row_ptr_ptr: int, row_ptr_bytes: int, col_ptr: int, labels_ptr: int,
                          stream: int = 0) -> None:
        """Load G from device buffers given by address (e.g. tensor.data_ptr()); the
        engine keeps using col in place, so the caller keeps it alive (gm_load_graph_device)."""
        self._check(self._lib.gm_load_graph_device(self._h, int(n), ctypes.c_void_p(row_ptr_ptr), int(row_ptr_bytes),
                                                   ctypes.c_void_p(col_ptr), ctypes.c_void_p(labels_ptr),
                                                   ctypes.c_void_p(stream)))
        self._n = int(n)

    def load_query(self, k: int, edges, labels) -> int:
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        lb = np.ascontiguousarray(labels, dtype=np.int32)
        qid = ctypes.c_int32()
        self._check(self._lib.gm_load_query(self._h, k, e.shape[0], _ptr(e), _ptr(lb), ctypes.byref(qid)))
        self._k[qid.value] = k
        return qid.value

    def set_order(self, qid: int, order: Optional[Sequence[int]]) -> None:
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
        self._check(self._lib.gm_set_order(self._h, qid, _ptr(o)))

    def get_order(self, qid: int) -> np.ndarray:
        out = np.zeros(self._k.get(qid, 32), dtype=np.int32)
        self._check(self._lib.gm_get_order(self._h, qid, _ptr(out)))
        return out

    @staticmethod
    def _result(r: _CResult, matches=None) -> Result:
        return Result(int(r.count), int(r.outcome), int(r.pool_depth), float(r.search_ms), int(r.pool_rows),
                      int(r.groups), int(r.tasks), int(r.lanes_active), int(r.lanes_issued), int(r.probes),
                      int(r.steals), int(r.rows), float(r.kernel_ms), int(r.grid_waves), int(r.kernel_tasks),
                      int(r.kernel_probes), int(r.kernel_groups), int(r.scanned), int(r.kernel_scanned),
                      int(r.kernel_lookups), matches, int(r.candidate_rounds), float(r.candidate_ms),
                      int(r.candidate_edges), int(r.kernel_bytes), int(r.kernel_bytes_late), float(r.query_ms))

    def count(self, qid: int, cap: int = 0, time_limit_s: float = 0.0) -> Result:
        r = _CResult()
        self._check(self._lib.gm_count(self._h, qid, int(cap), float(time_limit_s), ctypes.byref(r)))
        return self._result(r)

    def enumerate(self, qid: int, cap: int, time_limit_s: float = 0.0) -> Result:
        k = self._k.get(qid, 1)
        rows = np.zeros((int(cap), k), dtype=np.int32)
        r = _CResult()
        self._check(self._lib.gm_enumerate(self._h, qid, _ptr(rows), int(cap), float(time_limit_s),
                                           ctypes.byref(r)))
        return self._result(r, rows[: int(r.rows)])

    def count_noalloc(self, qid: int, cap: int = 0, time_limit_s: float = 0.0) -> Result:
        """gm_count_noalloc: one query, no device allocation (the library's fixed arena)."""
        r = _CResult()
        self._check(self._lib.gm_count_noalloc(self._h, qid, int(cap), float(time_limit_s), ctypes.byref(r)))
        return self._result(r)

    def count_batch(self, qids: Sequence[int], cap: int = 0, time_limit_s: float = 0.0):
        """Counts of several queries in shared launches: (list of Result, BatchInfo)."""
        ids = np.ascontiguousarray(qids, dtype=np.int32)
        res = (_CResult * max(len(ids), 1))()
        info = BatchInfo()
        self._check(self._lib.gm_count_batch(self._h, len(ids), _ptr(ids), int(cap), float(time_limit_s),
                                             ctypes.cast(res, ctypes.c_void_p), ctypes.byref(info)))
        return [self._result(res[i]) for i in range(len(ids))], info

    def tune_batch(self, qids: Sequence[int], cap: int = 0, time_limit_s: float = 0.0) -> Tuning:
        """Autotune the batched launch on a sample; the engine keeps the best setting."""
        ids = np.ascontiguousarray(qids, dtype=np.int32)
        t = Tuning()
        self._check(self._lib.gm_tune_batch(self._h, len(ids), _ptr(ids), int(cap), float(time_limit_s),
                                            ctypes.byref(t)))
        return t

    def options(self) -> Options:
        o = Options()
        self._check(self._lib.gm_get_options(self._h, ctypes.byref(o)))
        return o

    def order_features(self, qid: int, order: Optional[Sequence[int]] = None) -> np.ndarray:
        out = np.zeros(ORDER_FEATURES, dtype=np.float32)
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
        self._check(self._lib.gm_order_features(self._h, qid, _ptr(o), _ptr(out)))
        return out

    def candidate_orders(self, qid: int, max_orders: int = 8, seed: int = 0) -> List[np.ndarray]:
        k = self._k.get(qid, 32)
        buf = np.zeros((max_orders, k), dtype=np.int32)
        n = ctypes.c_int32()
        self._check(self._lib.gm_candidate_orders(self._h, qid, max_orders, seed, _ptr(buf), ctypes.byref(n)))
        return [buf[i].copy() for i in range(n.value)]

    def choose_order(self, model: "Model", qid: int, max_orders: int = 8, seed: int = 0, margin: float = 0.0):
        """Let the model pick the order of qid; returns (chosen index, predictions)."""
        chosen = ctypes.c_int32()
        pred = np.zeros(max_orders, dtype=np.float32)
        self._check(self._lib.gm_choose_order(self._h, model._h, qid, max_orders, seed, float(margin),
                                              ctypes.byref(chosen), _ptr(pred)))
        return chosen.value, pred

    def set_split(self, qid: int, split: int) -> None:
        """Task split of the query's two-phase pool (0 = the engine's; gm_set_split)."""
        self._check(self._lib.gm_set_split(self._h, qid, int(split)))

    def get_split(self, qid: int) -> int:
        s = ctypes.c_int32()
        self._check(self._lib.gm_get_split(self._h, qid, ctypes.byref(s)))
        return s.value

    def choose_plan(self, model: "Model", qid: int, splits=(1, 4, 16, 64), max_orders: int = 4, seed: int = 0,
                    margin: float = 0.0, probe_cap: int = 0, probe_limit_s: float = 0.0):
        """Let the model pick order and split (gm_choose_plan), judged by a measured probe when
        probe_cap > 0: (order index, split, predictions, probe ms)."""
        sp = np.ascontiguousarray(splits, dtype=np.int32)
        pred = np.zeros(1 + max_orders * sp.shape[0], dtype=np.float32)
        co, cs, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(self._lib.gm_choose_plan(self._h, model._h, qid, max_orders, seed, _ptr(sp), sp.shape[0],
                                             float(margin), int(probe_cap), float(probe_limit_s), ctypes.byref(co),
                                             ctypes.byref(cs), _ptr(pred), ctypes.byref(ms)))
        return co.value, cs.value, pred, ms.value

    def set_symmetry_breaking(self, qid: int, enable: bool = True) -> int:
        """Count one map per automorphism class of the query; returns |Aut(Q)|."""
        aut = ctypes.c_uint64()
        self._check(self._lib.gm_set_symmetry_breaking(self._h, qid, int(enable), ctypes.byref(aut)))
        return aut.value

    def candidate_sets(self, qid: int):
        """Candidate sets of the query (boolean k x n, row u = C(u)), G' list entries, filter sweeps."""
        k, n = self._k[qid], self._n
        words = (n + 31) // 32
        bits = np.zeros(max(k * words, 1), dtype=np.uint32)
        edges, rounds = ctypes.c_uint64(), ctypes.c_int32()
        self._check(self._lib.gm_candidate_sets(self._h, qid, _ptr(bits), ctypes.byref(edges), ctypes.byref(rounds)))
        sets = np.unpackbits(bits[:k * words].view(np.uint8), bitorder="little").reshape(k, words * 32)[:, :n]
        return sets.astype(bool), edges.value, rounds.value

    def serve(self, slots: int = 0, max_batch: int = 0, waves_per_cu: int = 0, batch_streams: int = 0,
              max_pending: int = 0, memory_mib: int = 0) -> "Server":
        """Open a continuous-batching server on this engine's resident graph."""
        return Server(self, slots, max_batch, waves_per_cu, batch_streams, max_pending, memory_mib)

    def free_query(self, qid: int) -> None:
        self._check(self._lib.gm_free_query(self._h, qid))
        self._k.pop(qid, None)

    # convenience for workloads.Graph / workloads.Query
    def load(self, g) -> None:
        self.load_graph(g.row_ptr, g.col, g.labels)

    def add(self, q) -> int:
        return self.load_query(q.k, q.edges, q.labels)


class Server:
    """Continuous batching over the engine's resident graph (gm_serve_*)."""

    def __init__(self, engine: Engine, slots: int = 0, max_batch: int = 0, waves_per_cu: int = 0,
                 batch_streams: int = 0, max_pending: int = 0, memory_mib: int = 0):
        self._engine = engine
        self._lib = engine._lib
        o = ServeOptions()
        o.slots, o.max_batch, o.waves_per_cu = slots, max_batch, waves_per_cu
        o.batch_streams, o.max_pending = batch_streams, max_pending
        o.memory_mib = memory_mib
        h = ctypes.c_void_p()
        engine._check(self._lib.gm_serve_open(engine._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._buf = (_CServeResult * 4096)()

    def submit(self, qid: int, cap: int = 0, time_limit_s: float = 0.0) -> int:
        t = ctypes.c_uint64()
        self._engine._check(self._lib.gm_serve_submit(self._h, qid, int(cap), float(time_limit_s), ctypes.byref(t)))
        return t.value

    def poll(self, wait_s: float = 0.0, max_results: int = 4096) -> List[ServeResult]:
        n = ctypes.c_int32()
        m = min(max_results, len(self._buf))
        self._engine._check(self._lib.gm_serve_poll(self._h, ctypes.cast(self._buf, ctypes.c_void_p), m,
                                                    float(wait_s), ctypes.byref(n)))
        out = []
        for i in range(n.value):
            r = self._buf[i]
            out.append(ServeResult(int(r.ticket), int(r.qid), int(r.slot), float(r.submit_ms), float(r.start_ms),
                                   float(r.done_ms), Engine._result(r.result), int(r.status)))
        return out

    def request_bytes(self, qid: int) -> int:
        """Launch-state bytes admission charges for qid running alone (gm_serve_request_bytes)."""
        b = ctypes.c_int64()
        self._engine._check(self._lib.gm_serve_request_bytes(self._h, qid, ctypes.byref(b)))
        return b.value

    def stats(self):
        p, r, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._engine._check(self._lib.gm_serve_stats(self._h, ctypes.byref(p), ctypes.byref(r), ctypes.byref(d)))
        return p.value, r.value, d.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            self._engine._check(self._lib.gm_serve_close(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Model:
    """Order cost model (gm_model_*): a two-hidden-layer perceptron on the GPU."""

    def __init__(self, in_dim: int = ORDER_FEATURES, hidden: int = 128, seed: int = 0, device: int = 0):
        self._lib = load_library()
        h = ctypes.c_void_p()
        st = self._lib.gm_model_create(device, in_dim, hidden, seed, ctypes.byref(h))
        if st != GM_OK:
            raise GmError(st, "model creation failed")
        self._h = h
        self.in_dim = in_dim
        self.padded = (in_dim + 31) // 32 * 32
        self.hidden = hidden

    def _check(self, st: int):
        if st != GM_OK:
            raise GmError(st, self._lib.gm_model_last_error(self._h).decode())

    def predict(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros(x.shape[0], dtype=np.float32)
        self._check(self._lib.gm_model_predict(self._h, _ptr(x), x.shape[0], x.shape[1], _ptr(y)))
        return y

    def train(self, x, t, epochs: int = 10, batch: int = 256, lr: float = 1e-3, seed: int = 0) -> float:
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        loss = ctypes.c_float()
        self._check(self._lib.gm_model_train(self._h, _ptr(x), _ptr(t), x.shape[0], x.shape[1], epochs, batch,
                                             float(lr), seed, ctypes.byref(loss)))
        return float(loss.value)

    def get_params(self):
        D, H = self.padded, self.hidden
        w1, b1 = np.zeros((D, H), np.float32), np.zeros(H, np.float32)
        w2, b2 = np.zeros((H, H), np.float32), np.zeros(H, np.float32)
        w3, b3 = np.zeros(H, np.float32), np.zeros(1, np.float32)
        self._check(self._lib.gm_model_get_params(self._h, _ptr(w1), _ptr(b1), _ptr(w2), _ptr(b2), _ptr(w3),
                                                  _ptr(b3)))
        return w1, b1, w2, b2, w3, b3

    def set_params(self, w1, b1, w2, b2, w3, b3) -> None:
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (w1, b1, w2, b2, w3, b3)]
        self._check(self._lib.gm_model_set_params(self._h, *[_ptr(a) for a in arrs]))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.gm_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
