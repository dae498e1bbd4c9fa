"""CPU oracle for exact subgraph matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it imports nothing from the GPU package.

The arithmetic lives in ``oracle.c`` (plain C, pthreads); this module only
compiles and loads it with ctypes and marshals numpy arrays.  What it computes
is stated at the top of ``oracle.c``: the set of matches of Def. 1 found by the
depth-first search of Alg. 1 with the local-candidate rule of Sec. 4.1.

Parity status of the functions here:
  * match / count / enumerate -- pinned by brute force over all injective maps,
    by networkx's monomorphism matcher, by closed forms (cliques, labelled
    cliques, grids, complete bipartite graphs, trace identities, stars) and by
    invariants (order, relabelling, label permutation, disjoint union,
    automorphism divisibility); see tests/test_oracle_pins.py.
  * work counters (tasks, groups) -- pinned by closed forms on complete graphs
    and stars.
  * ri_order -- a heuristic; pinned only by validity (a connected permutation)
    and by hand-worked small cases.
  * The paper's Figure-1 example (112 matches) is parity unpinned: the figure
    holding that graph is not part of the paper text.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_GRAPH, ERR_QUERY, ERR_ORDER, ERR_NOMEM = 0, -1, -2, -3, -4, -5
DONE, CAPPED, TIMEOUT = 0, 1, 2


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class _Result(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_uint64),
        ("outcome", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("tasks", ctypes.c_uint64),
        ("groups", ctypes.c_uint64),
        ("rows", ctypes.c_uint64),
        ("seconds", ctypes.c_double),
    ]


@dataclasses.dataclass
class Result:
    count: int
    outcome: int
    threads: int
    tasks: int
    groups: int
    seconds: float
    rows: Optional[np.ndarray] = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, -O2, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i32, u64, dbl = ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        lib.orc_check_graph.argtypes = [i32, p, p, i32]
        lib.orc_check_query.argtypes = [i32, i32, p]
        lib.orc_check_order.argtypes = [i32, i32, p, p]
        lib.orc_ri_order.argtypes = [i32, i32, p, p]
        lib.orc_match.argtypes = [i32, p, p, p, i32, i32, p, p, p, u64, dbl, i32, p, u64,
                                  ctypes.POINTER(_Result)]
        for f in (lib.orc_check_graph, lib.orc_check_query, lib.orc_check_order, lib.orc_ri_order,
                  lib.orc_match):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(row_ptr, col, labels):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    lb = np.ascontiguousarray(labels, dtype=np.int32)
    return rp, cl, lb


def _query_arrays(edges, qlabels):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    ql = np.ascontiguousarray(qlabels, dtype=np.int32)
    return e, ql


def check_graph(row_ptr, col, check_symmetry: bool = True) -> int:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    return _load().orc_check_graph(rp.shape[0] - 1, _ptr(rp), _ptr(cl), int(check_symmetry))


def check_query(k: int, edges) -> int:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    return _load().orc_check_query(k, e.shape[0], _ptr(e))


def check_order(k: int, edges, order) -> int:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    o = np.ascontiguousarray(order, dtype=np.int32)
    return _load().orc_check_order(k, e.shape[0], _ptr(e), _ptr(o))


def ri_order(k: int, edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    out = np.zeros(k, dtype=np.int32)
    rc = _load().orc_ri_order(k, e.shape[0], _ptr(e), _ptr(out))
    if rc:
        raise OracleError(rc, "ri_order")
    return out


def match(row_ptr, col, labels, k: int, edges, qlabels, order=None, cap: int = 0,
          time_limit_s: float = 0.0, threads: int = 0, enumerate_rows: int = 0) -> Result:
    """Count matches (and list up to ``enumerate_rows`` of them, unsorted)."""
    rp, cl, lb = _graph_arrays(row_ptr, col, labels)
    e, ql = _query_arrays(edges, qlabels)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    rows = np.zeros((enumerate_rows, k), dtype=np.int32) if enumerate_rows > 0 else None
    res = _Result()
    rc = _load().orc_match(rp.shape[0] - 1, _ptr(rp), _ptr(cl), _ptr(lb), k, e.shape[0], _ptr(e),
                           _ptr(ql), _ptr(o), int(cap), float(time_limit_s), int(threads), _ptr(rows),
                           int(enumerate_rows), ctypes.byref(res))
    if rc:
        raise OracleError(rc, "match")
    out = Result(int(res.count), int(res.outcome), int(res.threads), int(res.tasks), int(res.groups),
                 float(res.seconds))
    if rows is not None:
        out.rows = rows[: int(res.rows)]
    return out


def count(g, q, **kw) -> Result:
    """match() on a workloads.Graph / workloads.Query pair (duck-typed)."""
    return match(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, **kw)


def enumerate_sorted(g, q, limit: int, **kw) -> np.ndarray:
    """All matches (at most ``limit``) as rows indexed by query vertex, sorted lexicographically."""
    r = match(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, enumerate_rows=limit, **kw)
    rows = r.rows
    if rows.shape[0] == 0:
        return rows
    idx = np.lexsort(rows.T[::-1])
    return rows[idx]
