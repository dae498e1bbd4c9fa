"""Seeded synthetic workloads: data graphs, vertex labels and extracted queries.

This module only builds inputs.  It holds none of the matching arithmetic, so
both the GPU path and the CPU oracle can be fed from it.  Every generator takes
an explicit integer seed and draws from numpy's PCG64 or from the counter-based
SplitMix64 streams of workloads_gen.c, so a (recipe, seed) pair names one input
exactly.

Recipes (the paper's own datasets are not available; these stand in for them):

* Erdos-Renyi G(n, M): M distinct undirected pairs drawn uniformly without
  replacement, no self-loops (uniform labels as in the experimental setup,
  Sec. 6.1, "Datasets").
* R-MAT (the generator family behind the paper's ``rm`` graph, Sec. 6.1 and
  Table 3): ``edge_factor * 2**scale`` draws; each of the ``scale`` bits of a
  draw picks one quadrant (a, b, c, d) with one uniform number; the result is
  symmetrised, self-loops and duplicates are dropped and vertex ids are
  permuted at random.  Built natively (workloads_gen.c).
* Zipf labels (App. A, "label distribution skewness"): P(l) proportional to
  (l+1)**-s for l in [0, |Sigma|-1].
* Queries (Sec. 6.1, "Query Sets"): a random walk from a random seed vertex
  adds unseen neighbours until k vertices are collected (restarting after
  100 * k steps without a new one); the query is the induced subgraph on them
  with labels copied, ids in discovery order.  Walks are native
  (workloads_gen.c), walk t of a set drawing from stream t of its seed.  Dense
  means average query degree >= 3 (App. A, "query graph density").
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "workloads_gen.c")
_GEN_LIB = os.path.join(_HERE, "libworkloads.so")
_gen = None
_gen_lock = threading.Lock()


def build_native(force: bool = False) -> str:
    """Compile workloads_gen.c into libworkloads.so next to it (gcc, pthreads)."""
    if force or not os.path.exists(_GEN_LIB) or os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
        tmp = _GEN_LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _GEN_SRC])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _native():
    global _gen
    with _gen_lock:
        if _gen is None:
            if not os.path.exists(_GEN_LIB) or os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
                build_native()
            lib = ctypes.CDLL(_GEN_LIB)
            vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
            lib.wg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, u64, vp, ctypes.c_int,
                                    ctypes.POINTER(vp)]
            lib.wg_rmat.restype = ctypes.c_int
            lib.wg_graph_nnz.argtypes = [vp]
            lib.wg_graph_nnz.restype = i64
            lib.wg_graph_fetch.argtypes = [vp, vp, vp]
            lib.wg_graph_fetch.restype = ctypes.c_int
            lib.wg_graph_free.argtypes = [vp]
            lib.wg_graph_free.restype = None
            lib.wg_walk.argtypes = [vp, vp, vp, i64, ctypes.c_int, u64, u64, i64, vp, vp, ctypes.POINTER(i32)]
            lib.wg_walk.restype = i64
            _gen = lib
        return _gen


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


@dataclasses.dataclass
class Graph:
    """Undirected labelled graph in CSR form (both directions stored).

    row_ptr: int64 [n+1]; col: int32 [row_ptr[n]], each row strictly ascending;
    labels: int32 [n].
    """

    row_ptr: np.ndarray
    col: np.ndarray
    labels: np.ndarray

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


@dataclasses.dataclass
class Query:
    """Connected query graph: k vertices, edges (m, 2) int32 with a < b, labels int32 [k].

    ``witness`` is the data-vertex tuple the query was cut from (one known
    embedding, indexed by query vertex id), or None for hand-built queries.
    """

    k: int
    edges: np.ndarray
    labels: np.ndarray
    witness: Optional[np.ndarray] = None

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])

    @property
    def dense(self) -> bool:
        return 2 * self.m >= 3 * self.k


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def csr_from_pairs(n: int, lo: np.ndarray, hi: np.ndarray) -> tuple:
    """CSR (row_ptr int64, col int32) of the undirected graph with edges {lo[i], hi[i]}.

    Pairs must already be distinct with lo != hi.
    """
    lo = np.asarray(lo, dtype=np.int64)
    hi = np.asarray(hi, dtype=np.int64)
    key = np.concatenate([lo * n + hi, hi * n + lo])
    key.sort(kind="stable")
    src = key // n
    dst = (key - src * n).astype(np.int32)
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, dst


def erdos_renyi(n: int, m: int, seed: int) -> tuple:
    """G(n, M): m distinct non-loop pairs drawn uniformly without replacement."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("too many edges for n")
    rng = _rng(seed)
    t = np.sort(rng.choice(total, size=m, replace=False)).astype(np.int64)
    i_idx = np.arange(n, dtype=np.int64)
    first = i_idx * (2 * n - i_idx - 1) // 2  # index of pair (i, i+1)
    lo = np.searchsorted(first, t, side="right") - 1
    hi = t - first[lo] + lo + 1
    return csr_from_pairs(n, lo, hi)


def _native_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, threads: int = 0) -> tuple:
    """Symmetrised, deduplicated, loop-free R-MAT graph with randomly permuted ids.

    The draws and the CSR build are native (workloads_gen.c: counter-based
    SplitMix64, so the graph does not depend on the thread count); the id
    permutation is numpy's PCG64 with seed + 1_000_003.
    """
    n = 1 << scale
    perm = np.ascontiguousarray(_rng(seed + 1_000_003).permutation(n).astype(np.int64))
    lib = _native()
    h = ctypes.c_void_p()
    rc = lib.wg_rmat(scale, edge_factor, a, b, c, ctypes.c_uint64(seed), _ptr(perm), threads or _native_threads(),
                     ctypes.byref(h))
    if rc != 0:
        raise RuntimeError(f"R-MAT generator failed with code {rc}")
    try:
        nnz = int(lib.wg_graph_nnz(h))
        row_ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        if lib.wg_graph_fetch(h, _ptr(row_ptr), _ptr(col)) != 0:
            raise RuntimeError("R-MAT generator: fetch failed")
    finally:
        lib.wg_graph_free(h)
    return row_ptr, col[:nnz]


def uniform_labels(n: int, num_labels: int, seed: int) -> np.ndarray:
    return _rng(seed).integers(0, num_labels, size=n).astype(np.int32)


def zipf_labels(n: int, num_labels: int, s: float, seed: int) -> np.ndarray:
    w = (np.arange(num_labels, dtype=np.float64) + 1.0) ** (-s)
    return _rng(seed).choice(num_labels, size=n, p=w / w.sum()).astype(np.int32)


def induced_query(g: Graph, verts: Sequence[int]) -> Query:
    """Induced subgraph of g on verts (ids = positions in verts), labels copied."""
    verts = np.asarray(verts, dtype=np.int64)
    k = len(verts)
    edges = []
    for a in range(k - 1):
        lo, hi = g.row_ptr[verts[a]], g.row_ptr[verts[a] + 1]
        nb = g.col[lo:hi]
        if nb.shape[0] == 0:
            continue
        later = verts[a + 1:]
        p = np.minimum(np.searchsorted(nb, later), nb.shape[0] - 1)
        for b in np.flatnonzero(nb[p] == later):
            edges.append((a, a + 1 + int(b)))
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    return Query(k=k, edges=e, labels=g.labels[verts].astype(np.int32),
                 witness=verts.astype(np.int32))


def restricted(g: Graph, keep: np.ndarray) -> Graph:
    """The same vertex set with only the edges whose two ends have keep[v] set
    (vertices without keep become isolated); labels unchanged.  Random walks on
    it stay inside the kept vertices, and the induced edges among kept vertices
    are those of g."""
    keep = np.asarray(keep, dtype=bool)
    src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr))
    m = keep[src] & keep[g.col]
    deg = np.bincount(src[m], minlength=g.n)
    row_ptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return Graph(row_ptr, np.ascontiguousarray(g.col[m]), g.labels)


def hub_split_labels(g: Graph, max_degree: int, num_labels: int, seed: int) -> np.ndarray:
    """A test labelling of g's vertices: vertices of degree above max_degree get
    label num_labels (one label for all of them), every other vertex a uniform
    label in [0, num_labels)."""
    labels = uniform_labels(g.n, num_labels, seed)
    labels[np.diff(g.row_ptr) > max_degree] = num_labels
    return labels


def _live(g: Graph) -> np.ndarray:
    live = np.flatnonzero(np.diff(g.row_ptr) > 0).astype(np.int32)
    if live.shape[0] == 0:
        raise ValueError("graph has no edges")
    return live


def walk_query(g: Graph, k: int, seed: int, stream: int, live: Optional[np.ndarray] = None) -> Query:
    """The query cut out by random walk `stream` under `seed` (workloads_gen.c): k
    distinct vertices in discovery order, the induced edges among them, labels copied."""
    live = _live(g) if live is None else live
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    verts = np.empty(k, dtype=np.int32)
    edges = np.empty(max(1, k * (k - 1)), dtype=np.int32)
    m = ctypes.c_int32(0)
    rc = _native().wg_walk(_ptr(row_ptr), _ptr(col), _ptr(live), live.shape[0], k, ctypes.c_uint64(seed),
                           ctypes.c_uint64(stream), ctypes.c_int64(1_000_000), _ptr(verts), _ptr(edges),
                           ctypes.byref(m))
    if rc < 0:
        raise RuntimeError(f"random walk failed with code {rc} (k={k}: no component that large?)")
    e = edges[:2 * m.value].reshape(-1, 2).copy()
    return Query(k=k, edges=e, labels=g.labels[verts].astype(np.int32), witness=verts.copy())


def extract_queries(g: Graph, k_list: Sequence[int], n_dense: int, n_sparse: int, seed: int,
                    max_attempts: int = 1_000_000) -> List[Query]:
    """For every k in k_list: n_dense dense and n_sparse sparse random-walk queries.

    Attempt t (counted across all of k_list) is walk stream t under `seed`;
    queries whose density class is already full are rejected.
    Order of the result: grouped by k, dense first, then sparse.
    """
    live = _live(g)
    out: List[Query] = []
    t = 0
    for k in k_list:
        dense: List[Query] = []
        sparse: List[Query] = []
        attempts = 0
        while len(dense) < n_dense or len(sparse) < n_sparse:
            attempts += 1
            if attempts > max_attempts:
                raise RuntimeError(f"could not fill dense/sparse quotas for k={k}")
            q = walk_query(g, k, seed, t, live)
            t += 1
            if q.dense and len(dense) < n_dense:
                dense.append(q)
            elif (not q.dense) and len(sparse) < n_sparse:
                sparse.append(q)
        out.extend(dense)
        out.extend(sparse)
    return out


def extract_queries_any(g: Graph, k: int, count: int, seed: int) -> List[Query]:
    """count random-walk queries of size k (streams 0 .. count-1) with no density quota."""
    live = _live(g)
    return [walk_query(g, k, seed, i, live) for i in range(count)]


def walk_queries(g: Graph, sizes: Sequence[int], seed: int) -> List[Query]:
    """Random-walk queries of the given sizes, query i from walk stream i under `seed`."""
    live = _live(g)
    return [walk_query(g, int(k), seed, i, live) for i, k in enumerate(sizes)]


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    graph: Graph
    queries: List[Query]
    cap: int            # 0 = no cap
    time_limit_s: float  # <= 0 = none


def small_er(num_queries: int = 20) -> Workload:
    """ER n=2,000, |E|=8,000 (average degree 8), 4 uniform labels, 4-vertex queries."""
    row_ptr, col = erdos_renyi(2000, 8000, seed=101)
    g = Graph(row_ptr, col, uniform_labels(2000, 4, seed=102))
    qs = extract_queries_any(g, 4, num_queries, seed=103)
    return Workload("er2k_deg8_l4_q4", g, qs, cap=0, time_limit_s=0.0)


def rmat20_graph() -> Graph:
    """R-MAT scale 20, edge factor 16, (0.57, 0.19, 0.19, 0.05), 16 Zipf(1.0) labels."""
    row_ptr, col = rmat(20, 16, seed=20)
    return Graph(row_ptr, col, zipf_labels(1 << 20, 16, 1.0, seed=21))


def medium_rmat20(n_dense: int = 50, n_sparse: int = 50) -> Workload:
    """R-MAT scale 20 with 8-vertex queries, half dense and half sparse, cap 1e8."""
    g = rmat20_graph()
    qs = extract_queries(g, [8], n_dense, n_sparse, seed=22)
    return Workload("rmat20_ef16_zipf16_q8", g, qs, cap=100_000_000, time_limit_s=0.0)


def rmat24_graph() -> Graph:
    """R-MAT scale 24, edge factor 16, 8 Zipf(1.2) labels (about 2.2 GB as int32 CSR)."""
    row_ptr, col = rmat(24, 16, seed=24)
    return Graph(row_ptr, col, zipf_labels(1 << 24, 8, 1.2, seed=25))


def large_rmat24(per_class: int = 25, g: Optional[Graph] = None) -> Workload:
    """R-MAT scale 24 with 12/16/24/32-vertex queries, cap 1e9, 60 s per query."""
    g = rmat24_graph() if g is None else g
    qs = extract_queries(g, [12, 16, 24, 32], per_class, per_class, seed=26)
    return Workload("rmat24_ef16_zipf8_q12-32", g, qs, cap=1_000_000_000, time_limit_s=60.0)


def rmat22_graph() -> Graph:
    """R-MAT scale 22, edge factor 16, 16 Zipf(1.0) labels (the scale-20 recipe, larger)."""
    row_ptr, col = rmat(22, 16, seed=52)
    return Graph(row_ptr, col, zipf_labels(1 << 22, 16, 1.0, seed=53))


def order_sizes(n: int, seed: int) -> np.ndarray:
    """Sizes uniform in 8..32 for the learned-order query sets."""
    return _rng(seed).integers(8, 33, size=n)


def batch_rmat20(num_queries: int = 10_000, seed: int = 40, g: Optional[Graph] = None) -> Workload:
    """The R-MAT scale-20 graph with num_queries random-walk queries whose sizes are
    uniform in 4..32 (labels copied from G, so they follow G's label frequencies).
    Per query: cap 1e6 embeddings, 1 s time limit."""
    g = rmat20_graph() if g is None else g
    sizes = _rng(seed).integers(4, 33, size=num_queries)
    qs = walk_queries(g, sizes, seed)
    return Workload("rmat20_ef16_zipf16_q4-32_mixed", g, qs, cap=1_000_000, time_limit_s=1.0)


def cg_er20(per_size: int = 20, sizes: Sequence[int] = (16, 24, 32)) -> Workload:
    """Large queries over a labelled graph without hubs: G(n, M) with n = 2^20
    and M = 2^23 (average degree 16), 16 labels drawn uniformly, random-walk
    queries of each size.  Cap 1e9 per query, 5 s limit."""
    row_ptr, col = erdos_renyi(1 << 20, 1 << 23, seed=72)
    g = Graph(row_ptr, col, uniform_labels(1 << 20, 16, seed=73))
    qs = walk_queries(g, np.repeat(np.asarray(sizes), per_size), seed=74)
    return Workload("er20_d16_uniform16_q16-32", g, qs, cap=1_000_000_000, time_limit_s=5.0)


def cg_rmat20(per_size: int = 20, sizes: Sequence[int] = (16, 24, 32), g: Optional[Graph] = None) -> Workload:
    """Large queries over a labelled graph, the workload class the paper searches
    on a candidate graph: the scale-20 R-MAT edges with 16 labels drawn uniformly
    at random (how the paper labels its graphs for large queries), and per_size
    random-walk queries of each size (induced edges kept, labels copied).
    Cap 1e9 per query and a 5 s limit, as for the large queries on scale 24."""
    if g is None:
        row_ptr, col = rmat(20, 16, seed=20)
        g = Graph(row_ptr, col, uniform_labels(1 << 20, 16, seed=70))
    qs = walk_queries(g, np.repeat(np.asarray(sizes), per_size), seed=71)
    return Workload("rmat20_ef16_uniform16_q16-32", g, qs, cap=1_000_000_000, time_limit_s=5.0)

