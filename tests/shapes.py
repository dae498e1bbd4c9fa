"""Small hand-shaped graphs and queries for the tests (inputs only, no matching logic)."""
from __future__ import annotations

import itertools
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from paper_2604_10601_amd.workloads import Graph, Query, csr_from_pairs


def graph_from_edges(n: int, edges: Iterable[Tuple[int, int]], labels=None) -> Graph:
    pairs = {(min(a, b), max(a, b)) for a, b in edges if a != b}
    pairs = sorted(pairs)
    lo = np.array([p[0] for p in pairs], dtype=np.int64)
    hi = np.array([p[1] for p in pairs], dtype=np.int64)
    row_ptr, col = csr_from_pairs(n, lo, hi)
    if labels is None:
        labels = np.zeros(n, dtype=np.int32)
    return Graph(row_ptr, col, np.asarray(labels, dtype=np.int32))


def query(k: int, edges: Sequence[Tuple[int, int]], labels=None) -> Query:
    e = np.array([(min(a, b), max(a, b)) for a, b in edges], dtype=np.int32).reshape(-1, 2)
    if labels is None:
        labels = np.zeros(k, dtype=np.int32)
    return Query(k=k, edges=e, labels=np.asarray(labels, dtype=np.int32))


def complete(n: int, labels=None) -> Graph:
    return graph_from_edges(n, itertools.combinations(range(n), 2), labels)


def grid(a: int, b: int) -> Graph:
    def vid(i, j):
        return i * b + j
    e = []
    for i in range(a):
        for j in range(b):
            if i + 1 < a:
                e.append((vid(i, j), vid(i + 1, j)))
            if j + 1 < b:
                e.append((vid(i, j), vid(i, j + 1)))
    return graph_from_edges(a * b, e)


def complete_bipartite(m: int, n: int) -> Graph:
    return graph_from_edges(m + n, [(i, m + j) for i in range(m) for j in range(n)])


def star_graph(s: int) -> Graph:
    return graph_from_edges(s + 1, [(0, i) for i in range(1, s + 1)])


def gnp(n: int, p: float, rng: np.random.Generator, num_labels: int = 1) -> Graph:
    e = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
    return graph_from_edges(n, e, rng.integers(0, num_labels, size=n))


def path_q(k: int) -> Query:
    return query(k, [(i, i + 1) for i in range(k - 1)])


def cycle_q(k: int) -> Query:
    return query(k, [(i, (i + 1) % k) for i in range(k)])


def clique_q(k: int) -> Query:
    return query(k, list(itertools.combinations(range(k), 2)))


def star_q(s: int) -> Query:
    return query(s + 1, [(0, i) for i in range(1, s + 1)])


def random_connected_query(k: int, rng: np.random.Generator, extra_p: float = 0.3,
                           num_labels: int = 1) -> Query:
    """Random spanning tree plus extra edges with probability extra_p."""
    e = set()
    for v in range(1, k):
        u = int(rng.integers(0, v))
        e.add((u, v))
    for a, b in itertools.combinations(range(k), 2):
        if (a, b) not in e and rng.random() < extra_p:
            e.add((a, b))
    perm = rng.permutation(k)
    e = [(int(perm[a]), int(perm[b])) for a, b in e]
    return query(k, e, rng.integers(0, num_labels, size=k))


def relabel_graph(g: Graph, perm: np.ndarray) -> Graph:
    """Vertex v of g becomes perm[v]."""
    n = g.n
    src = np.repeat(np.arange(n), np.diff(g.row_ptr))
    keep = src < g.col
    lo, hi = perm[src[keep]], perm[g.col[keep]]
    row_ptr, col = csr_from_pairs(n, np.minimum(lo, hi), np.maximum(lo, hi))
    labels = np.empty(n, dtype=np.int32)
    labels[perm] = g.labels
    return Graph(row_ptr, col, labels)


def disjoint_union(g1: Graph, g2: Graph) -> Graph:
    n1 = g1.n
    def pairs(g, off):
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        keep = src < g.col
        return src[keep] + off, g.col[keep].astype(np.int64) + off
    a1, b1 = pairs(g1, 0)
    a2, b2 = pairs(g2, n1)
    row_ptr, col = csr_from_pairs(n1 + g2.n, np.concatenate([a1, a2]), np.concatenate([b1, b2]))
    return Graph(row_ptr, col, np.concatenate([g1.labels, g2.labels]).astype(np.int32))


def connected_orders(q: Query) -> List[List[int]]:
    adj = [set() for _ in range(q.k)]
    for a, b in q.edges:
        adj[a].add(int(b))
        adj[b].add(int(a))
    out = []
    for perm in itertools.permutations(range(q.k)):
        seen = {perm[0]}
        ok = True
        for u in perm[1:]:
            if not (adj[u] & seen):
                ok = False
                break
            seen.add(u)
        if ok:
            out.append(list(perm))
    return out
