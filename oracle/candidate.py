"""Candidate-graph filtering, written out plainly -- test infrastructure only.

Only tests/ may import this module; the engine never calls it.

When the paper compares with EGSM it runs its own search on EGSM's candidate
graph G' (experimental setup, Sec. 6.1); App. C describes G' as the product of
a light filtering pass over vertex labels and query structure, after which the
search reads G' instead of G.  The paper fixes neither the filter nor the
layout, so this module takes the usual reading of such a pass
(neighbourhood-support filtering, as in the CPU matchers App. C cites):

    C0(u) = { v in V(G) : L(v) = L(u) and d_G(v) >= d_Q(u) }
    C     = the largest family C(u) subset of C0(u) in which every v in C(u)
            has, for every neighbour u' of u in Q, a neighbour in C(u').

The condition only gets harder as sets shrink, so this largest family exists
and is what repeated removal of unsupported vertices reaches, whatever the
order of removals.  Every embedding M keeps M(u) in C(u) (the images of u's
query neighbours support it at every step), so a search restricted to G'
finds exactly the matches of Q in G.

G' has, for each query edge {u, u'}, the pairs (v, w) with v in C(u),
w in C(u') and {v, w} in E(G); `candidate_edges` counts them over all query
edges.

Pins (tests/test_oracle_candidate.py): a hand-worked fixture in
tests/golden/candidate_sets.txt, soundness against brute-force embeddings,
maximality against an exhaustive search over all candidate families on tiny
instances, and independence from the order of removals.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np


def _adjacency(k: int, edges) -> List[List[int]]:
    adj: List[List[int]] = [[] for _ in range(k)]
    for a, b in edges:
        adj[int(a)].append(int(b))
        adj[int(b)].append(int(a))
    return adj


def initial_sets(row_ptr, labels, k: int, edges, qlabels) -> np.ndarray:
    """C0 as a boolean k x n matrix: label equal and degree at least the query degree."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    labels = np.asarray(labels)
    deg = np.diff(row_ptr)
    qdeg = [len(a) for a in _adjacency(k, edges)]
    return np.stack([(labels == qlabels[u]) & (deg >= qdeg[u]) for u in range(k)]) if k else \
        np.zeros((0, len(deg)), dtype=bool)


def supported(row_ptr, col, v: int, cand: np.ndarray) -> bool:
    """True iff data vertex v has a neighbour w with cand[w] set."""
    return bool(cand[col[row_ptr[v]:row_ptr[v + 1]]].any())


def candidate_sets(row_ptr, col, labels, k: int, edges, qlabels,
                   rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """The largest supported family (boolean k x n; row u is C(u)).

    Sweeps over every (u, v) with v in C(u), removing v when some query
    neighbour u' of u finds no neighbour of v in C(u'), until a sweep removes
    nothing.  rng, if given, shuffles the order of every sweep (the result must
    not depend on it).
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    adj = _adjacency(k, edges)
    c = initial_sets(row_ptr, labels, k, edges, qlabels)
    while True:
        pairs = [(u, int(v)) for u in range(k) for v in np.flatnonzero(c[u])]
        if rng is not None:
            pairs = [pairs[i] for i in rng.permutation(len(pairs))]
        removed = False
        for u, v in pairs:
            for u2 in adj[u]:
                if not supported(row_ptr, col, v, c[u2]):
                    c[u, v] = False
                    removed = True
                    break
        if not removed:
            return c


def candidate_edges(row_ptr, col, k: int, edges, c: np.ndarray) -> int:
    """Edges of G': the sum over query edges {u, u'} of the number of pairs
    (v, w) with v in C(u), w in C(u') and {v, w} in E(G).  Each query edge
    counts once (its pairs read from the other end are the same edges of G')."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    total = 0
    for a, b in edges:
        for v in np.flatnonzero(c[int(a)]):
            total += int(c[int(b)][col[row_ptr[v]:row_ptr[v + 1]]].sum())
    return total


def sets_as_lists(c: np.ndarray) -> List[np.ndarray]:
    return [np.flatnonzero(row).astype(np.int32) for row in c]


def is_supported_family(row_ptr, col, k: int, edges, c: np.ndarray) -> bool:
    """Every v in C(u) has a neighbour in C(u') for every query neighbour u' of u."""
    adj = _adjacency(k, edges)
    for u in range(k):
        for v in np.flatnonzero(c[u]):
            for u2 in adj[u]:
                if not supported(row_ptr, col, int(v), c[u2]):
                    return False
    return True

