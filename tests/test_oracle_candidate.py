"""Pins of the candidate-graph oracle (oracle/candidate.py), CPU only.

* hand-worked sets, G' sizes and match counts (tests/golden/candidate_sets.txt);
* soundness: every match found by brute force over all injective maps keeps
  M(u) in C(u), and no match exists once some C(u) is empty;
* maximality: on tiny instances, C equals the union of every supported family
  inside the label and degree sets, found by trying all of them;
* the result does not depend on the order of removals;
* counting on the subgraph of G induced by the union of the sets gives the
  count on G.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import candidate as cand
from tests import shapes as S

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def sets(g, q, rng=None):
    return cand.candidate_sets(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, rng=rng)


def brute_force(g, q):
    adj = {(v, int(w)) for v in range(g.n) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]}
    out = []
    for M in itertools.permutations(range(g.n), q.k):
        if any(g.labels[M[u]] != q.labels[u] for u in range(q.k)):
            continue
        if all((M[a], M[b]) in adj for a, b in q.edges):
            out.append(M)
    return out


def test_candidate_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "candidate_sets.txt")
    seen = 0
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        name, gspec, qspec, want_sets, want_edges, want_count = [x.strip() for x in line.split("|")]

        def parse(spec):
            n_s, lab_s, edge_s = spec.split(";")
            n = int(n_s)
            labels = [int(x) for x in lab_s.split(",")] if lab_s.strip() else [0] * n
            edges = [tuple(int(v) for v in e.split("-")) for e in edge_s.split(",") if e.strip()]
            return n, labels, edges

        gn, gl, ge = parse(gspec)
        qk, ql, qe = parse(qspec)
        g = S.graph_from_edges(gn, ge, gl)
        q = S.query(qk, qe, ql)
        c = sets(g, q)
        got = [",".join(str(int(v)) for v in np.flatnonzero(row)) or "-" for row in c]
        assert "/".join(got) == want_sets, name
        assert cand.candidate_edges(g.row_ptr, g.col, q.k, q.edges, c) == int(want_edges), name
        assert oracle.count(g, q).count == int(want_count), name
        assert len(brute_force(g, q)) == int(want_count), name
        seen += 1
    assert seen == 5


def test_candidate_sound_against_brute_force():
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(150):
        n = int(rng.integers(2, 8))
        k = int(rng.integers(2, min(n, 4) + 1))
        nl = int(rng.integers(1, 3))
        g = S.gnp(n, float(rng.uniform(0.25, 0.8)), rng, nl)
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.6)), num_labels=nl)
        c = sets(g, q)
        matches = brute_force(g, q)
        for M in matches:
            assert all(c[u, M[u]] for u in range(q.k)), trial
        if not c.any(axis=1).all():
            assert not matches, trial
        assert cand.is_supported_family(g.row_ptr, g.col, q.k, q.edges, c), trial
        checked += len(matches)
    assert checked > 100


def test_candidate_maximal_by_exhaustion():
    """C is the union of all supported families inside C0 (so it is the largest one)."""
    rng = np.random.default_rng(12)
    done = 0
    for trial in range(400):
        n = int(rng.integers(3, 7))
        k = int(rng.integers(2, 4))
        nl = int(rng.integers(1, 3))
        g = S.gnp(n, float(rng.uniform(0.2, 0.6)), rng, nl)
        q = S.random_connected_query(k, rng, extra_p=0.5, num_labels=nl)
        c0 = cand.initial_sets(g.row_ptr, g.labels, q.k, q.edges, q.labels)
        bits = list(zip(*np.nonzero(c0)))
        if len(bits) > 11:
            continue
        union = np.zeros_like(c0)
        for mask in range(1 << len(bits)):
            f = np.zeros_like(c0)
            for i, (u, v) in enumerate(bits):
                if (mask >> i) & 1:
                    f[u, v] = True
            if cand.is_supported_family(g.row_ptr, g.col, q.k, q.edges, f):
                union |= f
        assert (sets(g, q) == union).all(), trial
        done += 1
    assert done >= 100


def test_candidate_independent_of_removal_order():
    rng = np.random.default_rng(13)
    for trial in range(6):
        g = S.gnp(120, 0.04, rng, 3)
        q = S.random_connected_query(int(rng.integers(3, 7)), rng, extra_p=0.3, num_labels=3)
        want = sets(g, q)
        for s in range(3):
            assert (sets(g, q, rng=np.random.default_rng(100 * trial + s)) == want).all(), trial


def test_candidate_induced_subgraph_keeps_the_count():
    rng = np.random.default_rng(14)
    reduced = 0
    for trial in range(12):
        g = S.gnp(200, 0.03, rng, 3)
        q = S.random_connected_query(int(rng.integers(3, 6)), rng, extra_p=0.3, num_labels=3)
        c = sets(g, q)
        keep = np.flatnonzero(c.any(axis=0))
        idx = -np.ones(g.n, dtype=np.int64)
        idx[keep] = np.arange(len(keep))
        e = [(int(idx[v]), int(idx[w])) for v in keep for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
             if idx[w] >= 0 and v < w]
        h = S.graph_from_edges(len(keep), e, g.labels[keep])
        assert oracle.count(h, q).count == oracle.count(g, q).count, trial
        reduced += len(keep) < g.n
    assert reduced >= 6
