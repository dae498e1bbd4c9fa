"""Pins for the CPU oracle: it is checked against things other than itself.

* Def. 1 written out as brute force over every injective map (tiny graphs);
* networkx's subgraph-monomorphism matcher (a library routine for the same
  non-induced, label-preserving definition) on mid-size graphs;
* closed forms for cliques, labelled cliques, grids, complete bipartite graphs,
  stars and trace identities of the adjacency matrix;
* invariants: matching order, vertex relabelling, label-value permutation,
  disjoint union, automorphism divisibility, edge monotonicity;
* closed forms for the work counters (groups, tasks) on cliques and stars;
* cap and time-limit semantics.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S


def brute_force(g, q):
    """Every injective map V(Q) -> V(G) that keeps labels and sends edges to edges (Def. 1)."""
    n = g.n
    adj = set()
    for v in range(n):
        for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
            adj.add((v, int(w)))
    out = []
    for M in itertools.permutations(range(n), q.k):
        if any(g.labels[M[u]] != q.labels[u] for u in range(q.k)):
            continue
        if all((M[a], M[b]) in adj for a, b in q.edges):
            out.append(M)
    return sorted(out)


def ocount(g, q, **kw):
    return oracle.count(g, q, **kw).count


def orows(g, q, limit=100000, **kw):
    return [tuple(int(x) for x in r) for r in oracle.enumerate_sorted(g, q, limit, **kw)]


# ---------------------------------------------------------------------------
# Brute force and library
# ---------------------------------------------------------------------------

def test_brute_force_random_tiny():
    rng = np.random.default_rng(7)
    cases = 0
    for trial in range(160):
        n = int(rng.integers(1, 8))
        k = int(rng.integers(1, min(n, 5) + 1))
        nl = int(rng.integers(1, 4))
        g = S.gnp(n, float(rng.uniform(0.2, 0.9)), rng, nl)
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.7)), num_labels=nl)
        want = brute_force(g, q)
        for threads in (1, 3):
            got = orows(g, q, threads=threads)
            assert got == want, (trial, n, k)
            assert ocount(g, q, threads=threads) == len(want)
        cases += 1
    assert cases == 160


def test_networkx_monomorphisms():
    nx = pytest.importorskip("networkx")
    from networkx.algorithms import isomorphism as iso
    rng = np.random.default_rng(11)
    for trial in range(12):
        n = int(rng.integers(20, 45))
        nl = int(rng.integers(1, 3))
        g = S.gnp(n, float(rng.uniform(0.08, 0.2)), rng, nl)
        k = int(rng.integers(3, 6))
        q = S.random_connected_query(k, rng, extra_p=0.3, num_labels=nl)
        G = nx.Graph()
        G.add_nodes_from((v, {"l": int(g.labels[v])}) for v in range(n))
        for v in range(n):
            for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]:
                G.add_edge(v, int(w))
        Q = nx.Graph()
        Q.add_nodes_from((u, {"l": int(q.labels[u])}) for u in range(k))
        Q.add_edges_from((int(a), int(b)) for a, b in q.edges)
        gm = iso.GraphMatcher(G, Q, node_match=lambda x, y: x["l"] == y["l"])
        want = sorted(tuple(inv[u] for u in range(k))
                      for inv in ({qv: gv for gv, qv in m.items()}
                                  for m in gm.subgraph_monomorphisms_iter()))
        assert orows(g, q) == want, trial


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [5, 7, 9])
def test_clique_any_connected_query(n):
    rng = np.random.default_rng(n)
    qs = [S.path_q(3), S.cycle_q(4), S.clique_q(4), S.star_q(3), S.path_q(5),
          S.random_connected_query(5, rng), S.clique_q(min(n, 6))]
    for q in qs:
        assert ocount(S.complete(n), q) == math.perm(n, q.k)


def test_labelled_clique():
    rng = np.random.default_rng(3)
    for trial in range(10):
        n = 10
        glab = rng.integers(0, 3, size=n)
        g = S.complete(n, glab)
        k = int(rng.integers(2, 6))
        q = S.random_connected_query(k, rng, num_labels=3)
        want = 1
        for lab in range(3):
            nl = int((glab == lab).sum())
            cl = int((q.labels == lab).sum())
            want *= math.perm(nl, cl) if cl <= nl else 0
        assert ocount(g, q) == want


@pytest.mark.parametrize("a,b", [(3, 3), (3, 4), (4, 4), (5, 7), (9, 6)])
def test_grid_closed_forms(a, b):
    g = S.grid(a, b)
    d = g.degrees()
    assert ocount(g, S.path_q(2)) == 2 * (2 * a * b - a - b)
    assert ocount(g, S.path_q(3)) == int((d * (d - 1)).sum())
    assert ocount(g, S.cycle_q(4)) == 8 * (a - 1) * (b - 1)
    assert ocount(g, S.cycle_q(6)) == 12 * ((a - 1) * (b - 2) + (a - 2) * (b - 1))
    assert ocount(g, S.clique_q(3)) == 0
    assert ocount(g, S.cycle_q(5)) == 0


@pytest.mark.parametrize("m,n", [(2, 2), (3, 4), (5, 3)])
def test_complete_bipartite_c4(m, n):
    assert ocount(S.complete_bipartite(m, n), S.cycle_q(4)) == 2 * m * (m - 1) * n * (n - 1)


def test_trace_identities_random_graphs():
    rng = np.random.default_rng(5)
    for trial in range(6):
        n = int(rng.integers(30, 80))
        g = S.gnp(n, float(rng.uniform(0.05, 0.25)), rng)
        A = np.zeros((n, n), dtype=np.int64)
        for v in range(n):
            A[v, g.col[g.row_ptr[v]:g.row_ptr[v + 1]]] = 1
        d = A.sum(1)
        E = int(A.sum()) // 2
        A3 = A @ A @ A
        A4 = A3 @ A
        assert ocount(g, S.clique_q(3)) == int(np.trace(A3))
        assert ocount(g, S.cycle_q(4)) == int(np.trace(A4)) - 2 * E - 2 * int((d * (d - 1)).sum())
        assert ocount(g, S.path_q(3)) == int((d * (d - 1)).sum())
        for s in (2, 3, 4):
            want = sum(math.perm(int(x), s) for x in d if x >= s)
            assert ocount(g, S.star_q(s)) == want


def test_self_match_equals_automorphisms():
    rng = np.random.default_rng(9)
    for trial in range(8):
        k = int(rng.integers(3, 7))
        q = S.random_connected_query(k, rng, extra_p=0.4, num_labels=2)
        g = S.graph_from_edges(k, [tuple(map(int, e)) for e in q.edges], q.labels)
        E = {(int(a), int(b)) for a, b in q.edges} | {(int(b), int(a)) for a, b in q.edges}
        aut = sum(1 for p in itertools.permutations(range(k))
                  if all(q.labels[p[u]] == q.labels[u] for u in range(k))
                  and all((p[a], p[b]) in E for a, b in E))
        assert ocount(g, q) == aut


def test_hand_worked_fixtures():
    """Small cases counted by hand, stored in tests/golden/hand_counts.txt."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_counts.txt")
    seen = 0
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        name, gspec, qspec, want = [x.strip() for x in line.split("|")]
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
        assert ocount(g, q) == int(want), name
        seen += 1
    assert seen >= 5


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------

def test_order_invariance_and_counters_depend_on_order_only():
    rng = np.random.default_rng(21)
    for trial in range(6):
        g = S.gnp(40, 0.15, rng, 2)
        q = S.random_connected_query(5, rng, extra_p=0.3, num_labels=2)
        counts = set()
        for order in S.connected_orders(q):
            r1 = oracle.count(g, q, order=order, threads=1)
            r4 = oracle.count(g, q, order=order, threads=4)
            counts.add(r1.count)
            assert (r1.count, r1.tasks, r1.groups) == (r4.count, r4.tasks, r4.groups)
        assert len(counts) == 1


def test_relabelling_and_label_permutation():
    rng = np.random.default_rng(31)
    for trial in range(6):
        g = S.gnp(50, 0.12, rng, 3)
        q = S.random_connected_query(4, rng, extra_p=0.3, num_labels=3)
        rows = orows(g, q)
        perm = rng.permutation(g.n)
        g2 = S.relabel_graph(g, perm)
        rows2 = orows(g2, q)
        assert sorted(tuple(int(perm[v]) for v in r) for r in rows) == rows2
        lp = rng.permutation(3)
        g3 = wl.Graph(g.row_ptr, g.col, lp[g.labels].astype(np.int32))
        q3 = wl.Query(q.k, q.edges, lp[q.labels].astype(np.int32))
        assert ocount(g3, q3) == len(rows)


def test_disjoint_union_additive():
    rng = np.random.default_rng(41)
    for trial in range(5):
        g1 = S.gnp(30, 0.2, rng, 2)
        g2 = S.gnp(25, 0.25, rng, 2)
        q = S.random_connected_query(4, rng, num_labels=2)
        assert ocount(S.disjoint_union(g1, g2), q) == ocount(g1, q) + ocount(g2, q)


def test_divisible_by_automorphisms_and_edge_monotone():
    rng = np.random.default_rng(51)
    for trial in range(6):
        g = S.gnp(45, 0.2, rng)
        q = S.random_connected_query(5, rng, extra_p=0.2)
        c = ocount(g, q)
        qg = S.graph_from_edges(q.k, [tuple(map(int, e)) for e in q.edges])
        aut = ocount(qg, q)
        assert aut >= 1 and c % aut == 0
        present = {(int(a), int(b)) for a, b in q.edges}
        missing = [e for e in itertools.combinations(range(q.k), 2) if e not in present]
        if missing:
            e = missing[int(rng.integers(len(missing)))]
            q2 = S.query(q.k, list(present) + [e])
            assert ocount(g, q2) <= c


def test_extracted_queries_contain_their_witness():
    w = wl.small_er(num_queries=8)
    for q in w.queries:
        rows = orows(w.graph, q)
        assert len(rows) >= 1
        assert tuple(int(x) for x in q.witness) in set(rows)


# ---------------------------------------------------------------------------
# Work counters, cap, time limit
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,q", [(6, "tri"), (8, "path4"), (7, "clique4")])
def test_counters_on_cliques(n, q):
    qq = {"tri": S.clique_q(3), "path4": S.path_q(4), "clique4": S.clique_q(4)}[q]
    r = oracle.count(S.complete(n), qq)
    # every partial match of length i (1 <= i < k) is valid and has n-1 local candidates
    groups = sum(math.perm(n, i) for i in range(1, qq.k))
    assert r.groups == groups
    assert r.tasks == (n - 1) * groups


def test_counters_on_star():
    s = 9
    r = oracle.count(S.star_graph(s), S.path_q(2))
    assert r.count == 2 * s
    assert r.groups == s + 1      # every vertex is a root
    assert r.tasks == 2 * s       # sum of degrees


def test_cap_semantics():
    g = S.complete(8)
    q = S.path_q(4)
    truth = math.perm(8, 4)
    for cap in (1, 7, truth - 1, truth, truth + 1, 10 ** 9):
        for threads in (1, 4):
            r = oracle.count(g, q, cap=cap, threads=threads)
            assert r.count == min(truth, cap)
            assert r.outcome == (oracle.CAPPED if truth >= cap else oracle.DONE)


def test_time_limit_gives_lower_bound():
    g = S.complete(40)
    q = S.clique_q(7)
    r = oracle.count(g, q, time_limit_s=0.05, threads=2)
    assert r.outcome == oracle.TIMEOUT
    assert r.count < math.perm(40, 7)


def test_input_checks():
    g = S.complete(4)
    assert oracle.check_graph(g.row_ptr, g.col) == oracle.OK
    bad = g.col.copy()
    bad[0], bad[1] = bad[1], bad[0]                      # unsorted row
    assert oracle.check_graph(g.row_ptr, bad) == oracle.ERR_GRAPH
    rp = np.array([0, 1, 1], dtype=np.int64)              # edge 0->1 without 1->0
    assert oracle.check_graph(rp, np.array([1], np.int32)) == oracle.ERR_GRAPH
    assert oracle.check_graph(rp, np.array([1], np.int32), check_symmetry=False) == oracle.OK
    assert oracle.check_graph(np.array([0, 1], np.int64), np.array([0], np.int32)) == oracle.ERR_GRAPH
    assert oracle.check_query(3, [(0, 1)]) == oracle.ERR_QUERY            # disconnected
    assert oracle.check_query(2, [(0, 1), (1, 0)]) == oracle.ERR_QUERY    # duplicate
    assert oracle.check_query(33, [(i, i + 1) for i in range(32)]) == oracle.ERR_QUERY
    assert oracle.check_query(32, [(i, i + 1) for i in range(31)]) == oracle.OK
    assert oracle.check_order(3, [(0, 1), (1, 2)], [0, 2, 1]) == oracle.ERR_ORDER
    assert oracle.check_order(3, [(0, 1), (1, 2)], [0, 1, 1]) == oracle.ERR_ORDER
    assert oracle.check_order(3, [(0, 1), (1, 2)], [2, 1, 0]) == oracle.OK


def test_ri_order_hand_cases_and_validity():
    assert list(oracle.ri_order(4, [(0, 1), (1, 2), (2, 3)])) == [1, 2, 0, 3]
    assert list(oracle.ri_order(4, [(0, 1), (1, 2), (0, 2), (2, 3)])) == [2, 0, 1, 3]
    assert list(oracle.ri_order(1, [])) == [0]
    rng = np.random.default_rng(61)
    for trial in range(50):
        k = int(rng.integers(1, 33))
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.3)))
        o = oracle.ri_order(q.k, q.edges)
        assert oracle.check_order(q.k, q.edges, o) == oracle.OK


def test_empty_and_degenerate_inputs():
    empty = wl.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert ocount(empty, S.path_q(2)) == 0
    assert ocount(empty, S.query(1, [])) == 0
    lonely = wl.Graph(np.zeros(4, np.int64), np.zeros(0, np.int32), np.array([0, 1, 0], np.int32))
    assert ocount(lonely, S.query(1, [], [0])) == 2      # single vertex query: label match only
    assert ocount(lonely, S.path_q(2)) == 0
    assert ocount(S.complete(3), S.path_q(4)) == 0        # query larger than the graph


@pytest.mark.parametrize("s", [3, 6, 11])
def test_counters_follow_min_degree_list(s):
    """Star (centre 0, leaves 1..s) plus the edge 1-2; triangle query along order (0, 1, 2).

    Roots need degree >= 2: the centre (degree s) and leaves 1, 2 (degree 2), so
    level-1 tasks = s + 2 + 2.  The six valid pairs are the ordered pairs of
    {0, 1, 2}; each contains a leaf of degree 2, whose list (2 entries) is the
    local candidate set (Sec. 4.1 takes the smaller list), so level-2 tasks = 12.
    """
    g = S.graph_from_edges(s + 1, [(0, i) for i in range(1, s + 1)] + [(1, 2)])
    r = oracle.count(g, S.clique_q(3), order=[0, 1, 2])
    assert r.count == 6
    assert r.groups == 3 + 6
    assert r.tasks == (s + 4) + 12
