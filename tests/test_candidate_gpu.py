"""GPU parity of the candidate-graph path (gm_options.candidate_graph) against the oracle.

* candidate sets and the number of list entries of G' are bit-exact against
  oracle/candidate.py: the hand-worked fixtures, ER and R-MAT graphs whose
  sizes span many 64-vertex words and end in a ragged one;
* counts and outcomes on G' equal the oracle's on G (the filter keeps every
  match), exact and under a cap, and enumerated rows (sorted) are the same;
* symmetry breaking on G', degenerate queries (a label G lacks, one vertex,
  one edge, every root filtered out), time limits;
* the batched and serving calls refuse the mode.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import candidate as cand
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def want_sets(g, q):
    return cand.candidate_sets(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels)


def sort_rows(rows):
    rows = np.asarray(rows)
    return rows if rows.shape[0] == 0 else rows[np.lexsort(rows.T[::-1])]


def golden_cases():
    path = os.path.join(os.path.dirname(__file__), "golden", "candidate_sets.txt")
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        name, gspec, qspec, sets, edges, count = [x.strip() for x in line.split("|")]

        def parse(spec):
            n_s, lab_s, edge_s = spec.split(";")
            n = int(n_s)
            labels = [int(x) for x in lab_s.split(",")] if lab_s.strip() else [0] * n
            es = [tuple(int(v) for v in e.split("-")) for e in edge_s.split(",") if e.strip()]
            return n, labels, es

        gn, gl, ge = parse(gspec)
        qk, ql, qe = parse(qspec)
        yield name, S.graph_from_edges(gn, ge, gl), S.query(qk, qe, ql), sets, int(edges), int(count)


def test_golden_sets_edges_and_counts():
    with gm.Engine(device=0, candidate_graph=True) as e:
        seen = 0
        for name, g, q, sets, edges, count in golden_cases():
            _say(f"candidate golden {name}")
            e.load(g)
            qid = e.add(q)
            got, got_edges, rounds = e.candidate_sets(qid)
            txt = "/".join(",".join(str(int(v)) for v in np.flatnonzero(row)) or "-" for row in got)
            assert txt == sets, name
            assert got_edges == edges, name
            r = e.count(qid)
            assert (r.count, r.outcome) == (count, gm.GM_DONE), name
            seen += 1
        assert seen == 5


def graph_cases():
    rp, col = wl.erdos_renyi(2000, 8000, seed=3101)
    yield "er2000", wl.Graph(rp, col, wl.uniform_labels(2000, 4, seed=3102)), (4, 6, 8)
    rp, col = wl.erdos_renyi(5000, 30000, seed=3103)       # 5000 = 78 words of 64 + 8
    yield "er5000", wl.Graph(rp, col, wl.uniform_labels(5000, 8, seed=3104)), (6, 10, 12)
    rp, col = wl.rmat(12, 16, seed=3105)
    yield "rmat12", wl.Graph(rp, col, wl.zipf_labels(1 << 12, 8, 1.2, seed=3106)), (5, 8, 12, 16)


def test_sets_match_oracle_on_random_graphs():
    with gm.Engine(device=0) as e:          # the sets are available with the option off too
        for name, g, sizes in graph_cases():
            e.load(g)
            for k in sizes:
                for i, q in enumerate(wl.extract_queries_any(g, k, 3, seed=3200 + k)):
                    _say(f"candidate sets {name} k={k} #{i}")
                    qid = e.add(q)
                    got, got_edges, rounds = e.candidate_sets(qid)
                    want = want_sets(g, q)
                    assert np.array_equal(got, want), (name, k, i)
                    assert got_edges == cand.candidate_edges(g.row_ptr, g.col, q.k, q.edges, want), (name, k, i)
                    assert rounds >= 1
                    # the sets do not depend on the matching order
                    phi = e.get_order(qid)
                    if _connected_reverse(q, phi):
                        e.set_order(qid, phi[::-1].copy())
                        assert np.array_equal(e.candidate_sets(qid)[0], want), (name, k, i)
                    e.free_query(qid)


def _connected_reverse(q, phi):
    """True if the reversed order is a valid matching order (every vertex after the first has an earlier neighbour)."""
    adj = {u: set() for u in range(q.k)}
    for a, b in q.edges:
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    seen = set()
    for i, u in enumerate(phi[::-1]):
        if i and not (adj[int(u)] & seen):
            return False
        seen.add(int(u))
    return True


def test_counts_on_candidate_graph_match_oracle():
    rp, col = wl.erdos_renyi(4000, 20000, seed=1701)
    g = wl.Graph(rp, col, wl.uniform_labels(4000, 8, seed=1702))
    qs = []
    for k, seed in ((8, 3301), (12, 1703), (16, 1704), (24, 1705), (32, 1706)):
        qs += wl.extract_queries_any(g, k, 3, seed=seed)
    with gm.Engine(device=0, candidate_graph=True) as e:
        e.load(g)
        for i, q in enumerate(qs):
            _say(f"candidate count er4000 #{i} k={q.k}")
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            assert (r.count, r.outcome) == (o.count, o.outcome), (i, q.k)
            assert r.candidate_rounds >= 1 and r.candidate_edges > 0
            if o.count <= 100000 and i % 3 == 0:
                er = e.enumerate(qid, 100000)
                want = oracle.match(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, order=e.get_order(qid),
                                    enumerate_rows=100000)
                assert np.array_equal(sort_rows(er.matches), sort_rows(want.rows)), (i, q.k)
            e.free_query(qid)


def test_capped_counts_on_rmat():
    rp, col = wl.rmat(16, 16, seed=1601)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 16, 8, 1.2, seed=1602))
    qs = wl.extract_queries(g, [12, 16, 24, 32], 2, 2, seed=1603)
    with gm.Engine(device=0, candidate_graph=True) as e:
        e.load(g)
        for i, q in enumerate(qs):
            _say(f"candidate rmat16 #{i} k={q.k}")
            qid = e.add(q)
            for cap in (1, 200000):
                r = e.count(qid, cap=cap)
                o = oracle.count(g, q, order=e.get_order(qid), cap=cap, time_limit_s=30)
                if o.outcome == oracle.TIMEOUT:
                    continue
                assert (r.count, r.outcome) == (o.count, o.outcome), (i, q.k, cap)


def test_tiny_random_graphs_count_and_rows():
    rng = np.random.default_rng(3401)
    with gm.Engine(device=0, candidate_graph=True, steal_threshold=2) as e:
        for trial in range(100):
            n = int(rng.integers(1, 40))
            k = int(rng.integers(1, 7))
            nl = int(rng.integers(1, 4))
            g = S.gnp(n, float(rng.uniform(0.05, 0.8)), rng, nl)
            q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.6)), num_labels=nl)
            e.load(g)
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            assert (r.count, r.outcome) == (o.count, o.outcome), trial
            if o.count <= 5000:
                er = e.enumerate(qid, 5000)
                assert np.array_equal(sort_rows(er.matches), sort_rows(oracle.enumerate_sorted(g, q, 5000))), trial
            e.free_query(qid)


def test_degenerate_queries():
    with gm.Engine(device=0, candidate_graph=True) as e:
        g = S.graph_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)], [0, 0, 1, 1, 0, 0])
        e.load(g)
        # a label G does not have
        r = e.count(e.add(S.query(2, [(0, 1)], [0, 7])))
        assert (r.count, r.outcome) == (0, gm.GM_DONE)
        # one vertex: its candidates
        r = e.count(e.add(S.query(1, [], [1])))
        assert r.count == 2
        # one edge
        q = S.query(2, [(0, 1)], [0, 1])
        r = e.count(e.add(q))
        assert r.count == oracle.count(g, q).count == 2
        # every root filtered out: both labels are present, but no A vertex has a B neighbour
        e.load(S.graph_from_edges(4, [(0, 1), (2, 3)], [0, 0, 1, 1]))
        q = S.query(2, [(0, 1)], [0, 1])
        qid = e.add(q)
        sets, edges, _ = e.candidate_sets(qid)
        assert not sets.any() and edges == 0
        r = e.count(qid)
        assert (r.count, r.outcome, r.pool_rows) == (0, gm.GM_DONE, 0)
        # a time limit still ends the search
        g = S.complete(60)
        e.load(g)
        r = e.count(e.add(S.clique_q(9)), time_limit_s=0.02)
        assert r.outcome in (gm.GM_TIMEOUT, gm.GM_DONE)


def test_symmetry_breaking_on_candidate_graph():
    rp, col = wl.erdos_renyi(3000, 24000, seed=3501)
    g = wl.Graph(rp, col, wl.uniform_labels(3000, 2, seed=3502))
    with gm.Engine(device=0, candidate_graph=True) as e:
        e.load(g)
        for q in (S.clique_q(3), S.cycle_q(4), S.path_q(4), S.star_q(3)):
            qid = e.add(q)
            full = oracle.count(g, q, order=e.get_order(qid)).count
            aut = e.set_symmetry_breaking(qid, True)
            r = e.count(qid)
            assert r.count * aut == full, (q.k, q.m)


def test_batched_calls_refuse_the_mode():
    g = S.complete(10)
    with gm.Engine(device=0, candidate_graph=True) as e:
        e.load(g)
        qid = e.add(S.clique_q(3))
        with pytest.raises(gm.GmError) as ex:
            e.count_batch([qid])
        assert ex.value.status == gm.GM_ERR_STATE
        with pytest.raises(gm.GmError) as ex:
            e.serve()
        assert ex.value.status == gm.GM_ERR_STATE
        assert e.count(qid).count == 720
