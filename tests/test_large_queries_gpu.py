"""Queries of 12 to 32 vertices (the large-query workload's sizes), which run the
K = 16 and K = 32 stack variants, against the oracle.

* ER graph, 8 uniform labels: searches finish, so counts, groups, tasks and
  sorted rows must match exactly.
* R-MAT scale 16 with 8 Zipf(1.2) labels (the large workload's recipe at a
  smaller scale): hubs make every query reach the cap, so counts and outcomes
  are compared under a cap.
"""
import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def er_case():
    rp, col = wl.erdos_renyi(4000, 20000, seed=1701)
    g = wl.Graph(rp, col, wl.uniform_labels(4000, 8, seed=1702))
    qs = []
    for k, seed in ((12, 1703), (16, 1704), (24, 1705), (32, 1706)):
        qs += wl.extract_queries_any(g, k, 3, seed=seed)
    return g, qs


@pytest.mark.parametrize("tau,threshold", [(0, 0), (-1, 2)])
def test_large_queries_exact(tau, threshold):
    g, qs = er_case()
    with gm.Engine(device=0, tau=tau, steal_threshold=threshold) as e:
        e.load(g)
        for i, q in enumerate(qs):
            _say(f"er large tau={tau} query {i} k={q.k} m={q.m}")
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            assert o.outcome == oracle.DONE
            assert (r.count, r.groups, r.tasks, r.outcome) == (o.count, o.groups, o.tasks, o.outcome), (i, q.k)
            assert r.count >= 1


def test_large_queries_enumerate():
    g, qs = er_case()
    with gm.Engine(device=0) as e:
        e.load(g)
        for q in (qs[2], qs[6], qs[9]):
            qid = e.add(q)
            o = oracle.match(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, order=e.get_order(qid),
                             enumerate_rows=200000)
            if o.count > 200000:
                continue
            r = e.enumerate(qid, 200000)
            got = r.matches[np.lexsort(r.matches.T[::-1])]
            want = o.rows[np.lexsort(o.rows.T[::-1])]
            assert np.array_equal(got, want), q.k
            assert tuple(q.witness) in {tuple(x) for x in got}


def test_large_queries_rmat_capped():
    rp, col = wl.rmat(16, 16, seed=1601)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 16, 8, 1.2, seed=1602))
    qs = wl.extract_queries(g, [12, 16, 24, 32], 2, 2, seed=1603)
    with gm.Engine(device=0) as e:
        e.load(g)
        for i, q in enumerate(qs):
            _say(f"rmat16 query {i} k={q.k} dense={q.dense}")
            qid = e.add(q)
            for cap in (1, 200000):
                r = e.count(qid, cap=cap)
                o = oracle.count(g, q, order=e.get_order(qid), cap=cap, time_limit_s=30)
                if o.outcome == oracle.TIMEOUT:
                    continue
                assert (r.count, r.outcome) == (o.count, o.outcome), (i, q.k, cap)


def test_large_query_time_limit():
    rp, col = wl.rmat(16, 16, seed=1601)
    g = wl.Graph(rp, col, np.zeros(1 << 16, np.int32))
    q = wl.extract_queries_any(g, 32, 1, seed=1607)[0]
    with gm.Engine(device=0) as e:
        e.load(g)
        r = e.count(e.add(q), time_limit_s=0.05)
        assert r.outcome in (gm.GM_TIMEOUT, gm.GM_DONE)
        if r.outcome == gm.GM_TIMEOUT:
            assert r.search_ms < 5000
