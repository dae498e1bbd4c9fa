"""Allocation-free count (gm_count_noalloc) against gm_count_batch on the same
query, through the C ABI: two calls in a row, the second with a smaller input
(a smaller query on a smaller graph), so that what the first call left in the
library's fixed arena cannot leak into the second.  Finished searches are also
checked against the oracle."""
import sys

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(r, b, tag):
    assert (r.count, r.outcome) == (b.count, b.outcome), (tag, r.count, b.count, r.outcome, b.outcome)
    if r.outcome == gm.GM_DONE:
        assert (r.groups, r.tasks) == (b.groups, b.tasks), (tag, r.groups, b.groups, r.tasks, b.tasks)
    assert r.pool_rows == b.pool_rows and r.pool_depth == 1


def test_two_calls_in_a_row_second_smaller():
    # first input: a 12-vertex query on an R-MAT graph with hubs, capped
    rp, col = wl.rmat(13, 16, seed=6101)
    g1 = wl.Graph(rp, col, wl.zipf_labels(1 << 13, 6, 1.0, seed=6102))
    q1 = wl.extract_queries_any(g1, 12, 1, seed=6103)[0]
    # second input: a 4-vertex query on a small ER graph, exact
    rp, col = wl.erdos_renyi(2000, 8000, seed=6104)
    g2 = wl.Graph(rp, col, wl.uniform_labels(2000, 4, seed=6105))
    q2 = wl.extract_queries_any(g2, 4, 1, seed=6106)[0]
    with gm.Engine(device=0) as e1, gm.Engine(device=0) as e2:
        e1.load(g1)
        e2.load(g2)
        a = e1.add(q1)
        b = e2.add(q2)
        _say("call 1: 12-vertex query, cap 5e6")
        r1 = e1.count_noalloc(a, cap=5_000_000)
        want1, _ = e1.count_batch([a], cap=5_000_000)
        _same(r1, want1[0], "call 1")
        _say("call 2: 4-vertex query on the smaller graph")
        r2 = e2.count_noalloc(b)
        want2, _ = e2.count_batch([b])
        _same(r2, want2[0], "call 2")
        o2 = oracle.count(g2, q2, order=e2.get_order(b))
        assert (r2.count, r2.outcome, r2.groups, r2.tasks) == (o2.count, o2.outcome, o2.groups, o2.tasks)
        assert r2.count >= 1
        # the first engine again after the second: its arena contents are the second call's
        r3 = e1.count_noalloc(a, cap=5_000_000)
        assert (r3.count, r3.outcome) == (r1.count, r1.outcome)


def test_finished_searches_equal_the_oracle_and_options_hold():
    rp, col = wl.erdos_renyi(3000, 15000, seed=6201)
    g = wl.Graph(rp, col, wl.uniform_labels(3000, 4, seed=6202))
    qs = wl.extract_queries_any(g, 5, 4, seed=6203) + wl.extract_queries_any(g, 8, 3, seed=6204)
    for opts in ({}, {"disable_stealing": True}, {"merge_ratio": -1}, {"steal_threshold": 2}):
        with gm.Engine(device=0, **opts) as e:
            e.load(g)
            for i, q in enumerate(qs):
                qid = e.add(q)
                r = e.count_noalloc(qid, cap=10_000_000, time_limit_s=30.0)
                want, _ = e.count_batch([qid], cap=10_000_000, time_limit_s=30.0)
                _same(r, want[0], f"{opts} q{i}")
                if r.outcome == gm.GM_DONE:
                    o = oracle.count(g, q, order=e.get_order(qid), cap=10_000_000)
                    assert (r.count, r.groups, r.tasks) == (o.count, o.groups, o.tasks), (opts, i)


def test_degenerate_and_refused_calls():
    g = S.complete(6)
    with gm.Engine(device=0) as e:
        e.load(g)
        absent = e.add(S.query(2, [(0, 1)], [0, 5]))     # label 5 is not in G: no candidates, no launch
        r = e.count_noalloc(absent)
        assert (r.count, r.outcome) == (0, gm.GM_DONE)
        one = e.add(S.query(1, [], [0]))
        assert e.count_noalloc(one).count == 6
        tri = e.add(S.clique_q(3))
        assert e.count_noalloc(tri, cap=7).count == 7
        assert e.count_noalloc(tri).count == 120
    with gm.Engine(device=0, candidate_graph=True) as e:
        e.load(g)
        with pytest.raises(gm.GmError) as ei:
            e.count_noalloc(e.add(S.clique_q(3)))
        assert ei.value.status == gm.GM_ERR_STATE
