"""Work stealing (Sec. 4.3, dynamic balancing): donated task ranges are explored
exactly once.  groups and tasks count every partial match extended and every
candidate examined, so a range run twice or dropped would change them."""
import sys

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from tests import shapes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def hub_graph():
    edges = [(0, i) for i in range(1, 3001)]
    rng = np.random.default_rng(8)
    for a in range(1, 200):
        for b in range(a + 1, 200):
            if rng.random() < 0.2:
                edges.append((a, b))
    labels = np.array([0] + [1] * 199 + [2] * 2801, dtype=np.int32)
    return S.graph_from_edges(3001, edges, labels)


HUB_QUERIES = [S.query(4, [(0, 1), (0, 2), (0, 3)], [0, 1, 1, 2]),
               S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [1, 1, 1, 1]),
               S.query(5, [(0, 1), (1, 2), (2, 0), (0, 3), (3, 4)], [0, 1, 1, 1, 1]),
               S.query(4, [(0, 1), (1, 2), (2, 0), (2, 3)], [1, 1, 1, 0])]


@pytest.mark.parametrize("tau,threshold", [(-1, 2), (-1, 0), (0, 2), (100, 16)])
def test_stealing_explores_every_task_once(tau, threshold):
    g = hub_graph()
    steals = 0
    with gm.Engine(device=0, tau=tau, steal_threshold=threshold) as e:
        e.load(g)
        for i, q in enumerate(HUB_QUERIES):
            _say(f"tau={tau} threshold={threshold} query {i}")
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            assert (r.count, r.groups, r.tasks, r.outcome) == (o.count, o.groups, o.tasks, o.outcome), i
            steals += r.steals
    if tau == -1:
        assert steals > 0          # the hub's subtree starts in one wavefront


def test_stealing_off_matches_on():
    g = hub_graph()
    res = {}
    for off in (False, True):
        with gm.Engine(device=0, tau=-1, disable_stealing=off, steal_threshold=4) as e:
            e.load(g)
            out = []
            for q in HUB_QUERIES:
                r = e.count(e.add(q))
                out.append((r.count, r.groups, r.tasks))
                if off:
                    assert r.steals == 0
            res[off] = out
    assert res[False] == res[True]


def test_stealing_enumerate_rows():
    g = hub_graph()
    q = HUB_QUERIES[3]
    with gm.Engine(device=0, tau=-1, steal_threshold=2) as e:
        e.load(g)
        qid = e.add(q)
        o = oracle.match(g.row_ptr, g.col, g.labels, q.k, q.edges, q.labels, order=e.get_order(qid),
                         enumerate_rows=2_000_000)
        r = e.enumerate(qid, 2_000_000)
        assert r.outcome == gm.GM_DONE and r.count == o.count == r.rows
        got = r.matches[np.lexsort(r.matches.T[::-1])]
        want = o.rows[np.lexsort(o.rows.T[::-1])]
        assert np.array_equal(got, want)


def test_stealing_with_cap_and_time_limit():
    g = hub_graph()
    q = HUB_QUERIES[0]
    with gm.Engine(device=0, tau=-1, steal_threshold=2) as e:
        e.load(g)
        qid = e.add(q)
        truth = oracle.count(g, q).count
        for cap in (1, 1000, truth - 1, truth, truth + 5):
            r = e.count(qid, cap=cap)
            assert r.count == min(cap, truth)
            assert r.outcome == (gm.GM_CAPPED if truth >= cap else gm.GM_DONE)
        big = S.complete(60)
        e.load(big)
        qid = e.add(S.clique_q(7))
        r = e.count(qid, time_limit_s=0.05)
        assert r.outcome == gm.GM_TIMEOUT
