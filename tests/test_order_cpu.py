"""Host logic of the learned-order path (no GPU): order features and candidate
orders on a graph small enough to work out by hand."""
import math

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from tests import shapes as S


def hand_graph():
    # K4 on 0..3 (label 0); vertex 4 (label 1) next to 0 and 1; vertex 5 (label 1) next to 4
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4), (1, 4), (4, 5)]
    return S.graph_from_edges(6, edges, [0, 0, 0, 0, 1, 1])


@pytest.fixture()
def eng():
    e = gm.Engine(device=-1)
    e.load(hand_graph())
    yield e
    e.close()


def lg(x):
    return math.log2(1 + x) / 24


def test_features_worked_by_hand(eng):
    # path a - b - c with labels 0, 1, 1: candidates a: 4 (label 0, deg >= 1), b: 1 (vertex 4),
    # c: 2 (vertices 4, 5); label counts 4 and 2
    qid = eng.add(S.query(3, [(0, 1), (1, 2)], labels=[0, 1, 1]))
    f = eng.order_features(qid, [1, 0, 2])
    want = np.zeros(gm.ORDER_FEATURES)
    want[0:5] = [lg(1), 2 / 8, 0, 0, lg(2)]
    want[5:10] = [lg(4), 1 / 8, 1 / 8, lg(1), lg(4)]
    want[10:15] = [lg(2), 1 / 8, 1 / 8, lg(1), lg(2)]
    want[160], want[161] = 3 / 32, 2 / 64
    want[162] = math.log2(1) / 8           # the task split: the default 1
    assert np.allclose(f, want, atol=1e-7)
    eng.set_split(qid, 64)
    assert eng.get_split(qid) == 64
    assert abs(eng.order_features(qid, [1, 0, 2])[162] - 6 / 8) < 1e-7
    eng.set_split(qid, 0)                  # back to the engine's setting
    assert eng.get_split(qid) == 1
    with pytest.raises(gm.GmError):
        eng.set_split(qid, -1)


def test_candidate_orders(eng):
    qid = eng.add(S.query(3, [(0, 1), (1, 2)], labels=[0, 1, 1]))
    cands = eng.candidate_orders(qid, max_orders=8, seed=3)
    assert list(cands[0]) == list(oracle.ri_order(3, np.array([(0, 1), (1, 2)])))
    assert list(cands[1]) == [1, 2, 0]            # fewest candidates first: b (1), then c (2), then a (4)
    seen = set()
    for o in cands:
        assert sorted(o) == [0, 1, 2] and tuple(o) not in seen
        seen.add(tuple(o))
        assert o[1] == 1 or o[0] == 1             # a path: the second vertex is next to the first
    assert len(cands) == 4                        # a 3-vertex path has 4 connected orders
    again = eng.candidate_orders(qid, max_orders=8, seed=3)
    assert all(np.array_equal(a, b) for a, b in zip(cands, again))


def test_candidate_orders_on_larger_queries(eng):
    rng = np.random.default_rng(11)
    for trial in range(40):
        k = int(rng.integers(4, 20))
        q = S.random_connected_query(k, rng, extra_p=0.3, num_labels=2)
        qid = eng.add(q)
        cands = eng.candidate_orders(qid, max_orders=8, seed=trial)
        assert 1 <= len(cands) <= 8
        adj = [set() for _ in range(k)]
        for a, b in q.edges:
            adj[a].add(b)
            adj[b].add(a)
        for o in cands:
            assert sorted(o) == list(range(k))
            for i in range(1, k):
                assert adj[o[i]] & set(o[:i]), (trial, list(o))
            f = eng.order_features(qid, o)
            assert f[160] == k / 32 and abs(f[161] - len(q.edges) / 64) < 1e-7


def test_order_errors(eng):
    qid = eng.add(S.path_q(3))
    with pytest.raises(gm.GmError) as ei:
        eng.order_features(qid, [0, 2, 1])
    assert ei.value.status == gm.GM_ERR_ORDER
    with pytest.raises(gm.GmError) as ei:
        eng.candidate_orders(999)
    assert ei.value.status == gm.GM_ERR_STATE
