"""Both LDS stack layouts (full: cached list ranges; slim: membership tests on
label slices) against the oracle, with and without the label index, on small
random graphs, a hub graph with forced stealing, and large queries."""
import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu


def same(r, o, tag):
    assert (r.count, r.outcome) == (o.count, o.outcome), tag
    if r.outcome == gm.GM_DONE:
        assert (r.groups, r.tasks) == (o.groups, o.tasks), tag


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("no_index", [False, True])
def test_random_graphs_both_layouts(layout, no_index):
    rng = np.random.default_rng(4321 + layout + 10 * no_index)
    with gm.Engine(device=0, stack_layout=layout, disable_label_index=no_index) as e:
        for trial in range(60):
            n = int(rng.integers(5, 60))
            nl = int(rng.integers(1, 5))
            g = S.gnp(n, float(rng.uniform(0.05, 0.5)), rng, nl)
            q = S.random_connected_query(int(rng.integers(2, 8)), rng, extra_p=float(rng.uniform(0, 0.6)),
                                         num_labels=nl)
            e.load(g)
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            same(r, o, (layout, no_index, trial))
            if o.count <= 3000:
                rows = e.enumerate(qid, 3000).matches
                want = oracle.enumerate_sorted(g, q, 3000, order=e.get_order(qid))
                assert np.array_equal(rows[np.lexsort(rows.T[::-1])], want), trial
            e.free_query(qid)


@pytest.mark.parametrize("layout", [1, 2])
def test_hub_forced_stealing_both_layouts(layout):
    edges = [(0, i) for i in range(1, 3001)]
    rng = np.random.default_rng(8)
    for a in range(1, 200):
        for b in range(a + 1, 200):
            if rng.random() < 0.2:
                edges.append((a, b))
    labels = np.array([0] + [1] * 199 + [2] * 2801, dtype=np.int32)
    g = S.graph_from_edges(3001, edges, labels)
    qs = [S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [1, 1, 1, 1]),
          S.query(5, [(0, 1), (1, 2), (2, 0), (0, 3), (3, 4)], [0, 1, 1, 1, 1]),
          S.query(4, [(0, 1), (1, 2), (2, 0), (2, 3)], [1, 1, 1, 0])]
    with gm.Engine(device=0, tau=-1, steal_threshold=2, stack_layout=layout) as e:
        e.load(g)
        for i, q in enumerate(qs):
            qid = e.add(q)
            same(e.count(qid), oracle.count(g, q, order=e.get_order(qid)), (layout, i))


@pytest.mark.parametrize("layout", [1, 2])
def test_large_queries_both_layouts(layout):
    rp, col = wl.erdos_renyi(4000, 20000, seed=1701)
    g = wl.Graph(rp, col, wl.uniform_labels(4000, 8, seed=1702))
    qs = wl.extract_queries_any(g, 12, 2, seed=1703) + wl.extract_queries_any(g, 24, 2, seed=1705) + \
        wl.extract_queries_any(g, 32, 2, seed=1706)
    with gm.Engine(device=0, stack_layout=layout) as e:
        e.load(g)
        for i, q in enumerate(qs):
            qid = e.add(q)
            same(e.count(qid), oracle.count(g, q, order=e.get_order(qid)), (layout, i, q.k))


def test_graph_above_2_24_vertices_takes_the_full_layout():
    """The slim stack keeps vertex ids in 24 bits, so a graph of more than 2^24
    vertices must be searched with the full layout.  Matches here use vertices
    above 2^24 (a dense random cluster placed there, joined to a few low ids), so
    truncated ids would change counts and rows; both are compared with the
    oracle, and a candidate-graph engine refuses the graph."""
    n = (1 << 24) + 64
    rng = np.random.default_rng(2424)
    hi = np.arange((1 << 24), n, dtype=np.int64)
    lo = np.arange(0, 16, dtype=np.int64)
    verts = np.concatenate([lo, hi])
    pairs = set()
    for _ in range(900):
        a, b = rng.choice(verts, size=2, replace=False)
        pairs.add((int(min(a, b)), int(max(a, b))))
    src = np.array([a for a, b in pairs], dtype=np.int64)
    dst = np.array([b for a, b in pairs], dtype=np.int64)
    rp, col = wl.csr_from_pairs(n, src, dst)
    labels = np.zeros(n, dtype=np.int32)
    labels[verts] = rng.integers(0, 2, size=verts.shape[0])
    g = wl.Graph(rp, col, labels)
    qs = [S.query(3, [(0, 1), (1, 2), (2, 0)], [0, 0, 1]), S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0, 1, 0, 1]),
          S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)], [1, 1, 0, 0])]
    with gm.Engine(device=0) as e:
        e.load(g)
        for i, q in enumerate(qs):
            qid = e.add(q)
            r = e.count(qid)
            o = oracle.count(g, q, order=e.get_order(qid))
            same(r, o, ("above 2^24", i))
            assert o.count > 0
            rows = e.enumerate(qid, o.count + 1).matches
            want = oracle.enumerate_sorted(g, q, o.count + 1, order=e.get_order(qid))
            assert np.array_equal(rows[np.lexsort(rows.T[::-1])], want), i
            assert rows.max() >= (1 << 24), "the matches should reach the ids above 2^24"
    with gm.Engine(device=0, candidate_graph=True) as e:
        with pytest.raises(gm.GmError) as ei:
            e.load(g)
        assert ei.value.status == gm.GM_ERR_GRAPH
