"""Full-size parity on the two benchmark graphs, every edge loaded and searched at
its real size: R-MAT scale 20 (2^20 vertices, 15.7M edges) and R-MAT scale 24
(2^24 vertices, 260M edges, about 2.2 GB as an int32 CSR).

* Exact counts (Def. 1).  With the workloads' own Zipf labels the hubs push the
  number of matches of a random-walk query of six or more vertices past 1e8, and
  on scale 24 past that already at four vertices: far beyond what the oracle
  finishes in seconds.  So two query sets are compared, each query by count,
  outcome, groups and tasks, alone and in one batched launch:
    - scale 20 with its own labels: random walks of 4-6 vertices among the four
      rarest labels (up to about 1e8 matches);
    - both scales with a test labelling of the same edges, loaded from device
      buffers (gm_load_graph_device): every vertex of degree above 128 carries
      one label that no query uses, every other vertex one of 8 uniform labels,
      and the queries are random walks of 8-24 vertices among the other
      vertices (1e5-1e7 matches).
  Every query the oracle finishes within its budget is compared.  A query it
  does not finish ("oracle-unsolved") is cross-checked by order invariance
  instead: counted on the GPU under two different connected orders without a
  cap, both runs must finish with the same count.  Each set must keep a stated
  minimum of oracle-compared queries.
* Capped enumerations of the workloads' own queries (8 vertices on scale 20; 12,
  16, 24 and 32 on scale 24): 100,000 rows each, every row checked: injective,
  labels kept, every query edge an edge of G, and the rows distinct.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl

pytestmark = pytest.mark.gpu

HUB_DEGREE = 128      # test labelling: vertices above this degree share one unused label
TEST_LABELS = 8
ENUM_ROWS = 100_000
GPU_LIMIT_S = 10.0    # order-invariance runs of oracle-unsolved queries


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=[20, 24], ids=["rmat20", "rmat24"])
def full(request):
    import torch
    scale = request.param
    _say(f"generating the R-MAT scale-{scale} graph")
    g = wl.rmat20_graph() if scale == 20 else wl.rmat24_graph()
    _say(f"n={g.n} |E|={g.num_edges}: host load")
    e = gm.Engine(device=0)
    e.load(g)
    # the same edges with the test labelling, from device buffers
    gt = wl.Graph(g.row_ptr, g.col, wl.hub_split_labels(g, HUB_DEGREE, TEST_LABELS, seed=4700 + scale))
    rp_t = torch.from_numpy(g.row_ptr).cuda()
    col_t = torch.from_numpy(g.col).cuda()
    lab_t = torch.from_numpy(gt.labels.astype(np.uint8)).cuda()
    torch.cuda.synchronize()
    _say("device load (test labelling)")
    et = gm.Engine(device=0)
    et.load_graph_device(g.n, rp_t.data_ptr(), 8, col_t.data_ptr(), lab_t.data_ptr())
    del rp_t, lab_t
    yield scale, g, e, gt, et
    et.close()
    e.close()
    del col_t


def _order_invariance(e, qid, i, tag):
    """An oracle-unsolved query: its exact count under two different connected
    orders (the heuristic one and the next candidate order: fewest candidates
    first, else a seeded random one) must agree.  Returns True if both runs
    finished (and agreed)."""
    orders = e.candidate_orders(qid, max_orders=3, seed=1000 + i)
    if len(orders) < 2:
        return False
    runs = []
    for phi in (orders[0], orders[1]):
        e.set_order(qid, phi)
        runs.append(e.count(qid, cap=0, time_limit_s=GPU_LIMIT_S))
    if any(r.outcome != gm.GM_DONE for r in runs):
        _say(f"{tag} query {i}: not finished on the GPU within {GPU_LIMIT_S} s under both orders")
        return False
    _say(f"{tag} query {i}: {runs[0].count} matches under both orders")
    assert runs[0].count == runs[1].count, (tag, i, runs[0].count, runs[1].count)
    return True


def _compare(e, g, queries, budget_s, tag):
    """Count every query the oracle finishes within budget_s on both sides; returns the qids compared."""
    done = []
    for i, q in enumerate(queries):
        qid = e.add(q)
        phi = e.get_order(qid)
        o = oracle.count(g, q, order=phi, time_limit_s=budget_s)
        if o.outcome != oracle.DONE:
            _say(f"{tag} query {i} (k={q.k}): oracle unsolved in {budget_s} s, order invariance instead")
            _order_invariance(e, qid, i, tag)
            e.free_query(qid)
            continue
        _say(f"{tag} query {i} (k={q.k} m={q.m}): oracle {o.count} matches, groups {o.groups}, tasks {o.tasks}")
        r = e.count(qid)
        assert (r.count, r.outcome) == (o.count, o.outcome), (tag, i, r, o)
        assert (r.groups, r.tasks) == (o.groups, o.tasks), (tag, i, r.groups, r.tasks, o.groups, o.tasks)
        assert r.count >= 1  # the walk's own vertices are a match
        done.append((qid, o))
    if done:
        res, _ = e.count_batch([qid for qid, _ in done])
        for (qid, o), r in zip(done, res):
            assert (r.count, r.outcome, r.groups, r.tasks) == (o.count, o.outcome, o.groups, o.tasks), (tag, qid)
    for qid, _ in done:
        e.free_query(qid)
    return done


def test_exact_counts_rare_labels(full):
    scale, g, e, _, _ = full
    if scale != 20:
        pytest.skip("on scale 24 even 4-vertex queries on the rarest labels exceed 1e8 matches")
    counts = np.bincount(g.labels)
    rare = np.argsort(counts, kind="stable")[:4]
    sub = wl.restricted(g, np.isin(g.labels, rare))
    qs = (wl.extract_queries_any(sub, 4, 8, seed=4800) + wl.extract_queries(sub, [5], 4, 0, seed=4801) +
          wl.extract_queries(sub, [6], 4, 0, seed=4802))
    done = _compare(e, g, qs, 3.0, f"rmat{scale} rare labels")
    assert len(done) >= 8, f"only {len(done)} queries finished on the oracle"
    assert {o.count for _, o in done} != {0}


def test_exact_counts_test_labelling(full):
    scale, g, _, gt, et = full
    sub = wl.restricted(gt, np.diff(g.row_ptr) <= HUB_DEGREE)
    qs = []
    for k in (8, 12, 16, 24):
        qs += wl.extract_queries_any(sub, k, 3, seed=4900 + 10 * scale + k)
    done = _compare(et, gt, qs, 5.0, f"rmat{scale} test labelling")
    assert len(done) >= 9, f"only {len(done)} queries finished on the oracle"
    assert max(o.count for _, o in done) >= 100_000


def is_edge(g, u, v):
    """Vectorised bisection: v[i] in N(u[i])."""
    u = u.astype(np.int64)
    v = v.astype(np.int64)
    lo = g.row_ptr[u].copy()
    end = g.row_ptr[u + 1]
    hi = end.copy()
    last = max(g.nnz - 1, 0)
    while True:
        go = lo < hi
        if not go.any():
            break
        mid = (lo + hi) // 2
        c = g.col[np.minimum(mid, last)]
        lo = np.where(go & (c < v), mid + 1, lo)
        hi = np.where(go & (c >= v), mid, hi)
    return (lo < end) & (g.col[np.minimum(lo, last)] == v)


def check_rows(g, q, rows):
    assert rows.ndim == 2 and rows.shape[1] == q.k
    assert rows.min() >= 0 and rows.max() < g.n
    srt = np.sort(rows, axis=1)
    assert np.all(np.diff(srt, axis=1) != 0), "a row maps two query vertices to one data vertex"
    assert np.array_equal(g.labels[rows], np.broadcast_to(q.labels, rows.shape)), "a label differs"
    for a, b in q.edges.tolist():
        assert is_edge(g, rows[:, a], rows[:, b]).all(), f"query edge ({a}, {b}) not in G"
    assert np.unique(rows, axis=0).shape[0] == rows.shape[0], "repeated rows"


def test_capped_enumerations_are_valid(full):
    scale, g, e, _, _ = full
    if scale == 20:
        qs = wl.extract_queries(g, [8], 50, 50, seed=22)[::12]      # the 8-vertex workload's queries
        limit = 0.0
    else:
        qs = wl.large_rmat24(g=g).queries[::25]                     # 12, 16, 24 and 32 vertices
        limit = 60.0
    for i, q in enumerate(qs):
        qid = e.add(q)
        _say(f"rmat{scale} enumerate query {i} (k={q.k} m={q.m})")
        r = e.enumerate(qid, ENUM_ROWS, time_limit_s=limit)
        e.free_query(qid)
        assert r.outcome in (gm.GM_CAPPED, gm.GM_DONE)
        assert r.rows == r.matches.shape[0] == r.count
        if r.outcome == gm.GM_CAPPED:
            assert r.count == ENUM_ROWS
        check_rows(g, q, r.matches)
        assert tuple(q.witness) in {tuple(x) for x in r.matches} or r.outcome == gm.GM_CAPPED


def test_order_invariance_of_oracle_unsolved_queries(full):
    """Queries with too many matches for the oracle's budget (long walks on the
    test labelling): the GPU's exact counts under two connected orders agree."""
    scale, g, _, gt, et = full
    sub = wl.restricted(gt, np.diff(g.row_ptr) <= HUB_DEGREE)
    qs = wl.extract_queries_any(sub, 24, 3, seed=5100 + scale) + wl.extract_queries_any(sub, 32, 3, seed=5200 + scale)
    checked = 0
    for i, q in enumerate(qs):
        qid = et.add(q)
        o = oracle.count(gt, q, order=et.get_order(qid), time_limit_s=0.3)
        if o.outcome == oracle.DONE:
            _say(f"rmat{scale} long walk {i} (k={q.k}): the oracle finished ({o.count}); not an unsolved case")
        else:
            checked += _order_invariance(et, qid, i, f"rmat{scale} long walk")
        et.free_query(qid)
    assert checked >= 2, f"only {checked} oracle-unsolved queries were cross-checked"
