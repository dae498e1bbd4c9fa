"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Counts, enumerated rows (sorted) and the work counters (groups, tasks) must be
bit-exact for finished searches; both sides use the same matching order.
"""
import math
import os
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


@pytest.fixture(scope="module")
def engine():
    e = gm.Engine(device=0)
    yield e
    e.close()


def run_pair(e, g, q, cap=0, order=None, enum_limit=0):
    qid = e.add(q)
    if order is not None:
        e.set_order(qid, order)
    phi = e.get_order(qid)
    r = e.count(qid, cap=cap)
    o = oracle.count(g, q, order=phi, cap=cap)
    rows = None
    if enum_limit:
        er = e.enumerate(qid, enum_limit)
        rows = er.matches
    e.free_query(qid)
    return r, o, rows


def assert_same(r, o, tag=""):
    assert r.count == o.count, (tag, r.count, o.count)
    assert r.outcome == o.outcome, (tag, r.outcome, o.outcome)
    if r.outcome == gm.GM_DONE:
        assert r.groups == o.groups, (tag, "groups", r.groups, o.groups)
        assert r.tasks == o.tasks, (tag, "tasks", r.tasks, o.tasks)


def sort_rows(rows):
    rows = np.asarray(rows)
    if rows.shape[0] == 0:
        return rows
    return rows[np.lexsort(rows.T[::-1])]


def test_small_er_workload_counts_and_counters(engine):
    w = wl.small_er()
    engine.load(w.graph)
    for i, q in enumerate(w.queries):
        _say(f"small_er query {i} k={q.k} m={q.m}")
        r, o, _ = run_pair(engine, w.graph, q)
        assert_same(r, o, f"q{i}")
        assert r.count >= 1


def test_small_er_enumerate_sorted_rows(engine):
    w = wl.small_er(num_queries=6)
    engine.load(w.graph)
    for i, q in enumerate(w.queries):
        qid = engine.add(q)
        phi = engine.get_order(qid)
        o = oracle.match(w.graph.row_ptr, w.graph.col, w.graph.labels, q.k, q.edges, q.labels, order=phi,
                         enumerate_rows=100000)
        er = engine.enumerate(qid, 100000)
        engine.free_query(qid)
        assert er.outcome == gm.GM_DONE and er.count == o.count == er.rows
        got = sort_rows(er.matches)
        want = sort_rows(o.rows)
        assert np.array_equal(got, want), i
        assert tuple(q.witness) in {tuple(x) for x in got}


def test_random_tiny_graphs_against_oracle(engine):
    rng = np.random.default_rng(1234)
    for trial in range(120):
        n = int(rng.integers(1, 40))
        k = int(rng.integers(1, 7))
        nl = int(rng.integers(1, 4))
        g = S.gnp(n, float(rng.uniform(0.05, 0.8)), rng, nl)
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.6)), num_labels=nl)
        engine.load(g)
        r, o, rows = run_pair(engine, g, q, enum_limit=5000)
        assert_same(r, o, f"trial {trial}")
        if o.count <= 5000:
            want = sort_rows(oracle.enumerate_sorted(g, q, 5000))
            assert np.array_equal(sort_rows(rows), want), trial


@pytest.mark.parametrize("n,k", [(12, 3), (20, 5), (70, 3), (9, 9)])
def test_cliques_closed_form(engine, n, k):
    g = S.complete(n)
    engine.load(g)
    for q in (S.clique_q(k), S.path_q(k), S.star_q(k - 1)):
        _say(f"clique n={n} k={k} query m={q.m}")
        r, o, _ = run_pair(engine, g, q)
        assert r.count == math.perm(n, k)
        groups = sum(math.perm(n, i) for i in range(1, k))
        assert r.groups == groups and r.tasks == (n - 1) * groups
        assert_same(r, o)


@pytest.mark.parametrize("opts", [dict(), dict(steal_threshold=2), dict(disable_stealing=True),
                                  dict(stack_layout=1, steal_threshold=2), dict(pool_roots_per_item=1),
                                  dict(pool_roots_per_item=7, steal_threshold=2)])
def test_first_vertex_lists_around_the_two_phase_cut(opts):
    """Roots with 63..130 candidates at position 1: the first phase keeps 64
    tasks per root and the second phase the rest, also when position 1 is
    donated (steal threshold 2)."""
    with gm.Engine(device=0, **opts) as e:
        for n in (64, 65, 66, 100, 131):
            g = S.complete(n)
            e.load(g)
            for k in (2, 3, 4):
                for q in (S.clique_q(k), S.path_q(k)):
                    _say(f"two-phase cut n={n} k={k} m={q.m} {opts}")
                    qid = e.add(q)
                    r = e.count(qid)
                    assert r.count == math.perm(n, k), (n, k)
                    groups = sum(math.perm(n, i) for i in range(1, k))
                    assert (r.groups, r.tasks) == (groups, (n - 1) * groups), (n, k)
                    e.free_query(qid)


@pytest.mark.parametrize("rpi", [1, 5, 64])
def test_roots_per_item_against_oracle(rpi):
    """First-phase items of 1, 5 and 64 roots (ragged last items): counts and counters."""
    rng = np.random.default_rng(77 + rpi)
    with gm.Engine(device=0, pool_roots_per_item=rpi) as e:
        for trial in range(25):
            g = S.gnp(int(rng.integers(20, 140)), float(rng.uniform(0.05, 0.3)), rng, 2)
            q = S.random_connected_query(int(rng.integers(2, 6)), rng, extra_p=0.4, num_labels=2)
            e.load(g)
            _say(f"roots per item {rpi} trial {trial}")
            r, o, _ = run_pair(e, g, q)
            assert_same(r, o, f"rpi {rpi} trial {trial}")


@pytest.mark.parametrize("disable", [False, True])
def test_hub_bitmaps(disable):
    """Lists of 256+ neighbours are tested through adjacency bitmaps (unless
    disabled): K_300 (every list a bitmap) against closed forms, and a dense
    labelled random graph against the oracle under a cap."""
    rng = np.random.default_rng(2024)
    with gm.Engine(device=0, disable_hub_bitmaps=disable) as e:
        g = S.complete(300)
        e.load(g)
        for k in (2, 3, 4):
            for q in (S.clique_q(k), S.path_q(k), S.star_q(k - 1)):
                _say(f"hub bitmaps disable={disable} K300 k={k} m={q.m}")
                qid = e.add(q)
                r = e.count(qid)
                assert r.count == math.perm(300, k), (k, q.m)
                groups = sum(math.perm(300, i) for i in range(1, k))
                assert (r.groups, r.tasks) == (groups, 299 * groups)
        g = S.gnp(700, 0.45, rng, 3)
        e.load(g)
        for trial in range(8):
            q = S.random_connected_query(int(rng.integers(3, 6)), rng, extra_p=0.5, num_labels=3)
            qid = e.add(q)
            r = e.count(qid, cap=300000)
            o = oracle.count(g, q, order=e.get_order(qid), cap=300000)
            assert (r.count, r.outcome) == (o.count, o.outcome), trial


def test_grid_closed_forms(engine):
    a, b = 40, 33
    g = S.grid(a, b)
    engine.load(g)
    d = g.degrees()
    cases = [(S.cycle_q(4), 8 * (a - 1) * (b - 1)),
             (S.cycle_q(6), 12 * ((a - 1) * (b - 2) + (a - 2) * (b - 1))),
             (S.path_q(3), int((d * (d - 1)).sum())),
             (S.clique_q(3), 0)]
    for q, want in cases:
        r, o, _ = run_pair(engine, g, q)
        assert r.count == want
        assert_same(r, o)


def test_every_connected_order_gives_same_count(engine):
    rng = np.random.default_rng(5)
    g = S.gnp(150, 0.08, rng, 2)
    engine.load(g)
    q = S.random_connected_query(5, rng, extra_p=0.35, num_labels=2)
    want = oracle.count(g, q).count
    for order in S.connected_orders(q)[::3]:
        r, o, _ = run_pair(engine, g, q, order=order)
        assert r.count == want
        assert_same(r, o, str(order))


def test_pool_depth_and_tau_do_not_change_results():
    """tau only moves work between the breadth-first phase and the DFS kernel."""
    rng = np.random.default_rng(17)
    g = S.gnp(400, 0.05, rng, 2)
    qs = [S.random_connected_query(k, rng, extra_p=0.25, num_labels=2) for k in (3, 4, 5, 6)]
    ref = [oracle.count(g, q) for q in qs]
    depths = set()
    for tau in (-1, 1, 7, 100, 5000, 0):
        with gm.Engine(device=0, tau=tau) as e:
            e.load(g)
            for q, o in zip(qs, ref):
                qid = e.add(q)
                o2 = oracle.count(g, q, order=e.get_order(qid))
                r = e.count(qid)
                depths.add(r.pool_depth)
                assert (r.count, r.groups, r.tasks) == (o2.count, o2.groups, o2.tasks), (tau, q.k)
                assert r.count == o.count
    assert len(depths) >= 3


def test_cap_semantics(engine):
    g = S.complete(16)
    engine.load(g)
    q = S.path_q(5)
    truth = math.perm(16, 5)
    for cap in (1, 63, 64, 65, 1000, truth - 1, truth, truth + 1):
        qid = engine.add(q)
        r = engine.count(qid, cap=cap)
        engine.free_query(qid)
        assert r.count == min(truth, cap), cap
        assert r.outcome == (gm.GM_CAPPED if truth >= cap else gm.GM_DONE), cap


def test_enumerate_with_cap_returns_distinct_valid_rows(engine):
    g = S.complete(12)
    engine.load(g)
    q = S.cycle_q(4)
    qid = engine.add(q)
    r = engine.enumerate(qid, 500)
    engine.free_query(qid)
    assert r.outcome == gm.GM_CAPPED and r.count == 500 and r.rows == 500
    rows = r.matches
    assert len({tuple(x) for x in rows}) == 500
    for x in rows:
        assert len(set(x.tolist())) == 4 and x.min() >= 0 and x.max() < 12


def test_time_limit_gives_lower_bound(engine):
    g = S.complete(60)
    engine.load(g)
    q = S.clique_q(7)
    qid = engine.add(q)
    r = engine.count(qid, time_limit_s=0.02)
    engine.free_query(qid)
    assert r.outcome == gm.GM_TIMEOUT
    assert r.count < math.perm(60, 7)


def test_degenerate_inputs(engine):
    empty = wl.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    engine.load(empty)
    for q in (S.query(1, []), S.path_q(3)):
        qid = engine.add(q)
        assert engine.count(qid).count == 0
        engine.free_query(qid)
    lonely = wl.Graph(np.zeros(5, np.int64), np.zeros(0, np.int32), np.array([0, 1, 0, 0], np.int32))
    engine.load(lonely)
    qid = engine.add(S.query(1, [], [0]))
    r = engine.enumerate(qid, 10)
    assert r.count == 3 and sorted(r.matches[:, 0].tolist()) == [0, 2, 3]
    qid = engine.add(S.query(2, [(0, 1)], [7, 7]))            # label absent from G
    assert engine.count(qid).count == 0
    g = S.complete(3)
    engine.load(g)
    qid = engine.add(S.path_q(4))                             # query larger than G
    assert engine.count(qid).count == 0


@pytest.mark.parametrize("tau", [-1, 0])
def test_single_parent_with_long_list(tau):
    """One parent whose local candidate list is much longer than a wavefront, alone
    in its scatter rounds (star centre, 1000 leaves, edge query)."""
    g = S.star_graph(1000)
    with gm.Engine(device=0, tau=tau) as e:
        e.load(g)
        qid = e.add(S.path_q(2))
        r = e.count(qid)
        assert (r.count, r.groups, r.tasks) == (2000, 1001, 2000)
        qid = e.add(S.path_q(3))
        r = e.count(qid)
        o = oracle.count(g, S.path_q(3), order=e.get_order(qid))
        assert r.count == 1000 * 999   # paths leaf-centre-leaf
        assert_same(r, o)


def test_hub_and_long_lists():
    """A hub (label 0) with 5000 neighbours: 119 core vertices (label 1, dense among
    themselves) and 4881 leaves (label 2).  Lists are far longer than a wavefront and
    the hub's subtree dwarfs every other one."""
    edges = [(0, i) for i in range(1, 5001)]
    rng = np.random.default_rng(3)
    core = list(range(1, 120))
    for a in core:
        for b in core:
            if a < b and rng.random() < 0.3:
                edges.append((a, b))
    labels = np.array([0] + [1] * 119 + [2] * 4881, dtype=np.int32)
    g = S.graph_from_edges(5001, edges, labels)
    qs = [S.query(3, [(0, 1), (1, 2), (0, 2)], [0, 1, 1]),          # hub + core edge
          S.query(3, [(0, 1), (1, 2)], [1, 0, 2]),                   # core - hub - leaf
          S.query(4, [(0, 1), (0, 2), (0, 3)], [0, 1, 1, 2]),        # star at the hub
          S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0)], [1, 1, 1, 1]),  # 4-cycles in the core
          S.query(4, [(0, 1), (1, 2), (2, 0), (0, 3)], [0, 1, 1, 1])]  # triangle + tail
    for tau in (-1, 0):
        with gm.Engine(device=0, tau=tau) as e:
            e.load(g)
            for i, q in enumerate(qs):
                _say(f"hub tau={tau} query {i}")
                qid = e.add(q)
                r = e.count(qid)
                o = oracle.count(g, q, order=e.get_order(qid))
                assert_same(r, o, f"tau={tau} q{i}")


def test_rmat20_sampled_queries_full_size(engine):
    """Full-size medium workload graph; a sample of its queries with a cap the oracle reaches quickly."""
    _say("generating R-MAT scale 20")
    w = wl.medium_rmat20(n_dense=4, n_sparse=4)
    engine.load(w.graph)
    for i, q in enumerate(w.queries):
        qid = engine.add(q)
        phi = engine.get_order(qid)
        cap = 200000
        _say(f"rmat20 query {i} dense={q.dense}")
        r = engine.count(qid, cap=cap)
        o = oracle.count(w.graph, q, order=phi, cap=cap, time_limit_s=60)
        engine.free_query(qid)
        if o.outcome != oracle.TIMEOUT:
            assert_same(r, o, f"rmat q{i}")


def test_label_index_on_off_same_results():
    """Label-partitioned scans give the same matches and the same paper-defined
    work counters as whole-list scans; they only read fewer candidates."""
    rng = np.random.default_rng(99)
    g = S.gnp(600, 0.03, rng, 5)
    qs = [S.random_connected_query(k, rng, extra_p=0.3, num_labels=5) for k in (2, 3, 4, 5, 6)]
    out = {}
    for off in (False, True):
        with gm.Engine(device=0, disable_label_index=off) as e:
            e.load(g)
            res = []
            for q in qs:
                qid = e.add(q)
                r = e.count(qid)
                o = oracle.count(g, q, order=e.get_order(qid))
                assert_same(r, o, f"label index off={off} k={q.k}")
                assert r.scanned <= r.tasks
                if off:
                    assert r.scanned == r.tasks
                res.append((r.count, r.groups, r.tasks))
            out[off] = res
    assert out[False] == out[True]
