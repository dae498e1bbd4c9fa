"""Batched counting (gm_count_batch) and its autotuner on the GPU.

Every query's result in a shared launch must equal what the query gets alone
(gm_count) and what the oracle gives: counts, outcomes and, for finished
searches, the work counters (groups, tasks), which do not depend on how work
is split between wavefronts or queries.
"""
import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def mixed_er_case():
    """ER(4000, 20000), 8 uniform labels; queries of 1..32 vertices."""
    rp, col = wl.erdos_renyi(4000, 20000, seed=2101)
    g = wl.Graph(rp, col, wl.uniform_labels(4000, 8, seed=2102))
    rng = np.random.default_rng(2103)
    qs = []
    for k in (1, 2, 3, 4, 5, 6, 8, 10, 12, 13, 16, 20, 24, 28, 32):
        qs += wl.extract_queries_any(g, k, 2, seed=int(rng.integers(1 << 30)))
    # a label G does not carry: no candidates, count 0
    qs.append(S.query(3, [(0, 1), (1, 2)], labels=[7, 99, 7]))
    return g, qs


def oracle_results(e, g, qs, qids, cap=0):
    return [oracle.count(g, q, order=e.get_order(qid), cap=cap) for q, qid in zip(qs, qids)]


def assert_matches_oracle(res, orc, tag):
    for i, (r, o) in enumerate(zip(res, orc)):
        assert (r.count, r.outcome) == (o.count, o.outcome), (tag, i, r.count, o.count, r.outcome, o.outcome)
        if o.outcome == oracle.DONE:
            assert (r.groups, r.tasks) == (o.groups, o.tasks), (tag, i)


@pytest.mark.parametrize("opts", [dict(), dict(batch_single_launch=True), dict(disable_stealing=True),
                                  dict(stack_layout=1), dict(steal_threshold=2), dict(batch_streams=1),
                                  dict(batch_streams=7, disable_stealing=True), dict(batch_streams=1000)])
def test_mixed_sizes_batched_equals_oracle(opts):
    g, qs = mixed_er_case()
    with gm.Engine(device=0, **opts) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        orc = oracle_results(e, g, qs, qids)
        _say(f"batch of {len(qids)} queries, options {opts}")
        res, info = e.count_batch(qids)
        assert_matches_oracle(res, orc, str(opts))
        assert info.count == sum(o.count for o in orc)
        assert info.launches >= 1
        assert res[-1].count == 0 and res[-1].outcome == gm.GM_DONE


def test_batched_equals_alone_and_repeats():
    g, qs = mixed_er_case()
    with gm.Engine(device=0) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        alone = [e.count(qid) for qid in qids]
        order = list(reversed(qids)) + qids[:5]  # another order, with repeats
        res, _ = e.count_batch(order)
        by_id = dict(zip(qids, alone))
        for qid, r in zip(order, res):
            a = by_id[qid]
            assert (r.count, r.outcome, r.groups, r.tasks) == (a.count, a.outcome, a.groups, a.tasks), qid


def test_empty_batch_and_errors():
    g, qs = mixed_er_case()
    with gm.Engine(device=0) as e:
        e.load(g)
        res, info = e.count_batch([])
        assert res == [] and info.launches == 0
        qid = e.add(qs[3])
        with pytest.raises(gm.GmError) as ei:
            e.count_batch([qid, 12345])
        assert ei.value.status == gm.GM_ERR_STATE


def test_small_er_workload_batched():
    w = wl.small_er()
    with gm.Engine(device=0) as e:
        e.load(w.graph)
        qids = [e.add(q) for q in w.queries]
        res, _ = e.count_batch(qids)
        assert_matches_oracle(res, oracle_results(e, w.graph, w.queries, qids), "small_er")


def rmat16_case():
    rp, col = wl.rmat(16, 16, seed=2201)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 16, 8, 1.2, seed=2202))
    rng = np.random.default_rng(2203)
    qs = []
    for k in (4, 6, 8, 12, 16, 24, 32):
        qs += wl.extract_queries_any(g, k, 3, seed=int(rng.integers(1 << 30)))
    return g, qs


@pytest.mark.parametrize("cap", [1, 1000, 200000])
def test_caps_on_hub_graph(cap):
    g, qs = rmat16_case()
    with gm.Engine(device=0) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        res, _ = e.count_batch(qids, cap=cap)
        for i, (q, qid, r) in enumerate(zip(qs, qids, res)):
            o = oracle.count(g, q, order=e.get_order(qid), cap=cap, time_limit_s=20)
            if o.outcome == oracle.TIMEOUT:
                continue
            assert (r.count, r.outcome) == (o.count, o.outcome), (i, q.k, cap)


def union(g1, g2, label_shift):
    """Disjoint union of two graphs; g2's ids and labels are shifted."""
    n1 = g1.row_ptr.shape[0] - 1
    rp = np.concatenate([g1.row_ptr, g2.row_ptr[1:] + g1.row_ptr[-1]]).astype(np.int64)
    col = np.concatenate([g1.col, g2.col + n1]).astype(np.int32)
    lab = np.concatenate([g1.labels, g2.labels + label_shift]).astype(np.int32)
    return wl.Graph(rp, col, lab)


def test_time_limit_finished_queries_are_exact():
    """Light queries (an ER part) next to explosive ones (an R-MAT part with its
    own labels) under a tight per-query limit: the explosive ones time out, and
    every query that reports DONE must carry the exact count."""
    ge, qe = mixed_er_case()
    gr, qr = rmat16_case()
    g = union(ge, gr, 8)
    qr = [wl.Query(k=q.k, edges=q.edges, labels=q.labels + 8) for q in qr if q.k >= 12]
    qs = qe[:-1] + qr
    with gm.Engine(device=0) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        res, _ = e.count_batch(qids, time_limit_s=0.005)
        outcomes = [r.outcome for r in res]
        _say(f"outcomes {outcomes}")
        assert gm.GM_TIMEOUT in outcomes and gm.GM_DONE in outcomes
        for i, (q, qid, r) in enumerate(zip(qs, qids, res)):
            if r.outcome == gm.GM_TIMEOUT:
                continue
            o = oracle.count(g, q, order=e.get_order(qid), time_limit_s=60)
            assert (r.count, r.outcome) == (o.count, o.outcome), (i, q.k)
            assert (r.groups, r.tasks) == (o.groups, o.tasks), (i, q.k)


def test_rmat20_queries_batched_equal_alone():
    """Full-size graph of the medium workload: a batch of its 8-vertex queries
    under a cap gives, query by query, what gm_count gives."""
    w = wl.medium_rmat20(n_dense=10, n_sparse=10)
    cap = 200_000
    with gm.Engine(device=0) as e:
        e.load(w.graph)
        qids = [e.add(q) for q in w.queries]
        alone = [e.count(qid, cap=cap) for qid in qids]
        res, info = e.count_batch(qids, cap=cap)
        for i, (a, r) in enumerate(zip(alone, res)):
            assert (r.count, r.outcome) == (a.count, a.outcome), i
            if a.outcome == gm.GM_DONE:
                assert (r.groups, r.tasks) == (a.groups, a.tasks), i
        _say(f"rmat20 batch {info.kernel_ms:.2f} ms kernel, alone {sum(a.kernel_ms for a in alone):.2f} ms")


def test_autotuner_keeps_counts_and_sets_options():
    g, qs = mixed_er_case()
    with gm.Engine(device=0) as e:
        e.load(g)
        qids = [e.add(q) for q in qs]
        t = e.tune_batch(qids)
        assert 10 <= t.trials <= 15
        assert t.best_ms <= t.default_ms
        o = e.options()
        assert (o.waves_per_cu, o.steal_threshold, o.stack_layout, o.batch_single_launch, o.batch_streams) == (
            t.waves_per_cu, t.steal_threshold, t.stack_layout, t.batch_single_launch, t.batch_streams)
        res, _ = e.count_batch(qids)
        assert_matches_oracle(res, oracle_results(e, g, qs, qids), "tuned")
