"""LDS-staged intersection (merge path) against the oracle.

A list is staged in LDS and intersected by merge path when it is short against
the run of candidates testing it (n <= merge_ratio x the run's lanes); longer
lists are bisected in device memory.  Counts, outcomes and the paper's work
counters (groups, tasks) must not depend on that choice: every case runs with
staging never (-1), by default (0: 1 entry per lane unless the staging area
would lower the wavefronts a CU keeps resident, as for the deepest queries),
always at 1 entry per lane (1) and at the largest buffer (8), with hub bitmaps
on and off, and matches the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu

RATIOS = (-1, 0, 1, 8)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(g, queries, cap=0, tag="", hubs=True):
    """Run every query under each ratio; all must equal the oracle.  Returns probes per ratio."""
    probes = {}
    for ratio in RATIOS:
        with gm.Engine(device=0, merge_ratio=ratio, disable_hub_bitmaps=not hubs) as e:
            e.load(g)
            got = []
            for i, q in enumerate(queries):
                qid = e.add(q)
                phi = e.get_order(qid)
                r = e.count(qid, cap=cap)
                o = oracle.count(g, q, order=phi, cap=cap)
                assert (r.count, r.outcome) == (o.count, o.outcome), (tag, ratio, i, r.count, o.count)
                if r.outcome == gm.GM_DONE:
                    assert (r.groups, r.tasks) == (o.groups, o.tasks), (tag, ratio, i)
                got.append(r.probes)
                e.free_query(qid)
            probes[ratio] = got
    return probes


@pytest.mark.parametrize("a,b", [(3, 5), (20, 200), (63, 64), (64, 64), (65, 130), (200, 20)])
def test_four_cycles_in_complete_bipartite_graphs(a, b):
    """K_{a,b}: a 4-cycle query tests a run of up to 64 candidates against a
    list of a or b entries (lengths on both sides of 64 and of the staging
    capacity).  Count = 2 a(a-1) b(b-1)."""
    _say(f"K_{a},{b}")
    g = S.complete_bipartite(a, b)
    probes = _check(g, [S.cycle_q(4)], tag=f"K{a},{b}")
    with gm.Engine(device=0, merge_ratio=8) as e:
        e.load(g)
        assert e.count(e.add(S.cycle_q(4))).count == 2 * a * (a - 1) * b * (b - 1)
    if min(a, b) >= 20:
        assert probes[-1] != probes[8], "staging should change the membership reads"


def test_deep_cycles_under_each_setting():
    """30- and 32-vertex cycles in K_{40,40}: the depths at which the default
    drops the staging area (LDS bounds residency there) while ratio 1 keeps it.
    Both stop at the cap; the count must be the cap under every setting."""
    _say("K_40,40 deep cycles")
    _check(S.complete_bipartite(40, 40), [S.cycle_q(30), S.cycle_q(32)], cap=1_000_000, tag="K40,40 C30/C32")


def test_cliques_and_labelled_cliques():
    qs = [S.clique_q(3), S.clique_q(4), S.clique_q(5)]
    _check(S.complete(40), qs, tag="K40")
    rng = np.random.default_rng(5101)
    labels = rng.integers(0, 3, size=70)
    g = S.complete(70, labels)
    lq = [S.query(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)], [0, 1, 0, 2]),
          S.query(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (1, 3)], [1, 1, 2, 0, 0])]
    _check(g, lq, cap=5_000_000, tag="labelled K70")


@pytest.mark.parametrize("hubs", [True, False])
def test_random_graphs_and_walk_queries(hubs):
    rp, col = wl.rmat(12, 16, seed=5201)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 12, 20, 0.5, seed=5202))
    qs = []
    for k in (4, 6, 8, 12, 16):
        qs += wl.extract_queries_any(g, k, 3, seed=5210 + k)
    _say(f"rmat12 walks, hubs={hubs}")
    _check(g, qs, cap=3_000_000, tag=f"rmat12 hubs={hubs}", hubs=hubs)
    rp, col = wl.erdos_renyi(3000, 30000, seed=5203)
    ge = wl.Graph(rp, col, wl.uniform_labels(3000, 8, seed=5204))
    qe = []
    for k in (5, 8, 12):
        qe += wl.extract_queries_any(ge, k, 4, seed=5220 + k)
    _say(f"ER walks, hubs={hubs}")
    _check(ge, qe, cap=3_000_000, tag=f"er3000 hubs={hubs}", hubs=hubs)


def test_enumerated_rows_do_not_depend_on_staging():
    g = S.complete_bipartite(12, 40)
    q = S.cycle_q(4)
    rows = {}
    for ratio in RATIOS:
        with gm.Engine(device=0, merge_ratio=ratio) as e:
            e.load(g)
            er = e.enumerate(e.add(q), 2 * 12 * 11 * 40 * 39 + 1)  # one more than the matches: DONE
            assert er.outcome == gm.GM_DONE
            m = er.matches
            rows[ratio] = m[np.lexsort(m.T[::-1])]
    assert all(np.array_equal(rows[-1], rows[r]) for r in RATIOS)
    want = oracle.enumerate_sorted(g, q, rows[-1].shape[0] + 1)
    assert np.array_equal(rows[-1], want)


def test_option_range():
    for bad in (-2, 9):
        with pytest.raises(gm.GmError) as ei:
            gm.Engine(device=0, merge_ratio=bad)
        assert ei.value.status == gm.GM_ERR_ARG
