"""Opt-in symmetry breaking on the GPU: with it on, count x |Aut(Q)| equals the
oracle's count of every map, and the listed representatives, closed under the
automorphisms of Q, are exactly the oracle's full list."""
import itertools
import math

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu


def automorphisms(q):
    edges = {(min(a, b), max(a, b)) for a, b in q.edges}
    for p in itertools.permutations(range(q.k)):
        if all(q.labels[i] == q.labels[p[i]] for i in range(q.k)) and \
                all((min(p[a], p[b]), max(p[a], p[b])) in edges for a, b in edges):
            yield p


@pytest.mark.parametrize("opts", [dict(), dict(tau=100), dict(tau=-1), dict(stack_layout=1, steal_threshold=2)])
def test_counts_times_aut_equal_all_maps(opts):
    rng = np.random.default_rng(71)
    with gm.Engine(device=0, **opts) as e:
        for n, k in ((9, 4), (12, 5)):
            g = S.complete(n)
            e.load(g)
            for q in (S.clique_q(k), S.path_q(k), S.cycle_q(k), S.star_q(k - 1)):
                qid = e.add(q)
                aut = e.set_symmetry_breaking(qid)
                assert e.count(qid).count * aut == math.perm(n, k)
        for trial in range(25):
            g = S.gnp(int(rng.integers(10, 40)), float(rng.uniform(0.1, 0.5)), rng, int(rng.integers(1, 3)))
            q = S.random_connected_query(int(rng.integers(2, 7)), rng, extra_p=0.4, num_labels=2)
            e.load(g)
            qid = e.add(q)
            aut = e.set_symmetry_breaking(qid)
            r = e.count(qid)
            o = oracle.count(g, q)
            assert r.count * aut == o.count, (trial, r.count, aut, o.count)


def test_batched_and_er_workload():
    w = wl.small_er()
    with gm.Engine(device=0) as e:
        e.load(w.graph)
        qids = [e.add(q) for q in w.queries]
        auts = [e.set_symmetry_breaking(qid) for qid in qids]
        res, _ = e.count_batch(qids)
        for q, a, r in zip(w.queries, auts, res):
            assert r.count * a == oracle.count(w.graph, q).count


def test_representatives_cover_every_map_once():
    rng = np.random.default_rng(72)
    with gm.Engine(device=0) as e:
        for trial in range(12):
            g = S.gnp(int(rng.integers(8, 16)), 0.5, rng, 2)
            q = S.random_connected_query(int(rng.integers(3, 6)), rng, extra_p=0.5, num_labels=2)
            e.load(g)
            qid = e.add(q)
            aut = e.set_symmetry_breaking(qid)
            rows = e.enumerate(qid, 100000).matches
            full = {tuple(r) for r in oracle.enumerate_sorted(g, q, 100000)}
            closure = set()
            for row in rows:
                for p in automorphisms(q):
                    closure.add(tuple(row[list(p)]))     # the map u -> M(p(u))
            assert closure == full and len(rows) * aut == len(full), trial
