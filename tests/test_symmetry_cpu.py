"""Opt-in symmetry breaking, host side (no GPU): |Aut(Q)| as the product of the
stabilizer chain's orbit sizes, against closed forms and brute force over all
permutations of small queries."""
import itertools
import math

import numpy as np

import paper_2604_10601_amd as gm
from tests import shapes as S


def brute_aut(q):
    k = q.k
    edges = {(min(a, b), max(a, b)) for a, b in q.edges}
    n = 0
    for p in itertools.permutations(range(k)):
        if any(q.labels[i] != q.labels[p[i]] for i in range(k)):
            continue
        if all((min(p[a], p[b]), max(p[a], p[b])) in edges for a, b in edges):
            n += 1
    return n


def test_closed_forms():
    e = gm.Engine(device=-1)
    e.load(S.complete(4))
    cases = [(S.clique_q(5), math.factorial(5)), (S.path_q(6), 2), (S.cycle_q(7), 14), (S.star_q(5), math.factorial(5)),
             (S.query(3, [(0, 1), (1, 2)], labels=[1, 2, 1]), 2), (S.query(3, [(0, 1), (1, 2)], labels=[1, 2, 3]), 1),
             (S.clique_q(12), math.factorial(12)), (S.star_q(20), math.factorial(20))]
    for q, want in cases:
        qid = e.add(q)
        assert e.set_symmetry_breaking(qid) == want, (q.k, q.m)
    e.close()


def test_random_queries_against_brute_force():
    rng = np.random.default_rng(9)
    e = gm.Engine(device=-1)
    e.load(S.complete(4))
    for trial in range(60):
        k = int(rng.integers(2, 8))
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.7)), num_labels=int(rng.integers(1, 3)))
        qid = e.add(q)
        assert e.set_symmetry_breaking(qid) == brute_aut(q), trial
    e.close()
