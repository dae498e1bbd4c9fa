"""The seeded input generators (CPU only): the native R-MAT build and the random
walks give well-formed inputs that do not depend on the thread count."""
import numpy as np

from paper_2604_10601_amd import workloads as wl


def _check_csr(row_ptr, col, n):
    assert row_ptr.shape == (n + 1,) and row_ptr[0] == 0 and np.all(np.diff(row_ptr) >= 0)
    assert col.shape == (row_ptr[-1],) and (col.size == 0 or (col.min() >= 0 and col.max() < n))
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    assert np.all(src != col), "self-loop"
    inner = np.ones(col.size, dtype=bool)
    inner[row_ptr[:-1][np.diff(row_ptr) > 0]] = False  # first entry of each row
    assert np.all(np.diff(col.astype(np.int64))[inner[1:]] > 0), "rows must be strictly ascending"
    fwd = np.sort(src * n + col)
    bwd = np.sort(col.astype(np.int64) * n + src)
    assert np.array_equal(fwd, bwd), "not symmetric"


def test_rmat_is_a_simple_symmetric_csr_independent_of_threads():
    rp1, c1 = wl.rmat(12, 16, seed=5, threads=1)
    rp8, c8 = wl.rmat(12, 16, seed=5, threads=8)
    assert np.array_equal(rp1, rp8) and np.array_equal(c1, c8)
    _check_csr(rp1, c1, 1 << 12)
    # duplicates and loops were dropped: fewer undirected edges than draws, most survive
    assert 0.5 * (16 << 12) < rp1[-1] // 2 < (16 << 12)
    rp_other, _ = wl.rmat(12, 16, seed=6)
    assert not np.array_equal(rp1, rp_other)


def test_rmat_degree_skew_follows_the_quadrant_weights():
    # a = 0.57 concentrates edges on few vertices; uniform weights spread them
    rp, _ = wl.rmat(14, 16, seed=1)
    rpu, _ = wl.rmat(14, 16, seed=1, a=0.25, b=0.25, c=0.25)
    assert np.diff(rp).max() > 20 * np.diff(rpu).max()
    assert np.diff(rpu).max() < 100


def test_walk_queries_are_connected_induced_and_witnessed():
    rp, col = wl.rmat(14, 16, seed=9)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 14, 8, 1.2, seed=10))
    qs = wl.extract_queries(g, [6, 12], 3, 3, seed=11)
    assert [q.k for q in qs] == [6] * 6 + [12] * 6
    assert [q.dense for q in qs] == ([True] * 3 + [False] * 3) * 2
    for q in qs:
        w = q.witness
        assert len(set(w.tolist())) == q.k
        assert np.array_equal(q.labels, g.labels[w])
        # exactly the induced edges
        adj = {(a, b) for a, b in q.edges.tolist()}
        for a in range(q.k):
            nb = set(col[rp[w[a]]:rp[w[a] + 1]].tolist())
            for b in range(a + 1, q.k):
                assert ((a, b) in adj) == (int(w[b]) in nb)
        # connected
        seen, todo = {0}, [0]
        while todo:
            x = todo.pop()
            for a, b in q.edges.tolist():
                for s, t in ((a, b), (b, a)):
                    if s == x and t not in seen:
                        seen.add(t)
                        todo.append(t)
        assert len(seen) == q.k
    # same seed, same queries; the stream index decides a query
    again = wl.extract_queries(g, [6, 12], 3, 3, seed=11)
    assert all(np.array_equal(a.witness, b.witness) for a, b in zip(qs, again))
    one = wl.walk_query(g, 12, seed=11, stream=0)
    assert np.array_equal(one.witness, wl.extract_queries_any(g, 12, 1, seed=11)[0].witness)
