"""Graph load from caller-owned device buffers (gm_load_graph_device) and the
device-side graph checks shared by both load calls.

The same graph loaded from host arrays and from torch device tensors (only
their addresses cross the ABI) gives identical counts, work counters and
enumerated rows, equal to the oracle's.  Malformed graphs are refused with
GM_ERR_GRAPH by both calls, and a refused load leaves the previous graph in
place.
"""
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
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _graph():
    """An ER part (its queries finish) beside an R-MAT part with hubs (rows far
    longer than a wavefront; its queries reach the cap), labels 0-3 and 4-9."""
    rp, col = wl.erdos_renyi(3000, 15000, seed=4605)
    ge = wl.Graph(rp, col, wl.uniform_labels(3000, 4, seed=4606))
    rp, col = wl.rmat(13, 16, seed=4601)
    gr = wl.Graph(rp, col, wl.zipf_labels(1 << 13, 6, 1.0, seed=4602) + 4)
    return S.disjoint_union(ge, gr)


def _queries(g):
    return wl.extract_queries_any(g, 4, 6, seed=4603) + wl.extract_queries_any(g, 6, 4, seed=4604)


def _run(e, g, qs):
    out = []
    for q in qs:
        qid = e.add(q)
        r = e.count(qid, cap=2_000_000)
        er = e.enumerate(qid, 3000)
        rows = b""
        if er.outcome == gm.GM_DONE:  # a capped enumeration may return any 3000 of the rows
            m = er.matches
            rows = (m[np.lexsort(m.T[::-1])] if m.shape[0] else m).tobytes()
        # the work counters of a capped search depend on the schedule; those of a finished one do not
        work = (r.groups, r.tasks) if r.outcome == gm.GM_DONE else None
        out.append((r.count, r.outcome, work, e.get_order(qid).tolist(), rows))
        e.free_query(qid)
    return out


@pytest.mark.parametrize("rp_bytes", [8, 4])
def test_device_buffers_give_the_host_load_results(torch_cuda, rp_bytes):
    torch = torch_cuda
    g = _graph()
    qs = _queries(g)
    with gm.Engine(device=0) as e:
        e.load(g)
        want = _run(e, g, qs)
    for (count, outcome, work, phi, _), q in zip(want, qs):
        o = oracle.count(g, q, order=np.asarray(phi, dtype=np.int32), cap=2_000_000)
        assert (count, outcome) == (o.count, o.outcome)
        if outcome == gm.GM_DONE:
            assert work == (o.groups, o.tasks)
    assert any(w is not None for _, _, w, _, _ in want)
    dev = torch.device("cuda:0")
    rp_t = torch.from_numpy(g.row_ptr.astype(np.int64 if rp_bytes == 8 else np.int32)).to(dev)
    col_t = torch.from_numpy(g.col.astype(np.int32)).to(dev)
    lab_t = torch.from_numpy(g.labels.astype(np.uint8)).to(dev)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with gm.Engine(device=0) as e:
        _say(f"device load, row_ptr {rp_bytes} bytes")
        e.load_graph_device(g.n, rp_t.data_ptr(), rp_bytes, col_t.data_ptr(), lab_t.data_ptr(), stream.cuda_stream)
        got = _run(e, g, qs)
        assert got == want
    del col_t  # the engine that used it is gone


def test_device_load_refuses_host_pointers_and_bad_widths(torch_cuda):
    torch = torch_cuda
    g = S.complete(5)
    rp_t = torch.from_numpy(g.row_ptr).cuda()
    col_t = torch.from_numpy(g.col).cuda()
    lab_t = torch.zeros(5, dtype=torch.uint8, device="cuda")
    with gm.Engine(device=0) as e:
        with pytest.raises(gm.GmError) as ei:
            e.load_graph_device(5, g.row_ptr.ctypes.data, 8, col_t.data_ptr(), lab_t.data_ptr())
        assert ei.value.status == gm.GM_ERR_ARG
        with pytest.raises(gm.GmError) as ei:
            e.load_graph_device(5, rp_t.data_ptr(), 2, col_t.data_ptr(), lab_t.data_ptr())
        assert ei.value.status == gm.GM_ERR_ARG
        with pytest.raises(gm.GmError) as ei:
            e.load_graph_device(5, rp_t.data_ptr(), 8, g.col.ctypes.data, lab_t.data_ptr())
        assert ei.value.status == gm.GM_ERR_ARG
        torch.cuda.synchronize()
        e.load_graph_device(5, rp_t.data_ptr(), 8, col_t.data_ptr(), lab_t.data_ptr())
        qid = e.add(S.query(3, [(0, 1), (1, 2), (0, 2)]))
        assert e.count(qid).count == 60


def _bad_graphs():
    """(name, n, row_ptr, col) cases every load call must refuse."""
    ok = S.complete(4)
    cases = []
    rp, col = ok.row_ptr.copy(), ok.col.copy()
    col[0], col[1] = col[1], col[0]
    cases.append(("unsorted row", 4, rp, col))
    rp, col = ok.row_ptr.copy(), ok.col.copy()
    col[0] = 0
    cases.append(("self-loop", 4, rp, col))
    rp, col = ok.row_ptr.copy(), ok.col.copy()
    col[2] = 7
    cases.append(("id out of range", 4, rp, col))
    # edge 0-1 stored only at 0
    g = S.graph_from_edges(3, [(0, 1), (1, 2)])
    rp = np.array([0, 1, 2, 3], dtype=np.int64)
    col = np.array([1, 2, 1], dtype=np.int32)
    cases.append(("asymmetric", 3, rp, col))
    rp, col = ok.row_ptr.copy(), ok.col.copy()
    rp[2] = rp[1] - 1
    cases.append(("decreasing row_ptr", 4, rp, col))
    return cases


def test_malformed_graphs_are_refused_and_the_old_graph_stays(torch_cuda):
    torch = torch_cuda
    good = S.complete(6)
    q = S.query(3, [(0, 1), (1, 2), (0, 2)])
    with gm.Engine(device=0) as e:
        e.load(good)
        qid = e.add(q)
        assert e.count(qid).count == 120
        for name, n, rp, col in _bad_graphs():
            _say(f"bad graph: {name}")
            labels = np.zeros(n, dtype=np.int32)
            with pytest.raises(gm.GmError) as ei:
                e.load_graph(rp, col, labels)
            assert ei.value.status == gm.GM_ERR_GRAPH, name
            assert e.count(qid).count == 120, name  # the previous graph is still loaded
            rp_t = torch.from_numpy(rp.astype(np.int64)).cuda()
            col_t = torch.from_numpy(col.astype(np.int32)).cuda()
            lab_t = torch.zeros(n, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            with pytest.raises(gm.GmError) as ei:
                e.load_graph_device(n, rp_t.data_ptr(), 8, col_t.data_ptr(), lab_t.data_ptr())
            assert ei.value.status == gm.GM_ERR_GRAPH, name
            assert e.count(qid).count == 120, name


def test_label_values_and_empty_graphs(torch_cuda):
    torch = torch_cuda
    # 255 distinct uint8 values are accepted, 256 are not
    n = 256
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(0, dtype=np.int32)
    with gm.Engine(device=0) as e:
        rp_t = torch.from_numpy(rp).cuda()
        col_t = torch.zeros(1, dtype=torch.int32, device="cuda")
        lab_t = torch.arange(256, dtype=torch.int32).to(torch.uint8).cuda()
        torch.cuda.synchronize()
        with pytest.raises(gm.GmError) as ei:
            e.load_graph_device(n, rp_t.data_ptr(), 8, col_t.data_ptr(), lab_t.data_ptr())
        assert ei.value.status == gm.GM_ERR_GRAPH
        lab_t = torch.arange(255, dtype=torch.int32).to(torch.uint8).cuda()
        rp_t = torch.from_numpy(np.zeros(256, dtype=np.int64)).cuda()
        torch.cuda.synchronize()
        e.load_graph_device(255, rp_t.data_ptr(), 8, col_t.data_ptr(), lab_t.data_ptr())
        qid = e.add(S.query(1, [], [7]))
        assert e.count(qid).count == 1          # one isolated vertex carries label 7
        # an empty graph through both calls
        e.load_graph(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.int32))
        qid = e.add(S.query(2, [(0, 1)]))
        assert e.count(qid).count == 0
