"""C-ABI checks that need no GPU: the library loads, exports what the header
declares, struct layouts agree with the binding, and the host-side logic
(input checks, matching-order plan, error codes) behaves as documented."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmatch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = gm.load_library()
    names = declared_functions()
    assert set(names) == set(gm.ABI_FUNCTIONS)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gmatch.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gm_options),'
                   ' sizeof(gm_result), offsetof(gm_result, kernel_ms), offsetof(gm_options, stack_layout),'
                   ' offsetof(gm_result, rows), offsetof(gm_options, batch_single_launch),'
                   ' sizeof(gm_batch_info), offsetof(gm_batch_info, count), sizeof(gm_tuning));'
                   'printf("%zu %zu %zu %zu\\n", sizeof(gm_serve_options), offsetof(gm_serve_options, max_pending),'
                   ' sizeof(gm_serve_result), offsetof(gm_serve_result, result));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    vals = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert vals == [ctypes.sizeof(gm.Options), ctypes.sizeof(gm._CResult), gm._CResult.kernel_ms.offset,
                    gm.Options.stack_layout.offset, gm._CResult.rows.offset, gm.Options.batch_single_launch.offset,
                    ctypes.sizeof(gm.BatchInfo), gm.BatchInfo.count.offset, ctypes.sizeof(gm.Tuning),
                    ctypes.sizeof(gm.ServeOptions), gm.ServeOptions.max_pending.offset,
                    ctypes.sizeof(gm._CServeResult), gm._CServeResult.result.offset]


@pytest.fixture()
def host_engine():
    e = gm.Engine(device=-1)
    yield e
    e.close()


def expect(status, fn, *args):
    with pytest.raises(gm.GmError) as ei:
        fn(*args)
    assert ei.value.status == status, str(ei.value)


def test_graph_checks(host_engine):
    e = host_engine
    g = S.complete(5)
    e.load(g)                                                   # accepted
    bad = g.col.copy()
    bad[0], bad[1] = bad[1], bad[0]
    expect(gm.GM_ERR_GRAPH, e.load_graph, g.row_ptr, bad, g.labels)              # unsorted row
    expect(gm.GM_ERR_GRAPH, e.load_graph, np.array([0, 1, 1]), np.array([1]), np.zeros(2))   # one direction only
    expect(gm.GM_ERR_GRAPH, e.load_graph, np.array([0, 1]), np.array([0]), np.zeros(1))      # self-loop
    expect(gm.GM_ERR_GRAPH, e.load_graph, np.array([0, 1, 2]), np.array([1, 5]), np.zeros(2))  # out of range
    expect(gm.GM_ERR_GRAPH, e.load_graph, np.array([1, 1]), np.array([0]), np.zeros(1))      # row_ptr[0] != 0
    expect(gm.GM_ERR_GRAPH, e.load_graph, np.array([0, 2, 1]), np.array([1, 0]), np.zeros(2))  # decreasing
    dup = np.array([0, 2, 4], np.int64), np.array([1, 1, 0, 0], np.int32)
    expect(gm.GM_ERR_GRAPH, e.load_graph, dup[0], dup[1], np.zeros(2))          # multi-edge
    many = S.complete(300)
    expect(gm.GM_ERR_GRAPH, e.load_graph, many.row_ptr, many.col, np.arange(300))  # > 255 labels
    e.load_graph(many.row_ptr, many.col, np.arange(300) % 255)                  # 255 labels fine
    e2 = gm.Engine(device=-1, skip_symmetry_check=True)
    e2.load_graph(np.array([0, 1, 1]), np.array([1]), np.zeros(2))              # trusted input
    e2.close()
    empty = wl.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    e.load(empty)


def test_query_and_order_checks(host_engine):
    e = host_engine
    expect(gm.GM_ERR_QUERY, e.load_query, 0, [], [])
    expect(gm.GM_ERR_QUERY, e.load_query, 33, [(i, i + 1) for i in range(32)], [0] * 33)
    expect(gm.GM_ERR_QUERY, e.load_query, 3, [(0, 1)], [0, 0, 0])               # disconnected
    expect(gm.GM_ERR_QUERY, e.load_query, 2, [(0, 1), (1, 0)], [0, 0])          # duplicate
    expect(gm.GM_ERR_QUERY, e.load_query, 2, [(0, 0)], [0, 0])                  # self-loop
    expect(gm.GM_ERR_QUERY, e.load_query, 2, [(0, 2)], [0, 0])                  # out of range
    q32 = e.load_query(32, [(i, i + 1) for i in range(31)], [0] * 32)
    assert sorted(e.get_order(q32)) == list(range(32))
    qid = e.load_query(3, [(0, 1), (1, 2)], [0, 0, 0])
    expect(gm.GM_ERR_ORDER, e.set_order, qid, [0, 2, 1])                        # not connected
    expect(gm.GM_ERR_ORDER, e.set_order, qid, [0, 1, 1])                        # not a permutation
    e.set_order(qid, [2, 1, 0])
    assert list(e.get_order(qid)) == [2, 1, 0]
    e.set_order(qid, None)
    assert list(e.get_order(qid)) == [1, 0, 2]
    e.free_query(qid)
    expect(gm.GM_ERR_STATE, e.get_order, qid)
    expect(gm.GM_ERR_STATE, e.count, 1234)


def test_heuristic_order_agrees_with_independent_oracle_copy(host_engine):
    """The library and the oracle implement RI's rule separately; they must agree."""
    e = host_engine
    rng = np.random.default_rng(77)
    for trial in range(300):
        k = int(rng.integers(1, 33))
        q = S.random_connected_query(k, rng, extra_p=float(rng.uniform(0, 0.5)))
        qid = e.add(q)
        assert list(e.get_order(qid)) == list(oracle.ri_order(q.k, q.edges)), trial


def test_host_engine_refuses_to_search(host_engine):
    e = host_engine
    qid = e.add(S.path_q(2))
    expect(gm.GM_ERR_STATE, e.count, qid)                                       # no graph yet
    e.load(S.complete(4))
    expect(gm.GM_ERR_DEVICE, e.count, qid)
    expect(gm.GM_ERR_DEVICE, e.enumerate, qid, 10)
    expect(gm.GM_ERR_DEVICE, e.count_batch, [qid, qid])
    expect(gm.GM_ERR_STATE, e.count_batch, [qid, 999])
    expect(gm.GM_ERR_DEVICE, e.tune_batch, [qid])
    expect(gm.GM_ERR_DEVICE, e.serve)                                           # no GPU: no server
    expect(gm.GM_ERR_ARG, e.serve, 99)                                          # slots out of range
    res, info = e.count_batch([])                                                # empty batch: nothing to do
    assert res == [] and info.launches == 0
    o = e.options()
    assert (o.stack_layout, o.batch_single_launch) == (0, 0)


def test_bad_options():
    with pytest.raises(gm.GmError) as ei:
        gm.Engine(device=-1, stack_layout=7)
    assert ei.value.status == gm.GM_ERR_ARG
    opt = gm.Options()
    opt.batch_single_launch = 2
    h = ctypes.c_void_p()
    assert gm.load_library().gm_create(-1, ctypes.byref(opt), ctypes.byref(h)) == gm.GM_ERR_ARG
    with pytest.raises(gm.GmError) as ei:
        gm.Engine(device=-2)
    assert ei.value.status == gm.GM_ERR_ARG
    # the candidate graph runs on the two-phase pool with the slim stack only
    for bad in (dict(tau=1000), dict(tau=-1), dict(stack_layout=1)):
        with pytest.raises(gm.GmError) as ei:
            gm.Engine(device=-1, candidate_graph=True, **bad)
        assert ei.value.status == gm.GM_ERR_ARG, bad
    for bad in (dict(hub_bitmap_mib=-1), dict(pool_roots_per_item=-1), dict(pool_roots_per_item=65)):
        with pytest.raises(gm.GmError) as ei:
            gm.Engine(device=-1, **bad)
        assert ei.value.status == gm.GM_ERR_ARG, bad
    opt = gm.Options()
    opt.candidate_graph = 2
    assert gm.load_library().gm_create(-1, ctypes.byref(opt), ctypes.byref(h)) == gm.GM_ERR_ARG


def test_candidate_graph_host_checks():
    with gm.Engine(device=-1, candidate_graph=True) as e:
        qid = e.add(S.path_q(3))
        expect(gm.GM_ERR_STATE, e.candidate_sets, qid)                              # no graph yet
        e.load(S.complete(5))
        expect(gm.GM_ERR_DEVICE, e.candidate_sets, qid)
        expect(gm.GM_ERR_STATE, e.count_batch, [qid])                               # built per query
        expect(gm.GM_ERR_STATE, e.tune_batch, [qid])
        expect(gm.GM_ERR_DEVICE, e.count, qid)
        assert e.options().candidate_graph == 1
