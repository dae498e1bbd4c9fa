"""The order cost model on the GPU (bf16 MFMA products, fp32 accumulation)
against the float64 reference in oracle/mlp.py, which rounds the same values
to bf16 at the same points.

Tolerances, from the arithmetic: the two sides differ by summation order and
float32 accumulation (relative error about K * 2^-24, K <= 192 terms, i.e.
~1e-5) and, rarely, by an activation that falls on the other side of a bf16
rounding boundary because of that (a change of 2^-8 relative in one hidden
unit).  So predictions must agree to 2e-2 * (1 + |y|) everywhere and to 1e-3 *
(1 + |y|) for at least 99 % of rows."""
import numpy as np
import pytest

import oracle
import paper_2604_10601_amd as gm
from oracle import mlp
from paper_2604_10601_amd import workloads as wl
from tests import shapes as S

pytestmark = pytest.mark.gpu

D, H = gm.ORDER_FEATURES, 128


def params(rng, scale=0.15):
    return {"w1": rng.normal(size=(D, H)) * scale, "b1": rng.normal(size=H) * 0.05,
            "w2": rng.normal(size=(H, H)) * scale, "b2": rng.normal(size=H) * 0.05,
            "w3": rng.normal(size=H) * scale, "b3": np.array([0.3])}


def load(model, p):
    model.set_params(p["w1"], p["b1"], p["w2"], p["b2"], p["w3"], p["b3"])


def test_predict_matches_reference():
    rng = np.random.default_rng(41)
    p = params(rng)
    x = rng.uniform(0, 1, size=(300, D))
    with gm.Model(D, H, seed=1) as m:
        load(m, p)
        got = m.predict(x)
        back = m.get_params()
    want = mlp.forward(p, x)["y"]
    err = np.abs(got - want) / (1 + np.abs(want))
    assert err.max() <= 2e-2, err.max()
    assert np.mean(err <= 1e-3) >= 0.99
    assert np.array_equal(back[0], p["w1"].astype(np.float32))  # master weights kept exactly


def test_two_adam_steps_match_reference():
    """One batch of 64 rows, two epochs: two Adam steps on the same rows (row
    order inside a batch does not change the gradient).  Compared: the updates
    w_after - w_before, which depend on the gradients' magnitudes from the
    second step on.  An entry may differ by more than 5 % of lr only where a
    gradient is near zero (its sign can differ); at most 1 % of entries."""
    rng = np.random.default_rng(42)
    p = params(rng)
    x = rng.uniform(0, 1, size=(64, D))
    t = rng.normal(size=64)
    lr = 1e-3
    with gm.Model(D, H, seed=1) as m:
        load(m, p)
        m.train(x, t, epochs=2, batch=64, lr=lr, seed=5)
        got = dict(zip(("w1", "b1", "w2", "b2", "w3", "b3"), m.get_params()))
    ref = {k: v.copy() for k, v in p.items()}
    state = {}
    for _ in range(2):
        mlp.adam_step(ref, mlp.grads(ref, x, t), state, lr=lr)
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        du_dev = got[name].astype(np.float64) - p[name].astype(np.float32).astype(np.float64)
        du_ref = ref[name] - p[name]
        off = np.abs(du_dev - du_ref) > 0.05 * lr
        assert off.mean() <= 0.01, (name, off.mean())


def test_training_fits_a_learnable_target():
    rng = np.random.default_rng(43)
    x = rng.uniform(0, 1, size=(4096, D)).astype(np.float32)
    v = rng.normal(size=D) / np.sqrt(D)
    t = (np.maximum(x @ v, 0) + 0.5 * np.sin(3 * x[:, 0])).astype(np.float32)
    var = float(np.var(t))
    with gm.Model(D, H, seed=2) as m:
        first = m.train(x, t, epochs=1, batch=256, lr=1e-3, seed=1)
        last = m.train(x, t, epochs=40, batch=256, lr=1e-3, seed=2)
        pred = m.predict(x[:512])
    # a constant predictor scores var; the fit must explain most of it
    assert last < 0.25 * var and last < first, (first, last, var)
    assert np.mean((pred - t[:512]) ** 2) < 0.3 * var


def test_chosen_orders_keep_counts():
    """Whatever order the model picks, counts equal the oracle's (every
    connected order gives the same matches)."""
    rp, col = wl.erdos_renyi(3000, 15000, seed=4401)
    g = wl.Graph(rp, col, wl.uniform_labels(3000, 6, seed=4402))
    qs = wl.extract_queries_any(g, 8, 6, seed=4403) + wl.extract_queries_any(g, 12, 4, seed=4404)
    rng = np.random.default_rng(44)
    with gm.Engine(device=0) as e, gm.Model(D, H, seed=3) as m:
        e.load(g)
        load(m, params(rng, scale=0.3))
        for i, q in enumerate(qs):
            qid = e.add(q)
            chosen, pred = e.choose_order(m, qid, max_orders=6, seed=i, margin=-10.0)  # always take the argmin
            cands = e.candidate_orders(qid, max_orders=6, seed=i)
            assert list(e.get_order(qid)) == list(cands[chosen])
            assert chosen == int(np.argmin(pred[:len(cands)]))
            r = e.count(qid)
            o = oracle.count(g, q)
            assert (r.count, r.outcome) == (o.count, o.outcome), i
        qid = e.add(qs[0])
        chosen, _ = e.choose_order(m, qid, max_orders=6, seed=0, margin=100.0)  # never beaten by 100
        assert chosen == 0 and list(e.get_order(qid)) == list(oracle.ri_order(qs[0].k, qs[0].edges))


def test_splits_keep_counts_and_the_model_picks_plans():
    """The task split changes how the pool is cut into work items, never the
    matches or the paper's work counters; the plan the model picks (order and
    split) is the one applied, and its counts equal the oracle's."""
    rp, col = wl.rmat(13, 16, seed=4501)
    g = wl.Graph(rp, col, wl.zipf_labels(1 << 13, 12, 0.5, seed=4502))
    qs = wl.extract_queries_any(g, 4, 3, seed=4503) + wl.extract_queries_any(g, 6, 3, seed=4504)
    rng = np.random.default_rng(45)
    splits = (8, 16, 32, 64)
    with gm.Engine(device=0) as e, gm.Model(D, H, seed=4) as m:
        e.load(g)
        load(m, params(rng, scale=0.3))
        for i, q in enumerate(qs):
            qid = e.add(q)
            o = oracle.count(g, q, order=e.get_order(qid), cap=2_000_000)
            for sp in (1, 8, 64, 5000):
                e.set_split(qid, sp)
                r = e.count(qid, cap=2_000_000)
                assert (r.count, r.outcome) == (o.count, o.outcome), (i, sp)
                if r.outcome == gm.GM_DONE:
                    assert (r.groups, r.tasks) == (o.groups, o.tasks), (i, sp)
            e.set_split(qid, 0)
            co, cs, pred, _ = e.choose_plan(m, qid, splits=splits, max_orders=4, seed=i, margin=-10.0)
            cands = e.candidate_orders(qid, max_orders=4, seed=i)
            assert list(e.get_order(qid)) == list(cands[co]) and e.get_split(qid) == cs
            n = 1 + len(cands) * len(splits)
            assert np.isfinite(pred[:n]).all()
            r = e.count(qid, cap=2_000_000)
            assert (r.count, r.outcome) == (o.count, o.outcome), i
        qid = e.add(qs[0])
        co, cs, _, probe = e.choose_plan(m, qid, splits=splits, max_orders=4, seed=0, margin=100.0, probe_cap=1000)
        assert (co, cs) == (0, 1) and e.get_split(qid) == 1 and probe == 0.0   # nothing to judge
        # a proposal judged by measured runtime: whichever plan stays, counts are the oracle's
        for i, q in enumerate(qs):
            qid = e.add(q)
            co, cs, _, probe = e.choose_plan(m, qid, splits=splits, max_orders=4, seed=i, margin=-10.0,
                                             probe_cap=10_000, probe_limit_s=1.0)
            assert probe >= 0.0 and e.get_split(qid) in (1, cs)
            o = oracle.count(g, q, order=e.get_order(qid), cap=2_000_000)
            r = e.count(qid, cap=2_000_000)
            assert (r.count, r.outcome) == (o.count, o.outcome), i
