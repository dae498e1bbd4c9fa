"""Pins of the CPU reference of the order cost model (oracle/mlp.py)."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_known_values():
    vals = {1.0: 1.0, 1 / 3: 0.333984375, -2.5: -2.5,
            1 + 2 ** -8: 1.0,                    # halfway: ties to even (1.0)
            1 + 3 * 2 ** -8: 1 + 2 ** -6,        # halfway: ties to even (1.015625)
            1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7,  # just above halfway: up
            0.0: 0.0}
    for x, want in vals.items():
        assert mlp.bf16(x) == want, x


def _params(d, h, rng):
    return {"w1": rng.normal(size=(d, h)) * 0.3, "b1": rng.normal(size=h) * 0.1,
            "w2": rng.normal(size=(h, h)) * 0.3, "b2": rng.normal(size=h) * 0.1,
            "w3": rng.normal(size=h) * 0.3, "b3": np.array([0.2])}


def test_forward_worked_by_hand():
    d = h = 4
    p = {"w1": np.eye(d), "b1": np.zeros(h), "w2": np.eye(h), "b2": np.array([0.0, 0.0, 0.0, -1.0]),
         "w3": np.array([1.0, 2.0, 0.0, 1.0]), "b3": np.array([0.5])}
    x = np.array([[1.0, -2.0, 3.0, 4.0], [0.5, 0.25, -1.0, 0.75]])
    # h1 = relu(x); h2 = relu(h1 + b2); y = h2 . w3 + 0.5
    # row 0: h1 = (1, 0, 3, 4), h2 = (1, 0, 3, 3), y = 1 + 0 + 0 + 3 + 0.5
    # row 1: h1 = (0.5, 0.25, 0, 0.75), h2 = (0.5, 0.25, 0, 0), y = 0.5 + 0.5 + 0.5
    y = mlp.forward(p, x)["y"]
    assert np.array_equal(y, [4.5, 1.5])


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(5)
    d, h, n = 6, 5, 7
    p = _params(d, h, rng)
    x = rng.normal(size=(n, d))
    t = rng.normal(size=n)
    g = mlp.grads(p, x, t, exact=True)
    eps = 1e-6
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        for idx in list(np.ndindex(p[name].shape))[:12]:
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += eps
            up = mlp.loss(q, x, t, exact=True)
            q[name][idx] -= 2 * eps
            down = mlp.loss(q, x, t, exact=True)
            num = (up - down) / (2 * eps)
            assert abs(num - g[name][idx]) <= 1e-6 * max(1.0, abs(num)), (name, idx, num, g[name][idx])


def test_adam_step_written_out():
    p = {"w": np.array([1.0])}
    state = {}
    mlp.adam_step(p, {"w": np.array([0.5])}, state, lr=0.1)
    # m = 0.05, v = 0.00025, mhat = 0.5, vhat = 0.25 -> w = 1 - 0.1 * 0.5 / (0.5 + 1e-8)
    assert abs(p["w"][0] - (1 - 0.1 * 0.5 / (0.5 + 1e-8))) < 1e-15
    mlp.adam_step(p, {"w": np.array([-0.25])}, state, lr=0.1)
    m = 0.9 * 0.05 + 0.1 * -0.25
    v = 0.999 * 0.00025 + 0.001 * 0.0625
    w2 = (1 - 0.1 * 0.5 / (0.5 + 1e-8)) - 0.1 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert abs(p["w"][0] - w2) < 1e-14
