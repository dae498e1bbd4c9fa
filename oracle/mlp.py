"""CPU reference of the order cost model -- test infrastructure only.

Only tests/ may import this module; the engine never calls it.

The model is a perceptron with two hidden relu layers and one output,
y = relu(relu(x W1 + b1) W2 + b2) w3 + b3, trained on the mean squared error
with Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015,
Algorithm 1).  Arithmetic is float64.  Where the GPU rounds a value to bf16
before a product (inputs, weights, activations, output gradients), this
reference rounds the same value the same way -- float32 first, then to the
nearest bf16 with ties to even -- so the two sides differ only by summation
order and float32 accumulation.  `exact=True` turns every rounding off (the
plain mathematics, used by the finite-difference pin).

Pins (tests/test_oracle_mlp.py): bf16 rounding of known values, a forward pass
worked out by hand, analytic gradients against central finite differences, and
one Adam step against the update written out for a scalar.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def bf16(a) -> np.ndarray:
    """Round to float32, then to the nearest bfloat16 (ties to even); returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(a, exact: bool) -> np.ndarray:
    return np.asarray(a, dtype=np.float64) if exact else bf16(a)


def forward(p: Dict[str, np.ndarray], x, exact: bool = False) -> Dict[str, np.ndarray]:
    """Activations of the rows of x; p holds w1 (in x hidden), b1, w2, b2, w3 (hidden), b3."""
    xb = _r(x, exact)
    z1 = xb @ _r(p["w1"], exact) + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1b = _r(h1, exact)
    z2 = h1b @ _r(p["w2"], exact) + p["b2"]
    h2 = np.maximum(z2, 0.0)
    h2b = _r(h2, exact)
    y = h2b @ _r(p["w3"], exact) + p["b3"][0]
    return {"xb": xb, "h1": h1, "h1b": h1b, "h2": h2, "h2b": h2b, "y": y}


def loss(p, x, t, exact: bool = False) -> float:
    y = forward(p, x, exact)["y"]
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grads(p, x, t, exact: bool = False) -> Dict[str, np.ndarray]:
    """Gradients of the mean squared error over the rows of x (backpropagation)."""
    a = forward(p, x, exact)
    n = x.shape[0]
    dy = 2.0 * (a["y"] - np.asarray(t, dtype=np.float64)) / n          # dL/dy per row
    dyb = _r(dy, exact)
    g = {"w3": a["h2b"].T @ dyb, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dyb, _r(p["w3"], exact)) * (a["h2"] > 0)
    dh2b = _r(dh2, exact)
    g["w2"] = a["h1b"].T @ dh2b
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2b @ _r(p["w2"], exact).T) * (a["h1"] > 0)
    g["w1"] = a["xb"].T @ _r(dh1, exact)
    g["b1"] = dh1.sum(axis=0)
    return g


def adam_step(p, g, state, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update of every parameter in place; state holds m, v per name and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for name, grad in g.items():
        m = state.setdefault("m_" + name, np.zeros_like(grad))
        v = state.setdefault("v_" + name, np.zeros_like(grad))
        m[...] = b1 * m + (1 - b1) * grad
        v[...] = b2 * v + (1 - b2) * grad * grad
        mhat = m / (1 - b1 ** t)
        vhat = v / (1 - b2 ** t)
        p[name] = p[name] - lr * mhat / (np.sqrt(vhat) + eps)
