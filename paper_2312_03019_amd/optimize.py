"""The classical half of the QAOA loop (Section 1, the QAOA workflow figure):
an optimizer that maximises <C>(gamma, beta) over the 2p angles, driven by
the library's adjoint gradient.

Several random starts are optimised together: every Adam step submits one
gradient request per start to the continuous-batching server, so the starts'
passes share launches on the device, and the host only does the 2p-element
Adam updates.  The result is the best start's angles, <C> and the
approximation ratio <C> / max_z C(z) (the quality measure of Section 3.4).

Adam: Kingma and Ba, "Adam: A Method for Stochastic Optimization" (2015),
used here for ascent (x += step).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class OptResult:
    expect: float
    gamma: np.ndarray
    beta: np.ndarray
    max_cut: float
    ratio: float
    steps: int
    history: list            # best <C> after each step


def adam_ascent(grad_batch, x0: np.ndarray, steps: int, lr: float = 0.05, b1: float = 0.9, b2: float = 0.999,
                eps: float = 1e-8):
    """Batched Adam ascent.  x0: (starts, dim).  grad_batch(x) -> (values (starts,), grads (starts, dim)).
    Returns the final points, their values and the best value seen after each step."""
    x = np.array(x0, dtype=np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    hist = []
    val = None
    for t in range(1, steps + 1):
        val, gr = grad_batch(x)
        hist.append(float(np.max(val)))
        m = b1 * m + (1 - b1) * gr
        v = b2 * v + (1 - b2) * gr * gr
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        x = x + lr * mh / (np.sqrt(vh) + eps)
    val, _ = grad_batch(x)
    hist.append(float(np.max(val)))
    return x, val, hist


def optimize(q, n, edges, weights, p: int, starts: int = 8, steps: int = 80, lr: float = 0.05, seed: int = 0,
             prec: str = "c64", budget_bytes: int = 64 << 30) -> OptResult:
    """Maximise <C> over (gamma, beta) in R^2p from `starts` random starts
    (gamma, beta uniform in [0, pi/2)), all starts batched through one server."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, math.pi / 2, size=(starts, 2 * p))
    srv = q.Server(budget_bytes, max_slots=max(4, starts), prec=prec)
    try:
        def grad_batch(x):
            tix = [srv.submit(n, edges, weights, xi[:p], xi[p:], want_grad=True) for xi in x]
            res = [srv.wait(t) for t in tix]
            for r in res:
                if r["status"] != 0:
                    raise q.QAOAError(r["status"], "gradient request failed")
            vals = np.array([r["expect"] for r in res])
            grads = np.array([np.concatenate([r["dgamma"], r["dbeta"]]) for r in res])
            return vals, grads

        x, val, hist = adam_ascent(grad_batch, x0, steps, lr)
    finally:
        srv.close()
    best = int(np.argmax(val))
    sim = q.Simulator(n, edges, weights, prec)
    try:
        mc, _ = sim.max_cut()
    finally:
        sim.close()
    return OptResult(float(val[best]), x[best, :p].copy(), x[best, p:].copy(), mc,
                     float(val[best]) / mc if mc > 0 else float("nan"), steps, hist)
