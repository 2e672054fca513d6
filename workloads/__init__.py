"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module draws graphs, edge weights, QAOA angles and serving traces.  It
holds none of the simulation method's arithmetic (no cut values, phases,
mixers or expectations): it only produces the problem instances both sides
are fed.  Everything is deterministic from an integer seed through a
splitmix64 stream (Steele, Lea and Flood 2014; Vigna's public-domain
reference), so the same seed gives the same instance on every machine.

Graph families follow the workloads named for the max-cut QAOA study:
random 3-regular graphs (configuration / pairing model), Erdos-Renyi
G(n, p), and complete graphs, each optionally weighted with U[0, 1) weights.
Edges are returned canonicalised (u < v) and sorted lexicographically, which
is the upper-triangular ``graph``/``w`` encoding of the paper's Table 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 generator; ``u01`` uses the top 53 bits."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def u01(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by rejection (no modulo bias)."""
        if m <= 0:
            raise ValueError("m must be positive")
        limit = (1 << 64) - ((1 << 64) % m)
        while True:
            x = self.next_u64()
            if x < limit:
                return x % m

    def shuffle(self, a: list) -> None:
        """In-place Fisher-Yates shuffle."""
        for i in range(len(a) - 1, 0, -1):
            j = self.below(i + 1)
            a[i], a[j] = a[j], a[i]


def derive_seed(*parts: int) -> int:
    """Combine integers into one 64-bit seed (splitmix64 finaliser chain)."""
    s = 0x243F6A8885A308D3
    for p in parts:
        r = SplitMix64(s ^ (p & MASK64))
        s = r.next_u64()
    return s


def _canon(edges: Sequence[Tuple[int, int]]) -> np.ndarray:
    e = sorted((min(u, v), max(u, v)) for u, v in edges)
    return np.asarray(e, dtype=np.int32).reshape(-1, 2)


def random_regular(n: int, d: int, rng: SplitMix64, max_tries: int = 100000) -> np.ndarray:
    """Simple d-regular graph from the pairing (configuration) model.

    n*d stubs are shuffled and paired consecutively; a draw with a self-loop
    or a repeated pair is discarded and redrawn from the same stream.
    """
    if (n * d) % 2 != 0 or d >= n:
        raise ValueError(f"no simple {d}-regular graph on {n} vertices")
    for _ in range(max_tries):
        stubs = [v for v in range(n) for _ in range(d)]
        rng.shuffle(stubs)
        seen = set()
        ok = True
        for k in range(0, len(stubs), 2):
            u, v = stubs[k], stubs[k + 1]
            if u == v:
                ok = False
                break
            key = (min(u, v), max(u, v))
            if key in seen:
                ok = False
                break
            seen.add(key)
        if ok:
            return _canon(list(seen))
    raise RuntimeError("pairing model did not produce a simple graph")


def gnp(n: int, prob: float, rng: SplitMix64) -> np.ndarray:
    """Erdos-Renyi G(n, p): pairs u < v in lexicographic order, kept if u01 < p."""
    out = []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.u01() < prob:
                out.append((u, v))
    return _canon(out)


def complete(n: int) -> np.ndarray:
    return _canon([(u, v) for u in range(n) for v in range(u + 1, n)])


def uniform_weights(num_edges: int, rng: SplitMix64) -> np.ndarray:
    """One U[0, 1) weight per canonical edge, in edge order."""
    return np.asarray([rng.u01() for _ in range(num_edges)], dtype=np.float64)


def uniform_angles(p: int, rng: SplitMix64, lo: float = 0.0, hi: float = math.pi):
    """p draws for gamma, then p for beta, each uniform in [lo, hi)."""
    g = np.asarray([lo + (hi - lo) * rng.u01() for _ in range(p)], dtype=np.float64)
    b = np.asarray([lo + (hi - lo) * rng.u01() for _ in range(p)], dtype=np.float64)
    return g, b


@dataclass
class Problem:
    """One max-cut QAOA instance: n vertices/qubits, canonical edges, weights."""
    n: int
    edges: np.ndarray                 # (m, 2) int32, u < v, sorted
    weights: Optional[np.ndarray]     # (m,) float64 or None for unweighted
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def total_weight(self) -> float:
        if self.weights is None:
            return float(self.num_edges)
        return float(np.sum(self.weights))


# ---------------------------------------------------------------------------
# The five workloads (seeds 1..5).  Each returns the problem plus angles.
# ---------------------------------------------------------------------------

def plain_n12(seed: int = 1):
    """n=12 unweighted random 3-regular graph (18 edges), p=1, gamma=0.6, beta=0.4."""
    rng = SplitMix64(seed)
    e = random_regular(12, 3, rng)
    prob = Problem(12, e, None, "3reg12")
    return prob, np.array([0.6]), np.array([0.4])


def gnp_n26(seed: int = 2, n: int = 26, p: int = 4):
    """G(26, 0.5) unweighted, p=4, angles uniform in [0, pi)."""
    rng = SplitMix64(seed)
    e = gnp(n, 0.5, rng)
    g, b = uniform_angles(p, rng)
    return Problem(n, e, None, f"gnp{n}_0.5"), g, b


def weighted_3reg_n30(seed: int = 3, n: int = 30, p: int = 10):
    """Random 3-regular graph with U[0,1) FP64 edge weights, p=10, angles U[0, pi)."""
    rng = SplitMix64(seed)
    e = random_regular(n, 3, rng)
    w = uniform_weights(e.shape[0], rng)
    g, b = uniform_angles(p, rng)
    return Problem(n, e, w, f"w3reg{n}"), g, b


def grad_gnp_n24(seed: int = 4, n: int = 24, p: int = 8, sets: int = 64):
    """G(24, 0.3) unweighted, p=8, `sets` random parameter sets U[0, pi)."""
    rng = SplitMix64(seed)
    e = gnp(n, 0.3, rng)
    params = [uniform_angles(p, rng) for _ in range(sets)]
    return Problem(n, e, None, f"gnp{n}_0.3"), params


@dataclass
class Request:
    idx: int
    arrival: float
    problem: Problem
    gamma: np.ndarray
    beta: np.ndarray
    want_grad: bool
    family: str


def serving_trace(num: int = 2048, seed: int = 5, rate: float = 1000.0,
                  n_lo: int = 14, n_hi: int = 28, p_lo: int = 1, p_hi: int = 12,
                  grad_frac: float = 0.3) -> List[Request]:
    """Poisson arrivals of mixed max-cut QAOA requests.

    Family is uniform over {3-regular, G(n, 0.3), complete}; n uniform in
    [n_lo, n_hi] (even values only for 3-regular, since n*3 must be even);
    edge weights U[0, 1); p uniform in [p_lo, p_hi]; a request wants the
    gradient with probability ``grad_frac``.  ``rate`` is arrivals per second.
    """
    top = SplitMix64(seed)
    t = 0.0
    out = []
    for i in range(num):
        t += -math.log(1.0 - top.u01()) / rate
        rng = SplitMix64(derive_seed(seed, i))
        fam = ("3reg", "gnp", "complete")[rng.below(3)]
        if fam == "3reg":
            lo = n_lo + (n_lo & 1)
            n = lo + 2 * rng.below((n_hi - lo) // 2 + 1)
            e = random_regular(n, 3, rng)
        else:
            n = n_lo + rng.below(n_hi - n_lo + 1)
            e = gnp(n, 0.3, rng) if fam == "gnp" else complete(n)
        w = uniform_weights(e.shape[0], rng)
        p = p_lo + rng.below(p_hi - p_lo + 1)
        g, b = uniform_angles(p, rng)
        want = rng.u01() < grad_frac
        out.append(Request(i, t, Problem(n, e, w, f"{fam}{n}"), g, b, want, fam))
    return out


def random_problem(n: int, rng: SplitMix64, kind: str = "gnp", weighted: bool = False,
                   prob: float = 0.5) -> Problem:
    """Small helper for tests: one random instance of the given family."""
    if kind == "3reg":
        e = random_regular(n, 3, rng)
    elif kind == "complete":
        e = complete(n)
    else:
        e = gnp(n, prob, rng)
    w = uniform_weights(e.shape[0], rng) if weighted else None
    return Problem(n, e, w, f"{kind}{n}")
