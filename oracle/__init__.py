"""FP64 oracle for QAOA max-cut simulation (arXiv:2312.03019).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path, and it shares no
code with the HIP library.

Two independent layers live here:

* ``liboracle.so`` (``qaoa_oracle.c``): the plain definition of the simulated
  circuit in double precision -- cut table by the per-edge loop, |+>^n start,
  per layer the diagonal cost phase exp(-i gamma C(z)) then exp(-i beta X_q)
  qubit by qubit, compensated <C>/norm, and the adjoint gradient.
* NumPy/SciPy references for tiny n that build the same circuit a different
  way: dense Pauli Kronecker products and matrix exponentials, the p = 1
  closed form for max-cut QAOA, the paper's own printed convention
  (Algorithm 2's +/- w rotation sum, RX(beta) = exp(-i beta X / 2)), and the
  light-cone reduction.  Tests use these to pin the C oracle.

Angle convention of the library and the C oracle: cost exp(-i gamma C),
mixer exp(-i beta sum_q X_q) (RX(2 beta) per qubit), qubit q = bit q of z.
"""
from __future__ import annotations

import ctypes
import math
import os
from functools import reduce
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def load(path: Optional[str] = None):
    """Load (building first if absent) the C oracle; returns the ctypes handle."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        from . import build as _b
        _b.build(p, quiet=True)
    lib = ctypes.CDLL(p)
    I, D = ctypes.c_int, ctypes.c_double
    lib.oracle_cut_table.argtypes = [I, I, _ip, _dp, _dp]
    lib.oracle_evolve.argtypes = [I, I, _ip, _dp, I, _dp, _dp, _dp]
    lib.oracle_expect.argtypes = [I, _dp, _dp, _dp, _dp]
    lib.oracle_run_expect.argtypes = [I, I, _ip, _dp, I, _dp, _dp, _dp, _dp]
    lib.oracle_grad.argtypes = [I, I, _ip, _dp, I, _dp, _dp, _dp, _dp, _dp]
    lib.oracle_fidelity.argtypes = [I, _dp, _dp, _dp]
    lib.oracle_num_threads.argtypes = []
    lib.oracle_amplitude_p1.argtypes = [I, I, _ip, _dp, D, D, ctypes.c_int64, _dp]
    for f in ("oracle_cut_table", "oracle_evolve", "oracle_expect", "oracle_run_expect",
              "oracle_grad", "oracle_fidelity", "oracle_num_threads", "oracle_amplitude_p1"):
        getattr(lib, f).restype = I
    if path is None:
        _lib = lib
    return lib


def _edges_ptr(edges):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    return e, e.ctypes.data_as(_ip), int(e.shape[0])


def _w_ptr(weights):
    if weights is None:
        return None, None
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    return w, w.ctypes.data_as(_dp)


def _arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    return a, a.ctypes.data_as(_dp)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


# ---------------------------------------------------------------------------
# C oracle wrappers
# ---------------------------------------------------------------------------

def cut_table(n, edges, weights=None, lib=None) -> np.ndarray:
    """C(z) for every z (float64; exact integers when unweighted)."""
    lib = lib or load()
    e, ep, m = _edges_ptr(edges)
    w, wp = _w_ptr(weights)
    out = np.empty(1 << n, dtype=np.float64)
    _check(lib.oracle_cut_table(n, m, ep, wp, out.ctypes.data_as(_dp)), "oracle_cut_table")
    return out


def evolve(n, edges, weights, gamma, beta, lib=None) -> np.ndarray:
    """Final state psi_p as complex128."""
    lib = lib or load()
    e, ep, m = _edges_ptr(edges)
    w, wp = _w_ptr(weights)
    g, gp = _arr(gamma)
    b, bp = _arr(beta)
    psi = np.empty(2 << n, dtype=np.float64)
    _check(lib.oracle_evolve(n, m, ep, wp, len(g), gp, bp, psi.ctypes.data_as(_dp)),
           "oracle_evolve")
    return psi.view(np.complex128)


def amplitude_p1(n, edges, weights, gamma, beta, z, lib=None) -> complex:
    """One amplitude psi_z of the depth-1 state, summed over the 2^n basis states
    by its definition (no state vector): at n = 30 it needs seconds, not 8 GiB."""
    lib = lib or load()
    e, ep, m = _edges_ptr(edges)
    w, wp = _w_ptr(weights)
    out = np.empty(2, dtype=np.float64)
    _check(lib.oracle_amplitude_p1(n, m, ep, wp, float(gamma), float(beta), int(z), out.ctypes.data_as(_dp)),
           "oracle_amplitude_p1")
    return complex(out[0], out[1])


def expect_of_state(n, psi, cut) -> Tuple[float, float]:
    lib = load()
    s = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    c = np.ascontiguousarray(np.asarray(cut, dtype=np.float64))
    e, nrm = ctypes.c_double(), ctypes.c_double()
    _check(lib.oracle_expect(n, s.ctypes.data_as(_dp), c.ctypes.data_as(_dp),
                             ctypes.byref(e), ctypes.byref(nrm)), "oracle_expect")
    return e.value, nrm.value


def run_expect(n, edges, weights, gamma, beta, lib=None) -> Tuple[float, float]:
    """(<C>, norm) after p layers from |+>^n."""
    lib = lib or load()
    e, ep, m = _edges_ptr(edges)
    w, wp = _w_ptr(weights)
    g, gp = _arr(gamma)
    b, bp = _arr(beta)
    ex, nrm = ctypes.c_double(), ctypes.c_double()
    _check(lib.oracle_run_expect(n, m, ep, wp, len(g), gp, bp, ctypes.byref(ex),
                                 ctypes.byref(nrm)), "oracle_run_expect")
    return ex.value, nrm.value


def grad(n, edges, weights, gamma, beta, lib=None):
    """(<C>, d<C>/dgamma[p], d<C>/dbeta[p]) by the FP64 adjoint recurrence."""
    lib = lib or load()
    e, ep, m = _edges_ptr(edges)
    w, wp = _w_ptr(weights)
    g, gp = _arr(gamma)
    b, bp = _arr(beta)
    p = len(g)
    dg = np.zeros(max(p, 1))
    db = np.zeros(max(p, 1))
    ex = ctypes.c_double()
    _check(lib.oracle_grad(n, m, ep, wp, p, gp, bp, ctypes.byref(ex),
                           dg.ctypes.data_as(_dp), db.ctypes.data_as(_dp)), "oracle_grad")
    return ex.value, dg[:p], db[:p]


def grad_fd(n, edges, weights, gamma, beta, h=1e-6, lib=None):
    """Central finite differences of <C> (FP64), step h, for every parameter."""
    g = np.asarray(gamma, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    dg, db = np.zeros_like(g), np.zeros_like(b)
    for l in range(len(g)):
        gp, gm = g.copy(), g.copy()
        gp[l] += h
        gm[l] -= h
        dg[l] = (run_expect(n, edges, weights, gp, b, lib)[0]
                 - run_expect(n, edges, weights, gm, b, lib)[0]) / (2 * h)
        bp_, bm = b.copy(), b.copy()
        bp_[l] += h
        bm[l] -= h
        db[l] = (run_expect(n, edges, weights, g, bp_, lib)[0]
                 - run_expect(n, edges, weights, g, bm, lib)[0]) / (2 * h)
    return dg, db


def fidelity(n, a, b) -> float:
    lib = load()
    x = np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)
    y = np.ascontiguousarray(np.asarray(b, dtype=np.complex128)).view(np.float64)
    f = ctypes.c_double()
    _check(lib.oracle_fidelity(n, x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                               ctypes.byref(f)), "oracle_fidelity")
    return f.value


def sample_cdf(psi) -> np.ndarray:
    """CDF(z) = sum_{y <= z} |psi_y|^2 over the natural index order, FP64, added
    left to right."""
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    return np.cumsum(p)


def sample(psi, uniforms) -> np.ndarray:
    """Measurement of the final state in the computational basis (the bitstrings
    a QAOA run hands to the classical side, Section 1's workflow), by inverse
    CDF: sample k is the smallest z with CDF(z) > u_k * CDF(N-1); the uniforms
    u_k in [0, 1) are inputs."""
    c = sample_cdf(psi)
    t = np.asarray(uniforms, dtype=np.float64) * c[-1]
    z = np.searchsorted(c, t, side="right")
    return np.minimum(z, len(c) - 1).astype(np.uint64)


def num_threads() -> int:
    return int(load().oracle_num_threads())


# ---------------------------------------------------------------------------
# Independent NumPy/SciPy references (tiny n)
# ---------------------------------------------------------------------------

_I2 = np.eye(2)
_X = np.array([[0.0, 1.0], [1.0, 0.0]])
_Zd = np.array([1.0, -1.0])


def _kron_diag_z(n, q):
    """Diagonal of Z_q; the Kronecker factor for qubit 0 is the rightmost."""
    facs = [(_Zd if k == q else np.ones(2)) for k in reversed(range(n))]
    return reduce(np.kron, facs)


def _kron_x(n, q):
    facs = [(_X if k == q else _I2) for k in reversed(range(n))]
    return reduce(np.kron, facs)


def dense_cost_diag(n, edges, weights=None) -> np.ndarray:
    """Diagonal of C = sum_e w_e (I - Z_u Z_v)/2 from Pauli Kronecker products."""
    d = np.zeros(1 << n)
    for k, (u, v) in enumerate(np.asarray(edges).reshape(-1, 2)):
        w = 1.0 if weights is None else float(weights[k])
        d += w * 0.5 * (1.0 - _kron_diag_z(n, int(u)) * _kron_diag_z(n, int(v)))
    return d


def dense_mixer(n) -> np.ndarray:
    """B = sum_q X_q as a dense real symmetric matrix (n <= 10)."""
    return sum(_kron_x(n, q) for q in range(n))


def dense_evolve(n, edges, weights, gamma, beta) -> np.ndarray:
    """psi_p via full matrix exponentials: H^n|0>, then diag(e^{-i g C}), e^{-i b B}."""
    import scipy.linalg as sla
    had = np.array([[1.0, 1.0], [1.0, -1.0]]) / math.sqrt(2.0)
    e0 = np.zeros(1 << n, dtype=np.complex128)
    e0[0] = 1.0
    psi = reduce(np.kron, [had] * n) @ e0
    cd = dense_cost_diag(n, edges, weights)
    B = dense_mixer(n)
    for g, b in zip(gamma, beta):
        psi = np.exp(-1j * g * cd) * psi
        psi = sla.expm(-1j * b * B) @ psi
    return psi


def dense_expect(n, edges, weights, gamma, beta) -> float:
    psi = dense_evolve(n, edges, weights, gamma, beta)
    cd = dense_cost_diag(n, edges, weights)
    return float(np.real(np.vdot(psi, cd * psi)))


def _neighbours(n, edges, weights):
    nb = [dict() for _ in range(n)]
    for k, (u, v) in enumerate(np.asarray(edges).reshape(-1, 2)):
        w = 1.0 if weights is None else float(weights[k])
        nb[int(u)][int(v)] = w
        nb[int(v)][int(u)] = w
    return nb


def closed_form_p1(n, edges, weights, gamma, beta) -> float:
    """<C> at p = 1 for any (weighted) graph, edge by edge.

    For edge (u, v) with weight w: let A = N(u)\\{v}, Bv = N(v)\\{u}, T = A & Bv.
    <Z_u Z_v> = -1/2 sin(4b) sin(g w) [prod_{k in A} cos(g w_uk) + prod_{k in Bv} cos(g w_vk)]
                + 1/2 sin^2(2b) prod_{A\\T} cos(g w_uk) prod_{Bv\\T} cos(g w_vk)
                  * [prod_T cos(g (w_uk - w_vk)) - prod_T cos(g (w_uk + w_vk))]
    and <C> = sum_e w_e (1 - <Z_u Z_v>) / 2.  (Unweighted form: Wang, Hadfield,
    Jiang and Rieffel, Phys. Rev. A 97, 022304 (2018).)
    """
    g, b = float(gamma), float(beta)
    nb = _neighbours(n, edges, weights)
    tot = 0.0
    for k, (u, v) in enumerate(np.asarray(edges).reshape(-1, 2)):
        u, v = int(u), int(v)
        w = 1.0 if weights is None else float(weights[k])
        A = set(nb[u]) - {v}
        Bv = set(nb[v]) - {u}
        T = A & Bv
        pa = np.prod([math.cos(g * nb[u][x]) for x in A]) if A else 1.0
        pb = np.prod([math.cos(g * nb[v][x]) for x in Bv]) if Bv else 1.0
        qa = np.prod([math.cos(g * nb[u][x]) for x in A - T]) if A - T else 1.0
        qb = np.prod([math.cos(g * nb[v][x]) for x in Bv - T]) if Bv - T else 1.0
        tm = np.prod([math.cos(g * (nb[u][x] - nb[v][x])) for x in T]) if T else 1.0
        tp = np.prod([math.cos(g * (nb[u][x] + nb[v][x])) for x in T]) if T else 1.0
        zz = (-0.5 * math.sin(4 * b) * math.sin(g * w) * (pa + pb)
              + 0.5 * math.sin(2 * b) ** 2 * qa * qb * (tm - tp))
        tot += w * (1.0 - zz) / 2.0
    return tot


def closed_form_p1_unweighted(n, edges, gamma, beta) -> float:
    """Unweighted p = 1 form: per edge 1/2 + 1/4 sin4b sin g (c^du + c^dv)
    - 1/4 sin^2 2b c^(du+dv-2t) (1 - cos^t 2g), c = cos g, d = deg - 1, t = triangles."""
    g, b = float(gamma), float(beta)
    nb = _neighbours(n, edges, None)
    c = math.cos(g)
    tot = 0.0
    for u, v in np.asarray(edges).reshape(-1, 2):
        u, v = int(u), int(v)
        du, dv = len(nb[u]) - 1, len(nb[v]) - 1
        t = len((set(nb[u]) - {v}) & (set(nb[v]) - {u}))
        tot += (0.5 + 0.25 * math.sin(4 * b) * math.sin(g) * (c ** du + c ** dv)
                - 0.25 * math.sin(2 * b) ** 2 * c ** (du + dv - 2 * t) * (1 - math.cos(2 * g) ** t))
    return tot


def paper_convention_expect(n, edges, weights, gamma, beta) -> float:
    """<C> under the paper's printed convention, Algorithm 2 taken literally.

    Cost layer: per basis state, a rotation total that adds w for an uncut
    edge and subtracts w for a cut one, then psi_b *= exp(-1/2 i gamma total)
    (Eq. UC_opt).  Mixer: RX(beta) = exp(-i beta X / 2) on every qubit.
    Tiny n only (dense mixer).
    """
    import scipy.linalg as sla
    N = 1 << n
    e = np.asarray(edges).reshape(-1, 2)
    tot = np.zeros(N)
    cutv = np.zeros(N)
    for z in range(N):
        r = 0.0
        c = 0.0
        for k, (i, j) in enumerate(e):
            w = 1.0 if weights is None else float(weights[k])
            if ((z >> int(i)) & 1) ^ ((z >> int(j)) & 1):
                r -= w
                c += w
            else:
                r += w
        tot[z] = r
        cutv[z] = c
    psi = np.full(N, 2.0 ** (-n / 2), dtype=np.complex128)
    B = dense_mixer(n)
    for g, b in zip(gamma, beta):
        psi = psi * np.exp(-0.5j * g * tot)
        psi = sla.expm(-0.5j * b * B) @ psi
    return float(np.real(np.vdot(psi, cutv * psi)))


def brute_max_cut(n, edges, weights=None) -> float:
    """Best cut by enumerating every bipartition with explicit vertex sets."""
    e = np.asarray(edges).reshape(-1, 2)
    best = 0.0
    for z in range(1 << (n - 1)):          # fix vertex n-1 on side 0 (C(z) = C(~z))
        side = [(z >> v) & 1 for v in range(n)]
        val = 0.0
        for k, (u, v) in enumerate(e):
            if side[int(u)] != side[int(v)]:
                val += 1.0 if weights is None else float(weights[k])
        best = max(best, val)
    return best


def light_cone_expect(n, edges, weights, gamma, beta, sub_expect) -> float:
    """<C> = sum_e w_e (1 - <Z_u Z_v>)/2 with each <Z_u Z_v> from the subgraph
    induced by the vertices within distance p of {u, v}.

    ``sub_expect(ns, sub_edges, sub_weights, gamma, beta, a, b)`` must return
    <Z_a Z_b> on the relabelled subgraph.
    """
    p = len(gamma)
    e = np.asarray(edges).reshape(-1, 2)
    adj = [[] for _ in range(n)]
    for u, v in e:
        adj[int(u)].append(int(v))
        adj[int(v)].append(int(u))
    tot = 0.0
    for k, (u, v) in enumerate(e):
        u, v = int(u), int(v)
        dist = {u: 0, v: 0}
        frontier = [u, v]
        for d in range(p):
            nxt = []
            for x in frontier:
                for y in adj[x]:
                    if y not in dist:
                        dist[y] = d + 1
                        nxt.append(y)
            frontier = nxt
        verts = sorted(dist)
        lab = {x: i for i, x in enumerate(verts)}
        se, sw = [], []
        for kk, (a, b) in enumerate(e):
            a, b = int(a), int(b)
            if a in lab and b in lab:
                se.append((lab[a], lab[b]))
                sw.append(1.0 if weights is None else float(weights[kk]))
        zz = sub_expect(len(verts), np.asarray(se, dtype=np.int32), np.asarray(sw),
                        gamma, beta, lab[u], lab[v])
        w = 1.0 if weights is None else float(weights[k])
        tot += w * (1.0 - zz) / 2.0
    return tot
