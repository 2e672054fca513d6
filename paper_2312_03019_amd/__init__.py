"""MI355X (gfx950) QAOA max-cut state-vector simulator.

Python binding over ``libqaoa.so``, the C ABI declared in ``include/qaoa.h``.
Every function here only marshals arguments: all simulation work runs in the
library's HIP kernels.  There is no CPU fallback; importing this package
raises if the library has not been built.

The functions carry the C names (``qaoa_create``, ``qaoa_run``, ...).
``Simulator`` wraps one context, ``QAOAExpectation`` is the autograd
Function whose backward uses the library's adjoint sweep, and ``Server``
wraps the continuous-batching serving API.

Convention (fixed by the ABI): qubit q is bit q of the basis index, the cost
layer is exp(-i gamma C(z)) with C(z) the cut weight, the mixer is
exp(-i beta X_q) on every qubit, and the start state is |+>^n.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

try:  # torch first: the library then binds to the HIP runtime torch already loaded
    import torch
except ImportError:  # pragma: no cover - torch is part of the supported stack
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqaoa.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "qaoa.h")

QAOA_OK, QAOA_EINVAL, QAOA_ENOMEM, QAOA_EDEVICE = 0, -1, -2, -3
QAOA_EPENDING, QAOA_ECANCELED, QAOA_ESTATE = -4, -5, -6
QAOA_C128, QAOA_C64 = 0, 1
_PREC = {"c128": QAOA_C128, "complex128": QAOA_C128, "c64": QAOA_C64, "complex64": QAOA_C64,
         QAOA_C128: QAOA_C128, QAOA_C64: QAOA_C64}
_NAMES = {0: "QAOA_OK", -1: "QAOA_EINVAL", -2: "QAOA_ENOMEM", -3: "QAOA_EDEVICE",
          -4: "QAOA_EPENDING", -5: "QAOA_ECANCELED", -6: "QAOA_ESTATE"}


class QAOAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class qaoa_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("num_edges", ctypes.c_int),
                ("edges", ctypes.POINTER(ctypes.c_int32)), ("weights", ctypes.POINTER(ctypes.c_double)),
                ("p", ctypes.c_int), ("gamma", ctypes.POINTER(ctypes.c_double)),
                ("beta", ctypes.POINTER(ctypes.c_double)), ("want_grad", ctypes.c_int)]


class qaoa_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("expect", ctypes.c_double), ("norm", ctypes.c_double),
                ("dgamma", ctypes.POINTER(ctypes.c_double)), ("dbeta", ctypes.POINTER(ctypes.c_double)),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_I, _D, _P, _SZ = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
_IP = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "qaoa_create": (_I, [_I, _I, _IP, _DP, _I, ctypes.POINTER(_P)]),
    "qaoa_destroy": (None, [_P]),
    "qaoa_max_qubits": (_I, [_I, _I]),
    "qaoa_run": (_I, [_P, _I, _DP, _DP]),
    "qaoa_expect": (_I, [_P, _DP, _DP]),
    "qaoa_grad": (_I, [_P, _I, _DP, _DP, _DP, _DP, _DP]),
    "qaoa_run_gates": (_I, [_P, _I, _DP, _DP]),
    "qaoa_max_cut": (_I, [_P, _DP, ctypes.POINTER(ctypes.c_uint64)]),
    "qaoa_sample": (_I, [_P, ctypes.c_int64, _DP, ctypes.POINTER(ctypes.c_uint64)]),
    "qaoa_cut_table": (_I, [_P, _P, _SZ]),
    "qaoa_get_state": (_I, [_P, _P, _SZ]),
    "qaoa_fidelity": (_I, [_P, _P, _DP]),
    "qaoa_fidelity_noalloc": (_I, [_P, _P, _DP]),
    "qaoa_bind_stream": (_I, [_P, _P]),
    "qaoa_bind_state": (_I, [_P, _P, _SZ]),
    "qaoa_set_profiling": (_I, [_P, _I]),
    "qaoa_pass_times": (_I, [_P, ctypes.POINTER(ctypes.c_float), _DP, _I, ctypes.POINTER(_I)]),
    "qaoa_set_chunking": (_I, [_P, _SZ, _SZ, _I]),
    "qaoa_pass_span": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_float)]),
    "qaoa_chunk_plan": (_I, [_I, _I, _I, _SZ, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_uint64), _I,
                             ctypes.POINTER(_I)]),
    "qaoa_chunk_tiles": (_I, [_I, _I, _I, ctypes.c_uint64, _I, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "qaoa_pass_kernel": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.c_char_p, _SZ]),
    "qaoa_plan_info": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I), _I]),
    "qaoa_tile_map": (_I, [_I, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(ctypes.c_int8),
                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int8)]),
    "qaoa_copy_probe": (_I, [_P, _P, _SZ, _I, _P]),
    "qaoa_last_error": (ctypes.c_char_p, []),
    "qaoa_serve_create": (_I, [_SZ, _I, _I, ctypes.POINTER(_P)]),
    "qaoa_serve_submit": (_I, [_P, ctypes.POINTER(qaoa_request), _D, ctypes.POINTER(ctypes.c_uint64)]),
    "qaoa_serve_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(qaoa_result)]),
    "qaoa_serve_wait": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(qaoa_result), _D]),
    "qaoa_serve_cancel": (_I, [_P, ctypes.c_uint64]),
    "qaoa_serve_stats": (_I, [_P, _DP, _DP, _DP]),
    "qaoa_serve_clock": (_D, [_P]),
    "qaoa_serve_destroy": (_I, [_P]),
}


def header_symbols(path: str = HEADER):
    """Function names declared in include/qaoa.h."""
    txt = open(path).read()
    return sorted(set(re.findall(r"\b(qaoa_[a-z_0-9]+)\s*\(", txt)))


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          f"or `python paper_2312_03019_amd/build.py`; there is no fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = load_library()


def _err(rc: int):
    if rc != QAOA_OK:
        msg = _lib.qaoa_last_error()
        raise QAOAError(rc, msg.decode() if msg else "")


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_DP)


def _edges(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


# ---------------------------------------------------------------------------
# C-named functions
# ---------------------------------------------------------------------------

def qaoa_create(n: int, edges, weights=None, prec="c128") -> ctypes.c_void_p:
    e = _edges(edges)
    w = None if weights is None else _f64(weights)
    if w is not None and w.shape[0] != e.shape[0]:
        raise QAOAError(QAOA_EINVAL, "one weight per edge")
    h = ctypes.c_void_p()
    _err(_lib.qaoa_create(int(n), int(e.shape[0]), e.ctypes.data_as(_IP), _dptr(w), _PREC[prec],
                          ctypes.byref(h)))
    return h


def qaoa_destroy(ctx) -> None:
    _lib.qaoa_destroy(ctx)


def qaoa_max_qubits(prec="c128", with_grad=False) -> int:
    return int(_lib.qaoa_max_qubits(_PREC[prec], int(bool(with_grad))))


def qaoa_run(ctx, gamma, beta) -> None:
    g, b = _f64(gamma), _f64(beta)
    if g.shape != b.shape:
        raise QAOAError(QAOA_EINVAL, "gamma and beta differ in length")
    _err(_lib.qaoa_run(ctx, int(g.shape[0]), _dptr(g), _dptr(b)))


def qaoa_run_gates(ctx, gamma, beta) -> None:
    g, b = _f64(gamma), _f64(beta)
    if g.shape != b.shape:
        raise QAOAError(QAOA_EINVAL, "gamma and beta differ in length")
    _err(_lib.qaoa_run_gates(ctx, int(g.shape[0]), _dptr(g), _dptr(b)))


def qaoa_max_cut(ctx):
    v, z = ctypes.c_double(), ctypes.c_uint64()
    _err(_lib.qaoa_max_cut(ctx, ctypes.byref(v), ctypes.byref(z)))
    return v.value, int(z.value)


def qaoa_sample(ctx, uniforms) -> np.ndarray:
    u = _f64(uniforms).reshape(-1)
    out = np.zeros(u.shape[0], dtype=np.uint64)
    _err(_lib.qaoa_sample(ctx, int(u.shape[0]), _dptr(u), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return out


def qaoa_expect(ctx):
    e, nrm = ctypes.c_double(), ctypes.c_double()
    _err(_lib.qaoa_expect(ctx, ctypes.byref(e), ctypes.byref(nrm)))
    return e.value, nrm.value


def qaoa_grad(ctx, gamma, beta):
    g, b = _f64(gamma), _f64(beta)
    if g.shape != b.shape:
        raise QAOAError(QAOA_EINVAL, "gamma and beta differ in length")
    p = g.shape[0]
    dg, db = np.zeros(max(p, 1)), np.zeros(max(p, 1))
    e = ctypes.c_double()
    _err(_lib.qaoa_grad(ctx, p, _dptr(g), _dptr(b), ctypes.byref(e), _dptr(dg), _dptr(db)))
    return e.value, dg[:p], db[:p]


def qaoa_cut_table(ctx, n: int, weighted: bool) -> np.ndarray:
    out = np.empty(1 << n, dtype=np.float64 if weighted else np.int32)
    _err(_lib.qaoa_cut_table(ctx, out.ctypes.data_as(_P), out.nbytes))
    return out


def qaoa_get_state(ctx, n: int, prec="c128") -> np.ndarray:
    dt = np.complex128 if _PREC[prec] == QAOA_C128 else np.complex64
    out = np.empty(1 << n, dtype=dt)
    _err(_lib.qaoa_get_state(ctx, out.ctypes.data_as(_P), out.nbytes))
    return out


def qaoa_fidelity(a, b) -> float:
    f = ctypes.c_double()
    _err(_lib.qaoa_fidelity(a, b, ctypes.byref(f)))
    return f.value


def qaoa_fidelity_noalloc(a, b) -> float:
    """qaoa_fidelity with the library's static device workspace (no allocation)."""
    f = ctypes.c_double()
    _err(_lib.qaoa_fidelity_noalloc(a, b, ctypes.byref(f)))
    return f.value


def qaoa_bind_stream(ctx, stream) -> None:
    """``stream``: a torch.cuda.Stream, a raw hipStream_t integer, or None (null stream)."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _err(_lib.qaoa_bind_stream(ctx, ctypes.c_void_p(stream) if stream else None))


def qaoa_bind_state(ctx, buf, nbytes: Optional[int] = None) -> None:
    """``buf``: a device tensor (kept alive by the caller) or a raw device address."""
    if hasattr(buf, "data_ptr"):
        nbytes = buf.numel() * buf.element_size() if nbytes is None else nbytes
        buf = buf.data_ptr()
    _err(_lib.qaoa_bind_state(ctx, ctypes.c_void_p(buf), int(nbytes)))


def qaoa_set_profiling(ctx, enable: bool) -> None:
    _err(_lib.qaoa_set_profiling(ctx, int(bool(enable))))


def qaoa_pass_times(ctx, max_passes: int = 4096):
    ms = (ctypes.c_float * max_passes)()
    by = (ctypes.c_double * max_passes)()
    cnt = ctypes.c_int()
    _err(_lib.qaoa_pass_times(ctx, ms, by, max_passes, ctypes.byref(cnt)))
    k = min(cnt.value, max_passes)
    return np.array(ms[:k], dtype=np.float64), np.array(by[:k], dtype=np.float64)


def qaoa_set_chunking(ctx, chunk_bytes: int, min_state_bytes: int = 512 << 20, streams: int = 3) -> None:
    """Chunked pass pairs: chunks of at least chunk_bytes for states from min_state_bytes (0 = off),
    spread over `streams` streams (2, 3 or 4)."""
    _err(_lib.qaoa_set_chunking(ctx, int(chunk_bytes), int(min_state_bytes), int(streams)))


def qaoa_pass_span(ctx, first: int, last: int) -> float:
    """ms from the start of pass `first` to the end of pass `last` of the last timed run."""
    ms = ctypes.c_float()
    _err(_lib.qaoa_pass_span(ctx, int(first), int(last), ctypes.byref(ms)))
    return ms.value


def qaoa_chunk_plan(n: int, prec: str, p: int, chunk_bytes: int):
    """(chunk bits F, [fixed memory-bit mask of each pass pair]) of a plan; no GPU needed."""
    F, cnt = ctypes.c_int(), ctypes.c_int()
    fixed = (ctypes.c_uint64 * max(p, 1))()
    _err(_lib.qaoa_chunk_plan(int(n), _PREC[prec], int(p), int(chunk_bytes), ctypes.byref(F), fixed, max(p, 1),
                              ctypes.byref(cnt)))
    return F.value, [int(fixed[i]) for i in range(cnt.value)]


def qaoa_chunk_tiles(n: int, prec: str, set_index: int, fixed_mem: int, chunk_bits: int, k: int) -> np.ndarray:
    """Tile indices of qubit set `set_index` covered by chunk k's launch; no GPU needed."""
    K = 13 if _PREC[prec] == QAOA_C64 else 12
    count = (1 << max(0, n - min(n, K))) >> chunk_bits
    out = np.zeros(max(count, 1), dtype=np.int64)
    _err(_lib.qaoa_chunk_tiles(int(n), _PREC[prec], int(set_index), ctypes.c_uint64(fixed_mem), int(chunk_bits),
                               int(k), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out[:count]


def qaoa_pass_kernel(ctx, index: int):
    """(qubit set, kernel name) of pass `index` of the last run."""
    st = ctypes.c_int()
    buf = ctypes.create_string_buffer(160)
    _err(_lib.qaoa_pass_kernel(ctx, int(index), ctypes.byref(st), buf, 160))
    return st.value, buf.value.decode()


def qaoa_plan_info(ctx, p: int):
    passes, sets = ctypes.c_int(), ctypes.c_int()
    sizes = (ctypes.c_int * 64)()
    _err(_lib.qaoa_plan_info(ctx, int(p), ctypes.byref(passes), ctypes.byref(sets), sizes, 64))
    return passes.value, list(sizes[:sets.value])


def qaoa_tile_map(n: int, prec: str, set_index: int):
    """Memory layout of one qubit set: (tpos, gpos, gmask, gshift) as numpy arrays
    (tile bit -> memory bit, tile-index bit -> memory bit, and the index map as runs)."""
    k = ctypes.c_int()
    tp = (ctypes.c_int8 * 16)()
    gp = (ctypes.c_int8 * 64)()
    gm = (ctypes.c_uint64 * 12)()
    gs = (ctypes.c_int8 * 12)()
    _err(_lib.qaoa_tile_map(int(n), _PREC[prec], int(set_index), ctypes.byref(k), tp, gp, gm, gs))
    K = k.value
    return (np.array(tp[:K], dtype=np.int64), np.array(gp[:n - K], dtype=np.int64),
            np.array(gm[:], dtype=np.uint64), np.array(gs[:], dtype=np.int64))


def qaoa_copy_probe(src, dst, nbytes: int, stream=None, block_bytes: int = 16384) -> None:
    if hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    s = src.data_ptr() if hasattr(src, "data_ptr") else src
    d = dst.data_ptr() if hasattr(dst, "data_ptr") else dst
    _err(_lib.qaoa_copy_probe(ctypes.c_void_p(s), ctypes.c_void_p(d), int(nbytes), int(block_bytes),
                              ctypes.c_void_p(stream) if stream else None))


def qaoa_last_error() -> str:
    m = _lib.qaoa_last_error()
    return m.decode() if m else ""


# ---------------------------------------------------------------------------
# Convenience wrappers
# ---------------------------------------------------------------------------

class Simulator:
    """One QAOA max-cut instance on the current HIP device."""

    def __init__(self, n: int, edges, weights=None, prec="c128", stream=None):
        self.n = int(n)
        self.edges = _edges(edges)
        self.weights = None if weights is None else _f64(weights)
        self.prec = prec
        self._h = qaoa_create(self.n, self.edges, self.weights, prec)
        if stream is not None:
            qaoa_bind_stream(self._h, stream)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            qaoa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, gamma, beta):
        qaoa_run(self._h, gamma, beta)
        return self

    def expect(self, gamma=None, beta=None):
        if gamma is not None:
            qaoa_run(self._h, gamma, beta)
        return qaoa_expect(self._h)

    def grad(self, gamma, beta):
        return qaoa_grad(self._h, gamma, beta)

    def run_gates(self, gamma, beta):
        """The same evolution gate by gate (one sweep per gate), as the uncompressed reference."""
        qaoa_run_gates(self._h, gamma, beta)
        return self

    def sample(self, uniforms):
        """Bitstrings from |psi|^2 of the last run, one per uniform in [0, 1) (inverse CDF)."""
        return qaoa_sample(self._h, uniforms)

    def max_cut(self):
        """(max_z C(z), lowest z attaining it)."""
        return qaoa_max_cut(self._h)

    def cut_table(self):
        return qaoa_cut_table(self._h, self.n, self.weights is not None)

    def state(self):
        return qaoa_get_state(self._h, self.n, self.prec)

    def fidelity(self, other: "Simulator") -> float:
        return qaoa_fidelity(self._h, other._h)

    def plan(self, p: int):
        return qaoa_plan_info(self._h, p)


if torch is not None:
    class QAOAExpectation(torch.autograd.Function):
        """<C>(gamma, beta) with the gradient from the library's adjoint sweep.

        When an input requires grad, forward runs the forward and adjoint
        sweeps together (one call) and backward scales the stored gradient.
        """

        @staticmethod
        def forward(ctx, gamma, beta, sim: Simulator):
            g = gamma.detach().to("cpu", torch.float64).numpy()
            b = beta.detach().to("cpu", torch.float64).numpy()
            if gamma.requires_grad or beta.requires_grad:
                e, dg, db = sim.grad(g, b)
                ctx.save_for_backward(torch.from_numpy(dg), torch.from_numpy(db))
            else:
                e, _ = sim.expect(g, b)
            ctx.dev, ctx.dt = gamma.device, gamma.dtype
            return torch.tensor(e, dtype=gamma.dtype, device=gamma.device)

        @staticmethod
        def backward(ctx, grad_out):
            dg, db = ctx.saved_tensors
            go = grad_out.detach().to("cpu", torch.float64)
            return ((go * dg).to(ctx.dev, ctx.dt), (go * db).to(ctx.dev, ctx.dt), None)

    def expectation(gamma, beta, sim: Simulator):
        return QAOAExpectation.apply(gamma, beta, sim)


class Server:
    """Continuous-batching server (qaoa_serve_*)."""

    def __init__(self, budget_bytes: int, max_slots: int = 256, prec="c64"):
        self._h = ctypes.c_void_p()
        _err(_lib.qaoa_serve_create(int(budget_bytes), int(max_slots), _PREC[prec], ctypes.byref(self._h)))
        self._keep = {}

    def clock(self) -> float:
        return float(_lib.qaoa_serve_clock(self._h))

    def submit(self, n, edges, weights, gamma, beta, want_grad=False, arrival=-1.0) -> int:
        e = _edges(edges)
        w = None if weights is None else _f64(weights)
        g, b = _f64(gamma), _f64(beta)
        req = qaoa_request(int(n), int(e.shape[0]), e.ctypes.data_as(_IP), _dptr(w), int(g.shape[0]),
                           _dptr(g), _dptr(b), int(bool(want_grad)))
        t = ctypes.c_uint64()
        _err(_lib.qaoa_serve_submit(self._h, ctypes.byref(req), float(arrival), ctypes.byref(t)))
        self._keep[t.value] = int(g.shape[0])
        return t.value

    def _result(self, ticket, fn, *extra):
        p = self._keep.get(ticket, 0)
        dg, db = np.zeros(max(p, 1)), np.zeros(max(p, 1))
        r = qaoa_result()
        r.dgamma, r.dbeta = _dptr(dg), _dptr(db)
        rc = fn(self._h, ctypes.c_uint64(ticket), ctypes.byref(r), *extra)
        if rc == QAOA_EPENDING:
            return None
        self._keep.pop(ticket, None)
        return {"status": rc, "expect": r.expect, "norm": r.norm, "dgamma": dg[:p], "dbeta": db[:p],
                "t_arrival": r.t_arrival, "t_admit": r.t_admit, "t_done": r.t_done}

    def poll(self, ticket):
        return self._result(ticket, _lib.qaoa_serve_poll)

    def wait(self, ticket, timeout: float = -1.0):
        return self._result(ticket, _lib.qaoa_serve_wait, ctypes.c_double(timeout))

    def cancel(self, ticket):
        _err(_lib.qaoa_serve_cancel(self._h, ctypes.c_uint64(ticket)))

    def stats(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _err(_lib.qaoa_serve_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"req_per_s": a.value, "p50_s": b.value, "p99_s": c.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.qaoa_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
