"""Serving on the GPU: continuous batching, results vs the oracle, alone == in the mix."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_03019_amd as q  # noqa: E402


def _check(r, x, prec):
    assert x["status"] == q.QAOA_OK, x
    E = max(1, r.problem.num_edges)
    if r.want_grad:
        e, dg, db = oracle.grad(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta)
        tol = 1e-4 * E if prec == "c64" else 1e-9 * E
        assert np.max(np.abs(x["dgamma"] - dg)) <= tol and np.max(np.abs(x["dbeta"] - db)) <= tol
    else:
        e, _ = oracle.run_expect(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta)
    assert abs(x["expect"] - e) <= (1e-4 if prec == "c64" else 1e-10) * E


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_mixed_requests_match_oracle_and_alone(prec):
    tr = W.serving_trace(24, seed=11, n_lo=10, n_hi=20, p_lo=1, p_hi=6)
    srv = q.Server(8 << 30, max_slots=8, prec=prec)
    # staggered arrivals so requests join while others are on the GPU
    tix = []
    for r in tr:
        tix.append(srv.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, r.want_grad))
        time.sleep(0.002)
    res = [srv.wait(t, 60.0) for t in tix]
    st = srv.stats()
    srv.close()
    assert st["req_per_s"] > 0 and 0 < st["p50_s"] <= st["p99_s"]
    for r, x in zip(tr, res):
        _check(r, x, prec)
        assert x["t_arrival"] <= x["t_admit"] <= x["t_done"]
    # each request alone gives bitwise the same numbers
    for r, x in list(zip(tr, res))[:8]:
        s1 = q.Server(8 << 30, max_slots=1, prec=prec)
        y = s1.wait(s1.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, r.want_grad), 60.0)
        s1.close()
        assert y["expect"] == x["expect"] and y["norm"] == x["norm"]
        assert np.array_equal(y["dgamma"], x["dgamma"]) and np.array_equal(y["dbeta"], x["dbeta"])


def test_admission_budget_and_errors():
    tr = W.serving_trace(6, seed=12, n_lo=20, n_hi=20, p_lo=2, p_hi=3, grad_frac=0.0)
    # budget fits one n=20 c64 state (8 MiB) at a time, plus a little
    srv = q.Server(12 << 20, max_slots=4, prec="c64")
    big = W.random_problem(22, W.SplitMix64(1), "gnp", False, 0.3)
    with pytest.raises(q.QAOAError) as ei:
        srv.submit(22, big.edges, None, [0.1], [0.2])
    assert ei.value.code == q.QAOA_ENOMEM
    with pytest.raises(q.QAOAError):
        srv.submit(20, [[0, 20]], None, [0.1], [0.2])
    tix = [srv.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, False) for r in tr]
    res = [srv.wait(t, 60.0) for t in tix]
    srv.close()
    for r, x in zip(tr, res):
        _check(r, x, "c64")
    # serialised by the budget: each admitted only after the previous finished
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_admit"]


def test_cancel():
    tr = W.serving_trace(10, seed=13, n_lo=22, n_hi=24, p_lo=8, p_hi=12, grad_frac=0.5)
    srv = q.Server(4 << 30, max_slots=2, prec="c64")
    tix = [srv.submit(r.problem.n, r.problem.edges, r.problem.weights, r.gamma, r.beta, r.want_grad) for r in tr]
    srv.cancel(tix[-1])
    srv.cancel(tix[-2])
    res = [srv.wait(t, 60.0) for t in tix]
    srv.close()
    assert res[-1]["status"] == q.QAOA_ECANCELED and res[-2]["status"] == q.QAOA_ECANCELED
    for r, x in zip(tr[:4], res[:4]):
        _check(r, x, "c64")


# Expectation requests small enough for one workgroup's LDS (complex64 n <= 14,
# complex128 n <= 13) run whole inside one workgroup (state in LDS for every
# layer) within the step that admits them; larger and gradient requests take
# the pass path.  Both paths must match the oracle, and every request must give
# bitwise the same result alone and in a mix of both kinds.
@pytest.mark.parametrize("prec,nmax", [("c64", 14), ("c128", 13)])
def test_small_requests_in_one_workgroup(prec, nmax):
    rng = W.SplitMix64(77)
    reqs = []
    for i, (n, kind, weighted) in enumerate([(1, "complete", False), (2, "gnp", True), (3, "complete", True),
                                             (5, "gnp", False), (8, "3reg", True), (nmax - 1, "gnp", True),
                                             (nmax, "complete", True), (nmax - nmax % 2, "3reg", False), (nmax, "gnp", False)]):
        pr = W.random_problem(n, W.SplitMix64(700 + i), kind, weighted, 0.4)
        p = 1 + (i % 5)
        g, b = W.uniform_angles(p, rng)
        reqs.append((pr, g, b, False))
    # larger and gradient requests in the same mix
    for i, (n, grad) in enumerate([(nmax + 2, False), (nmax, True), (18, False)]):
        pr = W.random_problem(n, W.SplitMix64(800 + i), "gnp", True, 0.3)
        g, b = W.uniform_angles(3, rng)
        reqs.append((pr, g, b, grad))
    srv = q.Server(4 << 30, max_slots=16, prec=prec)
    tix = [srv.submit(pr.n, pr.edges, pr.weights, g, b, grad) for pr, g, b, grad in reqs]
    res = [srv.wait(t, 60.0) for t in tix]
    srv.close()
    for (pr, g, b, grad), x in zip(reqs, res):
        assert x["status"] == q.QAOA_OK, x
        E = max(1, pr.num_edges)
        if grad:
            e, dg, db = oracle.grad(pr.n, pr.edges, pr.weights, g, b)
            tol = 1e-4 * E if prec == "c64" else 1e-9 * E
            assert np.max(np.abs(x["dgamma"] - dg)) <= tol and np.max(np.abs(x["dbeta"] - db)) <= tol
        else:
            e, nrm = oracle.run_expect(pr.n, pr.edges, pr.weights, g, b)
            assert abs(x["norm"] - 1.0) <= (1e-5 if prec == "c64" else 1e-12)
        err = abs(x["expect"] - e)
        print(f"n={pr.n} grad={grad} {prec}: |d<C>|={err:.2e}")
        assert err <= (1e-4 if prec == "c64" else 1e-10) * E
    for (pr, g, b, grad), x in zip(reqs, res):
        s1 = q.Server(4 << 30, max_slots=1, prec=prec)
        y = s1.wait(s1.submit(pr.n, pr.edges, pr.weights, g, b, grad), 60.0)
        s1.close()
        assert y["expect"] == x["expect"] and y["norm"] == x["norm"]
        assert np.array_equal(y["dgamma"], x["dgamma"]) and np.array_equal(y["dbeta"], x["dbeta"])
