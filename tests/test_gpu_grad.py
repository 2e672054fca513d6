"""GPU adjoint gradient against the oracle's adjoint, finite differences and autograd."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_03019_amd as q  # noqa: E402


def _prob(seed, n, kind="gnp", weighted=False, prob=0.5):
    return W.random_problem(n, W.SplitMix64(seed), kind, weighted, prob)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("seed,n,kind,weighted,p", [
    (1, 3, "complete", False, 2), (2, 8, "gnp", True, 3), (3, 12, "3reg", False, 4),
    (4, 13, "gnp", True, 2), (5, 14, "gnp", False, 3), (6, 17, "3reg", True, 3),
    (7, 20, "gnp", False, 4), (8, 23, "gnp", True, 2)])
def test_gradient_matches_oracle(prec, seed, n, kind, weighted, p):
    if kind == "3reg" and n % 2:
        n += 1
    pr = _prob(seed, n, kind, weighted, 0.4)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 50))
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    e, dg, db = sim.grad(g, b)
    re, rdg, rdb = oracle.grad(n, pr.edges, pr.weights, g, b)
    E = max(1, pr.num_edges)
    tol = 1e-9 * E if prec == "c128" else 1e-4 * E
    print(f"n={n} p={p} {prec}: |dg err|={np.max(np.abs(dg - rdg)):.2e} |db err|={np.max(np.abs(db - rdb)):.2e}")
    assert abs(e - re) <= (1e-10 if prec == "c128" else 1e-4) * E
    assert np.max(np.abs(dg - rdg)) <= tol and np.max(np.abs(db - rdb)) <= tol


def test_gradient_vs_central_differences_c128():
    pr = _prob(11, 16, "gnp", False, 0.3)
    g, b = W.uniform_angles(4, W.SplitMix64(12))
    sim = q.Simulator(16, pr.edges, None, "c128")
    _, dg, db = sim.grad(g, b)
    h = 1e-6
    for l in range(4):
        for arr, d in ((g, dg), (b, db)):
            a1, a2 = arr.copy(), arr.copy()
            a1[l] += h
            a2[l] -= h
            if arr is g:
                fd = (sim.expect(a1, b)[0] - sim.expect(a2, b)[0]) / (2 * h)
            else:
                fd = (sim.expect(g, a1)[0] - sim.expect(g, a2)[0]) / (2 * h)
            assert abs(fd - d[l]) <= 1e-6 * pr.num_edges


def test_autograd_function():
    pr = _prob(21, 15, "gnp", True, 0.4)
    sim = q.Simulator(15, pr.edges, pr.weights, "c128")
    g0, b0 = W.uniform_angles(3, W.SplitMix64(22))
    gt = torch.tensor(g0, dtype=torch.float64, requires_grad=True)
    bt = torch.tensor(b0, dtype=torch.float64, requires_grad=True)
    e = q.expectation(gt, bt, sim)
    (3.0 * e).backward()
    re, rdg, rdb = oracle.grad(15, pr.edges, pr.weights, g0, b0)
    assert abs(e.item() - re) < 1e-10 * pr.num_edges
    assert np.allclose(gt.grad.numpy(), 3 * rdg, atol=3e-9 * pr.num_edges)
    assert np.allclose(bt.grad.numpy(), 3 * rdb, atol=3e-9 * pr.num_edges)
    # without requires_grad only the forward sweep runs
    e2 = q.expectation(torch.tensor(g0), torch.tensor(b0), sim)
    assert abs(e2.item() - re) < 1e-10 * pr.num_edges
