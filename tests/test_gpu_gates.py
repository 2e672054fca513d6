"""The gate-by-gate circuit (Algorithm 1) and the maximum-cut reduction on the
GPU, through the C ABI, against the FP64 oracle.

The gate path must reach the same state as the oracle (and as the fused
passes); the maximum cut is compared bit-exactly (value and lowest index),
since both sides evaluate C(z) the same way (integer popcounts, or FP64 sums
in canonical edge order)."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_03019_amd as q  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fullsize.json")


def _prob(seed, n, kind, weighted):
    return W.random_problem(n, W.SplitMix64(seed), kind, weighted, 0.5)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("seed,n,kind,weighted,p", [
    (1, 1, "complete", False, 2), (2, 5, "gnp", True, 3), (3, 10, "3reg", False, 2), (4, 13, "complete", True, 1),
    (5, 17, "gnp", False, 3), (6, 20, "3reg", True, 2)])
def test_gate_path_matches_oracle(prec, seed, n, kind, weighted, p):
    pr = _prob(seed, n, kind, weighted)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 300))
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    try:
        sim.run_gates(g, b)
        e, nrm = q.qaoa_expect(sim.handle)
        psi = sim.state().astype(np.complex128)
        fused = q.Simulator(n, pr.edges, pr.weights, prec).run(g, b)
        f = sim.fidelity(fused)
        fused.close()
    finally:
        sim.close()
    ref = oracle.evolve(n, pr.edges, pr.weights, g, b)
    re, _ = oracle.run_expect(n, pr.edges, pr.weights, g, b)
    m = max(1, pr.num_edges)
    tol_state = 1e-12 if prec == "c128" else 1e-5
    print(f"n={n} {kind} {prec}: |dpsi| {np.max(np.abs(psi - ref)):.2e} dE {e - re:.2e} 1-F(fused) {1 - f:.2e}")
    assert np.max(np.abs(psi - ref)) < tol_state
    assert abs(e - re) <= (1e-10 if prec == "c128" else 1e-4) * m
    assert abs(nrm - 1) <= (1e-12 if prec == "c128" else 1e-5)
    assert 1 - f <= (1e-12 if prec == "c128" else 1e-5)


@pytest.mark.parametrize("seed,n,kind,weighted", [
    (11, 1, "complete", False), (12, 6, "gnp", True), (13, 12, "3reg", False), (14, 15, "complete", True),
    (15, 20, "gnp", False), (16, 22, "3reg", True), (17, 24, "gnp", True)])
def test_max_cut_bit_exact(seed, n, kind, weighted):
    pr = _prob(seed, n, kind, weighted)
    sim = q.Simulator(n, pr.edges, pr.weights, "c64")
    v, z = sim.max_cut()
    sim.close()
    ct = oracle.cut_table(n, pr.edges, pr.weights)
    zr = int(np.argmax(ct))          # first (lowest) index of the maximum
    assert v == float(ct[zr]) and z == zr
    if pr.num_edges and not weighted:
        assert v == oracle.brute_max_cut(n, pr.edges)


def test_max_cut_empty_graph_and_complement_symmetry():
    s0 = q.Simulator(9, np.zeros((0, 2), np.int32), None, "c128")
    assert s0.max_cut() == (0.0, 0)
    s0.close()
    pr = _prob(18, 16, "gnp", True)
    sim = q.Simulator(16, pr.edges, pr.weights, "c128")
    v, z = sim.max_cut()
    sim.close()
    # C(z) = C(~z): the lowest maximiser has the top bit clear
    assert z < (1 << 15)
    assert float(oracle.cut_table(16, pr.edges, pr.weights)[z ^ ((1 << 16) - 1)]) == v


def test_max_cut_n30_matches_stored_oracle():
    if not os.path.exists(GOLDEN):
        pytest.skip("stored oracle values not generated")
    d = json.load(open(GOLDEN)).get("weighted_3reg_n30_max_cut")
    if d is None:
        pytest.skip("stored oracle values lack the n=30 maximum cut")
    prob, _, _ = W.weighted_3reg_n30()
    sim = q.Simulator(prob.n, prob.edges, prob.weights, "c64")
    v, z = sim.max_cut()
    sim.close()
    assert v == d["value"] and z == d["argmax"]
