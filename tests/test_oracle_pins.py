"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the paper's
worked bit example and its Algorithm 2 / Algorithm 3 reformulations, textbook
max-cut values, dense matrix exponentials, the p = 1 closed form, invariants,
the light-cone reduction, the paper's printed sign convention, and central
finite differences.  ``test_planted_mistakes_are_caught`` rebuilds the oracle
with deliberate errors and checks that this battery rejects every one.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(seed, n, kind="gnp", weighted=False, prob=0.5):
    return W.random_problem(n, W.SplitMix64(seed), kind, weighted, prob)


# --------------------------------------------------------------------------
# Cut values: paper's Fig. popcount, Algorithm 3, Algorithm 2, invariants
# --------------------------------------------------------------------------

def test_fig_popcount_worked_example():
    g = json.load(open(os.path.join(GOLD, "fig_popcount.json")))
    bits = g["bits"]
    full = (1 << bits) - 1
    b, gi = int(g["b"], 2), int(g["graph_I"], 2)
    b_I = int(g["b_I"], 2)
    assert b_I == full                              # figure's b_i is 1 (MSB-first label)
    assert (b ^ b_I) & full == int(g["xor_b_I_b"], 2)
    assert gi & (b ^ b_I) == int(g["and_graph_I"], 2)
    assert bin(gi & (b ^ b_I)).count("1") == g["count"]
    # MSB-first label i=3 is bit (bits-1-3) counted from the right.
    assert (b >> (bits - 1 - g["i"])) & 1 == 1


def _alg3_cut_counts(n, edges):
    """c_neg of Algorithm 3 for every b: sum_i popcount(graph_I[i] & (b_I ^ b))."""
    graph_I = [0] * n
    for u, v in edges:
        graph_I[int(u)] |= 1 << int(v)             # row i holds its j > i neighbours
    b = np.arange(1 << n, dtype=np.int64)
    c_neg = np.zeros_like(b)
    for i in range(n):
        b_I = -((b >> i) & 1)                      # all ones iff b_i = 1
        x = (graph_I[i] & (b_I ^ b))
        c_neg += np.array([bin(int(t)).count("1") for t in x], dtype=np.int64)
    return c_neg


@pytest.mark.parametrize("seed,n,kind", [(11, 9, "gnp"), (12, 10, "3reg"), (13, 8, "complete")])
def test_cut_table_equals_algorithm3_popcount(seed, n, kind):
    pr = _rand_problem(seed, n, kind)
    ct = oracle.cut_table(n, pr.edges)
    c_neg = _alg3_cut_counts(n, pr.edges)
    assert np.array_equal(ct.astype(np.int64), c_neg)
    # Algorithm 3's closing lines: c_pos = totEdge - c_neg, totRotation = c_pos - c_neg
    tot_rot = (pr.num_edges - c_neg) - c_neg
    assert np.array_equal(tot_rot, pr.num_edges - 2 * ct.astype(np.int64))


def test_cut_table_equals_algorithm2_sign_form():
    pr = _rand_problem(21, 7, "gnp", weighted=True)
    ct = oracle.cut_table(pr.n, pr.edges, pr.weights)
    graph = np.zeros((pr.n, pr.n), dtype=bool)
    wm = np.zeros((pr.n, pr.n))
    for k, (u, v) in enumerate(pr.edges):
        graph[u, v] = True
        wm[u, v] = pr.weights[k]
    for b in range(1 << pr.n):
        tot = 0.0
        for i in range(pr.n):
            for j in range(i + 1, pr.n):
                if graph[i, j]:
                    if ((b >> i) & 1) ^ ((b >> j) & 1):
                        tot -= wm[i, j]
                    else:
                        tot += wm[i, j]
        assert tot == pytest.approx(pr.total_weight - 2 * ct[b], abs=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
def test_cut_table_invariants(weighted):
    pr = _rand_problem(31, 11, "gnp", weighted=weighted)
    n = pr.n
    ct = oracle.cut_table(n, pr.edges, pr.weights)
    full = (1 << n) - 1
    z = np.arange(1 << n)
    assert ct[0] == 0.0
    assert np.allclose(ct, ct[full ^ z], rtol=0, atol=1e-12)        # C(z) = C(~z)
    assert ct.sum() == pytest.approx((1 << (n - 1)) * pr.total_weight, rel=1e-13)
    assert ct.max() == pytest.approx(oracle.brute_max_cut(n, pr.edges, pr.weights), abs=1e-12)
    # each single edge contributes w on exactly half of all z
    for k, (u, v) in enumerate(pr.edges[:5]):
        one = oracle.cut_table(n, pr.edges[k:k + 1],
                               None if pr.weights is None else pr.weights[k:k + 1])
        w = 1.0 if pr.weights is None else pr.weights[k]
        assert np.count_nonzero(one) == (1 << (n - 1))
        assert np.all((one == 0) | (one == w))


def test_textbook_max_cuts():
    gold = json.load(open(os.path.join(GOLD, "textbook_max_cuts.json")))
    for g in gold["graphs"]:
        e = np.asarray(g["edges"], dtype=np.int32)
        assert oracle.cut_table(g["n"], e).max() == g["max_cut"], g["name"]
        assert oracle.brute_max_cut(g["n"], e) == g["max_cut"], g["name"]


def test_empty_graph_and_single_qubit():
    e = np.zeros((0, 2), dtype=np.int32)
    assert np.all(oracle.cut_table(5, e) == 0)
    ex, nrm = oracle.run_expect(5, e, None, [0.3, 0.7], [0.2, 0.9])
    assert ex == 0.0 and nrm == pytest.approx(1.0, abs=1e-14)
    ex, nrm = oracle.run_expect(1, e, None, [0.3], [0.2])
    assert nrm == pytest.approx(1.0, abs=1e-15)


def test_invalid_inputs_rejected():
    with pytest.raises(ValueError):
        oracle.cut_table(4, np.array([[0, 0]]))
    with pytest.raises(ValueError):
        oracle.cut_table(4, np.array([[0, 4]]))
    with pytest.raises(ValueError):
        oracle.run_expect(4, np.array([[0, 1]]), None, [float("nan")], [0.1])


# --------------------------------------------------------------------------
# Evolution: dense matrix exponentials (n <= 8)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,weighted,p", [(41, 6, False, 1), (42, 7, True, 2),
                                               (43, 8, False, 3), (44, 5, True, 4)])
def test_state_matches_dense_matrix_exponential(seed, n, weighted, p):
    pr = _rand_problem(seed, n, "gnp", weighted)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 100))
    psi = oracle.evolve(n, pr.edges, pr.weights, g, b)
    ref = oracle.dense_evolve(n, pr.edges, pr.weights, g, b)
    assert np.max(np.abs(psi - ref)) < 1e-12
    ex, nrm = oracle.run_expect(n, pr.edges, pr.weights, g, b)
    assert ex == pytest.approx(oracle.dense_expect(n, pr.edges, pr.weights, g, b), abs=1e-12)
    assert nrm == pytest.approx(1.0, abs=1e-13)


# One amplitude of the depth-1 state as a sum over basis states (used for the
# element-wise checks at n = 30, where no state vector fits the oracle): every
# amplitude against the dense matrix exponentials, for angles in all four
# quadrants of beta (sin and cos of either sign) and both graph kinds.
@pytest.mark.parametrize("seed,n,kind,weighted", [(46, 3, "complete", True), (47, 5, "gnp", False),
                                                  (48, 8, "gnp", True), (49, 6, "3reg", False)])
def test_single_amplitude_p1_matches_dense_matrix_exponential(seed, n, kind, weighted):
    pr = _rand_problem(seed, n, kind, weighted)
    for g, b in ((0.83, 1.27), (0.4, 0.2), (2.1, 2.9), (-0.7, -1.9)):
        ref = oracle.dense_evolve(n, pr.edges, pr.weights, [g], [b])
        got = np.array([oracle.amplitude_p1(n, pr.edges, pr.weights, g, b, z) for z in range(1 << n)])
        assert np.max(np.abs(got - ref)) < 1e-13
    with pytest.raises(ValueError):
        oracle.amplitude_p1(n, pr.edges, pr.weights, 0.1, 0.2, 1 << n)


def test_cost_diagonal_matches_pauli_kronecker():
    pr = _rand_problem(45, 9, "gnp", True)
    assert np.allclose(oracle.cut_table(9, pr.edges, pr.weights),
                       oracle.dense_cost_diag(9, pr.edges, pr.weights), atol=1e-13)


# --------------------------------------------------------------------------
# <C> special cases and symmetries
# --------------------------------------------------------------------------

@pytest.mark.parametrize("weighted", [False, True])
def test_expectation_special_cases(weighted):
    pr = _rand_problem(51, 10, "gnp", weighted)
    Wt = pr.total_weight
    rng = W.SplitMix64(52)
    g, b = W.uniform_angles(3, rng)
    for gg, bb in [(g * 0, b * 0), (g, b * 0), (g * 0, b)]:
        ex, nrm = oracle.run_expect(10, pr.edges, pr.weights, gg, bb)
        assert ex == pytest.approx(Wt / 2, abs=1e-12 * max(1, Wt))
        assert nrm == pytest.approx(1.0, abs=1e-13)
    ex, _ = oracle.run_expect(10, pr.edges, pr.weights, [], [])
    assert ex == pytest.approx(Wt / 2, abs=1e-12)


def test_expectation_symmetries():
    pr = _rand_problem(61, 9, "gnp", False)
    g, b = W.uniform_angles(3, W.SplitMix64(62))
    e0 = oracle.run_expect(9, pr.edges, None, g, b)[0]
    assert oracle.run_expect(9, pr.edges, None, -g, -b)[0] == pytest.approx(e0, abs=1e-12)
    assert oracle.run_expect(9, pr.edges, None, g, b + math.pi / 2)[0] == pytest.approx(e0, abs=1e-12)
    assert oracle.run_expect(9, pr.edges, None, g + 2 * math.pi, b)[0] == pytest.approx(e0, abs=1e-11)
    # relabelling the vertices leaves <C> unchanged
    perm = np.array([3, 0, 8, 1, 7, 2, 6, 4, 5])
    pe = np.sort(perm[pr.edges], axis=1)
    assert oracle.run_expect(9, pe, None, g, b)[0] == pytest.approx(e0, abs=1e-12)


# --------------------------------------------------------------------------
# p = 1 closed forms (any n)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,kind,weighted", [(71, 10, "gnp", False), (72, 9, "gnp", True),
                                                  (73, 12, "3reg", False), (74, 8, "complete", True)])
def test_p1_closed_form(seed, n, kind, weighted):
    pr = _rand_problem(seed, n, kind, weighted, prob=0.4)
    g, b = W.uniform_angles(1, W.SplitMix64(seed + 1))
    ex = oracle.run_expect(n, pr.edges, pr.weights, g, b)[0]
    assert ex == pytest.approx(oracle.closed_form_p1(n, pr.edges, pr.weights, g[0], b[0]), abs=1e-12)
    if not weighted:
        assert ex == pytest.approx(oracle.closed_form_p1_unweighted(n, pr.edges, g[0], b[0]), abs=1e-12)


def test_plain_n12_config_closed_form():
    pr, g, b = W.plain_n12()
    assert pr.num_edges == 18
    ex = oracle.run_expect(12, pr.edges, None, g, b)[0]
    tri_free = oracle.closed_form_p1_unweighted(12, pr.edges, 0.6, 0.4)
    assert ex == pytest.approx(tri_free, abs=1e-12)


def test_farhi_triangle_free_3regular_optimum():
    """Per-edge optimum of p = 1 QAOA on triangle-free 3-regular graphs is 0.6924."""
    # 3-dimensional cube graph: 3-regular and triangle-free, n = 8, 12 edges
    e = np.array([(u, u ^ (1 << k)) for u in range(8) for k in range(3) if u < u ^ (1 << k)],
                 dtype=np.int32)
    best = 0.0
    for g in np.linspace(0.55, 0.68, 27):
        ex = oracle.run_expect(8, e, None, [g], [math.pi / 8])[0]
        best = max(best, ex / 12)
    assert 0.6923 < best < 0.6925


# --------------------------------------------------------------------------
# Light cone (p = 2) and the paper's printed convention
# --------------------------------------------------------------------------

def _zz_by_oracle(ns, se, sw, gamma, beta, a, b):
    psi = oracle.evolve(ns, se, sw, gamma, beta)
    z = np.arange(1 << ns)
    sgn = 1.0 - 2.0 * (((z >> a) ^ (z >> b)) & 1)
    return float(np.sum(np.abs(psi) ** 2 * sgn))


def test_light_cone_p2_n20():
    rng = W.SplitMix64(81)
    e = W.random_regular(20, 3, rng)
    w = W.uniform_weights(e.shape[0], rng)
    g, b = W.uniform_angles(2, rng)
    full = oracle.run_expect(20, e, w, g, b)[0]
    lc = oracle.light_cone_expect(20, e, w, g, b, _zz_by_oracle)
    assert full == pytest.approx(lc, abs=1e-11)


@pytest.mark.parametrize("weighted", [False, True])
def test_paper_convention_mapping(weighted):
    pr = _rand_problem(91, 6, "gnp", weighted)
    g, b = W.uniform_angles(2, W.SplitMix64(92))
    paper = oracle.paper_convention_expect(6, pr.edges, pr.weights, g, b)
    ours = oracle.run_expect(6, pr.edges, pr.weights, -g, b / 2)[0]
    assert paper == pytest.approx(ours, abs=1e-12)


# --------------------------------------------------------------------------
# Gradient: adjoint vs central differences and the p = 1 derivative
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n,weighted,p", [(101, 8, False, 3), (102, 7, True, 4)])
def test_adjoint_gradient_vs_central_differences(seed, n, weighted, p):
    pr = _rand_problem(seed, n, "gnp", weighted)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 7))
    ex, dg, db = oracle.grad(n, pr.edges, pr.weights, g, b)
    fg, fb = oracle.grad_fd(n, pr.edges, pr.weights, g, b, h=1e-6)
    tol = 1e-7 * pr.num_edges
    assert np.max(np.abs(dg - fg)) < tol and np.max(np.abs(db - fb)) < tol
    assert ex == pytest.approx(oracle.run_expect(n, pr.edges, pr.weights, g, b)[0], abs=1e-13)


def test_gradient_p1_analytic_triangle_free():
    e = np.array([(u, u ^ (1 << k)) for u in range(8) for k in range(3) if u < u ^ (1 << k)],
                 dtype=np.int32)
    g, b = 0.37, 0.91
    _, dg, db = oracle.grad(8, e, None, [g], [b])
    E = 12
    assert dg[0] == pytest.approx(E * 0.5 * math.sin(4 * b) *
                                  (math.cos(g) ** 3 - 2 * math.sin(g) ** 2 * math.cos(g)), abs=1e-12)
    assert db[0] == pytest.approx(E * 2 * math.cos(4 * b) * math.sin(g) * math.cos(g) ** 2, abs=1e-12)


def test_fidelity_definition():
    rng = np.random.default_rng(5)
    a = rng.normal(size=64) + 1j * rng.normal(size=64)
    b = rng.normal(size=64) + 1j * rng.normal(size=64)
    f = oracle.fidelity(6, a, b)
    ref = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
    assert f == pytest.approx(ref, rel=1e-13)
    assert oracle.fidelity(6, a, np.exp(0.3j) * 2 * a) == pytest.approx(1.0, abs=1e-14)
    # orthogonal states: disjoint supports, and a state against its Gram-Schmidt complement
    e0 = np.zeros(64, complex)
    e0[:32] = a[:32]
    e1 = np.zeros(64, complex)
    e1[32:] = b[32:]
    assert oracle.fidelity(6, e0, e1) == 0.0
    c = b - np.vdot(a, b) / np.vdot(a, a) * a
    assert oracle.fidelity(6, a, c) < 1e-28
    # a known angle: |<x|y>|^2 = cos^2(t) for unit x, y = cos(t) x + sin(t) x_perp
    x = a / np.linalg.norm(a)
    xp = c / np.linalg.norm(c)
    assert oracle.fidelity(6, x, np.cos(0.4) * x + np.sin(0.4) * xp) == pytest.approx(np.cos(0.4) ** 2, abs=1e-14)


# --------------------------------------------------------------------------
# Planted mistakes: every one must be caught by the battery above
# --------------------------------------------------------------------------

def _battery(lib):
    """Fast subset of the pins, run against an alternative oracle build."""
    fails = []
    pr = _rand_problem(11, 8, "gnp")
    try:
        ct = oracle.cut_table(8, pr.edges, lib=lib)
        if not np.array_equal(ct.astype(np.int64), _alg3_cut_counts(8, pr.edges)):
            fails.append("alg3")
        g, b = W.uniform_angles(2, W.SplitMix64(3))
        pw = _rand_problem(12, 6, "gnp", True)
        pw5 = _rand_problem(13, 5, "gnp", True)
        psi = oracle.evolve(6, pw.edges, pw.weights, g, b, lib=lib)
        if np.max(np.abs(psi - oracle.dense_evolve(6, pw.edges, pw.weights, g, b))) > 1e-12:
            fails.append("dense")
        ex, nrm = oracle.run_expect(8, pr.edges, None, g * 0, b, lib=lib)
        if abs(ex - pr.num_edges / 2) > 1e-12 or abs(nrm - 1) > 1e-12:
            fails.append("special")
        ref1 = oracle.dense_evolve(5, pw5.edges, pw5.weights, [0.83], [2.1])
        amps = [oracle.amplitude_p1(5, pw5.edges, pw5.weights, 0.83, 2.1, z, lib=lib) for z in range(32)]
        if np.max(np.abs(np.array(amps) - ref1)) > 1e-12:
            fails.append("amplitude")
        ex, dg, db = oracle.grad(6, pw.edges, pw.weights, g, b, lib=lib)
        fg, fb = oracle.grad_fd(6, pw.edges, pw.weights, g, b, lib=lib)
        if max(np.max(np.abs(dg - fg)), np.max(np.abs(db - fb))) > 1e-6:
            fails.append("grad")
    except ValueError:
        fails.append("error")
    return fails


MUTANTS = [
    ("mixer sign", "b[1] = -s * ar + c * bi;", "b[1] = s * ar + c * bi;"),
    ("transposed mixer operand", "a[0] = c * ar + s * bi;", "a[0] = c * ar + s * br;"),
    ("dropped edge", "for (int e = 0; e < m; ++e) {\n            int u = edges[2 * e], v = edges[2 * e + 1];\n            int cut",
     "for (int e = 1; e < m; ++e) {\n            int u = edges[2 * e], v = edges[2 * e + 1];\n            int cut"),
    ("wrong bit index", "(((z >> u) ^ (z >> v)) & 1)", "(((z >> u) ^ (z >> (v + 1))) & 1)"),
    ("cost phase sign", "double c = cos(th), s = -sin(th);", "double c = cos(th), s = sin(th);"),
    ("start amplitude", "pow(2.0, -0.5 * n)", "pow(2.0, -0.5 * (n - 1))"),
    ("gamma gradient factor", "dgamma[l] = 2.0 *", "dgamma[l] = 1.0 *"),
    ("adjoint conjugation", "ks_add(&s, lam[2 * z] * phi[2 * y + 1] - lam[2 * z + 1] * phi[2 * y]);",
     "ks_add(&s, lam[2 * z] * phi[2 * y + 1] + lam[2 * z + 1] * phi[2 * y]);"),
    ("mixer undo direction", "apply_rx(N, phi, q, -beta[l]);", "apply_rx(N, phi, q, beta[l]);"),
    ("amplitude: +i sin off the diagonal", "pi[4] = {0.0, -1.0, 0.0, 1.0}", "pi[4] = {0.0, 1.0, 0.0, -1.0}"),
    ("amplitude: distance from x alone", "__builtin_popcountll((uint64_t)(x ^ z))", "__builtin_popcountll((uint64_t)x)"),
    ("amplitude: cos and sin powers swapped", "pow(cb, n - d) * pow(sb, d)", "pow(sb, n - d) * pow(cb, d)"),
    ("amplitude: cost phase sign", "const double er = cos(th), ei = -sin(th);", "const double er = cos(th), ei = sin(th);"),
]


def test_battery_passes_on_true_oracle():
    assert _battery(oracle.load()) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes_are_caught(tmp_path, name, old, new):
    from oracle import build as ob
    src = open(ob.SRC).read()
    assert src.count(old) == 1, name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    import subprocess
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    str(mut), "-o", so, "-lm"], check=True, capture_output=True)
    assert _battery(oracle.load(so)) != [], f"planted mistake '{name}' not detected"


# --- sampling (inverse CDF) -------------------------------------------------
def test_sampling_distributions_with_known_cdf():
    # a basis state is always measured as itself
    psi = np.zeros(16, complex)
    psi[11] = 1j
    assert np.all(oracle.sample(psi, [0.0, 0.3, 0.999999]) == 11)
    # p = (1/4, 1/4, 1/2, 0): boundaries at 1/4 and 1/2, the zero-probability state never drawn
    psi = np.sqrt(np.array([0.25, 0.25, 0.5, 0.0])).astype(complex)
    u = [0.0, 0.24, 0.25, 0.49, 0.5, 0.75, 0.999999]
    assert oracle.sample(psi, u).tolist() == [0, 0, 1, 1, 2, 2, 2]
    # uniform state: u in the middle of cell k gives k
    psi = np.full(8, 8 ** -0.5, complex)
    assert oracle.sample(psi, [(k + 0.5) / 8 for k in range(8)]).tolist() == list(range(8))
    # unnormalised input: the CDF is scaled by the total
    assert oracle.sample(3.0 * np.sqrt(np.array([0.25, 0.75])), [0.2, 0.3]).tolist() == [0, 1]


def test_sampling_frequencies_match_probabilities():
    pr = _rand_problem(95, 6, "gnp", True)
    g, b = W.uniform_angles(2, W.SplitMix64(96))
    psi = oracle.evolve(6, pr.edges, pr.weights, g, b)
    rng = W.SplitMix64(97)
    u = np.array([rng.u01() for _ in range(40000)])
    z = oracle.sample(psi, u)
    counts = np.bincount(z.astype(np.int64), minlength=64)
    p = np.abs(psi) ** 2
    from scipy.stats import chisquare
    keep = p * len(u) >= 5
    exp = p[keep] * len(u)
    obs = counts[keep].astype(float)
    exp *= obs.sum() / exp.sum()
    assert chisquare(obs, exp).pvalue > 1e-4


def test_stored_oracle_adjoint_matches_stored_central_differences():
    # tests/golden/make_golden.py --only-fd: FP64 central differences (h = 1e-6) of the
    # oracle's <C> for the first four n=24 parameter sets; the stored adjoint gradients of
    # the same sets must agree within the FD error (truncation ~h^2, rounding ~eps |E| / h)
    import json
    d = json.load(open(os.path.join(GOLD, "oracle_fullsize.json")))
    E = d["grad_gnp_n24"]["num_edges"]
    fd = d["grad_gnp_n24_fd"]["sets"]
    assert len(fd) == 4
    for x in fd:
        r = d["grad_gnp_n24"]["sets"][x["set"]]
        assert np.max(np.abs(np.array(x["dgamma"]) - r["dgamma"])) < 1e-8 * E
        assert np.max(np.abs(np.array(x["dbeta"]) - r["dbeta"])) < 1e-8 * E
