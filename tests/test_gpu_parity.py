"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (stated for the method): integer cut tables bit-exact; complex128
<C> within 1e-10 |E|; complex64 <C> within 1e-4 |E| and 1 - fidelity to the
exact state <= 1e-5 for p <= 10.
"""
import math

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


def _tol(pr, prec):
    return (1e-10 if prec == "c128" else 1e-4) * max(1, pr.num_edges)


# n spans: single tile (n <= 12/13), one high set, two high sets, ragged sizes
CASES = [
    (1, 1, "complete", False, 2), (2, 2, "complete", True, 3), (3, 3, "complete", False, 1),
    (4, 5, "gnp", True, 4), (5, 8, "3reg", False, 3), (6, 12, "3reg", False, 1),
    (7, 13, "gnp", True, 2), (8, 14, "gnp", False, 3), (9, 15, "3reg", True, 2),
    (10, 17, "gnp", True, 5), (11, 20, "3reg", False, 4), (12, 22, "gnp", False, 2),
    (13, 23, "3reg", True, 3),
]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("seed,n,kind,weighted,p", CASES)
def test_expectation_matches_oracle(prec, seed, n, kind, weighted, p):
    if kind == "3reg" and n % 2:
        n += 1
    pr = _prob(seed, n, kind, weighted, 0.5)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 1000))
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    e, nrm = sim.expect(g, b)
    ref, _ = oracle.run_expect(n, pr.edges, pr.weights, g, b)
    print(f"n={n} {kind} w={weighted} p={p} {prec}: gpu={e!r} oracle={ref!r} diff={e - ref:.3e}")
    assert abs(e - ref) <= _tol(pr, prec)
    assert abs(nrm - 1.0) <= (1e-12 if prec == "c128" else 1e-5)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("seed,n,weighted,p", [(21, 6, False, 2), (22, 13, True, 3), (23, 16, False, 4),
                                               (24, 19, True, 3), (25, 21, False, 5)])
def test_state_matches_oracle(prec, seed, n, weighted, p):
    pr = _prob(seed, n, "gnp", weighted, 0.4)
    g, b = W.uniform_angles(p, W.SplitMix64(seed + 7))
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    sim.run(g, b)
    psi = sim.state().astype(np.complex128)
    ref = oracle.evolve(n, pr.edges, pr.weights, g, b)
    if prec == "c128":
        assert np.max(np.abs(psi - ref)) < 1e-12
    else:
        f = oracle.fidelity(n, psi, ref)
        assert 1 - f <= 1e-5 and np.max(np.abs(psi - ref)) < 1e-5


@pytest.mark.parametrize("seed,n,kind,weighted", [(31, 12, "3reg", False), (32, 9, "gnp", True),
                                                  (33, 16, "complete", False), (34, 18, "gnp", True),
                                                  (35, 20, "3reg", False), (36, 1, "complete", False)])
def test_cut_table_bit_exact(seed, n, kind, weighted):
    pr = _prob(seed, n, kind, weighted)
    sim = q.Simulator(n, pr.edges, pr.weights, "c64")
    ct = sim.cut_table()
    ref = oracle.cut_table(n, pr.edges, pr.weights)
    if weighted:
        assert ct.dtype == np.float64 and np.array_equal(ct, ref)     # same FP64 sum order
    else:
        assert ct.dtype == np.int32 and np.array_equal(ct.astype(np.int64), ref.astype(np.int64))


def test_plain_n12_config():
    prob, g, b = W.plain_n12()
    for prec in ("c128", "c64"):
        sim = q.Simulator(prob.n, prob.edges, None, prec)
        e, _ = sim.expect(g, b)
        cf = oracle.closed_form_p1_unweighted(prob.n, prob.edges, 0.6, 0.4)
        assert abs(e - cf) <= _tol(prob, prec)
        ct = sim.cut_table()
        assert np.array_equal(ct.astype(np.int64), oracle.cut_table(prob.n, prob.edges).astype(np.int64))
        assert ct.max() == oracle.brute_max_cut(prob.n, prob.edges)


def test_special_cases_any_size():
    pr = _prob(41, 21, "gnp", True, 0.3)
    sim = q.Simulator(21, pr.edges, pr.weights, "c128")
    Wt = pr.total_weight
    for g, b in [([0.0, 0.0], [0.3, 1.1]), ([0.7, 2.0], [0.0, 0.0]), ([], [])]:
        e, nrm = sim.expect(g, b)
        assert abs(e - Wt / 2) < 1e-10 * pr.num_edges and abs(nrm - 1) < 1e-12
    # empty graph
    s0 = q.Simulator(15, np.zeros((0, 2), np.int32), None, "c64")
    e, nrm = s0.expect([0.4], [0.3])
    assert e == 0.0 and abs(nrm - 1) < 1e-5


def test_deterministic_and_repeatable():
    pr = _prob(51, 22, "gnp", True, 0.3)
    g, b = W.uniform_angles(3, W.SplitMix64(52))
    sim = q.Simulator(22, pr.edges, pr.weights, "c64")
    e1 = sim.expect(g, b)
    s1 = sim.state()
    e2 = sim.expect(g, b)
    assert e1 == e2 and np.array_equal(s1, sim.state())


def test_fidelity_c64_vs_c128():
    pr = _prob(61, 20, "gnp", False, 0.5)
    g, b = W.uniform_angles(4, W.SplitMix64(62))
    a = q.Simulator(20, pr.edges, None, "c64").run(g, b)
    c = q.Simulator(20, pr.edges, None, "c128").run(g, b)
    f = a.fidelity(c)
    ref = oracle.fidelity(20, a.state().astype(np.complex128), c.state())
    assert abs(f - ref) < 1e-12 and 1 - f <= 1e-5
    c2 = q.Simulator(20, pr.edges, None, "c128").run(g, b)
    assert abs(c.fidelity(c2) - 1.0) < 1e-12


def test_bound_torch_state_and_stream():
    pr = _prob(71, 18, "3reg", False)
    g, b = W.uniform_angles(2, W.SplitMix64(72))
    buf = torch.empty(1 << 18, dtype=torch.complex128, device="cuda")
    st = torch.cuda.Stream()
    sim = q.Simulator(18, pr.edges, None, "c128", stream=st)
    q.qaoa_bind_state(sim.handle, buf)
    e, _ = sim.expect(g, b)
    st.synchronize()
    ref = oracle.evolve(18, pr.edges, None, g, b)
    assert np.max(np.abs(buf.cpu().numpy() - ref)) < 1e-12
    assert abs(e - oracle.run_expect(18, pr.edges, None, g, b)[0]) < 1e-10 * pr.num_edges


# A layer with |sin beta| > |cos beta| is applied in its shifted factored form,
# which leaves every qubit flipped; an odd number of them leaves the stored
# state complemented (psi(~z) at z).  Readback, bound buffers and overlaps
# must still see the natural order.
@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14, 17])
def test_state_after_shifted_angle_layers(prec, n):
    pr = _prob(90 + n, n, "gnp", True, 0.4)
    for g, b in (([0.7], [1.2]), ([0.7, 0.3], [1.2, 0.25]), ([0.7, 0.3, 1.1], [1.2, 1.4, 2.0])):
        sim = q.Simulator(n, pr.edges, pr.weights, prec)
        sim.run(g, b)
        psi = sim.state().astype(np.complex128)
        ref = oracle.evolve(n, pr.edges, pr.weights, g, b)
        sim.close()
        assert np.max(np.abs(psi - ref)) < (1e-12 if prec == "c128" else 1e-5)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_bound_state_after_shifted_angle_layer(prec):
    n = 16
    pr = _prob(95, n, "3reg", False)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    buf = torch.empty(1 << n, dtype=dt, device="cuda")
    sim = q.Simulator(n, pr.edges, None, prec)
    q.qaoa_bind_state(sim.handle, buf)
    sim.expect([0.5], [1.3])
    torch.cuda.synchronize()
    ref = oracle.evolve(n, pr.edges, None, [0.5], [1.3])
    assert np.max(np.abs(buf.cpu().numpy().astype(np.complex128) - ref)) < (1e-12 if prec == "c128" else 1e-5)


def test_fidelity_between_complemented_and_plain_states():
    n = 15
    pr = _prob(96, n, "gnp", False, 0.4)
    a = q.Simulator(n, pr.edges, None, "c128").run([0.4], [1.2])      # stored complemented
    b = q.Simulator(n, pr.edges, None, "c128").run([0.9], [0.3])      # natural order
    c = q.Simulator(n, pr.edges, None, "c64").run([0.4], [1.2])
    ra = oracle.evolve(n, pr.edges, None, [0.4], [1.2])
    rb = oracle.evolve(n, pr.edges, None, [0.9], [0.3])
    ref = oracle.fidelity(n, ra, rb)
    assert abs(a.fidelity(b) - ref) < 1e-12 and abs(b.fidelity(a) - ref) < 1e-12
    assert abs(c.fidelity(b) - ref) < 1e-5
    assert 1 - a.fidelity(c) < 1e-5


# Plans with three qubit sets (complex64 from n = 23, complex128 from n = 22):
# the low set runs second, two high sets take the upper qubits round-robin, and
# their tile maps have several runs.  This is the plan shape of the n = 30
# benchmark.  <C> and the gradient cannot see a permutation of the state that
# keeps C (the global complement the shifted mixer form leaves, or a wrong
# tile map that happens to preserve C), so the state is compared element by
# element.  Angle sets give an odd and an even number of layers with
# |sin beta| > |cos beta| (applied in the shifted form).
_BETA_ODD = [0.3, 1.2, 0.5]            # one shifted layer -> stored complemented
_BETA_EVEN = [1.0, 0.2, 1.3, 0.6]      # two shifted layers -> natural order


@pytest.mark.parametrize("prec,n", [("c64", 23), ("c64", 24), ("c128", 22), ("c128", 23)])
@pytest.mark.parametrize("beta", [_BETA_ODD, _BETA_EVEN], ids=["odd_shifted", "even_shifted"])
def test_state_three_set_plan(prec, n, beta):
    pr = _prob(300 + n, n, "3reg", True) if n % 2 == 0 else _prob(300 + n, n, "gnp", True, 0.2)
    g = list(W.uniform_angles(len(beta), W.SplitMix64(400 + n))[0])
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    passes, sizes = sim.plan(len(beta))
    assert len(sizes) == 3, sizes
    sim.run(g, beta)
    psi = sim.state().astype(np.complex128)
    sim.close()
    ref = oracle.evolve(n, pr.edges, pr.weights, g, beta)
    err = float(np.max(np.abs(psi - ref)))
    print(f"n={n} {prec} sets={sizes} passes={passes} beta={beta}: max|dpsi|={err:.3e}")
    assert err < (1e-12 if prec == "c128" else 1e-5)


@pytest.mark.parametrize("prec,n", [("c64", 24), ("c128", 22)])
def test_bound_state_three_set_plan(prec, n):
    pr = _prob(320 + n, n, "gnp", False, 0.3)
    g = [0.45, 1.1, 0.8]
    dt = torch.complex128 if prec == "c128" else torch.complex64
    buf = torch.empty(1 << n, dtype=dt, device="cuda")
    st = torch.cuda.Stream()
    sim = q.Simulator(n, pr.edges, None, prec, stream=st)
    q.qaoa_bind_state(sim.handle, buf)
    e, _ = sim.expect(g, _BETA_ODD)
    st.synchronize()
    ref = oracle.evolve(n, pr.edges, None, g, _BETA_ODD)
    err = float(np.max(np.abs(buf.cpu().numpy().astype(np.complex128) - ref)))
    print(f"bound n={n} {prec}: max|dpsi|={err:.3e}")
    assert err < (1e-12 if prec == "c128" else 1e-5)
    assert abs(e - oracle.run_expect(n, pr.edges, None, g, _BETA_ODD)[0]) <= _tol(pr, prec)
    sim.close()


# Chunked pass pairs (each low-set pass and the high-set pass after it run chunk
# by chunk, the second on its own stream) compute every tile exactly as the
# unchunked passes do, so the state, <C> and the gradient must be bitwise
# equal; small chunks force chunking at sizes the oracle checks element-wise.
@pytest.mark.parametrize("prec,n", [("c64", 23), ("c64", 24), ("c128", 22), ("c128", 23)])
def test_chunked_pass_pairs_bitwise_equal(prec, n):
    pr = _prob(340 + n, n, "gnp", True, 0.25)
    g = [0.45, 1.1, 0.8, 0.3]
    b = [0.3, 1.2, 0.5, 1.0]
    res = {}
    for label, chunk, streams in (("plain", 0, 2), ("chunked", 1 << 20, 2), ("chunked3", 1 << 20, 3),
                                  ("chunked4", 1 << 20, 4)):
        sim = q.Simulator(n, pr.edges, pr.weights, prec)
        q.qaoa_set_chunking(sim.handle, chunk, 0, streams)
        e, nrm = sim.expect(g, b)
        psi = sim.state()
        eg, dg, db = sim.grad(g, b)
        res[label] = (e, nrm, psi, eg, dg, db)
        sim.close()
    F, _ = q.qaoa_chunk_plan(n, prec, len(g), 1 << 20)
    assert F >= 1
    a = res["plain"]
    for key in ("chunked", "chunked3", "chunked4"):
        c = res[key]
        assert a[0] == c[0] and a[1] == c[1] and a[3] == c[3], key
        assert np.array_equal(a[2], c[2]) and np.array_equal(a[4], c[4]) and np.array_equal(a[5], c[5]), key
    c = res["chunked"]
    ref = oracle.evolve(n, pr.edges, pr.weights, g, b)
    err = float(np.max(np.abs(c[2].astype(np.complex128) - ref)))
    print(f"chunked n={n} {prec} F={F}: max|dpsi|={err:.3e}")
    assert err < (1e-12 if prec == "c128" else 1e-5)


# A chunked run on a caller's stream with a caller's buffer: the extra streams'
# work is joined back into the caller's stream before qaoa_run returns, so work
# the caller queues on its stream right after sees the finished state (here with
# an odd number of shifted layers, so the library also reorders the buffer).
@pytest.mark.parametrize("prec,n", [("c64", 24), ("c128", 23)])
def test_chunked_pairs_join_the_caller_stream(prec, n):
    pr = _prob(360 + n, n, "gnp", True, 0.3)
    g = [0.45, 1.1, 0.8]
    plain = q.Simulator(n, pr.edges, pr.weights, prec)
    q.qaoa_set_chunking(plain.handle, 0, 0)
    plain.expect(g, _BETA_ODD)
    want = plain.state()
    plain.close()
    dt = torch.complex128 if prec == "c128" else torch.complex64
    buf = torch.empty(1 << n, dtype=dt, device="cuda")
    st = torch.cuda.Stream()
    sim = q.Simulator(n, pr.edges, pr.weights, prec, stream=st)
    q.qaoa_bind_state(sim.handle, buf)
    q.qaoa_set_chunking(sim.handle, 1 << 20, 0, 3)
    assert q.qaoa_chunk_plan(n, prec, len(g), 1 << 20)[0] >= 1
    q.qaoa_run(sim.handle, g, _BETA_ODD)
    with torch.cuda.stream(st):
        snap = buf.clone()
    st.synchronize()
    assert np.array_equal(snap.cpu().numpy(), want)
    sim.close()


# The extra streams of chunked runs are shared by every context on the device:
# two contexts whose chunked runs alternate (and a third created between them)
# each still get bitwise their whole-pass result.
def test_chunked_contexts_share_streams():
    n64, n128 = 24, 23
    p64, p128 = _prob(380, n64, "gnp", True, 0.3), _prob(381, n128, "gnp", True, 0.3)
    g, b = [0.45, 1.1, 0.8], [0.3, 1.2, 0.5]
    want = {}
    for key, n, pr, prec in (("c64", n64, p64, "c64"), ("c128", n128, p128, "c128")):
        s = q.Simulator(n, pr.edges, pr.weights, prec)
        q.qaoa_set_chunking(s.handle, 0, 0)
        want[key] = (s.expect(g, b), s.state())
        s.close()
    a = q.Simulator(n64, p64.edges, p64.weights, "c64")
    c = q.Simulator(n128, p128.edges, p128.weights, "c128")
    for s in (a, c):
        q.qaoa_set_chunking(s.handle, 1 << 20, 0, 3)
    try:
        for rep in range(2):
            ea = a.expect(g, b)
            mid = q.Simulator(n64, p64.edges, p64.weights, "c64")
            q.qaoa_set_chunking(mid.handle, 1 << 20, 0, 3)
            em = mid.expect(g, b)
            mid.close()
            ec = c.expect(g, b)
            assert ea == want["c64"][0] and em == want["c64"][0], rep
            assert ec == want["c128"][0], rep
            assert np.array_equal(a.state(), want["c64"][1]) and np.array_equal(c.state(), want["c128"][1]), rep
    finally:
        a.close()
        c.close()


# Kernel choice for the complex128 low-set pass: the generic full-LDS kernel
# when launched whole, the half-LDS four-round kernel only in chunked pairs
# (and both give bitwise the same result, as the test above checks).
def test_c128_low_set_kernel_by_launch_mode():
    n = 23
    pr = _prob(390, n, "gnp", True, 0.3)
    g, b = [0.45, 1.1], [0.3, 1.2]
    sim = q.Simulator(n, pr.edges, pr.weights, "c128")
    try:
        names = {}
        for label, chunk in (("whole", 0), ("chunked", 1 << 20)):
            q.qaoa_set_chunking(sim.handle, chunk, 0, 3)
            sim.expect(g, b)
            names[label] = [q.qaoa_pass_kernel(sim.handle, i) for i in range(2 * len(g) + 1)]
        low = [i for i, (st, _) in enumerate(names["whole"]) if st == 0]
        assert low == [1, 3]
        for i in low:
            assert names["whole"][i][1] == "k_fwd<double, 4, 12, 0, 0, -1, -1, -1, 0>"
            assert names["chunked"][i][1] == "k_fwd<double, 4, 12, 4, 1, 0, 0, 0, 1>"
        for i in range(2 * len(g) + 1):
            if i not in low:
                assert names["whole"][i] == names["chunked"][i]
    finally:
        sim.close()


# Kernel choice for the complex64 merged pass: four waves per SIMD launched
# whole, its own three-wave instance for the chunk launches of a pass pair;
# every other pass keeps its kernel.
def test_c64_merged_kernel_by_launch_mode():
    n = 24
    pr = _prob(391, n, "gnp", True, 0.3)
    g, b = [0.45, 1.1, 0.8], [0.3, 1.2, 0.5]
    sim = q.Simulator(n, pr.edges, pr.weights, "c64")
    try:
        names = {}
        for label, chunk in (("whole", 0), ("chunked", 1 << 20)):
            q.qaoa_set_chunking(sim.handle, chunk, 0, 3)
            sim.expect(g, b)
            names[label] = [q.qaoa_pass_kernel(sim.handle, i)[1] for i in range(2 * len(g) + 1)]
        # sets 13 / 6 / 5 qubits: the 6-qubit set's merged pass has two rounds (pass 4),
        # the 5-qubit set's one (pass 2, kept as it is)
        merged = [i for i, k in enumerate(names["whole"]) if k == "k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>"]
        assert merged == [4]
        for i in range(2 * len(g) + 1):
            want = "k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 2>" if i in merged else names["whole"][i]
            assert names["chunked"][i] == want, i
    finally:
        sim.close()
