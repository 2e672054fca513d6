"""Sampling bitstrings from |psi|^2 on the GPU against the oracle's inverse CDF.

Both sides take the same uniforms.  Away from CDF boundaries the sample is
unique and must match exactly; within a rounding distance of a boundary (the
GPU adds the probabilities in another order) either neighbour is a valid
answer, and the sample must at least satisfy the CDF condition within that
distance.  The CDF is taken over the GPU's own state (read back), so a
complex64 state is judged on its own probabilities."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_03019_amd as q  # noqa: E402


def _accurate_cdf(psi, chunk=4096):
    """The CDF with small rounding at any size: pairwise sums per chunk, a
    compensated running sum over the chunks, then in-chunk cumulative sums.
    Each |psi_z|^2 is the exact FP64 sum of the squared components (abs() of
    a complex64 array would round the magnitude to float32 first)."""
    psi = np.asarray(psi)
    p = psi.real.astype(np.float64) ** 2
    p += psi.imag.astype(np.float64) ** 2
    n = len(p)
    if n <= chunk:
        return np.cumsum(p)
    pc = p.reshape(-1, chunk)
    sums = pc.sum(axis=1)
    pre = np.empty_like(sums)
    s = c = 0.0
    for i, x in enumerate(sums):   # Neumaier
        pre[i] = s + c
        t = s + x
        c += (s - t) + x if abs(s) >= abs(x) else (x - t) + s
        s = t
    return (np.cumsum(pc, axis=1) + pre[:, None]).reshape(-1)


def _check(psi, u, z, rel=1e-11):
    c = _accurate_cdf(psi)
    total = c[-1]
    t = np.asarray(u) * total
    ref = np.minimum(np.searchsorted(c, t, side="right"), len(c) - 1).astype(np.int64)
    small = len(c) <= 1 << 16
    if small:   # the oracle's own definition agrees with the accurate CDF away from boundaries
        oref = oracle.sample(psi, u).astype(np.int64)
    z = z.astype(np.int64)
    tol = rel * total
    prev = np.where(ref > 0, c[np.maximum(ref - 1, 0)], 0.0)
    clear = (t - prev > tol) & (c[ref] - t > tol)
    assert np.array_equal(z[clear], ref[clear])
    if small:
        assert np.array_equal(oref[clear], ref[clear])
    assert np.all(z < len(c))
    zp = np.where(z > 0, c[np.maximum(z - 1, 0)], 0.0)
    assert np.all((zp <= t + tol) & (c[z] > t - tol))
    p = np.abs(np.asarray(psi)) ** 2
    assert np.all(p[z] > 0)
    return int(clear.sum())


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("seed,n,kind,weighted,beta1", [
    (1, 1, "complete", False, 0.3), (9, 5, "gnp", True, 0.3), (2, 7, "gnp", True, 0.2), (3, 12, "3reg", False, 1.2),
    (4, 15, "gnp", True, 0.4),
    (5, 18, "3reg", True, 1.3), (6, 21, "gnp", False, 0.7)])
def test_samples_match_oracle(prec, seed, n, kind, weighted, beta1):
    pr = W.random_problem(n, W.SplitMix64(seed), kind, weighted, 0.4)
    g, b = W.uniform_angles(2, W.SplitMix64(seed + 600))
    b[0] = beta1                      # beta > pi/4 leaves the stored state complemented
    rng = W.SplitMix64(seed + 700)
    u = np.array([rng.u01() for _ in range(4000)] + [0.0, 0.5, 1.0 - 2.0 ** -53])
    sim = q.Simulator(n, pr.edges, pr.weights, prec)
    try:
        sim.run(g, b)
        z = sim.sample(u)
        psi = sim.state().astype(np.complex128)
    finally:
        sim.close()
    clear = _check(psi, u, z)
    assert clear >= len(u) - 10


def test_sample_rejects_bad_uniforms_and_missing_state():
    sim = q.Simulator(6, [[0, 1], [1, 2]], None, "c64")
    try:
        with pytest.raises(q.QAOAError) as ei:
            sim.sample([0.5])
        assert ei.value.code == q.QAOA_ESTATE
        sim.run([0.3], [0.2])
        for bad in ([1.0], [-0.1], [float("nan")]):
            with pytest.raises(q.QAOAError) as ei:
                sim.sample(bad)
            assert ei.value.code == q.QAOA_EINVAL
        assert sim.sample([]).shape == (0,)
    finally:
        sim.close()


def test_samples_n30_are_valid():
    """Full size: 2^16 samples of the n=30 workload's state, checked against
    its CDF at sampled points (the oracle's cumulative sum of the read-back state)."""
    prob, g, b = W.weighted_3reg_n30()
    sim = q.Simulator(prob.n, prob.edges, prob.weights, "c64")
    rng = W.SplitMix64(800)
    u = np.array([rng.u01() for _ in range(1 << 16)])
    try:
        sim.run(g[:3], b[:3])
        z = sim.sample(u)
        psi = sim.state()
    finally:
        sim.close()
    clear = _check(psi, u, z, rel=1e-11)
    assert clear >= 0.9 * len(u)
