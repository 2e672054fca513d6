"""Seeded generators: reproducibility and the structure each family promises."""
import numpy as np

import workloads as W


def test_splitmix64_reference_vector():
    # first outputs of splitmix64 seeded with 0 (public reference implementation)
    r = W.SplitMix64(0)
    assert r.next_u64() == 0xE220A8397B1DCDAF
    assert r.next_u64() == 0x6E789E6AA1B965F4


def test_u01_and_below_ranges():
    r = W.SplitMix64(7)
    xs = [r.u01() for _ in range(2000)]
    assert min(xs) >= 0.0 and max(xs) < 1.0
    ys = [r.below(7) for _ in range(7000)]
    assert set(ys) == set(range(7))
    assert 800 < min(np.bincount(ys))


def test_random_regular_is_simple_and_regular():
    for n in (12, 20, 30):
        e = W.random_regular(n, 3, W.SplitMix64(n))
        assert e.shape == (3 * n // 2, 2)
        assert np.all(e[:, 0] < e[:, 1])
        assert len({tuple(x) for x in e}) == e.shape[0]
        assert np.all(np.bincount(e.ravel(), minlength=n) == 3)


def test_plain_config_has_18_edges_and_is_deterministic():
    a, g, b = W.plain_n12()
    a2, _, _ = W.plain_n12()
    assert a.num_edges == 18 and np.array_equal(a.edges, a2.edges)
    assert g[0] == 0.6 and b[0] == 0.4


def test_gnp_and_weights():
    pr, g, b = W.gnp_n26()
    m = pr.num_edges
    assert 120 < m < 205                           # Binomial(325, 0.5): mean 162.5, sd 9
    assert len(g) == 4 and np.all((g >= 0) & (g < np.pi)) and np.all((b >= 0) & (b < np.pi))
    pw, gw, bw = W.weighted_3reg_n30()
    assert pw.num_edges == 45 and pw.weights.shape == (45,)
    assert np.all((pw.weights >= 0) & (pw.weights < 1)) and len(gw) == 10


def test_serving_trace_properties():
    tr = W.serving_trace(200)
    assert all(tr[i].arrival < tr[i + 1].arrival for i in range(len(tr) - 1))
    for r in tr:
        assert 14 <= r.problem.n <= 28 and 1 <= len(r.gamma) <= 12
        if r.family == "3reg":
            assert r.problem.n % 2 == 0
        if r.family == "complete":
            assert r.problem.num_edges == r.problem.n * (r.problem.n - 1) // 2
    frac = np.mean([r.want_grad for r in tr])
    assert 0.15 < frac < 0.45
    tr2 = W.serving_trace(20)
    assert all(np.array_equal(a.problem.edges, b.problem.edges) for a, b in zip(tr[:20], tr2))
