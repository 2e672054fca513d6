"""qaoa_fidelity_noalloc (static device workspace, no allocation) against
qaoa_fidelity, through the C ABI: two calls in a row, the second on a smaller
state, each equal to the allocating entry point's result (same kernels, same
reduction order) and to the FP64 oracle's fidelity of the read-back states."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_03019_amd as q  # noqa: E402


def _pair(n, seed, prec_a, prec_b, beta):
    pr = W.random_problem(n, W.SplitMix64(seed), "gnp", True, 0.3)
    g = list(W.uniform_angles(len(beta), W.SplitMix64(seed + 1))[0])
    a = q.Simulator(n, pr.edges, pr.weights, prec_a).run(g, beta)
    b = q.Simulator(n, pr.edges, pr.weights, prec_b).run(g[::-1], beta)
    return a, b


def test_noalloc_fidelity_matches_allocating_entry_point():
    # first call: n = 20 (complex64 against complex128, 2048 blocks: the
    # workspace's largest layout); second: n = 13, one state stored
    # complemented (an odd number of |sin beta| > |cos beta| layers)
    cases = [(20, 501, "c64", "c128", [0.3, 0.9]), (13, 502, "c128", "c128", [1.2, 0.4, 0.2])]
    for n, seed, pa, pb, beta in cases:
        a, b = _pair(n, seed, pa, pb, beta)
        f_alloc = q.qaoa_fidelity(a.handle, b.handle)
        f_static = q.qaoa_fidelity_noalloc(a.handle, b.handle)
        ref = oracle.fidelity(n, a.state().astype(np.complex128), b.state().astype(np.complex128))
        print(f"n={n} {pa}/{pb}: noalloc={f_static!r} alloc={f_alloc!r} oracle={ref!r}")
        assert f_static == f_alloc            # same kernels and reduction order: bit for bit
        assert abs(f_static - ref) < 1e-12
        # same pair again, the other way round (reads b reversed when only one is complemented)
        assert q.qaoa_fidelity_noalloc(b.handle, a.handle) == q.qaoa_fidelity(b.handle, a.handle)
        a.close()
        b.close()


def test_noalloc_fidelity_errors():
    a, b = _pair(12, 503, "c64", "c64", [0.5])
    with pytest.raises(q.QAOAError) as ei:
        q.qaoa_fidelity_noalloc(a.handle, a.handle)
    assert ei.value.code == q.QAOA_EINVAL
    pr = W.random_problem(11, W.SplitMix64(504), "gnp", False, 0.5)
    c = q.Simulator(11, pr.edges, None, "c64").run([0.2], [0.3])
    with pytest.raises(q.QAOAError) as ei:
        q.qaoa_fidelity_noalloc(a.handle, c.handle)
    assert ei.value.code == q.QAOA_EINVAL
    d = q.Simulator(12, pr.edges, None, "c64")          # no run yet: no state
    with pytest.raises(q.QAOAError) as ei:
        q.qaoa_fidelity_noalloc(a.handle, d.handle)
    assert ei.value.code == q.QAOA_ESTATE
