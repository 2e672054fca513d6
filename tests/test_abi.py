"""C ABI checks that need no GPU: exported symbols, validation, the pass planner."""
import ctypes

import numpy as np
import pytest

import paper_2312_03019_amd as q


def test_library_exports_every_header_symbol():
    lib = ctypes.CDLL(q.LIB_PATH)
    names = q.header_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) == set(q._SIGS), "binding signatures out of sync with the header"


@pytest.mark.parametrize("n,edges,w,prec", [
    (0, [[0, 1]], None, "c128"),            # n out of range
    (36, [[0, 1]], None, "c128"),
    (4, [[0, 4]], None, "c128"),             # vertex out of range
    (4, [[2, 2]], None, "c64"),              # self loop
    (4, [[0, 1], [1, 0]], None, "c64"),      # duplicate pair
    (4, [[0, 1]], [float("inf")], "c64"),    # non-finite weight
])
def test_create_rejects_invalid_graphs(n, edges, w, prec):
    with pytest.raises(q.QAOAError) as ei:
        q.qaoa_create(n, edges, w, prec)
    assert ei.value.code == q.QAOA_EINVAL
    assert q.qaoa_last_error() != ""


def test_bad_precision_and_null_out():
    lib = q._lib
    h = ctypes.c_void_p()
    e = np.array([[0, 1]], dtype=np.int32)
    assert lib.qaoa_create(3, 1, e.ctypes.data_as(q._IP), None, 7, ctypes.byref(h)) == q.QAOA_EINVAL
    assert lib.qaoa_create(3, 1, e.ctypes.data_as(q._IP), None, 0, None) == q.QAOA_EINVAL


def test_calls_out_of_order_and_bad_arguments():
    h = q.qaoa_create(5, [[0, 1], [1, 2]], None, "c128")
    try:
        with pytest.raises(q.QAOAError) as ei:
            q.qaoa_expect(h)
        assert ei.value.code == q.QAOA_ESTATE
        with pytest.raises(q.QAOAError) as ei:
            q.qaoa_run(h, [float("nan")], [0.1])
        assert ei.value.code == q.QAOA_EINVAL
        with pytest.raises(q.QAOAError) as ei:
            q.qaoa_get_state(h, 5)
        assert ei.value.code == q.QAOA_ESTATE
        with pytest.raises(q.QAOAError) as ei:
            q.qaoa_bind_state(h, 256, 12345)
        assert ei.value.code == q.QAOA_EINVAL
    finally:
        q.qaoa_destroy(h)
    with pytest.raises(q.QAOAError):
        q.qaoa_copy_probe(256, 512, 15)
    lib = q._lib
    assert lib.qaoa_serve_poll(None, 1, None) == q.QAOA_EINVAL
    assert lib.qaoa_serve_create(1 << 30, 0, 1, ctypes.byref(ctypes.c_void_p())) == q.QAOA_EINVAL


@pytest.mark.parametrize("prec,kmax,pas", [("c64", 13, 4), ("c128", 12, 3)])
@pytest.mark.parametrize("n", [1, 3, 7, 12, 13, 14, 17, 22, 23, 26, 30, 34, 35])
def test_plan_covers_every_qubit_once(prec, kmax, pas, n):
    h = q.qaoa_create(n, [], None, prec)
    try:
        for p in (0, 1, 2, 5, 10):
            passes, sizes = q.qaoa_plan_info(h, p)
            m = len(sizes)
            assert sum(sizes) == n
            if n <= kmax:
                assert sizes == [n]
            else:
                assert sizes[0] == kmax and all(1 <= s <= kmax - pas for s in sizes[1:])
                assert max(sizes[1:]) - min(sizes[1:]) <= 1          # balanced high sets
            # consecutive layers share their boundary set: p(m-1)+1 passes
            assert passes == (1 if p == 0 else p * (m - 1) + 1)
    finally:
        q.qaoa_destroy(h)


def test_three_qubit_sets_two_passes_per_layer_at_n30():
    for prec in ("c64", "c128"):
        h = q.qaoa_create(30, [], None, prec)
        passes, sizes = q.qaoa_plan_info(h, 10)
        q.qaoa_destroy(h)
        assert len(sizes) == 3 and passes == 21
