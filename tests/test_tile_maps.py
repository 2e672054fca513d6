"""Host checks of the tile layouts the planner hands to the pass kernels (no GPU).

For every n and both precisions, each qubit set's map must be a permutation
of the n memory bits, its run form must give the same tile base offsets as
the per-bit form, the low set must hold qubits [0, K) with each wave's
round-0 loads on one contiguous block, and the high sets must hold the
qubits above K dealt round-robin behind their passenger bits.  A wrong map
would silently mix the wrong amplitudes, so these are checked exhaustively
here and by the GPU parity tests at every size they run."""
import numpy as np
import pytest

import paper_2312_03019_amd as q

KMAX = {"c64": 13, "c128": 12}
LOGR = {"c64": 5, "c128": 4}


def _sets(n, prec):
    out, s = [], 0
    while True:
        try:
            out.append(q.qaoa_tile_map(n, prec, s))
        except q.QAOAError as e:
            assert e.code == q.QAOA_EINVAL
            return out
        s += 1


def _base(g, gmask, gshift):
    z = 0
    for m, sh in zip(gmask, gshift):
        z |= (g & int(m)) << int(sh)
    return z


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_maps_are_permutations_and_runs_agree(prec):
    rng = np.random.default_rng(5)
    for n in range(1, 35):
        sets = _sets(n, prec)
        assert len(sets) >= 1
        covered = []
        for si, (tp, gp, gm, gs) in enumerate(sets):
            K = len(tp)
            assert K == min(n, KMAX[prec])
            assert sorted(np.concatenate([tp, gp]).tolist()) == list(range(n)), (n, si)
            assert np.all(np.diff(gp) > 0)               # index bits fill the rest in ascending order
            for i in range(n - K):                      # runs reproduce the per-bit map, bit by bit
                assert _base(1 << i, gm, gs) == 1 << int(gp[i])
            for g in rng.integers(0, 1 << (n - K), size=16, dtype=np.uint64):
                g = int(g)
                want = sum(((g >> i) & 1) << int(gp[i]) for i in range(n - K))
                assert _base(g, gm, gs) == want
            covered.append(tp if si == 0 else tp[_passengers(tp):])   # the qubits this set mixes
        # every qubit is mixed by exactly one set
        qubits = np.concatenate(covered)
        assert sorted(qubits.tolist()) == list(range(n)), n


def _passengers(tp):
    """Leading tile bits that sit on memory bits 0, 1, 2, ... (a high set's passengers)."""
    L = 0
    while L < len(tp) and tp[L] == L:
        L += 1
    return L


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_low_set_is_wave_contiguous(prec):
    for n in (8, 12, 13, 20, 30, 34):
        tp = _sets(n, prec)[0][0]
        K = len(tp)
        logr = min(LOGR[prec], K)
        t0 = K - logr                                  # thread bits of round 0: lanes, then the wave index
        lanes = min(t0, 6)
        assert sorted(tp.tolist()) == list(range(K))
        assert tp[:lanes].tolist() == list(range(lanes))
        # round-0 register bits sit right above the lanes, the wave index on top
        assert tp[t0:].tolist() == list(range(lanes, lanes + logr))
        assert tp[lanes:t0].tolist() == list(range(lanes + logr, K))


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_high_sets_deal_qubits_round_robin(prec):
    for n in range(KMAX[prec] + 1, 35):
        sets = _sets(n, prec)
        K = KMAX[prec]
        mh = len(sets) - 1
        for j, (tp, _, _, _) in enumerate(sets[1:]):
            k = len(range(K + j, n, mh))
            L = K - k
            assert tp[:L].tolist() == list(range(L))       # passengers
            assert L >= (4 if prec == "c64" else 3)         # rows of at least 128 B
            assert tp[L:].tolist() == list(range(K + j, n, mh)), (n, j)


def test_tile_map_rejects_bad_arguments():
    for args in ((0, "c64", 0), (36, "c64", 0), (30, "c64", 3), (30, "c64", -1), (12, "c128", 1)):
        with pytest.raises(q.QAOAError) as ei:
            q.qaoa_tile_map(*args)
        assert ei.value.code == q.QAOA_EINVAL
