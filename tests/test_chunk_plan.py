"""Chunked pass pairs, checked on the CPU through the library's inspection calls.

With three qubit sets a layer is one pass over the low set followed by one over
a high set X.  Such a pair may run chunk by chunk: a chunk fixes some qubits of
the third set Y, so it is a union of whole tiles of both passes.  For every
plan this checks that the chunk plan fixes only qubits of Y (the top ones,
F of them), that the launches of each pass cover every tile exactly once over
the 2^F chunks, and that chunk k of both passes covers the same amplitudes:
exactly those whose fixed bits spell k.
"""
import numpy as np
import pytest

import paper_2312_03019_amd as q


def _mem_base(gpos, g):
    """Memory offset of tile index g (tile-index bit i at memory bit gpos[i])."""
    z = np.zeros_like(g)
    for i, b in enumerate(gpos):
        z |= ((g >> i) & 1) << int(b)
    return z


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n", [23, 24, 26, 28, 30, 31])
def test_chunk_plan_covers_pairs(prec, n):
    p = 3
    for chunk_bytes in (1 << 20, 8 << 20, 64 << 20):
        F, fixed = q.qaoa_chunk_plan(n, prec, p, chunk_bytes)
        sets = []
        s = 0
        while True:
            try:
                sets.append(q.qaoa_tile_map(n, prec, s))
            except q.QAOAError:
                break
            s += 1
        if len(sets) != 3:
            assert F == 0 and fixed == []
            continue
        state = (1 << n) * (8 if prec == "c64" else 16)
        if state // 2 < chunk_bytes:
            assert F == 0 and fixed == []
            continue
        assert F >= 1 and state >> F >= chunk_bytes and len(fixed) == p
        assert F == 9 or F == len([b for b in sets[1][0] if b >= len(sets[0][0])]) \
            or F == len([b for b in sets[2][0] if b >= len(sets[0][0])]) or state >> (F + 1) < chunk_bytes
        for i, fm in enumerate(fixed, start=1):
            x = 2 if i % 2 else 1                 # the high set of pair i (sets 2 and 1 alternate)
            y = 3 - x
            tp_y = [int(b) for b in sets[y][0]]
            L_y = len(tp_y) - sum(1 for b in tp_y if b >= len(sets[0][0]))
            qubits_y = sorted(tp_y[L_y:])
            want = 0
            for b in qubits_y[-F:]:
                want |= 1 << b
            assert fm == want and bin(fm).count("1") == F
            fixed_bits = [b for b in range(n) if (fm >> b) & 1]
            for st in (0, x):
                tpos, gpos, _, _ = sets[st]
                assert not any((fm >> int(b)) & 1 for b in tpos)      # chunks are unions of whole tiles
                seen = []
                for k in range(1 << F):
                    g = q.qaoa_chunk_tiles(n, prec, st, fm, F, k)
                    z = _mem_base(gpos, g)
                    kk = np.zeros_like(z)
                    for j, b in enumerate(fixed_bits):
                        kk |= ((z >> b) & 1) << j
                    assert np.all(kk == k)                          # chunk k = fixed bits spell k
                    seen.append(g)
                allg = np.sort(np.concatenate(seen))
                assert np.array_equal(allg, np.arange(1 << (n - len(tpos))))


def test_no_chunking_without_three_sets_or_when_off():
    assert q.qaoa_chunk_plan(20, "c64", 4, 1 << 20) == (0, [])      # two qubit sets
    assert q.qaoa_chunk_plan(30, "c64", 4, 0) == (0, [])            # off
    assert q.qaoa_chunk_plan(30, "c64", 0, 1 << 20) == (0, [])      # no layers
    F, fixed = q.qaoa_chunk_plan(30, "c64", 10, 64 << 20)
    assert F == 7 and len(fixed) == 10                               # 8 GiB in 128 chunks of 64 MiB


def test_inspection_calls_reject_bad_arguments():
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_plan(0, "c64", 4, 1 << 20)                      # n out of range
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_plan(40, "c64", 4, 1 << 20)
    F, fixed = q.qaoa_chunk_plan(24, "c64", 3, 1 << 20)
    assert F >= 1
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_tiles(24, "c64", 3, fixed[0], F, 0)             # no fourth set
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_tiles(24, "c64", 0, fixed[0], F, 1 << F)        # chunk index out of range
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_tiles(24, "c64", 0, fixed[0], F + 1, 0)         # bit count differs from the mask
    with pytest.raises(q.QAOAError):
        q.qaoa_chunk_tiles(24, "c64", 0, 1, 1, 0)                    # bit 0 is a tile bit, not an index bit
    assert len(q.qaoa_chunk_tiles(24, "c64", 0, fixed[0], F, 0)) == (1 << (24 - 13)) >> F
    # context calls on a NULL context
    assert q._lib.qaoa_set_chunking(None, 1 << 20, 0, 3) == q.QAOA_EINVAL
    assert q._lib.qaoa_pass_kernel(None, 0, None, None, 0) == q.QAOA_EINVAL
