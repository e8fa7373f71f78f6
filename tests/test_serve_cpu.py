"""Host logic of the serving loop: the arena's range allocator."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2108_04413_amd.serve import ALIGN, RangeAllocator  # noqa: E402


def test_alloc_alignment_and_exhaustion():
    a = RangeAllocator(10 * ALIGN + 17)
    assert a.nbytes == 10 * ALIGN
    r1 = a.alloc(1)
    r2 = a.alloc(ALIGN + 1)
    assert r1 == (0, ALIGN) and r2 == (ALIGN, 2 * ALIGN)
    assert a.alloc(8 * ALIGN) is None
    assert a.largest() == 7 * ALIGN


def test_release_coalesces_and_first_fit():
    a = RangeAllocator(8 * ALIGN)
    rs = [a.alloc(ALIGN) for _ in range(8)]
    assert a.alloc(1) is None
    for r in (rs[1], rs[3], rs[2]):
        a.release(*r)
    assert a.free == [(ALIGN, 3 * ALIGN)]
    assert a.alloc(2 * ALIGN) == (ALIGN, 2 * ALIGN)
    a.release(*rs[0])
    assert a.alloc(ALIGN) == (0, ALIGN)


def test_random_alloc_release_never_overlaps():
    rng = np.random.default_rng(5)
    a = RangeAllocator(1000 * ALIGN)
    live = []
    for _ in range(2000):
        if live and rng.random() < 0.45:
            a.release(*live.pop(int(rng.integers(len(live)))))
        else:
            r = a.alloc(int(rng.integers(1, 40 * ALIGN)))
            if r is not None:
                live.append(r)
        spans = sorted(live + a.free)
        pos = 0
        for o, s in spans:
            assert o == pos and s > 0
            pos = o + s
        assert pos == a.nbytes


def _teams(n_qubits, team, grid, concurrent):
    import ctypes
    from paper_2108_04413_amd._lib import check, lib
    c = len(n_qubits)
    n = (ctypes.c_int * c)(*n_qubits)
    K = (ctypes.c_int64 * c)(*[10 * q for q in n_qubits])
    S = (ctypes.c_int64 * c)(*[100 * q for q in n_qubits])
    T = None if team is None else (ctypes.c_int * c)(*team)
    W = (ctypes.c_int * c)()
    check(lib.qf_batch_teams(c, n, K, S, T, grid, concurrent, W), "qf_batch_teams")
    return list(W)


def test_batch_teams_respect_the_co_residency_cap():
    """Teams of overlapping persistent launches stay within grid / concurrent
    (host-only computation of the library's team sizes)."""
    big = [24, 22, 20, 18]
    alone = _teams(big, [-1] * 4, 512, 1)
    assert max(alone) > 256  # a lone large instance may take most of the grid
    for conc in (2, 3, 4):
        for team in ([-1] * 4, [512, 400, 300, 4], None, [-64, -64, 1, 1]):
            w = _teams(big, team, 512, conc)
            assert max(w) <= 512 // conc and min(w) >= 1
    # small instances are limited by their tiles, not by the cap
    assert _teams([12, 14], [64, 64], 512, 2) == [2, 8]
