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
