"""Pins of the balanced-heap model (oracle/heap.py) against the paper's chunk
figure and hand-worked layouts. CPU only."""
import pytest

from oracle.heap import BalancedHeap, UNIT


def test_chunk_layout_and_selection():
    # 16 KiB = 1024 units; 2 team shares of 512; 512 // (3 + 4 - 1) = 85 units per part
    h = BalancedHeap(16 * 1024, thread_slots=4, team_slots=2, first_ratio=3)
    assert [(c.base, c.cap) for c in h.chunks] == [(0, 255), (255, 85), (340, 85), (425, 85),
                                                   (512, 255), (767, 85), (852, 85), (937, 85)]
    assert h.chunk_index(tid=5, team=3) == 5          # (3 mod 2) * 4 + (5 mod 4)
    assert h.malloc(5, 3, 40) == (767 + 1) * UNIT     # header unit, then the user data


def test_the_papers_chunk_figure():
    """Three live entries; freeing the middle one changes nothing but its
    mark; freeing the top one reclaims it and the freed entry below it."""
    h = BalancedHeap(4096, 1, 1, 1)
    a = h.malloc(0, 0, 64)     # units 0 (header) + 1..4
    b = h.malloc(0, 0, 20)     # 5 + 6..7
    c = h.malloc(0, 0, 100)    # 8 + 9..15
    assert (a, b, c) == (16, 96, 144)
    assert h.tops() == [16]
    h.free(b)
    assert h.tops() == [16]
    h.free(c)
    assert h.tops() == [5]     # back to the end of the first entry
    d = h.malloc(0, 0, 16)     # placed on top again, not in the old hole
    assert d == 96 and h.tops() == [7]


def test_exhausted_chunk_reuses_the_first_free_entry_that_fits():
    h = BalancedHeap(15 * UNIT, 1, 1, 1)   # one chunk of 15 units
    # entries (header unit, data units): (0, 1-3), (4, 5), (6, 7-10), (11, 12-13)
    p = [h.malloc(0, 0, 48), h.malloc(0, 0, 16), h.malloc(0, 0, 64), h.malloc(0, 0, 32)]
    assert p == [16, 80, 112, 192] and h.tops() == [14]
    h.free(p[0])                            # 3-unit hole at the bottom
    h.free(p[2])                            # 4-unit hole
    assert h.malloc(0, 0, 80) is None       # 5 units: no room on top, no hole large enough
    assert h.malloc(0, 0, 60) == 112        # 4 units: the first hole is too small, the second fits
    assert h.find(112 + 63) == (112, 64)    # reused whole, not split
    assert h.malloc(0, 0, 33) == 16         # 3 units: the bottom hole
    assert h.malloc(0, 0, 1) is None
    assert h.malloc(0, 0, 0) is None        # a zero-byte request still takes a unit


def test_find_reports_live_allocations_only():
    h = BalancedHeap(4096, 2, 1, 2)
    a = h.malloc(0, 0, 50)
    b = h.malloc(1, 0, 8)
    assert h.find(a) == (a, 64) and h.find(a + 63) == (a, 64)
    assert h.find(a - 1) is None                   # the header
    assert h.find(b + 3) == (b, 16)
    h.free(a)
    assert h.find(a) is None


@pytest.mark.parametrize("order", ["lifo", "fifo", "interleaved"])
def test_every_chunk_is_empty_after_all_frees(order):
    h = BalancedHeap(1 << 16, 8, 4, 4)
    ptrs = [h.malloc(t, g, 16 + (t * 7 + g * 13) % 100) for g in range(6) for t in range(20)]
    assert all(p is not None for p in ptrs)
    if order == "lifo":
        ptrs = ptrs[::-1]
    elif order == "interleaved":
        ptrs = ptrs[::2] + ptrs[1::2]
    for p in ptrs:
        h.free(p)
    assert h.tops() == [0] * 32
