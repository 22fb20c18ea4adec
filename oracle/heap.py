"""The balanced heap allocator, as a plain sequential model.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests compare
the device allocator with it, and nothing here is shared with the library.

Follows the paper's description of its balanced allocator (Section 3.4,
"Heap Allocators and Allocation Tracking", and the chunk figure). The heap is
cut into N x M chunks, and a thread allocates from chunk (thread id mod N,
team id mod M). Within each team slot, the chunk of thread slot 0 is
`first_ratio` times the size of the others, because the initial thread
allocates the large objects of the serial code. Inside a chunk, entries are
placed bottom-up, each a header followed by the user data. An allocation goes
on top of the highest entry (the watermark). Freeing marks an entry unused.
If the freed entry is the top one, the watermark moves down over it and over
every unused entry directly below it. When the space above the watermark is
too small, the entries are searched from the bottom for an unused one that
is large enough, and that entry is reused whole. Otherwise the allocation
fails.

Sizes are counted in 16-byte units. A header is one unit. A request of b
bytes takes max(1, ceil(b / 16)) units of user data. Offsets returned are
byte offsets of the user data from the heap's start.

Readings where the paper is silent: the chunk sizes come from splitting the
heap into M equal team shares of whole units, and each share into
(first_ratio + N - 1) equal parts (rounded down, the remainder unused). The
search for a reusable entry is first-fit from the bottom, and does not split
the entry. `find` reports the live allocation that contains a byte offset:
its start and its size in bytes (units * 16).
"""
from __future__ import annotations

UNIT = 16
NONE = None


class _Chunk:
    def __init__(self, base_units: int, cap_units: int):
        self.base = base_units      # first unit of the chunk in the heap
        self.cap = cap_units        # units in the chunk
        self.top = 0                # first unit above the highest entry
        self.last = NONE            # header unit of the highest entry
        self.entries = {}           # header unit -> [prev header unit, size units, used]


class BalancedHeap:
    def __init__(self, nbytes: int, thread_slots: int, team_slots: int, first_ratio: int):
        if thread_slots < 1 or team_slots < 1 or first_ratio < 1:
            raise ValueError("slots and ratio must be >= 1")
        self.N, self.M, self.ratio = thread_slots, team_slots, first_ratio
        units = nbytes // UNIT
        share = units // team_slots
        per = share // (first_ratio + thread_slots - 1)
        self.chunks = []
        for m in range(team_slots):
            for n in range(thread_slots):
                start = m * share + (0 if n == 0 else first_ratio * per + (n - 1) * per)
                cap = first_ratio * per if n == 0 else per
                self.chunks.append(_Chunk(start, cap))

    # chunk of a thread, and of a heap unit
    def chunk_index(self, tid: int, team: int) -> int:
        return (team % self.M) * self.N + (tid % self.N)

    def _chunk_of_unit(self, u: int):
        for i, c in enumerate(self.chunks):
            if c.base <= u < c.base + c.cap:
                return i, c
        return None, None

    def malloc(self, tid: int, team: int, nbytes: int):
        units = max(1, -(-nbytes // UNIT))
        c = self.chunks[self.chunk_index(tid, team)]
        if c.top + 1 + units <= c.cap:
            e = c.top
            c.entries[e] = [c.last, units, True]
            c.last = e
            c.top = e + 1 + units
            return (c.base + e + 1) * UNIT
        e = 0
        while e < c.top:
            prev, size, used = c.entries[e]
            if not used and size >= units:
                c.entries[e][2] = True
                return (c.base + e + 1) * UNIT
            e += 1 + size
        return None

    def free(self, off):
        if off is None:
            return
        u = off // UNIT
        i, c = self._chunk_of_unit(u)
        if c is None:
            raise ValueError("pointer outside the heap")
        e = u - c.base - 1
        c.entries[e][2] = False
        if e == c.last:
            while c.last is not None and not c.entries[c.last][2]:
                c.top = c.last
                c.last = c.entries[c.last][0]
                del c.entries[c.top]

    def find(self, off: int):
        """(user start, bytes) of the live allocation containing byte `off`."""
        u = off // UNIT
        i, c = self._chunk_of_unit(u)
        if c is None:
            return None
        rel = u - c.base
        e = 0
        while e < c.top:
            prev, size, used = c.entries[e]
            if e + 1 <= rel < e + 1 + size:
                return ((c.base + e + 1) * UNIT, size * UNIT) if used else None
            e += 1 + size
        return None

    def tops(self):
        return [c.top for c in self.chunks]
