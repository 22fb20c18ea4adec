// gf_heap_dev.h -- device side of the balanced heap (paper, Section 3.4
// "Heap Allocators and Allocation Tracking"): chunk layout, per-chunk locks,
// malloc, free and the lookup of the live allocation holding a pointer.
// Used by the heap's own kernels and by the RPC client, which finds the
// object behind a heap pointer passed as a reference argument (Section 3.2).
//
// Chunk metadata (the chunk headers and the entry headers inside the heap)
// is read and written with agent-scope atomics under the chunk's lock. The
// lock is taken by a compare-and-swap with agent-scope acquire and released
// by a store with agent-scope release, so each holder sees every earlier
// holder's metadata updates on any XCD.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gf {
namespace heapdev {

constexpr uint32_t kUnit = 16;
constexpr uint32_t kNone = 0xFFFFFFFFu;

// One chunk: watermark (units in use or reserved from the chunk's start),
// header unit of the highest entry (kNone if empty), capacity and first unit
// in the heap. 32 bytes. The chunk's lock word lives on a 128-byte line of
// its own (the waiters' reads and compare-and-swaps do not touch the line the
// holder works on).
constexpr uint32_t kLockStride = 32;  // uint32 words per lock line
struct ChunkHdr {
    uint32_t unused_;
    uint32_t top;
    uint32_t last;
    uint32_t cap;
    uint32_t base;
    uint32_t pad_[3];
};
static_assert(sizeof(ChunkHdr) == 32, "chunk header size");

struct DHeap {
    char *base;
    ChunkHdr *chunks;
    uint32_t *locks;             // lock of chunk c at locks[c * kLockStride]
    unsigned long long *counts;  // NULL allocations, corrupt blocks, lock timeouts, bad frees
    uint64_t units;
    uint32_t N, M, share, per, ratio;
    uint32_t vendor;
    int64_t spin_ticks;
};

__device__ __forceinline__ uint32_t ald(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ast(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void count(const DHeap &h, int k)
{
    __hip_atomic_fetch_add(h.counts + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Entry header words at unit e of a chunk whose first unit is cbase:
// [0] header unit of the entry below (kNone for the first), [1] size in
// units, [2] in use.
__device__ __forceinline__ uint32_t *entry(const DHeap &h, uint32_t cbase, uint32_t e)
{
    return (uint32_t *)(h.base + (uint64_t)(cbase + e) * kUnit);
}

// Run f(chunk) holding chunk c's lock. False if the lock was not obtained
// within the time limit (counted). The critical section sits inside the
// retry loop, and the loop ends only when a ballot shows every active lane
// done. A lane that wins a lock therefore runs its critical section and
// releases the lock in the same pass. Had the winner left the loop first, it
// would wait there, still holding the lock, for lanes of its own wavefront
// that spin on that lock.
template <typename F>
__device__ inline bool with_chunk(const DHeap &h, uint32_t c, F f)
{
    ChunkHdr *ch = h.chunks + c;
    uint32_t *lock = h.locks + (uint64_t)c * kLockStride;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    bool done = false, ok = false;
    for (;;) {
        if (!done) {
            // read before trying: a held lock costs the holder nothing
            uint32_t expect = 0;
            // agent-scope acquire and release: the entry headers share cache
            // lines with user data, so a line cached by plain accesses is
            // invalidated before the holder reads headers, and the holder's
            // updates are written back before the next holder can take the lock
            if (ald(lock) == 0 &&
                __hip_atomic_compare_exchange_strong(lock, &expect, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                f(ch);
                __hip_atomic_store(lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                done = ok = true;
            } else if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > h.spin_ticks) {
                done = true;
            } else {
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (__builtin_amdgcn_ballot_w64(!done) == 0)
            break;
    }
    if (!ok)
        count(h, 2);
    return ok;
}

// Chunk of heap unit u, or kNone outside every chunk.
__device__ __forceinline__ uint32_t chunk_of_unit(const DHeap &h, uint64_t u)
{
    const uint64_t m = u / h.share;
    if (m >= h.M)
        return kNone;
    const uint64_t r = u - m * h.share;
    const uint64_t first = (uint64_t)h.ratio * h.per;
    uint64_t n = 0;
    if (r >= first) {
        n = 1 + (r - first) / h.per;
        if (n >= h.N)
            return kNone;
    }
    return (uint32_t)(m * h.N + n);
}

__device__ inline void *heap_malloc(const DHeap &h, uint32_t tid, uint32_t team, uint64_t bytes)
{
    const uint64_t want = bytes <= kUnit ? 1 : (bytes + kUnit - 1) / kUnit;
    const uint32_t c = (team % h.M) * h.N + (tid % h.N);
    void *res = nullptr;
    with_chunk(h, c, [&](ChunkHdr *ch) {
        const uint32_t cbase = ch->base, cap = ch->cap;
        const uint32_t top = ald(&ch->top);
        if ((uint64_t)top + 1 + want <= cap) {
            // on top of the highest entry
            uint32_t *e = entry(h, cbase, top);
            ast(e + 0, ald(&ch->last));
            ast(e + 1, (uint32_t)want);
            ast(e + 2, 1u);
            ast(&ch->last, top);
            ast(&ch->top, top + 1 + (uint32_t)want);
            res = h.base + (uint64_t)(cbase + top + 1) * kUnit;
            return;
        }
        // full: the first unused entry from the bottom that is large enough
        for (uint32_t x = 0; x < top;) {
            uint32_t *e = entry(h, cbase, x);
            const uint32_t size = ald(e + 1);
            if (ald(e + 2) == 0 && size >= want) {
                ast(e + 2, 1u);
                res = h.base + (uint64_t)(cbase + x + 1) * kUnit;
                return;
            }
            x += 1 + size;
        }
    });
    return res;
}

// False for a pointer that is not the user data of an entry in the heap.
__device__ inline bool heap_free(const DHeap &h, void *p)
{
    if (!p)
        return true;
    const char *q = (const char *)p;
    if (q < h.base || (uint64_t)(q - h.base) >= h.units * kUnit || (uint64_t)(q - h.base) % kUnit != 0) {
        count(h, 3);
        return false;
    }
    const uint64_t u = (uint64_t)(q - h.base) / kUnit;
    const uint32_t c = chunk_of_unit(h, u);
    if (c == kNone || u == h.chunks[c].base) {
        count(h, 3);
        return false;
    }
    with_chunk(h, c, [&](ChunkHdr *ch) {
        const uint32_t cbase = ch->base;
        const uint32_t e = (uint32_t)(u - cbase - 1);
        ast(entry(h, cbase, e) + 2, 0u);
        uint32_t last = ald(&ch->last);
        if (e == last) {
            // reclaim the top entry and every unused entry directly below it
            uint32_t top = ald(&ch->top);
            while (last != kNone && ald(entry(h, cbase, last) + 2) == 0) {
                const uint32_t below = ald(entry(h, cbase, last) + 0);
                top = last;
                // links point strictly downwards; stop on anything else
                last = (below == kNone || below < last) ? below : kNone;
            }
            ast(&ch->top, top);
            ast(&ch->last, last);
        }
    });
    return true;
}

// The live allocation holding pointer p: its user data and size in bytes.
__device__ inline bool heap_find(const DHeap &h, const void *p, uint64_t *start, uint64_t *bytes)
{
    const char *q = (const char *)p;
    if (q < h.base || (uint64_t)(q - h.base) >= h.units * kUnit)
        return false;
    const uint64_t u = (uint64_t)(q - h.base) / kUnit;
    const uint32_t c = chunk_of_unit(h, u);
    if (c == kNone)
        return false;
    bool found = false;
    with_chunk(h, c, [&](ChunkHdr *ch) {
        const uint32_t cbase = ch->base;
        const uint64_t rel = u - cbase;
        const uint32_t top = ald(&ch->top);
        for (uint32_t x = 0; x < top;) {
            uint32_t *e = entry(h, cbase, x);
            const uint32_t size = ald(e + 1);
            if (rel >= (uint64_t)x + 1 && rel < (uint64_t)x + 1 + size) {
                if (ald(e + 2)) {
                    *start = (uint64_t)(cbase + x + 1) * kUnit;
                    *bytes = (uint64_t)size * kUnit;
                    found = true;
                }
                return;
            }
            x += 1 + size;
        }
    });
    return found;
}


}  // namespace heapdev
}  // namespace gf

struct gf_heap;
namespace gf {
namespace heapdev {
// The device view of a heap (false for NULL or a vendor heap).
bool heap_view(const gf_heap *h, DHeap *out);
}  // namespace heapdev
}  // namespace gf
