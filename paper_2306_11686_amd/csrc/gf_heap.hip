// gf_heap.hip -- the balanced heap allocator on the device (paper, Section
// 3.4 "Heap Allocators and Allocation Tracking"), the script and
// microbenchmark kernels that exercise it (Section 5.1 "Allocator
// Performance"), and the C ABI of include/gf_heap.h.
//
// Chunk metadata (the chunk headers and the entry headers inside the heap)
// is read and written only with agent-scope atomics, which stay coherent
// across the XCDs without writing back or invalidating whole L2 caches. A
// chunk's lock is taken with a compare-and-swap. The holder's metadata
// stores are complete (s_waitcnt) before the lock word is cleared, and the
// next holder issues its loads only after its own compare-and-swap has
// returned. The lock is taken per lane: a lane that wins it finishes its
// critical section and releases it in the same pass of the retry loop, so
// lanes of one wavefront that map to the same chunk cannot deadlock.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "gf.h"
#include "gf_heap.h"

namespace {

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
__device__ bool with_chunk(const DHeap &h, uint32_t c, F f)
{
    ChunkHdr *ch = h.chunks + c;
    uint32_t *lock = h.locks + (uint64_t)c * kLockStride;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    bool done = false, ok = false;
    uint32_t backoff = 1;
    for (;;) {
        if (!done) {
            // read before trying: a held lock costs the holder nothing
            uint32_t expect = 0;
            if (ald(lock) == 0 &&
                __hip_atomic_compare_exchange_strong(lock, &expect, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                f(ch);
                // the metadata stores are complete before the lock is released
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                ast(lock, 0u);
                done = ok = true;
            } else if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > h.spin_ticks) {
                done = true;
            } else {
                // exponential back-off, up to 16 x 8 x 64 clocks
                for (uint32_t k = 0; k < backoff; ++k)
                    __builtin_amdgcn_s_sleep(8);
                backoff = backoff < 16 ? 2 * backoff : 16;
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

__device__ void *heap_malloc(const DHeap &h, uint32_t tid, uint32_t team, uint64_t bytes)
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
__device__ bool heap_free(const DHeap &h, void *p)
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
__device__ bool heap_find(const DHeap &h, const void *p, uint64_t *start, uint64_t *bytes)
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

__global__ void __launch_bounds__(64) k_heap_script(DHeap h, const int64_t *ops, int32_t n, int64_t *res)
{
    if (threadIdx.x != 0)
        return;
    for (int32_t i = 0; i < n; ++i) {
        const int64_t op = ops[3 * i], a = ops[3 * i + 1], b = ops[3 * i + 2];
        int64_t r0 = 0, r1 = 0;
        if (op == GF_HEAP_OP_MALLOC) {
            void *p = heap_malloc(h, (uint32_t)(b & 0xFFFFFFFF), (uint32_t)((uint64_t)b >> 32), (uint64_t)a);
            r0 = p ? (int64_t)((char *)p - h.base) : -1;
        } else if (op == GF_HEAP_OP_FREE) {
            const int64_t off = res[2 * a];
            heap_free(h, off < 0 ? nullptr : h.base + off);
        } else if (op == GF_HEAP_OP_FIND) {
            const int64_t off = res[2 * a];
            uint64_t s = 0, bytes = 0;
            r0 = -1;
            if (off >= 0 && heap_find(h, h.base + off + b, &s, &bytes)) {
                r0 = (int64_t)s;
                r1 = (int64_t)bytes;
            }
        }
        res[2 * i] = r0;
        res[2 * i + 1] = r1;
    }
}

// The microbenchmark body; VENDOR selects the HIP runtime's device malloc.
template <bool VENDOR>
__global__ void __launch_bounds__(1024) k_heap_bench(DHeap h, int64_t bytes, int32_t mode, void **ptrs)
{
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words = bytes / 8;
    uint64_t *p;
    if (mode == GF_HEAP_BENCH_RELEASE) {
        p = (uint64_t *)ptrs[gid];
    } else {
        if constexpr (VENDOR)
            p = (uint64_t *)malloc((size_t)bytes);
        else
            p = (uint64_t *)heap_malloc(h, threadIdx.x, blockIdx.x, (uint64_t)bytes);
        if (!p) {
            count(h, 0);
            if (mode == GF_HEAP_BENCH_HOLD)
                ptrs[gid] = nullptr;
            return;
        }
        for (int64_t k = 0; k < words; ++k)
            p[k] = (gid << 20) ^ (uint64_t)k;
        if (mode == GF_HEAP_BENCH_HOLD) {
            ptrs[gid] = p;
            return;
        }
    }
    if (!p)
        return;
    bool ok = true;
    for (int64_t k = 0; k < words; ++k)
        ok &= p[k] == ((gid << 20) ^ (uint64_t)k);
    if (!ok)
        count(h, 1);
    if constexpr (VENDOR)
        free(p);
    else
        heap_free(h, p);
}

__global__ void k_heap_tops(DHeap h, uint32_t *out, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = ald(&h.chunks[i].top);
}

hipStream_t stream_of(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

struct gf_heap {
    int device = 0;
    DHeap d{};
    std::vector<ChunkHdr> init;  // empty chunks, copied in by reset
    void *mem = nullptr;         // heap bytes | chunk headers | counters
};

extern "C" {

gf_status gf_heap_create(int32_t hip_device, const gf_heap_opts *opts, gf_heap **out)
{
    if (!opts || !out)
        return GF_EINVAL;
    *out = nullptr;
    const gf_heap_opts o = *opts;
    if (o.bytes < 16 || o.bytes > (int64_t(1) << 35))
        return GF_EINVAL;
    const bool vendor = o.vendor != 0;
    if (!vendor && (o.thread_slots < 1 || o.team_slots < 1 || o.first_ratio < 1 ||
                    (int64_t)o.thread_slots * o.team_slots > (1 << 20)))
        return GF_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess)
        return GF_EHIP;
    gf_heap *h = new (std::nothrow) gf_heap();
    if (!h)
        return GF_ENOMEM;
    h->device = hip_device;
    DHeap &d = h->d;
    d.vendor = vendor ? 1u : 0u;
    d.spin_ticks = (o.lock_timeout_us > 0 ? o.lock_timeout_us : 2 * 1000 * 1000) * 100;  // 100 MHz clock
    size_t heap_bytes = 0, nchunks = 0;
    if (vendor) {
        // the runtime's device malloc draws from a heap of this size
        hipDeviceSetLimit(hipLimitMallocHeapSize, (size_t)o.bytes);
        d.N = d.M = d.ratio = 1;
    } else {
        d.N = (uint32_t)o.thread_slots;
        d.M = (uint32_t)o.team_slots;
        d.ratio = (uint32_t)o.first_ratio;
        d.units = (uint64_t)o.bytes / kUnit;
        d.share = (uint32_t)(d.units / d.M);
        d.per = d.share / (d.ratio + d.N - 1);
        if (d.per < 2) {
            delete h;
            return GF_EINVAL;  // chunks too small to hold an entry
        }
        heap_bytes = (size_t)d.units * kUnit;
        nchunks = (size_t)d.N * d.M;
        h->init.resize(nchunks);
        for (uint32_t m = 0; m < d.M; ++m)
            for (uint32_t n = 0; n < d.N; ++n) {
                ChunkHdr &c = h->init[(size_t)m * d.N + n];
                std::memset(&c, 0, sizeof c);
                c.last = kNone;
                c.base = m * d.share + (n == 0 ? 0 : d.ratio * d.per + (n - 1) * d.per);
                c.cap = n == 0 ? d.ratio * d.per : d.per;
            }
    }
    const size_t hdr_off = (heap_bytes + 255) / 256 * 256;
    const size_t lock_off = hdr_off + (nchunks * sizeof(ChunkHdr) + 255) / 256 * 256;
    const size_t cnt_off = lock_off + nchunks * kLockStride * sizeof(uint32_t);
    if (hipMalloc(&h->mem, cnt_off + 4 * sizeof(unsigned long long)) != hipSuccess) {
        delete h;
        return GF_ENOMEM;
    }
    d.base = vendor ? nullptr : (char *)h->mem;
    d.chunks = (ChunkHdr *)((char *)h->mem + hdr_off);
    d.locks = (uint32_t *)((char *)h->mem + lock_off);
    d.counts = (unsigned long long *)((char *)h->mem + cnt_off);
    if (hipMemset(d.locks, 0, nchunks * kLockStride * sizeof(uint32_t) + 4 * sizeof(unsigned long long)) !=
            hipSuccess ||
        (!vendor && hipMemcpy(d.chunks, h->init.data(), nchunks * sizeof(ChunkHdr), hipMemcpyHostToDevice) !=
                        hipSuccess)) {
        hipFree(h->mem);
        delete h;
        return GF_EHIP;
    }
    *out = h;
    return GF_OK;
}

gf_status gf_heap_destroy(gf_heap *h)
{
    if (!h)
        return GF_OK;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    if (h->mem)
        hipFree(h->mem);
    delete h;
    return GF_OK;
}

gf_status gf_heap_reset(gf_heap *h, void *s)
{
    if (!h)
        return GF_EINVAL;
    if (h->d.vendor)
        return GF_EUNSUPPORTED;
    hipSetDevice(h->device);
    return hipMemcpyAsync(h->d.chunks, h->init.data(), h->init.size() * sizeof(ChunkHdr), hipMemcpyHostToDevice,
                          stream_of(s)) == hipSuccess
               ? GF_OK
               : GF_EHIP;
}

gf_status gf_heap_script(gf_heap *h, const int64_t *d_ops, int32_t n_ops, int64_t *d_res, void *s)
{
    if (!h || n_ops < 0 || (n_ops > 0 && (!d_ops || !d_res)))
        return GF_EINVAL;
    if (h->d.vendor)
        return GF_EUNSUPPORTED;
    if (n_ops == 0)
        return GF_OK;
    // the operations reference earlier results only: check on the host
    std::vector<int64_t> ops((size_t)n_ops * 3);
    hipSetDevice(h->device);
    if (hipMemcpy(ops.data(), d_ops, ops.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return GF_EHIP;
    for (int32_t i = 0; i < n_ops; ++i) {
        const int64_t op = ops[3 * i], a = ops[3 * i + 1];
        if (op == GF_HEAP_OP_MALLOC) {
            if (a < 0)
                return GF_EINVAL;
        } else if (op == GF_HEAP_OP_FREE || op == GF_HEAP_OP_FIND) {
            if (a < 0 || a >= i || ops[3 * a] != GF_HEAP_OP_MALLOC)
                return GF_EINVAL;
        } else {
            return GF_EINVAL;
        }
    }
    hipLaunchKernelGGL(k_heap_script, dim3(1), dim3(64), 0, stream_of(s), h->d, d_ops, n_ops, d_res);
    return hipGetLastError() == hipSuccess ? GF_OK : GF_EHIP;
}

gf_status gf_heap_bench(gf_heap *h, int32_t teams, int32_t threads, int64_t bytes, int32_t mode, void **d_ptrs,
                        void *s)
{
    if (!h || teams < 1 || threads < 1 || threads > 1024 || bytes < 8 || bytes % 8 != 0 ||
        mode < GF_HEAP_BENCH_ROUNDTRIP || mode > GF_HEAP_BENCH_RELEASE || (mode != GF_HEAP_BENCH_ROUNDTRIP && !d_ptrs))
        return GF_EINVAL;
    hipSetDevice(h->device);
    if (h->d.vendor)
        hipLaunchKernelGGL(k_heap_bench<true>, dim3(teams), dim3(threads), 0, stream_of(s), h->d, bytes, mode, d_ptrs);
    else
        hipLaunchKernelGGL(k_heap_bench<false>, dim3(teams), dim3(threads), 0, stream_of(s), h->d, bytes, mode,
                           d_ptrs);
    return hipGetLastError() == hipSuccess ? GF_OK : GF_EHIP;
}

gf_status gf_heap_counts(gf_heap *h, uint64_t out[4], int32_t reset)
{
    if (!h || !out)
        return GF_EINVAL;
    hipSetDevice(h->device);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(out, h->d.counts, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess)
        return GF_EHIP;
    if (reset && hipMemset(h->d.counts, 0, 4 * sizeof(unsigned long long)) != hipSuccess)
        return GF_EHIP;
    return GF_OK;
}

gf_status gf_heap_tops(gf_heap *h, uint32_t *tops, int32_t n)
{
    if (!h || !tops)
        return GF_EINVAL;
    if (h->d.vendor)
        return GF_EUNSUPPORTED;
    const uint32_t nc = h->d.N * h->d.M;
    if (n < (int64_t)nc)
        return GF_EINVAL;
    hipSetDevice(h->device);
    uint32_t *dtmp = nullptr;
    if (hipMalloc(&dtmp, nc * sizeof(uint32_t)) != hipSuccess)
        return GF_ENOMEM;
    hipLaunchKernelGGL(k_heap_tops, dim3((nc + 255) / 256), dim3(256), 0, nullptr, h->d, dtmp, nc);
    gf_status st = GF_OK;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(tops, dtmp, nc * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        st = GF_EHIP;
    hipFree(dtmp);
    return st;
}

}  // extern "C"
