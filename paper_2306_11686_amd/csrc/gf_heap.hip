// gf_heap.hip -- the balanced heap allocator (paper, Section 3.4 "Heap
// Allocators and Allocation Tracking"): the script and microbenchmark
// kernels that exercise it (Section 5.1 "Allocator Performance") and the C
// ABI of include/gf_heap.h. The allocator itself is in gf_heap_dev.h.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "gf.h"
#include "gf_heap.h"
#include "gf_heap_dev.h"

using namespace gf::heapdev;

namespace {

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

bool gf::heapdev::heap_view(const gf_heap *h, DHeap *out)
{
    if (!h || h->d.vendor)
        return false;
    *out = h->d;
    return true;
}

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

void *gf_heap_base(const gf_heap *h) { return h ? h->d.base : nullptr; }

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
