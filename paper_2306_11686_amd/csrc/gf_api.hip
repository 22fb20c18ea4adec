// gf_api.hip -- host runtime behind the C ABI declared in include/gf.h:
// context and device scratch, program validation, the two execution modes
// (persistent program kernel; one launch per region, optionally replayed
// from a captured HIP graph), the stand-alone reduction, and the host side
// of the RPC protocol (server loop and typed landing pads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <sys/prctl.h>
#include <cstring>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "gf_internal.h"
#include "gf_heap.h"

using namespace gf;

// ---------------------------------------------------------------------------
// RPC landing pads (paper, Section 3.2): one non-variadic host wrapper per
// argument-type signature of a variadic callee. The device sends opaque
// 64-bit argument words; the pad reinterprets each by its signature letter
// ('i' = 64-bit integer, 'd' = double) and makes the real call.
// ---------------------------------------------------------------------------

namespace {

using Pad = int (*)(char *buf, size_t cap, const char *fmt, const uint64_t *a);

template <typename T>
T from_word(uint64_t w)
{
    if constexpr (std::is_same<T, double>::value) {
        double d;
        std::memcpy(&d, &w, sizeof d);
        return d;
    } else {
        return (T)(int64_t)w;
    }
}

template <typename... T>
struct PrintfPad {
    template <size_t... I>
    static int call(char *buf, size_t cap, const char *fmt, const uint64_t *a, std::index_sequence<I...>)
    {
        return std::snprintf(buf, cap, fmt, from_word<T>(a[I])...);
    }
    static int pad(char *buf, size_t cap, const char *fmt, const uint64_t *a)
    {
        return call(buf, cap, fmt, a, std::index_sequence_for<T...>{});
    }
};

template <int Depth, typename... T>
void gen_pads(std::map<std::string, Pad> &m, const std::string &sig)
{
    m[sig] = &PrintfPad<T...>::pad;
    if constexpr (Depth > 0) {
        gen_pads<Depth - 1, T..., long long>(m, sig + "i");
        gen_pads<Depth - 1, T..., double>(m, sig + "d");
    }
}

const std::map<std::string, Pad> &printf_pads()
{
    static const std::map<std::string, Pad> m = [] {
        std::map<std::string, Pad> t;
        gen_pads<4>(t, "");
        return t;
    }();
    return m;
}

struct Format {
    std::string fmt;
    std::string sig;
    Pad pad;
};

// Landing pads of GF_S_CALL (Section 3.2): one non-variadic wrapper per
// callee and argument-type signature ('i' long long, 'd' double, 'p' a
// pointer: an opaque host value or a reference already translated into the
// request's payload). With output capture on, fprintf and fwrite aimed at
// stdout or stderr append to the capture buffer instead.
using CallPad = int64_t (*)(const uint64_t *w, std::string *cap);

template <typename T>
T word_as(uint64_t w)
{
    if constexpr (std::is_same<T, double>::value) {
        double d;
        std::memcpy(&d, &w, sizeof d);
        return d;
    } else if constexpr (std::is_pointer<T>::value) {
        return (T)(uintptr_t)w;
    } else {
        return (T)(int64_t)w;
    }
}

bool captured_stream(const void *f, const std::string *cap)
{
    return cap && (f == (const void *)stdout || f == (const void *)stderr);
}

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wformat-nonliteral"
#pragma clang diagnostic ignored "-Wformat-security"

template <typename... V>
struct FprintfPad {
    template <size_t... I>
    static int64_t run(const uint64_t *w, std::string *cap, std::index_sequence<I...>)
    {
        FILE *f = word_as<FILE *>(w[0]);
        const char *fmt = word_as<const char *>(w[1]);
        if (captured_stream(f, cap)) {
            char buf[4096];
            const int n = std::snprintf(buf, sizeof buf, fmt, word_as<V>(w[2 + I])...);
            if (n > 0)
                cap->append(buf, std::min<size_t>((size_t)n, sizeof buf - 1));
            return n;
        }
        return std::fprintf(f, fmt, word_as<V>(w[2 + I])...);
    }
    static int64_t pad(const uint64_t *w, std::string *cap) { return run(w, cap, std::index_sequence_for<V...>{}); }
};

template <typename... V>
struct SnprintfPad {
    template <size_t... I>
    static int64_t run(const uint64_t *w, std::index_sequence<I...>)
    {
        return std::snprintf(word_as<char *>(w[0]), (size_t)w[1], word_as<const char *>(w[2]),
                             word_as<V>(w[3 + I])...);
    }
    static int64_t pad(const uint64_t *w, std::string *) { return run(w, std::index_sequence_for<V...>{}); }
};

template <typename... V>
struct SscanfPad {
    template <size_t... I>
    static int64_t run(const uint64_t *w, std::index_sequence<I...>)
    {
        return std::sscanf(word_as<const char *>(w[0]), word_as<const char *>(w[1]), word_as<V>(w[2 + I])...);
    }
    static int64_t pad(const uint64_t *w, std::string *) { return run(w, std::index_sequence_for<V...>{}); }
};

#pragma clang diagnostic pop

int64_t fwrite_pad(const uint64_t *w, std::string *cap)
{
    const char *p = word_as<const char *>(w[0]);
    const size_t size = (size_t)w[1], n = (size_t)w[2];
    FILE *f = word_as<FILE *>(w[3]);
    if (captured_stream(f, cap)) {
        if (size > 0)
            cap->append(p, size * n);
        return (int64_t)n;
    }
    return (int64_t)std::fwrite(p, size, n, f);
}

int64_t fread_pad(const uint64_t *w, std::string *)
{
    return (int64_t)std::fread(word_as<void *>(w[0]), (size_t)w[1], (size_t)w[2], word_as<FILE *>(w[3]));
}

// Variadic tails: every combination of 'i', 'd', 'p' (AnyType) or of 'p'
// only, up to Depth arguments.
template <template <typename...> class P, bool AnyType, int Depth, typename... V>
void gen_call_pads(std::map<std::string, CallPad> &m, const std::string &key)
{
    m[key] = &P<V...>::pad;
    if constexpr (Depth > 0) {
        gen_call_pads<P, AnyType, Depth - 1, V..., void *>(m, key + "p");
        if constexpr (AnyType) {
            gen_call_pads<P, AnyType, Depth - 1, V..., long long>(m, key + "i");
            gen_call_pads<P, AnyType, Depth - 1, V..., double>(m, key + "d");
        }
    }
}

// key: callee number, ':', full type signature
const std::map<std::string, CallPad> &call_pads()
{
    static const std::map<std::string, CallPad> m = [] {
        std::map<std::string, CallPad> t;
        gen_call_pads<FprintfPad, true, 4>(t, std::to_string(GF_CALLEE_FPRINTF) + ":pp");
        gen_call_pads<SnprintfPad, true, 4>(t, std::to_string(GF_CALLEE_SNPRINTF) + ":pip");
        gen_call_pads<SscanfPad, false, 6>(t, std::to_string(GF_CALLEE_SSCANF) + ":pp");
        t[std::to_string(GF_CALLEE_FWRITE) + ":piip"] = &fwrite_pad;
        t[std::to_string(GF_CALLEE_FREAD) + ":piip"] = &fread_pad;
        return t;
    }();
    return m;
}

// A registered call site: its device record, landing pad, whether its
// device side copies objects back, and host stage times of timed calls.
struct CallSite {
    DCall dev;
    CallPad pad;
    bool copy_out;
    int64_t host_calls = 0;
    int64_t host_ns[3] = {0, 0, 0};  // decode, call, reply
};

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    gf_run_stats stats{};
};

struct gf_ctx {
    int device = 0;
    int num_cu = 0;
    std::string err;
    // resident workgroups of a per-region kernel, by (region kind, workgroup
    // size, rows per tile, prefetch)
    std::map<std::array<int, 4>, int> region_cap;

    Scratch scr{};
    void *d_scratch_lines = nullptr;

    // RPC
    RpcSlot *h_slots = nullptr;
    RpcSlot *d_slots = nullptr;
    uint64_t *d_ticket = nullptr;
    uint32_t nslots = 0;
    int64_t rpc_timeout_us = 0;
    uint64_t next_ticket = 0;
    std::mutex rpc_mu;
    std::vector<Format> formats;
    // general host calls: per-slot payloads (pinned), call-site table and
    // its device copy with the device-side stage counters
    char *h_payload = nullptr;
    char *d_payload = nullptr;
    uint32_t payload_bytes = 0;
    DCall *d_calls = nullptr;
    unsigned long long *d_call_stats = nullptr;
    std::vector<CallSite> calls;  // capacity GF_CALL_MAX_SITES, never reallocated
    heapdev::DHeap heap{};        // heap for GF_ARG_HEAPREF lookups (base NULL: none)
    bool capture = false;
    std::string captured;
    std::atomic<int64_t> serviced{0};
    std::thread server;
    std::atomic<bool> stop{false};

    hipStream_t capture_stream = nullptr;
    // kernel split: the run whose regions the main kernel requests by RPC
    // (valid while `active`), launched on split_stream
    hipStream_t split_stream = nullptr;
    struct {
        bool active = false;
        DProg p;
        gf_instance in;
        Tiling t;
        gf_launch l;
        bool has_l = false;
        int regions = 0, launches = 0, max_grid = 0;
    } split;
    std::unordered_map<std::string, GraphEntry> graphs;

    // batched persistent launches: device table, pinned staging, and an
    // event that marks when the staging buffer may be rewritten
    void *d_batch = nullptr;
    void *h_batch = nullptr;
    bool batch_align = true;  // keep each batched group on one XCD (GF_BATCH_ALIGN=0: lay groups out in order)
    uint32_t batch_check_epoch = 0;  // epoch of the last batched launch that checked placement (0: none)
    hipEvent_t batch_copied = nullptr;
    bool batch_pending = false;

    // Every enqueue shares the scratch above: work enqueued on a stream other
    // than the previous call's waits for the previous call's work first
    hipEvent_t last_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;

    // launches the autotuner chose when the predictor deferred, by program,
    // sizes, instance count and mode
    bool tune_fallback = true;
    struct Tuned {
        gf_launch launch;
        int32_t cand;
        std::vector<gf_launch> per;  // batched persistent runs: a shape per instance
    };
    std::unordered_map<std::string, Tuned> tuned;

    // set-up of gf_reduce_noalloc's static array on this device
    hipError_t noalloc_status = hipErrorNotInitialized;

    // predictor: device scratch for training, host copy for inference
    float *d_mlp = nullptr;       // gradient partials | grads | z1 | z2 | y | loss partials
    size_t d_mlp_floats = 0;
    std::vector<float> pred_params, pred_mean, pred_std;
};

constexpr size_t kBatchBytes = (size_t)4096 * sizeof(BatchEntry) + (size_t)GF_MAX_INSTANCES * sizeof(DInst);

namespace {

gf_status fail(gf_ctx *ctx, gf_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

gf_status hipfail(gf_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, GF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

RpcRing ring_of(const gf_ctx *ctx)
{
    RpcRing r;
    r.slots = ctx->d_slots;
    r.ticket = ctx->d_ticket;
    r.mask = ctx->nslots - 1;
    r.payload = ctx->payload_bytes;
    r.timeout_ticks = ctx->rpc_timeout_us * 100;  // s_memrealtime runs at 100 MHz
    r.payloads = ctx->d_payload;
    r.calls = ctx->d_calls;
    r.call_stats = ctx->d_call_stats;
    r.heap = ctx->heap;
    return r;
}

// Enqueues of one context are ordered even across streams, because they
// share the context's scratch (reduction partials, counter lines, the
// batched table, MLP buffers): before enqueueing on stream s, wait for the
// work the previous call enqueued if that was on another stream; afterwards
// mark the end of this call's work. Work enqueued while s is being captured
// into a graph by the caller is not tracked (an event recorded inside a
// capture cannot be waited on from outside it).
bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

gf_status order_before(gf_ctx *ctx, hipStream_t s)
{
    if (!ctx->have_last || s == ctx->last_stream || !ctx->last_done || capturing(s))
        return GF_OK;
    hipError_t e = hipStreamWaitEvent(s, ctx->last_done, 0);
    return e == hipSuccess ? GF_OK : hipfail(ctx, e, "stream wait on the previous call");
}

void mark_after(gf_ctx *ctx, hipStream_t s)
{
    if (!ctx->last_done || capturing(s))
        return;
    if (hipEventRecord(ctx->last_done, s) == hipSuccess) {
        ctx->last_stream = s;
        ctx->have_last = true;
    }
}

int64_t now_us()
{
    return std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t split_region(gf_ctx *ctx, int sidx, uint64_t perm);

// Service requests; caller holds rpc_mu.
int32_t poll_locked(gf_ctx *ctx, int32_t max_requests, int32_t timeout_us)
{
    int32_t done = 0;
    const int64_t deadline = now_us() + (timeout_us > 0 ? timeout_us : 0);
    char buf[1024];
    while (done < max_requests) {
        RpcSlot *slot = &ctx->h_slots[ctx->next_ticket & (ctx->nslots - 1)];
        const uint64_t seq = __atomic_load_n(&slot->seq, __ATOMIC_ACQUIRE);
        if (seq == ctx->next_ticket + 1) {
            int64_t ret = -1;
            bool device_frees = false;
            if (slot->callee == kCalleeCall && slot->fmt_id < ctx->calls.size()) {
                CallSite &cs = ctx->calls[slot->fmt_id];
                const bool timed = (slot->flags & GF_STEP_TIMED) != 0;
                const int64_t h0 = timed ? now_ns() : 0;
                // the device frees the slot itself after copying objects back
                device_frees = cs.copy_out && (slot->flags & GF_STEP_BLOCKING);
                if (slot->nargs == (uint32_t)cs.dev.nargs) {
                    char *pl = ctx->h_payload + (size_t)(ctx->next_ticket & (ctx->nslots - 1)) * ctx->payload_bytes;
                    uint64_t w[GF_CALL_MAX_ARGS];
                    for (int k = 0; k < cs.dev.nargs; ++k) {
                        const DCallArg &a = cs.dev.a[k];
                        if (a.kind == GF_ARG_REF) {
                            if (a.mode == GF_REF_WRITE)
                                std::memset(pl + a.pos, 0, (size_t)a.size);
                            w[k] = (uint64_t)(uintptr_t)(pl + a.pos + a.offset);
                        } else if (a.kind == GF_ARG_HEAPREF && !(slot->flags & (kHeapValueFlag0 << k))) {
                            // the heap found the object: {bytes << 32 | offset of the pointer}
                            const uint64_t bytes = slot->args[k] >> 32, off = slot->args[k] & 0xFFFFFFFFu;
                            if (a.mode == GF_REF_WRITE)
                                std::memset(pl + a.pos, 0, (size_t)bytes);
                            w[k] = (uint64_t)(uintptr_t)(pl + a.pos + off);
                        } else {
                            w[k] = slot->args[k];
                        }
                    }
                    const int64_t h1 = timed ? now_ns() : 0;
                    ret = cs.pad(w, ctx->capture ? &ctx->captured : nullptr);
                    const int64_t h2 = timed ? now_ns() : 0;
                    slot->ret = ret;
                    if (!device_frees)
                        __atomic_store_n(&slot->freed, ctx->next_ticket + 1, __ATOMIC_RELAXED);
                    __atomic_store_n(&slot->done, ctx->next_ticket + 1, __ATOMIC_RELEASE);
                    if (timed) {
                        const int64_t h3 = now_ns();
                        cs.host_calls += 1;
                        cs.host_ns[0] += h1 - h0;
                        cs.host_ns[1] += h2 - h1;
                        cs.host_ns[2] += h3 - h2;
                    }
                    ++ctx->next_ticket;
                    ++done;
                    ctx->serviced.fetch_add(1);
                    continue;
                }
            } else if (slot->callee == kCalleeRegion && slot->nargs == 3) {
                ret = split_region(ctx, (int)slot->args[0], slot->args[2]);
            } else if (slot->callee == kCalleePrintf && slot->fmt_id < ctx->formats.size()) {
                const Format &f = ctx->formats[slot->fmt_id];
                if (slot->nargs == f.sig.size()) {
                    int k = f.pad(buf, sizeof buf, f.fmt.c_str(), slot->args);
                    ret = k;
                    if (k > 0) {
                        const size_t len = std::min<size_t>((size_t)k, sizeof buf - 1);
                        if (ctx->capture) {
                            ctx->captured.append(buf, len);
                        } else {
                            std::fwrite(buf, 1, len, stdout);
                            std::fflush(stdout);
                        }
                    }
                }
            }
            slot->ret = ret;
            if (!device_frees)
                __atomic_store_n(&slot->freed, ctx->next_ticket + 1, __ATOMIC_RELAXED);
            __atomic_store_n(&slot->done, ctx->next_ticket + 1, __ATOMIC_RELEASE);
            ++ctx->next_ticket;
            ++done;
            ctx->serviced.fetch_add(1);
            continue;
        }
        if (done == 0 && now_us() < deadline) {
            std::this_thread::yield();
            continue;
        }
        break;
    }
    return done;
}

// After a device error, with no kernel of the device running: bring the
// ring back to a state the next run can use. A client takes its ticket
// before it waits for the slot to be freed; if that wait (or the wait for
// the reply) gave up, the ticket was never published, or its caller never
// freed the slot after copying back. Every request published in ticket order
// is serviced as usual; a ticket that was taken but never published is
// skipped (completed with return value -1, nothing run); finally each slot
// is marked free for the last ticket that used it, so that clients of later
// tickets do not wait for a caller that has gone.
void recover_ring(gf_ctx *ctx)
{
    uint64_t taken = 0;
    if (hipMemcpy(&taken, ctx->d_ticket, sizeof taken, hipMemcpyDeviceToHost) != hipSuccess)
        return;
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    while (ctx->next_ticket < taken) {
        if (poll_locked(ctx, 1 << 20, 0) > 0)
            continue;
        if (ctx->next_ticket >= taken)
            break;
        RpcSlot *slot = &ctx->h_slots[ctx->next_ticket & (ctx->nslots - 1)];
        slot->ret = -1;
        __atomic_store_n(&slot->freed, ctx->next_ticket + 1, __ATOMIC_RELAXED);
        __atomic_store_n(&slot->done, ctx->next_ticket + 1, __ATOMIC_RELEASE);
        ++ctx->next_ticket;
    }
    const uint64_t ns = ctx->nslots;
    for (uint64_t t = taken > ns ? taken - ns : 0; t < taken; ++t) {
        RpcSlot *slot = &ctx->h_slots[t & (ns - 1)];
        if (__atomic_load_n(&slot->freed, __ATOMIC_RELAXED) < t + 1)
            __atomic_store_n(&slot->freed, t + 1, __ATOMIC_RELEASE);
    }
}

}  // namespace

extern "C" {

gf_status gf_ctx_create(int32_t hip_device, const gf_ctx_opts *opts, gf_ctx **out)
{
    if (!out)
        return GF_EINVAL;
    *out = nullptr;
    gf_ctx *ctx = new (std::nothrow) gf_ctx();
    if (!ctx)
        return GF_ENOMEM;
    gf_ctx_opts o{};
    if (opts)
        o = *opts;
    hipError_t e = hipSetDevice(hip_device);
    if (e != hipSuccess) {
        delete ctx;
        return GF_EHIP;
    }
    ctx->device = hip_device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
        delete ctx;
        return GF_EHIP;
    }
    ctx->num_cu = prop.multiProcessorCount;
    // gf_reduce_noalloc's static array on this device: resolved once per
    // device here, so that the entry point itself allocates nothing
    ctx->noalloc_status = noalloc_setup(hip_device);

    // device scratch: partials (two halves), counter lines, error word
    const int64_t cap = 1 << 20;
    const size_t part_bytes = 2 * cap * sizeof(double);
    const size_t line_bytes = (size_t)kNumLines * 128;
    const size_t hist_bytes = (size_t)kHistRowsMax * 65536 * sizeof(uint16_t);
    const size_t total = part_bytes + line_bytes + 256 + hist_bytes;
    char *base = nullptr;
    if ((e = hipMalloc((void **)&base, total)) != hipSuccess) {
        delete ctx;
        return GF_ENOMEM;
    }
    ctx->d_scratch_lines = base;
    if ((e = hipMemset(base + part_bytes, 0, line_bytes + 256)) != hipSuccess) {
        hipFree(base);
        delete ctx;
        return GF_EHIP;
    }
    ctx->scr.partials = (double *)base;
    ctx->scr.partials_cap = cap;
    ctx->scr.lines = (uint32_t *)(base + part_bytes);
    ctx->scr.error = (int32_t *)(base + part_bytes + line_bytes);
    ctx->scr.hist_rows = (uint32_t *)(base + part_bytes + line_bytes + 256);
    const int64_t btus = o.barrier_timeout_us > 0 ? o.barrier_timeout_us : 10 * 1000 * 1000;
    ctx->scr.barrier_timeout_ticks = btus * 100;
    ctx->scr.epoch = 0;
    // XCD barrier by default; GF_BARRIER=tree selects the per-workgroup
    // publication of the tree barrier (for comparison)
    ctx->scr.barrier_kind = kBarrierXcd;
    if (const char *bk = std::getenv("GF_BARRIER"))
        ctx->scr.barrier_kind = std::strcmp(bk, "tree") == 0 ? kBarrierTree : kBarrierXcd;
    if (const char *ba = std::getenv("GF_BATCH_ALIGN"))
        ctx->batch_align = std::strcmp(ba, "0") != 0;

    // RPC ring
    uint32_t ns = o.rpc_slots > 0 ? (uint32_t)o.rpc_slots : 256u;
    if (ns < 8 || ns > 4096 || (ns & (ns - 1))) {
        hipFree(base);
        delete ctx;
        return GF_EINVAL;
    }
    ctx->nslots = ns;
    if ((e = hipHostMalloc((void **)&ctx->h_slots, ns * sizeof(RpcSlot), hipHostMallocCoherent | hipHostMallocMapped)) !=
        hipSuccess) {
        hipFree(base);
        delete ctx;
        return GF_ENOMEM;
    }
    std::memset(ctx->h_slots, 0, ns * sizeof(RpcSlot));
    if (hipHostGetDevicePointer((void **)&ctx->d_slots, ctx->h_slots, 0) != hipSuccess)
        ctx->d_slots = ctx->h_slots;
    // the ticket counter lives in the last scratch line (device memory)
    ctx->d_ticket = (uint64_t *)(base + part_bytes + line_bytes + 128);
    // payloads of general host calls, and the call-site table
    const int64_t pb = o.rpc_payload > 0 ? o.rpc_payload : 1024;
    if (pb < 16 || pb > 65536 || (pb & 15)) {
        gf_ctx_destroy(ctx);
        return GF_EINVAL;
    }
    ctx->payload_bytes = (uint32_t)pb;
    ctx->calls.reserve(GF_CALL_MAX_SITES);
    if (hipHostMalloc((void **)&ctx->h_payload, (size_t)ns * pb, hipHostMallocCoherent | hipHostMallocMapped) !=
            hipSuccess ||
        hipMalloc((void **)&ctx->d_calls,
                  GF_CALL_MAX_SITES * (sizeof(DCall) + kCallStatWords * sizeof(unsigned long long))) != hipSuccess) {
        gf_ctx_destroy(ctx);
        return GF_ENOMEM;
    }
    std::memset(ctx->h_payload, 0, (size_t)ns * pb);
    if (hipHostGetDevicePointer((void **)&ctx->d_payload, ctx->h_payload, 0) != hipSuccess)
        ctx->d_payload = ctx->h_payload;
    ctx->d_call_stats = (unsigned long long *)(ctx->d_calls + GF_CALL_MAX_SITES);
    if (hipMemset(ctx->d_calls, 0, GF_CALL_MAX_SITES * (sizeof(DCall) + kCallStatWords * sizeof(unsigned long long))) !=
        hipSuccess) {
        gf_ctx_destroy(ctx);
        return GF_EHIP;
    }
    ctx->rpc_timeout_us = o.rpc_timeout_us > 0 ? o.rpc_timeout_us : 2 * 1000 * 1000;
    ctx->tune_fallback = o.tune_fallback >= 0;
    ctx->capture = o.rpc_capture != 0;
    if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess)
        ctx->capture_stream = nullptr;
    if (hipStreamCreateWithFlags(&ctx->split_stream, hipStreamNonBlocking) != hipSuccess)
        ctx->split_stream = nullptr;
    if (hipMalloc(&ctx->d_batch, kBatchBytes) != hipSuccess ||
        hipHostMalloc(&ctx->h_batch, kBatchBytes, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->batch_copied, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->last_done, hipEventDisableTiming) != hipSuccess) {
        gf_ctx_destroy(ctx);
        return GF_ENOMEM;
    }
    if (o.rpc_thread) {
        // The server spins (yielding) for a while after the last request so a
        // burst of calls sees a PCIe round trip, not a sleep; after 2 ms of
        // silence it polls every 20 us (with a fine timer slack).
        ctx->server = std::thread([ctx] {
            prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
            int64_t last = now_us();
            while (!ctx->stop.load()) {
                int32_t k;
                {
                    std::lock_guard<std::mutex> g(ctx->rpc_mu);
                    k = poll_locked(ctx, 1 << 20, 0);
                }
                const int64_t t = now_us();
                if (k > 0)
                    last = t;
                else if (t - last < 2000)
                    std::this_thread::yield();
                else
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        });
    }
    *out = ctx;
    return GF_OK;
}

gf_status gf_ctx_destroy(gf_ctx *ctx)
{
    if (!ctx)
        return GF_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    if (ctx->server.joinable()) {
        ctx->stop.store(true);
        ctx->server.join();
    }
    for (auto &kv : ctx->graphs) {
        if (kv.second.exec)
            hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph)
            hipGraphDestroy(kv.second.graph);
    }
    if (ctx->capture_stream)
        hipStreamDestroy(ctx->capture_stream);
    if (ctx->split_stream)
        hipStreamDestroy(ctx->split_stream);
    if (ctx->batch_copied)
        hipEventDestroy(ctx->batch_copied);
    if (ctx->last_done)
        hipEventDestroy(ctx->last_done);
    if (ctx->h_batch)
        hipHostFree(ctx->h_batch);
    if (ctx->d_batch)
        hipFree(ctx->d_batch);
    if (ctx->h_slots)
        hipHostFree(ctx->h_slots);
    if (ctx->h_payload)
        hipHostFree(ctx->h_payload);
    if (ctx->d_calls)
        hipFree(ctx->d_calls);
    if (ctx->d_scratch_lines)
        hipFree(ctx->d_scratch_lines);
    if (ctx->d_mlp)
        hipFree(ctx->d_mlp);
    delete ctx;
    return GF_OK;
}

const char *gf_last_error(const gf_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

int32_t gf_rpc_register_format(gf_ctx *ctx, const char *fmt, const char *sig)
{
    if (!ctx || !fmt || !sig)
        return GF_EINVAL;
    auto it = printf_pads().find(sig);
    if (it == printf_pads().end())
        return fail(ctx, GF_EINVAL, "unsupported printf signature '%s' (up to 4 of 'i'/'d')", sig);
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    ctx->formats.push_back(Format{fmt, sig, it->second});
    return (int32_t)ctx->formats.size() - 1;
}

gf_status gf_ctx_set_heap(gf_ctx *ctx, gf_heap *heap)
{
    if (!ctx)
        return GF_EINVAL;
    heapdev::DHeap d{};
    if (heap && !heapdev::heap_view(heap, &d))
        return fail(ctx, GF_EINVAL, "a vendor heap keeps no record of its objects");
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    ctx->heap = d;
    return GF_OK;
}

int32_t gf_rpc_register_call(gf_ctx *ctx, int32_t callee, const gf_call_arg *args, int32_t nargs)
{
    if (!ctx)
        return GF_EINVAL;
    if (nargs < 0 || nargs > GF_CALL_MAX_ARGS || (nargs > 0 && !args))
        return fail(ctx, GF_EINVAL, "call site needs 0..%d argument records", GF_CALL_MAX_ARGS);
    if (callee < GF_CALLEE_FPRINTF || callee > GF_CALLEE_FREAD)
        return fail(ctx, GF_EINVAL, "unknown callee %d", callee);
    DCall d;
    std::memset(&d, 0, sizeof d);
    d.callee = callee;
    d.nargs = nargs;
    std::string sig;
    int64_t pos = 0;
    bool copy_out = false;
    for (int k = 0; k < nargs; ++k) {
        const gf_call_arg &a = args[k];
        DCallArg &o = d.a[k];
        o.kind = a.kind;
        o.type = a.type;
        o.slot = a.slot;
        o.mode = a.mode;
        o.value = a.value;
        o.ref = -1;
        switch (a.kind) {
        case GF_ARG_CONST:
            if (a.type != 'i' && a.type != 'd' && a.type != 'p')
                return fail(ctx, GF_EINVAL, "argument %d: type must be 'i', 'd' or 'p'", k);
            break;
        case GF_ARG_SCALAR:
            if (a.type != 'i' && a.type != 'd')
                return fail(ctx, GF_EINVAL, "argument %d: a scalar passes as 'i' or 'd'", k);
            if (a.slot < 0 || a.slot >= GF_MAX_SCALARS)
                return fail(ctx, GF_EINVAL, "argument %d: scalar slot out of range", k);
            break;
        case GF_ARG_ITER:
            if (a.type != 'i')
                return fail(ctx, GF_EINVAL, "argument %d: the iteration number passes as 'i'", k);
            break;
        case GF_ARG_HEAPREF:
            if (a.type != 'p')
                return fail(ctx, GF_EINVAL, "argument %d: a reference passes as 'p'", k);
            if (a.slot < 0 || a.slot >= GF_MAX_ARRAYS)
                return fail(ctx, GF_EINVAL, "argument %d: array slot out of range", k);
            if (a.mode < GF_REF_READ || a.mode > GF_REF_READWRITE)
                return fail(ctx, GF_EINVAL, "argument %d: access mode must be read, write or read-write", k);
            if (a.size < 16 || a.start < 0)
                return fail(ctx, GF_EINVAL, "argument %d: heap reference needs size >= 16 and start >= 0", k);
            if (d.nrefs == GF_CALL_MAX_REFS)
                return fail(ctx, GF_EINVAL, "more than %d reference arguments", GF_CALL_MAX_REFS);
            o.start = a.start;
            o.size = (a.size + 15) / 16 * 16;
            o.offset = 0;
            o.pos = (int32_t)pos;
            o.ref = d.nrefs++;
            pos += o.size;
            if (pos > (int64_t)ctx->payload_bytes)
                return fail(ctx, GF_EINVAL, "referenced objects need %lld payload bytes; the slot payload is %u",
                            (long long)pos, ctx->payload_bytes);
            copy_out |= (a.mode & GF_REF_WRITE) != 0;
            break;
        case GF_ARG_REF:
            if (a.type != 'p')
                return fail(ctx, GF_EINVAL, "argument %d: a reference passes as 'p'", k);
            if (a.slot < 0 || a.slot >= GF_MAX_ARRAYS)
                return fail(ctx, GF_EINVAL, "argument %d: array slot out of range", k);
            if (a.mode < GF_REF_READ || a.mode > GF_REF_READWRITE)
                return fail(ctx, GF_EINVAL, "argument %d: access mode must be read, write or read-write", k);
            if (a.size < 1 || a.start < 0 || a.offset < 0 || a.offset > a.size)
                return fail(ctx, GF_EINVAL, "argument %d: object needs size >= 1, start >= 0, 0 <= offset <= size", k);
            if (d.nrefs == GF_CALL_MAX_REFS)
                return fail(ctx, GF_EINVAL, "more than %d reference arguments", GF_CALL_MAX_REFS);
            o.start = a.start;
            o.size = a.size;
            o.offset = a.offset;
            o.pos = (int32_t)pos;
            o.ref = d.nrefs++;
            pos += (a.size + 15) / 16 * 16;
            if (pos > (int64_t)ctx->payload_bytes)
                return fail(ctx, GF_EINVAL, "referenced objects need %lld payload bytes; the slot payload is %u",
                            (long long)pos, ctx->payload_bytes);
            copy_out |= (a.mode & GF_REF_WRITE) != 0;
            break;
        default:
            return fail(ctx, GF_EINVAL, "argument %d: unknown kind %d", k, a.kind);
        }
        sig.push_back((char)a.type);
    }
    d.payload = (int32_t)pos;
    auto it = call_pads().find(std::to_string(callee) + ":" + sig);
    if (it == call_pads().end())
        return fail(ctx, GF_EUNSUPPORTED, "no landing pad for callee %d with argument types '%s'", callee,
                    sig.c_str());
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    if ((int)ctx->calls.size() == GF_CALL_MAX_SITES)
        return fail(ctx, GF_EINVAL, "at most %d call sites", GF_CALL_MAX_SITES);
    const int id = (int)ctx->calls.size();
    hipSetDevice(ctx->device);
    hipError_t e = hipMemcpy(ctx->d_calls + id, &d, sizeof d, hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return hipfail(ctx, e, "call-site upload");
    CallSite cs;
    cs.dev = d;
    cs.pad = it->second;
    cs.copy_out = copy_out;
    ctx->calls.push_back(cs);
    return id;
}

gf_status gf_rpc_call_stats(gf_ctx *ctx, int32_t call_id, gf_call_stats *out, int32_t reset)
{
    if (!ctx || !out)
        return GF_EINVAL;
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    if (call_id < 0 || call_id >= (int)ctx->calls.size())
        return fail(ctx, GF_EINVAL, "unknown call site %d", call_id);
    hipSetDevice(ctx->device);
    unsigned long long dev[kCallStatWords];
    unsigned long long *dptr = ctx->d_call_stats + (int64_t)call_id * kCallStatWords;
    hipError_t e = hipMemcpy(dev, dptr, sizeof dev, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hipfail(ctx, e, "call statistics");
    CallSite &cs = ctx->calls[call_id];
    std::memset(out, 0, sizeof *out);
    out->calls = (int64_t)dev[0];
    if (dev[0] > 0) {
        const double per = 0.01 / (double)dev[0];  // 100 MHz ticks -> us per call
        out->dev_args_us = (double)dev[1] * per;
        out->dev_copy_in_us = (double)dev[2] * per;
        out->dev_wait_us = (double)dev[3] * per;
        out->dev_copy_out_us = (double)dev[4] * per;
    }
    if (cs.host_calls > 0) {
        const double per = 1e-3 / (double)cs.host_calls;
        out->host_decode_us = (double)cs.host_ns[0] * per;
        out->host_call_us = (double)cs.host_ns[1] * per;
        out->host_reply_us = (double)cs.host_ns[2] * per;
    }
    out->transit_us = out->dev_wait_us - (out->host_decode_us + out->host_call_us + out->host_reply_us);
    if (reset) {
        if ((e = hipMemset(dptr, 0, sizeof dev)) != hipSuccess)
            return hipfail(ctx, e, "call statistics reset");
        cs.host_calls = 0;
        cs.host_ns[0] = cs.host_ns[1] = cs.host_ns[2] = 0;
    }
    return GF_OK;
}

int32_t gf_rpc_poll(gf_ctx *ctx, int32_t max_requests, int32_t timeout_us)
{
    if (!ctx || max_requests < 0)
        return GF_EINVAL;
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    return poll_locked(ctx, max_requests, timeout_us);
}

int64_t gf_rpc_take_output(gf_ctx *ctx, char *buf, int64_t cap)
{
    if (!ctx || !buf || cap <= 0)
        return GF_EINVAL;
    std::lock_guard<std::mutex> g(ctx->rpc_mu);
    const int64_t n = std::min<int64_t>((int64_t)ctx->captured.size(), cap - 1);
    std::memcpy(buf, ctx->captured.data(), (size_t)n);
    buf[n] = '\0';
    ctx->captured.erase(0, (size_t)n);
    return n;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Program validation and tiling
// ---------------------------------------------------------------------------

namespace {

bool is_region(int k) { return k >= GF_R_JACOBI2D && k <= GF_R_PHASES; }
bool is_serial(int k) { return k >= GF_S_SET && k <= GF_S_CALL; }

int region_nops(int k)
{
    switch (k) {
    case GF_R_JACOBI2D:
    case GF_R_JACOBI3D:
        return 2;
    case GF_R_SPMV:
        return 5;
    case GF_R_DOT:
        return 2;
    case GF_R_AXPBY:
        return 3;
    case GF_R_HIST:
        return 2;
    case GF_R_OWNER:
        return 1;
    case GF_R_PHASES:
        return 3;  // the owner map (operand 2) is optional
    default:
        return 0;
    }
}

// An operand a region may leave unbound (-1).
bool optional_operand(int kind, int k) { return kind == GF_R_PHASES && k == 2; }

gf_status check_step(gf_ctx *ctx, const gf_step &s, int idx)
{
    auto slot_ok = [](int a) { return a >= 0 && a < GF_MAX_ARRAYS; };
    auto sc_ok = [](int a) { return a >= 0 && a < GF_MAX_SCALARS; };
    if (is_region(s.kind)) {
        for (int k = 0; k < region_nops(s.kind); ++k)
            if (!slot_ok(s.arr[k]) && !(optional_operand(s.kind, k) && s.arr[k] == -1))
                return fail(ctx, GF_EINVAL, "step %d: array operand %d out of range", idx, k);
        if (s.np < 0 || s.np >= GF_MAX_IPARAMS)
            return fail(ctx, GF_EINVAL, "step %d: size index out of range", idx);
        int allowed = GF_OP_NONE;
        if (s.kind == GF_R_JACOBI2D || s.kind == GF_R_DOT)
            allowed = GF_OP_SUM;
        if (s.kind == GF_R_JACOBI3D)
            allowed = GF_OP_MAX;
        if (s.red_op != GF_OP_NONE && s.red_op != allowed)
            return fail(ctx, GF_EINVAL, "step %d: reduction op %d not defined for region kind %d", idx, s.red_op,
                        s.kind);
        if (s.kind == GF_R_DOT && s.red_op == GF_OP_NONE)
            return fail(ctx, GF_EINVAL, "step %d: DOT needs reduction(+)", idx);
        if (s.red_op != GF_OP_NONE && !sc_ok(s.sc[0]))
            return fail(ctx, GF_EINVAL, "step %d: reduction target out of range", idx);
        if (s.kind == GF_R_AXPBY && !sc_ok(s.sc[1]))
            return fail(ctx, GF_EINVAL, "step %d: AXPBY coefficient slot out of range", idx);
        if (s.kind == GF_R_HIST && ((s.mask & (s.mask + 1u)) != 0 || s.mask >= (1u << 20)))
            return fail(ctx, GF_EINVAL, "step %d: histogram mask must be 2^k - 1 with at most 2^20 bins", idx);
        if (s.kind == GF_R_OWNER && s.chunk < 0)
            return fail(ctx, GF_EINVAL, "step %d: negative chunk", idx);
        if (s.kind == GF_R_PHASES && (s.chunk < 1 || s.chunk > (1 << 20)))
            return fail(ctx, GF_EINVAL, "step %d: phase count must be 1 .. 2^20", idx);
        if (s.kind == GF_R_PHASES && (s.arr[0] == s.arr[1] || s.arr[2] == s.arr[0] || s.arr[2] == s.arr[1]))
            return fail(ctx, GF_EINVAL, "step %d: the two phase buffers and the owner map must be distinct slots",
                        idx);
        if (s.flags & ~GF_STEP_NOWAIT)
            return fail(ctx, GF_EINVAL, "step %d: a region takes only the nowait flag", idx);
        if ((s.flags & GF_STEP_NOWAIT) && s.red_op != GF_OP_NONE)
            return fail(ctx, GF_EINVAL, "step %d: nowait with a reduction clause (its value needs the barrier)", idx);
        if ((s.flags & GF_STEP_NOWAIT) && (s.kind == GF_R_HIST || s.kind == GF_R_PHASES))
            return fail(ctx, GF_EINVAL, "step %d: nowait on a region with barriers inside it", idx);
        return GF_OK;
    }
    if (!is_serial(s.kind))
        return fail(ctx, GF_EINVAL, "step %d: unknown kind %d", idx, s.kind);
    switch (s.kind) {
    case GF_S_SET:
        if (!sc_ok(s.sc[0]))
            return fail(ctx, GF_EINVAL, "step %d: scalar slot out of range", idx);
        break;
    case GF_S_COPY:
    case GF_S_SQRT:
        if (!sc_ok(s.sc[0]) || !sc_ok(s.sc[1]))
            return fail(ctx, GF_EINVAL, "step %d: scalar slot out of range", idx);
        break;
    case GF_S_DIV:
        if (!sc_ok(s.sc[0]) || !sc_ok(s.sc[1]) || !sc_ok(s.sc[2]))
            return fail(ctx, GF_EINVAL, "step %d: scalar slot out of range", idx);
        break;
    case GF_S_SWAP:
        if (!slot_ok(s.arr[0]) || !slot_ok(s.arr[1]))
            return fail(ctx, GF_EINVAL, "step %d: swap slot out of range", idx);
        break;
    case GF_S_RECORD:
        if (!slot_ok(s.arr[0]) || !sc_ok(s.sc[0]))
            return fail(ctx, GF_EINVAL, "step %d: record operand out of range", idx);
        break;
    case GF_S_PRINTF: {
        if (s.every < 1 || s.nargs < 1 || s.nargs > 4)
            return fail(ctx, GF_EINVAL, "step %d: printf needs every >= 1 and 1..4 arguments", idx);
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        if (s.fmt_id < 0 || s.fmt_id >= (int)ctx->formats.size())
            return fail(ctx, GF_EINVAL, "step %d: unregistered format id %d", idx, s.fmt_id);
        const std::string &sig = ctx->formats[s.fmt_id].sig;
        if ((int)sig.size() != s.nargs || sig[0] != 'i')
            return fail(ctx, GF_EINVAL, "step %d: format signature '%s' does not match (int iter, %d doubles)", idx,
                        sig.c_str(), s.nargs - 1);
        for (size_t k = 1; k < sig.size(); ++k)
            if (sig[k] != 'd' || !sc_ok(s.sc[k - 1]))
                return fail(ctx, GF_EINVAL, "step %d: printf argument %zu must be a scalar variable", idx, k);
        break;
    }
    case GF_S_CALL: {
        if (s.every < 1)
            return fail(ctx, GF_EINVAL, "step %d: call needs every >= 1", idx);
        if (s.sc[0] != -1 && !sc_ok(s.sc[0]))
            return fail(ctx, GF_EINVAL, "step %d: return slot out of range", idx);
        if (s.flags & ~(GF_STEP_BLOCKING | GF_STEP_TIMED))
            return fail(ctx, GF_EINVAL, "step %d: unknown flags 0x%x", idx, s.flags);
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        if (s.fmt_id < 0 || s.fmt_id >= (int)ctx->calls.size())
            return fail(ctx, GF_EINVAL, "step %d: unregistered call site %d", idx, s.fmt_id);
        if (!(s.flags & GF_STEP_BLOCKING) && (ctx->calls[s.fmt_id].copy_out || s.sc[0] >= 0))
            return fail(ctx, GF_EINVAL, "step %d: a call that copies objects back or returns a value must be blocking",
                        idx);
        break;
    }
    default:
        break;
    }
    return GF_OK;
}

DStep to_dev(const gf_step &s)
{
    DStep d;
    std::memset(&d, 0, sizeof d);
    d.kind = s.kind;
    for (int k = 0; k < 5; ++k)
        d.arr[k] = s.arr[k];
    for (int k = 0; k < 3; ++k)
        d.sc[k] = s.sc[k];
    d.red_op = is_region(s.kind) ? s.red_op : GF_OP_NONE;
    d.np = s.np;
    d.every = s.every;
    d.fmt_id = s.fmt_id;
    d.nargs = s.nargs;
    d.flags = s.flags;
    d.mask = s.mask;
    d.chunk = s.chunk;
    d.c = s.c;
    // operands a kind does not use are marked absent
    if (is_region(s.kind))
        for (int k = region_nops(s.kind); k < 5; ++k)
            d.arr[k] = -1;
    return d;
}

unsigned program_region_mask(const DProg &p)
{
    unsigned m = 0;
    for (int i = 0; i < p.n_steps; ++i)
        if (is_region(p.steps[i].kind))
            m |= 1u << p.steps[i].kind;
    return m;
}

// Defaults: 3D stencil 256-wide rows x 8 rows x 64-plane segments; 2D
// stencil single-row tiles (the 2D grid is small and latency-bound);
// streaming regions 4 elements per thread.
Tiling choose_tiling(const DProg &p, const gf_launch *l)
{
    Tiling t;
    std::memset(&t, 0, sizeof t);
    const unsigned m = program_region_mask(p);
    t.wg_size = program_is_hist_family(p) ? 1024 : 256;
    if (program_is_hist_family(p))
        t.items = 8;
    t.tile_y = (m & (1u << GF_R_JACOBI3D)) ? 8 : ((m & (1u << GF_R_JACOBI2D)) ? 16 : 1);
    t.tile_z = 64;
    t.prefetch = 1;
    if (!program_is_hist_family(p))
        t.items = 4;
    t.xcd_remap = 1;
    if (l) {
        if (l->wg_size)
            t.wg_size = l->wg_size;
        if (l->tile_y)
            t.tile_y = l->tile_y;
        if (l->tile_z)
            t.tile_z = l->tile_z;
        if (l->items)
            t.items = l->items;
        t.xcd_remap = l->xcd_remap;
        if (l->prefetch)
            t.prefetch = l->prefetch;
    }
    return t;
}

gf_status check_tiling(gf_ctx *ctx, const DProg &p, const Tiling &t)
{
    const int maxwg = program_is_hist_family(p) ? 1024 : 256;
    if (t.wg_size < 64 || t.wg_size > maxwg || (t.wg_size % 64))
        return fail(ctx, GF_EINVAL, "wg_size must be a multiple of 64 in [64, %d]", maxwg);
    // the 3D stencil keeps tile_y rows per thread in registers (compiled for
    // five heights); the 2D stencil marches segments of any length
    if ((program_region_mask(p) & (1u << GF_R_JACOBI3D)) &&
        !(t.tile_y == 1 || t.tile_y == 2 || t.tile_y == 4 || t.tile_y == 8 || t.tile_y == 16))
        return fail(ctx, GF_EINVAL, "tile_y must be 1, 2, 4, 8 or 16");
    if (t.tile_y < 1 || t.tile_y > 1 << 20)
        return fail(ctx, GF_EINVAL, "tile_y out of range");
    if (t.tile_z < 1 || t.tile_z > 1 << 20)
        return fail(ctx, GF_EINVAL, "tile_z out of range");
    if (t.items < 1 || t.items > 64)
        return fail(ctx, GF_EINVAL, "items must be 1..64");
    if (t.prefetch != 1 && t.prefetch != 2)
        return fail(ctx, GF_EINVAL, "prefetch must be 1 or 2");
    if (t.prefetch == 2 && t.tile_y > 8)
        return fail(ctx, GF_EINVAL, "prefetch 2 needs tile_y <= 8");
    if (program_is_hist_family(p) && !(t.items == 1 || t.items == 2 || t.items == 4 || t.items == 8))
        return fail(ctx, GF_EINVAL, "histogram items must be 1, 2, 4 or 8");
    if (program_is_hist_family(p) && (int64_t)t.wg_size * t.items * 4 > 32768)
        return fail(ctx, GF_EINVAL, "histogram chunks hold at most 32768 keys (wg_size * items * 4)");
    return GF_OK;
}

gf_status build_program(gf_ctx *ctx, const gf_program *prog, DProg *out)
{
    if (!prog)
        return fail(ctx, GF_EINVAL, "null program");
    if (prog->n_prologue < 0 || prog->n_body < 0 || prog->iters < 0)
        return fail(ctx, GF_EINVAL, "negative program counts");
    if (prog->n_prologue + prog->n_body > kMaxDevSteps)
        return fail(ctx, GF_EINVAL, "program has %d steps; at most %d", prog->n_prologue + prog->n_body,
                    kMaxDevSteps);
    if ((prog->n_prologue && !prog->prologue) || (prog->n_body && !prog->body))
        return fail(ctx, GF_EINVAL, "null step array");
    if (prog->iters > 0 && prog->n_body == 0)
        return fail(ctx, GF_EINVAL, "iters > 0 with an empty body");
    std::memset(out, 0, sizeof *out);
    out->n_pro = prog->n_prologue;
    out->n_body = prog->n_body;
    out->iters = prog->iters;
    out->n_steps = prog->n_prologue + prog->n_body;
    for (int i = 0; i < out->n_steps; ++i) {
        const gf_step &s = i < prog->n_prologue ? prog->prologue[i] : prog->body[i - prog->n_prologue];
        gf_status st = check_step(ctx, s, i);
        if (st != GF_OK)
            return st;
        out->steps[i] = to_dev(s);
    }
    if (program_mixes_hist(*out))
        return fail(ctx, GF_EUNSUPPORTED, "a histogram region can only share a program with schedule regions");
    // a host call with references between a nowait region and the next
    // region would copy in data that other workgroups may still be writing.
    // Steps are walked in execution order, the body taken as repeating.
    auto next_step = [&](int j) -> int {
        if (j + 1 < out->n_steps)
            return (j + 1 == out->n_pro && out->iters == 0) ? -1 : j + 1;
        return (out->n_body > 0 && out->iters > 0) ? out->n_pro : -1;
    };
    for (int i = 0; i < out->n_steps; ++i) {
        if (!is_region(out->steps[i].kind) || !(out->steps[i].flags & GF_STEP_NOWAIT))
            continue;
        int j = next_step(i);
        for (int guard = 0; j >= 0 && guard < out->n_steps && !is_region(out->steps[j].kind);
             ++guard, j = next_step(j))
            if (out->steps[j].kind == GF_S_CALL) {
                std::lock_guard<std::mutex> g(ctx->rpc_mu);
                if (ctx->calls[out->steps[j].fmt_id].dev.nrefs > 0)
                    return fail(ctx, GF_EINVAL, "step %d: a host call with references (step %d) follows a nowait "
                                "region before the next region", i, j);
            }
    }
    // last region in execution order and the number of grid barriers
    out->last_region = -1;
    int64_t bar_pro = 0, bar_body = 0;
    for (int i = 0; i < out->n_steps; ++i) {
        if (!is_region(out->steps[i].kind))
            continue;
        // a histogram region has one barrier inside it, a phase region one
        // between consecutive phases
        int64_t b = (out->steps[i].flags & GF_STEP_NOWAIT) ? 0 : 1;
        if (out->steps[i].kind == GF_R_HIST)
            b = 2;
        else if (out->steps[i].kind == GF_R_PHASES)
            b = out->steps[i].chunk;
        if (i < out->n_pro) {
            bar_pro += b;
            out->last_region = i;
        } else {
            bar_body += b;
        }
    }
    if (out->iters > 0)
        for (int i = out->n_pro; i < out->n_steps; ++i)
            if (is_region(out->steps[i].kind))
                out->last_region = (int64_t)out->n_pro + (int64_t)(out->iters - 1) * out->n_body + (i - out->n_pro);
    out->barriers = bar_pro + bar_body * out->iters;
    if (out->last_region >= 0) {
        // the persistent kernel skips the barrier after the last region
        // when that region has no reduction (a nowait region was not
        // counted)
        const int64_t lr = out->last_region;
        const int si = lr < out->n_pro ? (int)lr : out->n_pro + (int)((lr - out->n_pro) % out->n_body);
        if (out->steps[si].red_op == GF_OP_NONE && !(out->steps[si].flags & GF_STEP_NOWAIT))
            out->barriers -= 1;
    }
    // host calls: a grid barrier after each call that fires; a call that
    // reads objects may follow the last region, so every region keeps its
    // barrier
    bool call_refs = false;
    for (int i = 0; i < out->n_steps; ++i) {
        const DStep &st = out->steps[i];
        if (st.kind != GF_S_CALL)
            continue;
        out->barriers += i < out->n_pro ? 1 : (int64_t)(out->iters / st.every);
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        call_refs |= ctx->calls[st.fmt_id].dev.nrefs > 0;
    }
    if (call_refs && out->last_region >= 0) {
        const int64_t lr = out->last_region;
        const int si = lr < out->n_pro ? (int)lr : out->n_pro + (int)((lr - out->n_pro) % out->n_body);
        if (out->steps[si].red_op == GF_OP_NONE && !(out->steps[si].flags & GF_STEP_NOWAIT))
            out->barriers += 1;
        out->last_region = -1;
    }
    return GF_OK;
}

gf_status check_instance(gf_ctx *ctx, const DProg &p, const gf_instance &in, const Tiling &t, int idx)
{
    if (!in.scal)
        return fail(ctx, GF_EINVAL, "instance %d: null scalar array", idx);
    for (int i = 0; i < p.n_steps; ++i) {
        const DStep &s = p.steps[i];
        if (s.kind == GF_S_CALL) {
            std::lock_guard<std::mutex> g(ctx->rpc_mu);
            const DCall &c = ctx->calls[s.fmt_id].dev;
            for (int k = 0; k < c.nargs; ++k)
                if ((c.a[k].kind == GF_ARG_REF || c.a[k].kind == GF_ARG_HEAPREF) && !in.arr[c.a[k].slot])
                    return fail(ctx, GF_EINVAL, "instance %d step %d: call references empty array slot %d", idx, i,
                                c.a[k].slot);
            continue;
        }
        if (is_region(s.kind)) {
            for (int k = 0; k < region_nops(s.kind); ++k)
                if (s.arr[k] >= 0 && !in.arr[s.arr[k]])
                    return fail(ctx, GF_EINVAL, "instance %d step %d: null array in slot %d", idx, i, s.arr[k]);
            const int64_t n = in.ip[s.np];
            if (n < 0)
                return fail(ctx, GF_EINVAL, "instance %d step %d: negative size", idx, i);
            if ((s.kind == GF_R_JACOBI2D || s.kind == GF_R_JACOBI3D) && n > (1 << 20))
                return fail(ctx, GF_EINVAL, "instance %d step %d: grid side too large", idx, i);
            if (s.kind == GF_R_HIST && ((uintptr_t)in.arr[s.arr[0]] % 16) != 0)
                return fail(ctx, GF_EINVAL, "instance %d step %d: histogram keys must be 16-byte aligned", idx, i);
            if (s.kind == GF_R_OWNER && n > INT32_MAX)
                return fail(ctx, GF_EINVAL, "instance %d step %d: owner map larger than int32", idx, i);
            if (s.kind == GF_R_PHASES && n > 0 && (int64_t)s.mask >= n)
                return fail(ctx, GF_EINVAL, "instance %d step %d: phase shift %u must be below n = %lld", idx, i,
                            s.mask, (long long)n);
            if (s.kind == GF_R_PHASES && s.arr[2] >= 0 && n > INT32_MAX)
                return fail(ctx, GF_EINVAL, "instance %d step %d: owner map larger than int32", idx, i);
            if (s.red_op != GF_OP_NONE && region_items(s, n, t) > ctx->scr.partials_cap)
                return fail(ctx, GF_EINVAL, "instance %d step %d: %lld reduction tiles exceed the partials capacity",
                            idx, i, (long long)region_items(s, n, t));
        } else if (s.kind == GF_S_SWAP || s.kind == GF_S_RECORD) {
            if (!in.arr[s.arr[0]] || (s.kind == GF_S_SWAP && !in.arr[s.arr[1]]))
                return fail(ctx, GF_EINVAL, "instance %d step %d: null array slot", idx, i);
        }
    }
    return GF_OK;
}

int64_t max_items(const DProg &p, const gf_instance &in, const Tiling &t)
{
    int64_t m = 1;
    for (int i = 0; i < p.n_steps; ++i)
        if (is_region(p.steps[i].kind))
            m = std::max<int64_t>(m, region_items(p.steps[i], in.ip[p.steps[i].np], t));
    return m;
}

// Grid of a per-region launch: one workgroup per work item up to 16 per CU;
// SpMV, which is latency-bound and holds an LDS tile per workgroup, at most
// one resident round (CG at 128^3: 122 ms per 500 iterations with 1,280
// workgroups, five per CU, against 133 ms with 4,096 in rounds).
// Histogram grid: a multiple of the bin-part count, at most kHistRowsMax.
int hist_grid(int64_t want, uint32_t mask)
{
    const int64_t parts = hist_parts(mask);
    int64_t g = std::min<int64_t>(want, kHistRowsMax);
    g -= g % parts;
    return (int)std::max<int64_t>(g, parts);
}

int region_grid(gf_ctx *ctx, const DStep &s, int64_t items, const Tiling &t)
{
    if (s.kind == GF_R_OWNER)
        return std::max(1, ctx->num_cu);
    if (s.kind == GF_R_PHASES)
        return std::max(1, std::min(ctx->num_cu, phases_capacity(t.wg_size, ctx->num_cu)));
    if (s.kind == GF_R_HIST)
        return hist_grid(std::min<int64_t>(std::max<int64_t>(items, 1), (int64_t)ctx->num_cu * 2), s.mask);
    int64_t cap = (int64_t)ctx->num_cu * 16;
    if (s.kind == GF_R_SPMV) {
        const std::array<int, 4> key{s.kind, t.wg_size, t.tile_y, t.prefetch};
        auto it = ctx->region_cap.find(key);
        if (it == ctx->region_cap.end())
            it = ctx->region_cap.emplace(key, region_capacity(s.kind, t, ctx->num_cu)).first;
        if (it->second > 0)
            cap = it->second;
    }
    return (int)std::max<int64_t>(1, std::min<int64_t>(items, cap));
}

// Walk the flattened step sequence of one instance, enqueueing one launch per
// region; the serial steps that follow a region ride along as its glue (run
// by its last workgroup); SWAPs are applied to the host's binding table.
// Enqueue one region launch (a histogram region is two launches: counting,
// then the merge that also runs the glue) with the per-region grid.
gf_status launch_one(gf_ctx *ctx, const RegionLaunch &cur, const Tiling &t, const gf_launch *l, hipStream_t stream,
                     int *launches, int *max_grid)
{
    const RpcRing rpc = ring_of(ctx);
    int grid = 1;
    if (is_region(cur.step.kind)) {
        grid = region_grid(ctx, cur.step, cur.n_items, t);
        if (l && l->num_wg > 0)
            grid = cur.step.kind == GF_R_HIST ? hist_grid(l->num_wg, cur.step.mask) : l->num_wg;
    }
    if (cur.step.kind == GF_R_PHASES) {
        // every workgroup must be resident for the in-region barrier
        const int cap = phases_capacity(t.wg_size, ctx->num_cu);
        if (cap < 1)
            return fail(ctx, GF_EHIP, "phase region: no co-resident capacity");
        grid = std::max(1, std::min(grid, cap));
        hipError_t e = launch_phases(cur, t.wg_size, grid, ctx->scr, rpc, stream);
        if (e != hipSuccess)
            return hipfail(ctx, e, "phase region launch");
        *launches += 1;
    } else if (cur.step.kind == GF_R_HIST) {
        RegionLaunch p1 = cur;
        p1.n_glue = 0;
        hipError_t e = launch_region(p1, t, grid, ctx->scr, rpc, stream);
        if (e == hipSuccess)
            e = launch_hist_merge(cur, grid, ctx->scr, rpc, ctx->num_cu, stream);
        if (e != hipSuccess)
            return hipfail(ctx, e, "histogram launch");
        *launches += 2;
    } else {
        hipError_t e = launch_region(cur, t, grid, ctx->scr, rpc, stream);
        if (e != hipSuccess)
            return hipfail(ctx, e, "region launch");
        *launches += 1;
    }
    *max_grid = std::max(*max_grid, grid);
    return GF_OK;
}

// Kernel split: launch region step `sidx` of the active run for the main
// kernel, with the array slots permuted by `perm` (4 bits per slot), and
// wait for it. Returns 0, or -1 if nothing could be launched. Runs on the
// thread that polls the RPC ring (rpc_mu held).
int64_t split_region(gf_ctx *ctx, int sidx, uint64_t perm)
{
    auto &sp = ctx->split;
    if (!sp.active || sidx < 0 || sidx >= sp.p.n_steps || !is_region(sp.p.steps[sidx].kind) || !ctx->split_stream)
        return -1;
    const DStep &s = sp.p.steps[sidx];
    RegionLaunch cur;
    std::memset(&cur, 0, sizeof cur);
    cur.step = s;
    for (int k = 0; k < 5; ++k)
        cur.arr[k] = s.arr[k] >= 0 ? sp.in.arr[(perm >> (4 * s.arr[k])) & 15u] : nullptr;
    cur.scal = sp.in.scal;
    cur.n = sp.in.ip[s.np];
    cur.n_items = (int32_t)region_items(s, cur.n, sp.t);
    cur.inst = 0;

    if (launch_one(ctx, cur, sp.t, sp.has_l ? &sp.l : nullptr, ctx->split_stream, &sp.launches, &sp.max_grid) !=
        GF_OK)
        return -1;
    if (hipStreamSynchronize(ctx->split_stream) != hipSuccess)
        return -1;
    sp.regions += 1;
    return 0;
}

gf_status enqueue_per_region(gf_ctx *ctx, const DProg &p, const gf_instance &in, int inst_idx, const Tiling &t,
                             const gf_launch *l, hipStream_t stream, gf_run_stats *stats)
{
    void *arr[GF_MAX_ARRAYS];
    std::memcpy(arr, in.arr, sizeof arr);
    RegionLaunch cur;
    bool pending = false;
    int launches = 0, regions = 0, max_grid = 0;

    auto flush = [&]() -> gf_status {
        if (!pending)
            return GF_OK;
        pending = false;
        return launch_one(ctx, cur, t, l, stream, &launches, &max_grid);
    };
    auto start_serial_only = [&]() {
        std::memset(&cur, 0, sizeof cur);
        cur.step.kind = 0;
        cur.step.red_op = GF_OP_NONE;
        for (int k = 0; k < 5; ++k)
            cur.step.arr[k] = -1;
        cur.scal = in.scal;
        cur.inst = inst_idx;
        pending = true;
    };

    const int64_t total = (int64_t)p.n_pro + (int64_t)p.iters * p.n_body;
    for (int64_t si = 0; si < total; ++si) {
        int sidx;
        int32_t iter;
        if (si < p.n_pro) {
            sidx = (int)si;
            iter = -1;
        } else {
            const int64_t k = si - p.n_pro;
            sidx = p.n_pro + (int)(k % p.n_body);
            iter = (int32_t)(k / p.n_body);
        }
        const DStep &s = p.steps[sidx];
        if (is_region(s.kind)) {
            gf_status st = flush();
            if (st != GF_OK)
                return st;
            std::memset(&cur, 0, sizeof cur);
            cur.step = s;
            for (int k = 0; k < 5; ++k)
                cur.arr[k] = s.arr[k] >= 0 ? arr[s.arr[k]] : nullptr;
            cur.scal = in.scal;
            cur.n = in.ip[s.np];
            cur.n_items = (int32_t)region_items(s, cur.n, t);
            cur.inst = inst_idx;
            pending = true;
            ++regions;
        } else if (s.kind == GF_S_SWAP) {
            std::swap(arr[s.arr[0]], arr[s.arr[1]]);
        } else {
            if (!pending || cur.n_glue == kMaxGlue) {
                gf_status st = flush();
                if (st != GF_OK)
                    return st;
                start_serial_only();
            }
            Glue &g = cur.glue[cur.n_glue++];
            std::memset(&g, 0, sizeof g);
            g.kind = s.kind;
            for (int k = 0; k < 3; ++k)
                g.sc[k] = s.sc[k];
            g.every = s.every;
            g.fmt_id = s.fmt_id;
            g.nargs = s.nargs;
            g.iter = iter;
            g.flags = s.flags;
            g.c = s.c;
            g.rec = s.kind == GF_S_RECORD ? (double *)arr[s.arr[0]] : nullptr;
            if (s.kind == GF_S_CALL) {
                std::lock_guard<std::mutex> lk(ctx->rpc_mu);
                const DCall &c = ctx->calls[s.fmt_id].dev;
                for (int k = 0; k < c.nargs; ++k)
                    if ((c.a[k].kind == GF_ARG_REF || c.a[k].kind == GF_ARG_HEAPREF))
                        g.obj[c.a[k].ref] = arr[c.a[k].slot];
                if (c.nrefs > 0)
                    cur.publish = 1;
            }
        }
    }
    gf_status st = flush();
    if (st != GF_OK)
        return st;
    if (stats) {
        stats->regions += regions;
        stats->launches += launches;
        stats->num_wg = std::max(stats->num_wg, max_grid);
        stats->wg_size = t.wg_size;
    }
    return GF_OK;
}

std::string graph_key(const DProg &p, const gf_instance *inst, int n_inst, const Tiling &t, const gf_launch *l,
                      hipStream_t s)
{
    std::string k;
    k.append((const char *)&p, sizeof p);
    k.append((const char *)inst, sizeof(gf_instance) * (size_t)n_inst);
    k.append((const char *)&t, sizeof t);
    const int32_t nwg = l ? l->num_wg : 0;
    k.append((const char *)&nwg, sizeof nwg);
    k.append((const char *)&s, sizeof s);
    return k;
}

}  // namespace

// Per-instance shape of a batched run: rows per tile (0: the launch's) and
// the relative weight of its share of workgroups (<= 0: its work items).
struct InstShape {
    int32_t tile_y;
    double weight;
};

// Workgroups for the instances `ids` out of `budget` (each >= 1 and at most
// its item count). A group of g_i workgroups deals its items_i tiles
// round-robin, so its time per region is ceil(items_i / g_i) tiles at a cost
// of w_i / items_i each; the launch lasts as long as its slowest group.
// Greedy: every instance starts with one workgroup, and while the budget
// allows, the slowest group gets just enough workgroups to take one tile
// less each. Workgroups that would not shorten the slowest group stay
// unused.
void share_groups(const std::vector<int> &ids, int budget, const std::vector<double> &w,
                  const std::vector<int64_t> &items, std::vector<int> &g)
{
    auto cost = [&](int i) { return w[i] / (double)items[i]; };
    auto per_wg = [&](int i) { return (items[i] + g[i] - 1) / g[i]; };
    std::vector<std::pair<double, int>> heap;
    int used = 0;
    for (int i : ids) {
        g[i] = 1;
        ++used;
        heap.emplace_back((double)items[i] * cost(i), i);
    }
    std::make_heap(heap.begin(), heap.end());
    while (!heap.empty()) {
        std::pop_heap(heap.begin(), heap.end());
        const int i = heap.back().second;
        heap.pop_back();
        const int64_t k = per_wg(i);
        if (k <= 1)
            break;  // the slowest group takes one tile per workgroup already
        const int64_t want = (items[i] + (k - 1) - 1) / (k - 1);
        const int need = (int)(want - g[i]);
        if (used + need > budget)
            break;  // the slowest group cannot be shortened
        g[i] += need;
        used += need;
        heap.emplace_back((double)per_wg(i) * cost(i), i);
        std::push_heap(heap.begin(), heap.end());
    }
}

// The plan of a batched persistent launch: with `align`, instance i goes to
// XCD xcd[i] (heaviest first onto the least loaded XCD with a free slot)
// and each XCD's budget / 8 workgroups are shared among its instances;
// otherwise (or when an XCD would need more than its share of instances)
// xcd[] stays -1 and the whole budget is shared. g[i] receives the group
// sizes. Returns the grid: 8 times the largest XCD's workgroups when
// aligned, else the sum of the groups.
int plan_batch(int n, const std::vector<int64_t> &items, const std::vector<double> &w, int budget, bool align,
               std::vector<int> &g, std::vector<int> &xcd)
{
    const int per = budget / kNumXcd;
    bool aligned = per >= 1 && align;
    std::fill(xcd.begin(), xcd.end(), -1);
    if (aligned) {
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i)
            order[i] = i;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b] || (w[a] == w[b] && a < b); });
        double load[kNumXcd] = {0};
        int cnt[kNumXcd] = {0};
        for (int i : order) {
            int best = -1;
            for (int x = 0; x < kNumXcd; ++x)
                if (cnt[x] < per && (best < 0 || load[x] < load[best]))
                    best = x;
            if (best < 0) {
                aligned = false;
                break;
            }
            xcd[i] = best;
            load[best] += w[i];
            ++cnt[best];
        }
        if (!aligned)
            std::fill(xcd.begin(), xcd.end(), -1);
    }
    if (aligned) {
        int longest = 0;
        for (int x = 0; x < kNumXcd; ++x) {
            std::vector<int> ids;
            for (int i = 0; i < n; ++i)
                if (xcd[i] == x)
                    ids.push_back(i);
            share_groups(ids, per, w, items, g);
            int used = 0;
            for (int i : ids)
                used += g[i];
            longest = std::max(longest, used);
        }
        return longest * kNumXcd;
    }
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i)
        all[i] = i;
    share_groups(all, budget, w, items, g);
    int sum = 0;
    for (int i = 0; i < n; ++i)
        sum += g[i];
    return sum;
}

// Batched persistent launch (many uneven instances of one program in one
// cooperative launch). Instance i gets a group of g_i >= 1 workgroups, its
// own group barrier and its own slice of the reduction partials. The groups
// are kept on single XCDs: the instances are packed onto the eight XCDs
// (heaviest first onto the least loaded XCD; weight = work items unless the
// shape gives one), each XCD's share of the grid is divided among its
// instances, and workgroup b takes an entry of XCD b mod 8
// (the hardware's round-robin dispatch; the kernel checks it and falls back
// to the cross-XCD group barrier otherwise). A group on one XCD shares one
// L2, so its barrier needs no L2 write-back and its tiles share halo rows.
// Within an XCD the group sizes minimise the slowest group's time per region
// (share_groups). Without room for that packing the groups are laid out in
// order. The
// device table is staged through pinned memory; the staging buffer is
// rewritten only after the previous copy has executed.
gf_status run_batched(gf_ctx *ctx, const DProg &p, const gf_instance *inst, int n_inst, const Tiling &t,
                      const gf_launch *launch, int cap, gf_run_stats *stats, hipStream_t stream,
                      const InstShape *shape)
{
    if (program_is_hist_family(p))
        return fail(ctx, GF_EUNSUPPORTED, "batched persistent runs of histogram programs are not supported");
    int budget = cap;
    if (launch && launch->num_wg > 0)
        budget = std::min(budget, launch->num_wg);
    budget = std::min(budget, 4096);
    if (n_inst > budget)
        return fail(ctx, GF_EINVAL, "%d instances need at least %d co-resident workgroups, capacity %d", n_inst,
                    n_inst, budget);
    std::vector<int64_t> items(n_inst), red(n_inst);
    std::vector<double> w(n_inst);
    std::vector<int32_t> ty(n_inst, 0);
    for (int i = 0; i < n_inst; ++i) {
        Tiling ti = t;
        if (shape && shape[i].tile_y > 0)
            ti.tile_y = ty[i] = shape[i].tile_y;
        items[i] = std::max<int64_t>(1, max_items(p, inst[i], ti));
        int64_t r = 0;
        for (int k = 0; k < p.n_steps; ++k)
            if (is_region(p.steps[k].kind) && p.steps[k].red_op != GF_OP_NONE)
                r = std::max<int64_t>(r, region_items(p.steps[k], inst[i].ip[p.steps[k].np], ti));
        red[i] = r;
        w[i] = (shape && shape[i].weight > 0.0) ? shape[i].weight : (double)items[i];
    }
    // pack onto XCDs and size the groups
    std::vector<int> g(n_inst, 1), xcd_of(n_inst, -1);
    const int grid = plan_batch(n_inst, items, w, budget, ctx->batch_align, g, xcd_of);
    const bool aligned = xcd_of[0] >= 0;
    std::vector<std::vector<int>> on(kNumXcd);
    if (aligned)
        for (int i = 0; i < n_inst; ++i)
            on[xcd_of[i]].push_back(i);
    // partial slices
    std::vector<int64_t> off(n_inst);
    int64_t acc = 0;
    for (int i = 0; i < n_inst; ++i) {
        off[i] = acc;
        acc += red[i];
    }
    if (acc > ctx->scr.partials_cap)
        return fail(ctx, GF_EINVAL, "batched reductions need %lld partial slots, capacity %lld", (long long)acc,
                    (long long)ctx->scr.partials_cap);
    // stage the table (wait until the previous staging copy has executed)
    if (ctx->batch_pending) {
        hipError_t e = hipEventSynchronize(ctx->batch_copied);
        if (e != hipSuccess)
            return hipfail(ctx, e, "batch staging wait");
        ctx->batch_pending = false;
    }
    BatchEntry *hb = (BatchEntry *)ctx->h_batch;
    DInst *hi = (DInst *)((char *)ctx->h_batch + (size_t)4096 * sizeof(BatchEntry));
    auto entry = [&](int i, int m) {
        BatchEntry e;
        e.inst = i;
        e.member = m;
        e.gsize = g[i];
        e.tile_y = ty[i];
        e.part_off = off[i];
        return e;
    };
    int wg = 0;
    if (aligned) {
        std::vector<std::vector<BatchEntry>> lists(kNumXcd);
        size_t longest = 0;
        for (int x = 0; x < kNumXcd; ++x) {
            for (int i : on[x])
                for (int m = 0; m < g[i]; ++m)
                    lists[x].push_back(entry(i, m));
            longest = std::max(longest, lists[x].size());
        }
        wg = (int)(longest * kNumXcd);
        (void)grid;
        BatchEntry idle;
        std::memset(&idle, 0, sizeof idle);
        idle.inst = -1;
        for (int b = 0; b < wg; ++b) {
            const auto &l = lists[b % kNumXcd];
            const size_t r = (size_t)(b / kNumXcd);
            hb[b] = r < l.size() ? l[r] : idle;
        }
    } else {
        for (int i = 0; i < n_inst; ++i)
            for (int m = 0; m < g[i]; ++m)
                hb[wg++] = entry(i, m);
    }
    for (int i = 0; i < n_inst; ++i) {
        std::memcpy(hi[i].arr, inst[i].arr, sizeof hi[i].arr);
        hi[i].scal = inst[i].scal;
        std::memcpy(hi[i].ip, inst[i].ip, sizeof hi[i].ip);
    }
    BatchEntry *db = (BatchEntry *)ctx->d_batch;
    DInst *di = (DInst *)((char *)ctx->d_batch + (size_t)4096 * sizeof(BatchEntry));
    hipError_t e = hipMemcpyAsync(db, hb, (size_t)wg * sizeof(BatchEntry), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(di, hi, (size_t)n_inst * sizeof(DInst), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipEventRecord(ctx->batch_copied, stream);
    if (e != hipSuccess)
        return hipfail(ctx, e, "batch table copy");
    ctx->batch_pending = true;
    BatchTable bt{db, di, aligned ? 1 : 0};
    DInst dummy;
    std::memset(&dummy, 0, sizeof dummy);
    ctx->scr.epoch += 1;
    ctx->batch_check_epoch = aligned ? ctx->scr.epoch : 0;
    e = launch_persistent(p, dummy, t, wg, ctx->scr, ring_of(ctx), stream, &bt);
    if (e != hipSuccess)
        return hipfail(ctx, e, "batched persistent launch");
    if (stats) {
        stats->launches = 1;
        stats->num_wg = wg;
        stats->wg_size = t.wg_size;
        int nb = 0;
        for (int k = p.n_pro; k < p.n_steps; ++k)
            nb += is_region(p.steps[k].kind);
        stats->regions = n_inst * nb * p.iters;
        stats->barriers = (int32_t)p.barriers;
    }
    return GF_OK;
}

namespace {
int32_t predict_launch(gf_ctx *ctx, const DProg &p, const gf_instance *inst, int n_inst, int mode, hipStream_t s,
                       gf_launch *out);

// Writes the predictor's choice into the caller's stats when the run returns.
struct CandidateNote {
    gf_run_stats *stats;
    int32_t cand;
    int32_t source = GF_LAUNCH_GIVEN;
    ~CandidateNote()
    {
        if (stats) {
            stats->candidate = cand;
            stats->launch_source = source;
        }
    }
};

int32_t tune_fallback(gf_ctx *ctx, const gf_program *prog, const DProg &p, const gf_instance *inst, int n_inst,
                      int mode, hipStream_t s, gf_launch *out, bool *cached, std::vector<gf_launch> *per);
}  // namespace

// Kernel split: the main kernel (one thread) runs on `stream`; its region
// requests are serviced by whoever polls the RPC ring — the library's server
// thread, else this call, which polls until the main kernel has finished.
gf_status run_kernel_split(gf_ctx *ctx, const DProg &p, const gf_instance &in, int n_inst, const Tiling &t,
                           const gf_launch *launch, gf_run_stats *stats, hipStream_t stream)
{
    if (n_inst != 1)
        return fail(ctx, GF_EUNSUPPORTED, "the kernel split runs one instance");
    if (!ctx->split_stream)
        return fail(ctx, GF_EHIP, "no stream for the split regions");
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess)
        return hipfail(ctx, e, "event create");
    {
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        auto &sp = ctx->split;
        sp.active = true;
        sp.p = p;
        sp.in = in;
        sp.t = t;
        sp.has_l = launch != nullptr;
        if (launch)
            sp.l = *launch;
        sp.regions = sp.launches = sp.max_grid = 0;
    }
    DInst di;
    std::memcpy(di.arr, in.arr, sizeof di.arr);
    di.scal = in.scal;
    std::memcpy(di.ip, in.ip, sizeof di.ip);
    e = launch_main(p, di, ring_of(ctx), ctx->scr, stream);
    if (e == hipSuccess)
        e = hipEventRecord(ev, stream);
    if (e == hipSuccess) {
        const bool serve = !ctx->server.joinable();
        for (;;) {
            const hipError_t q = hipEventQuery(ev);
            if (q == hipSuccess)
                break;
            if (q != hipErrorNotReady) {
                e = q;
                break;
            }
            if (serve) {
                std::lock_guard<std::mutex> g(ctx->rpc_mu);
                poll_locked(ctx, 1 << 20, 0);
            } else {
                std::this_thread::yield();
            }
        }
    }
    {
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        // remaining posted requests (printf) are serviced before the run is released
        poll_locked(ctx, 1 << 20, 0);
        ctx->split.active = false;
        if (stats) {
            stats->regions = ctx->split.regions;
            stats->launches = ctx->split.launches + 1;
            stats->num_wg = ctx->split.max_grid;
            stats->wg_size = t.wg_size;
        }
    }
    hipEventDestroy(ev);
    if (e != hipSuccess)
        return hipfail(ctx, e, "kernel split run");
    return GF_OK;
}

extern "C" {

int32_t gf_persistent_capacity(gf_ctx *ctx, const gf_program *prog, int32_t wg_size)
{
    if (!ctx)
        return 0;
    DProg p;
    if (build_program(ctx, prog, &p) != GF_OK)
        return 0;
    gf_launch l{};
    l.wg_size = wg_size;
    Tiling t = choose_tiling(p, wg_size > 0 ? &l : nullptr);
    if (check_tiling(ctx, p, t) != GF_OK)
        return 0;
    hipSetDevice(ctx->device);
    return persistent_capacity(p, t, ctx->num_cu);
}

static gf_status region_run(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                            int32_t mode, const gf_launch *launch, gf_run_stats *stats, void *hip_stream,
                            const InstShape *shape = nullptr);

gf_status gf_region_run(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst, int32_t mode,
                        const gf_launch *launch, gf_run_stats *stats, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    gf_status st = order_before(ctx, s);
    if (st != GF_OK)
        return st;
    st = region_run(ctx, prog, inst, n_inst, mode, launch, stats, hip_stream);
    if (st == GF_OK)
        mark_after(ctx, s);
    return st;
}

static gf_status region_run(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                            int32_t mode, const gf_launch *launch, gf_run_stats *stats, void *hip_stream,
                            const InstShape *shape)
{
    if (!inst || n_inst < 1 || n_inst > GF_MAX_INSTANCES)
        return fail(ctx, GF_EINVAL, "need 1..%d instances", GF_MAX_INSTANCES);
    if (mode != GF_EXEC_PER_REGION && mode != GF_EXEC_PERSISTENT && mode != GF_EXEC_PER_REGION_GRAPH &&
        mode != GF_EXEC_KERNEL_SPLIT)
        return fail(ctx, GF_EINVAL, "unknown execution mode %d", mode);
    DProg p;
    gf_status st = build_program(ctx, prog, &p);
    if (st != GF_OK)
        return st;
    hipSetDevice(ctx->device);
    hipStream_t stream = (hipStream_t)hip_stream;
    gf_launch predicted;
    CandidateNote note{stats, -1};
    if (!launch && !shape && !ctx->pred_params.empty()) {
        int32_t k = predict_launch(ctx, p, inst, n_inst, mode, stream, &predicted);
        if (k < -1)
            return (gf_status)k;
        if (k >= 0) {
            note.cand = k;
            note.source = GF_LAUNCH_PREDICTED;
            launch = &predicted;
        } else if (ctx->tune_fallback && mode != GF_EXEC_KERNEL_SPLIT) {
            // the predictor defers (outside its training distribution, or
            // no runnable shape it knows): the autotuner decides
            bool cached = false;
            std::vector<gf_launch> per;
            k = tune_fallback(ctx, prog, p, inst, n_inst, mode, stream, &predicted, &cached, &per);
            if (k < -1)
                return (gf_status)k;
            if (!per.empty()) {
                // a batched persistent run: the autotuner chose a shape per instance
                std::vector<InstShape> sh(n_inst);
                for (int i = 0; i < n_inst; ++i) {
                    sh[i].tile_y = per[i].tile_y;
                    sh[i].weight = (double)per[i].num_wg;
                }
                gf_launch common = per[0];
                common.num_wg = 0;
                common.tile_y = 0;
                note.cand = -1;
                note.source = cached ? GF_LAUNCH_TUNED_CACHED : GF_LAUNCH_TUNED;
                return region_run(ctx, prog, inst, n_inst, mode, &common, stats, hip_stream, sh.data());
            }
            if (k >= 0) {
                note.cand = k;
                note.source = cached ? GF_LAUNCH_TUNED_CACHED : GF_LAUNCH_TUNED;
                launch = &predicted;
            }
        }
    }
    Tiling t = choose_tiling(p, launch);
    if ((st = check_tiling(ctx, p, t)) != GF_OK)
        return st;
    // per instance: its own rows per tile when a shape gives them (the 3D
    // stencil's rows are compiled into the kernel, so they must agree)
    std::vector<Tiling> ti(n_inst, t);
    for (int i = 0; i < n_inst; ++i) {
        if (shape && shape[i].tile_y > 0) {
            if ((program_region_mask(p) & (1u << GF_R_JACOBI3D)) && shape[i].tile_y != t.tile_y)
                return fail(ctx, GF_EINVAL, "instance %d: 3D stencil rows per tile %d differ from the launch's %d", i,
                            shape[i].tile_y, t.tile_y);
            ti[i].tile_y = shape[i].tile_y;
            if ((st = check_tiling(ctx, p, ti[i])) != GF_OK)
                return st;
        }
        if ((st = check_instance(ctx, p, inst[i], ti[i], i)) != GF_OK)
            return st;
    }
    if (stats)
        std::memset(stats, 0, sizeof *stats);

    if (mode == GF_EXEC_PERSISTENT) {
        // the barrier tree is sized for at most 4096 workgroups
        const int cap = std::min(4096, persistent_capacity(p, t, ctx->num_cu));
        if (cap <= 0)
            return fail(ctx, GF_EHIP, "occupancy query failed");
        if (n_inst > 1)
            return run_batched(ctx, p, inst, n_inst, t, launch, cap, stats, stream, shape);
        for (int i = 0; i < n_inst; ++i) {
            // default grid: at most two workgroups per CU (the grid barrier's
            // cost grows with the number of members), sized so that every
            // workgroup gets the same number of work items (balanced rounds)
            const int64_t gmax = std::min<int64_t>(cap, 2 * (int64_t)ctx->num_cu);
            const int64_t items = max_items(p, inst[i], t);
            const int64_t rounds = (items + gmax - 1) / gmax;
            int grid = (int)((items + rounds - 1) / rounds);
            if (launch && launch->num_wg > 0) {
                if (launch->num_wg > cap)
                    return fail(ctx, GF_EINVAL, "num_wg %d exceeds the co-resident capacity %d", launch->num_wg, cap);
                grid = launch->num_wg;
            }
            if (program_is_hist_family(p)) {
                uint32_t mask = 0;
                for (int k = 0; k < p.n_steps; ++k)
                    if (p.steps[k].kind == GF_R_HIST)
                        mask = std::max(mask, p.steps[k].mask);
                const int want = (launch && launch->num_wg > 0) ? launch->num_wg : cap;
                grid = hist_grid(want, mask);
                if (grid > cap)
                    return fail(ctx, GF_EINVAL, "histogram needs %d co-resident workgroups, capacity %d", grid, cap);
            }
            DInst di;
            std::memcpy(di.arr, inst[i].arr, sizeof di.arr);
            di.scal = inst[i].scal;
            std::memcpy(di.ip, inst[i].ip, sizeof di.ip);
            ctx->scr.epoch += 1;
            // the XCD barrier's per-launch registration costs a tree barrier:
            // programs with few barriers keep the tree barrier
            Scratch scr = ctx->scr;
            if (p.barriers < kXcdBarrierMinBarriers)
                scr.barrier_kind = kBarrierTree;
            hipError_t e = launch_persistent(p, di, t, grid, scr, ring_of(ctx), stream);
            if (e != hipSuccess)
                return hipfail(ctx, e, "persistent launch");
            if (stats) {
                stats->launches += 1;
                stats->num_wg = std::max(stats->num_wg, grid);
                stats->wg_size = t.wg_size;
                int nreg = 0;
                for (int k = 0; k < p.n_pro; ++k)
                    nreg += is_region(p.steps[k].kind);
                int nbody = 0;
                for (int k = p.n_pro; k < p.n_steps; ++k)
                    nbody += is_region(p.steps[k].kind);
                stats->regions += nreg + nbody * p.iters;
                stats->barriers = (int32_t)p.barriers;
            }
        }
        return GF_OK;
    }

    if (mode == GF_EXEC_KERNEL_SPLIT)
        return run_kernel_split(ctx, p, inst[0], n_inst, t, launch, stats, stream);

    if (mode == GF_EXEC_PER_REGION) {
        for (int i = 0; i < n_inst; ++i)
            if ((st = enqueue_per_region(ctx, p, inst[i], i, ti[i], launch, stream, stats)) != GF_OK)
                return st;
        return GF_OK;
    }

    // GF_EXEC_PER_REGION_GRAPH: capture the per-region launch sequence once
    // per (program, bindings, tilings, stream) and replay it.
    std::string key = graph_key(p, inst, n_inst, t, launch, stream);
    for (int i = 0; shape && i < n_inst; ++i)
        key.append((const char *)&ti[i].tile_y, sizeof ti[i].tile_y);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        hipStream_t cs = ctx->capture_stream;
        if (!cs)
            return fail(ctx, GF_EHIP, "no capture stream");
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            return hipfail(ctx, e, "begin capture");
        gf_run_stats tmp{};
        for (int i = 0; i < n_inst && st == GF_OK; ++i)
            st = enqueue_per_region(ctx, p, inst[i], i, ti[i], launch, cs, &tmp);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (st != GF_OK) {
            if (g)
                hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess)
            return hipfail(ctx, e, "end capture");
        GraphEntry ge;
        ge.graph = g;
        ge.stats = tmp;
        e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return hipfail(ctx, e, "graph instantiate");
        }
        it = ctx->graphs.emplace(key, ge).first;
    }
    if (stats)
        *stats = it->second.stats;
    hipError_t e = hipGraphLaunch(it->second.exec, stream);
    if (e != hipSuccess)
        return hipfail(ctx, e, "graph launch");
    return GF_OK;
}

gf_status gf_reduce(gf_ctx *ctx, int32_t op, int32_t dt, const void *d_in, int64_t n, void *d_out, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (op != GF_OP_SUM && op != GF_OP_MAX)
        return fail(ctx, GF_EINVAL, "unknown reduction op %d", op);
    if (dt < GF_F64 || dt > GF_I64)
        return fail(ctx, GF_EINVAL, "unknown dtype %d", dt);
    if (n < 0 || (n > 0 && !d_in) || !d_out)
        return fail(ctx, GF_EINVAL, "bad reduction arguments");
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    gf_status st = order_before(ctx, s);
    if (st != GF_OK)
        return st;
    hipError_t e = launch_reduce(op, dt, d_in, n, d_out, ctx->scr, ctx->num_cu, s);
    if (e != hipSuccess)
        return hipfail(ctx, e, "reduce launch");
    mark_after(ctx, s);
    return GF_OK;
}

gf_status gf_reduce_noalloc(gf_ctx *ctx, int32_t op, int32_t dt, const void *d_in, int64_t n, void *d_out,
                            void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (op != GF_OP_SUM && op != GF_OP_MAX)
        return fail(ctx, GF_EINVAL, "unknown reduction op %d", op);
    if (dt < GF_F64 || dt > GF_I64)
        return fail(ctx, GF_EINVAL, "unknown dtype %d", dt);
    if (n < 0 || (n > 0 && !d_in) || !d_out)
        return fail(ctx, GF_EINVAL, "bad reduction arguments");
    if (ctx->noalloc_status != hipSuccess)
        return hipfail(ctx, ctx->noalloc_status, "gf_reduce_noalloc: static scratch not set up on this device");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = noalloc_reduce(ctx->device, ctx->num_cu, op, dt, d_in, n, d_out, (hipStream_t)hip_stream, nullptr);
    if (e == hipErrorInvalidValue)
        return fail(ctx, GF_EINVAL, "gf_reduce_noalloc: the grid for n = %lld needs more partials than the static "
                    "array holds (%zu bytes)", (long long)n, noalloc_scratch_bytes());
    if (e != hipSuccess)
        return hipfail(ctx, e, "gf_reduce_noalloc launch");
    return GF_OK;
}

gf_status gf_copy(gf_ctx *ctx, void *d_dst, const void *d_src, int64_t nbytes, int32_t num_wg, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_dst || !d_src || nbytes < 0 || (nbytes % 16))
        return fail(ctx, GF_EINVAL, "copy needs non-null buffers and a multiple of 16 bytes");
    hipSetDevice(ctx->device);
    hipError_t e = launch_copy(d_dst, d_src, nbytes, num_wg, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hipfail(ctx, e, "copy launch");
    return GF_OK;
}

int64_t gf_batch_misplaced(gf_ctx *ctx)
{
    if (!ctx)
        return GF_EINVAL;
    if (!ctx->batch_check_epoch)
        return -1;
    hipSetDevice(ctx->device);
    if (hipDeviceSynchronize() != hipSuccess)
        return GF_EHIP;
    uint64_t v = 0;
    if (hipMemcpy(&v, ctx->scr.lines + (int64_t)kBatchPlaceLine * kLineWords, sizeof v, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return GF_EHIP;
    if ((uint32_t)(v >> 32) != ctx->batch_check_epoch)
        return -1;
    return (int64_t)(uint32_t)v;
}

gf_status gf_sync(gf_ctx *ctx, void *hip_stream, gf_run_stats *stats)
{
    if (!ctx)
        return GF_EINVAL;
    hipSetDevice(ctx->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    {
        std::lock_guard<std::mutex> g(ctx->rpc_mu);
        while (poll_locked(ctx, 1 << 20, 0) > 0) {
        }
    }
    if (stats)
        stats->rpc_posted = (int32_t)ctx->serviced.load();
    if (e != hipSuccess)
        return hipfail(ctx, e, "stream synchronize");
    int32_t code = 0;
    if ((e = hipMemcpy(&code, ctx->scr.error, sizeof code, hipMemcpyDeviceToHost)) != hipSuccess)
        return hipfail(ctx, e, "error word read");
    if (code != kErrNone) {
        // a kernel that stopped on the error may have left barrier counters
        // mid-count: clear every counter line with the error word; a caller
        // that gave up on an RPC slot may have left the ring mid-ticket:
        // re-synchronise it (both once no kernel of the device still runs)
        hipDeviceSynchronize();
        recover_ring(ctx);
        const int32_t zero = 0;
        hipMemset(ctx->scr.lines, 0, (size_t)kNumLines * kLineWords * sizeof(uint32_t));
        hipMemcpy(ctx->scr.error, &zero, sizeof zero, hipMemcpyHostToDevice);
        if (code == kErrBarrierTimeout)
            return fail(ctx, GF_ETIMEOUT, "device: grid barrier watchdog expired");
        if (code == kErrRegionLaunch)
            return fail(ctx, GF_EHIP, "device: the host could not launch a region the main kernel requested");
        if (code == kErrRpcTimeout)
            return fail(ctx, GF_ETIMEOUT, "device: RPC wait watchdog expired (is a server polling?)");
        return fail(ctx, GF_EDEVICE, "device error code %d", code);
    }
    return GF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------

namespace {

int64_t first_stencil_size(const DProg &p, const gf_instance &in)
{
    for (int i = 0; i < p.n_steps; ++i)
        if (p.steps[i].kind == GF_R_JACOBI3D || p.steps[i].kind == GF_R_JACOBI2D)
            return in.ip[p.steps[i].np];
    return 0;
}

gf_launch decode_candidate(const DProg &p, const gf_instance &in, int c, int num_cu)
{
    gf_launch l;
    std::memset(&l, 0, sizeof l);
    const int a = c & 3, b = (c >> 2) & 3, h = (c >> 4) & 1;
    const unsigned m = program_region_mask(p);
    static const int ty[4] = {1, 2, 4, 8};
    static const int zs[4] = {2, 3, 4, 6};
    static const int wg[4] = {64, 128, 192, 256};
    static const int hw[4] = {256, 512, 768, 1024};
    static const int it[4] = {1, 2, 4, 8};
    if (m & (1u << GF_R_HIST)) {
        l.wg_size = hw[a];
        l.items = it[b];
        l.num_wg = h ? num_cu : num_cu / 2;  // one 128 KiB-LDS workgroup per CU at most
        l.xcd_remap = 1;
    } else if (m & (1u << GF_R_JACOBI3D)) {
        const int64_t n = first_stencil_size(p, in);
        const int64_t interior = n > 2 ? n - 2 : 1;
        l.tile_y = ty[a];
        l.tile_z = (int32_t)std::max<int64_t>(1, (interior + zs[b] - 1) / zs[b]);
        l.xcd_remap = 1;
        l.num_wg = h ? 3 * num_cu : 0;  // three workgroups per CU, or the default grid
    } else if (m & (1u << GF_R_JACOBI2D)) {
        static const int seg[4] = {2, 8, 32, 128};
        l.tile_y = seg[a];
        l.wg_size = wg[b];
        l.xcd_remap = 1 - h;
    } else {
        l.wg_size = wg[a];
        l.items = it[b];
        l.num_wg = h ? 4 * num_cu : 0;
        l.xcd_remap = 1;
    }
    return l;
}

// Raw predictor features of the program's dominant region (largest trip
// count x bytes per iteration); see gf_nest_features.
gf_status nest_features(gf_ctx *ctx, const DProg &p, const gf_instance &in, int n_inst, hipStream_t s, double *f)
{
    double best = -1.0;
    for (int k = 0; k < GF_MLP_IN; ++k)
        f[k] = 0.0;
    for (int i = 0; i < p.n_steps; ++i) {
        const DStep &st = p.steps[i];
        if (!is_region(st.kind))
            continue;
        const int64_t n = in.ip[st.np];
        const double m = (double)std::max<int64_t>(n - 2, 0);
        const double red = st.red_op != GF_OP_NONE ? 1.0 : 0.0;
        double g[GF_MLP_IN] = {(double)n, 0.0, 0.0, 0.0, 0.0, 0.0, (double)n_inst, 8.0};
        switch (st.kind) {
        case GF_R_JACOBI2D:
            g[0] = m * m, g[1] = 16.0, g[2] = 7.0, g[3] = 1.0, g[4] = red;
            break;
        case GF_R_JACOBI3D:
            g[0] = m * m * m, g[1] = 16.0, g[2] = 9.0, g[3] = 1.0, g[4] = red;
            break;
        case GF_R_SPMV: {
            int32_t nnz = 0;
            if (n > 0) {
                const int32_t *rp = (const int32_t *)in.arr[st.arr[0]];
                hipError_t e = hipMemcpyAsync(&nnz, rp + n, sizeof nnz, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    return hipfail(ctx, e, "reading the row pointer");
            }
            const double nz = n > 0 ? (double)nnz / (double)n : 0.0;
            g[1] = 12.0 * nz + 20.0, g[2] = 2.0 * nz, g[5] = nz;
            break;
        }
        case GF_R_DOT:
            g[1] = 16.0, g[2] = 2.0, g[4] = 1.0;
            break;
        case GF_R_AXPBY:
            g[1] = 24.0, g[2] = 2.0;
            break;
        case GF_R_HIST:
            g[1] = 4.0, g[4] = (double)st.mask + 1.0, g[7] = 4.0;
            break;
        default:  // GF_R_OWNER
            g[1] = 4.0, g[7] = 4.0;
            break;
        }
        const double w = g[0] * g[1];
        if (w > best) {
            best = w;
            std::memcpy(f, g, sizeof g);
        }
    }
    return GF_OK;
}

// Whether `l` passes every check gf_region_run makes before enqueueing
// (tiling, instances, co-residency of the persistent grid). Leaves the
// context's error message untouched.
bool launch_runnable(gf_ctx *ctx, const DProg &p, const gf_instance *inst, int n_inst, int mode, const gf_launch &l)
{
    const std::string saved = ctx->err;
    bool ok = true;
    const Tiling t = choose_tiling(p, &l);
    if (check_tiling(ctx, p, t) != GF_OK)
        ok = false;
    for (int i = 0; ok && i < n_inst; ++i)
        ok = check_instance(ctx, p, inst[i], t, i) == GF_OK;
    if (ok && mode == GF_EXEC_PERSISTENT) {
        const int cap = std::min(4096, persistent_capacity(p, t, ctx->num_cu));
        ok = cap > 0 && l.num_wg <= cap;
        if (ok && n_inst > 1)
            ok = !program_is_hist_family(p) && n_inst <= (l.num_wg > 0 ? l.num_wg : cap);
        if (ok && program_is_hist_family(p)) {
            uint32_t mask = 0;
            for (int k = 0; k < p.n_steps; ++k)
                if (p.steps[k].kind == GF_R_HIST)
                    mask = std::max(mask, p.steps[k].mask);
            ok = hist_grid(l.num_wg > 0 ? l.num_wg : cap, mask) <= cap;
        }
    }
    ctx->err = saved;
    return ok;
}

int32_t predict_launch(gf_ctx *ctx, const DProg &p, const gf_instance *inst, int n_inst, int mode, hipStream_t s,
                       gf_launch *out)
{
    double f[GF_MLP_IN];
    const gf_status st = nest_features(ctx, p, inst[0], n_inst, s, f);
    if (st != GF_OK)
        return st;
    uint8_t valid[GF_NUM_CANDIDATES];
    gf_launch cand[GF_NUM_CANDIDATES];
    bool any = false;
    for (int c = 0; c < GF_NUM_CANDIDATES; ++c) {
        cand[c] = decode_candidate(p, inst[0], c, ctx->num_cu);
        valid[c] = launch_runnable(ctx, p, inst, n_inst, mode, cand[c]) ? 1 : 0;
        any = any || valid[c];
    }
    if (!any)
        return -1;
    const int32_t k = gf_predict(ctx, f, valid, nullptr);
    if (k >= 0)
        *out = cand[k];
    return k;
}

// Bytes of each array slot that the program's regions and records touch in
// instance `in` (0: unused). SpMV's column and value arrays take their
// length from the row pointer's last entry, read from the device on s.
gf_status slot_bytes(gf_ctx *ctx, const DProg &p, const gf_instance &in, hipStream_t s, int64_t *bytes)
{
    for (int k = 0; k < GF_MAX_ARRAYS; ++k)
        bytes[k] = 0;
    auto need = [&](int slot, int64_t b) {
        if (slot >= 0 && slot < GF_MAX_ARRAYS)
            bytes[slot] = std::max(bytes[slot], b);
    };
    for (int i = 0; i < p.n_steps; ++i) {
        const DStep &st = p.steps[i];
        const int64_t n = is_region(st.kind) ? in.ip[st.np] : 0;
        switch (st.kind) {
        case GF_R_JACOBI2D:
            need(st.arr[0], 8 * n * n), need(st.arr[1], 8 * n * n);
            break;
        case GF_R_JACOBI3D:
            need(st.arr[0], 8 * n * n * n), need(st.arr[1], 8 * n * n * n);
            break;
        case GF_R_SPMV: {
            int32_t nnz = 0;
            if (n > 0) {
                hipError_t e = hipMemcpyAsync(&nnz, (const int32_t *)in.arr[st.arr[0]] + n, sizeof nnz,
                                              hipMemcpyDeviceToHost, s);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(s);
                if (e != hipSuccess)
                    return hipfail(ctx, e, "reading the row pointer");
            }
            need(st.arr[0], 4 * (n + 1)), need(st.arr[1], 4 * (int64_t)nnz), need(st.arr[2], 8 * (int64_t)nnz);
            need(st.arr[3], 8 * n), need(st.arr[4], 8 * n);
            break;
        }
        case GF_R_DOT:
            need(st.arr[0], 8 * n), need(st.arr[1], 8 * n);
            break;
        case GF_R_AXPBY:
            need(st.arr[0], 8 * n), need(st.arr[1], 8 * n), need(st.arr[2], 8 * n);
            break;
        case GF_R_HIST:
            need(st.arr[0], (4 * n + 15) / 16 * 16), need(st.arr[1], 4 * ((int64_t)st.mask + 1));
            break;
        case GF_R_OWNER:
            need(st.arr[0], 4 * n);
            break;
        case GF_R_PHASES:
            need(st.arr[0], 8 * n), need(st.arr[1], 8 * n), need(st.arr[2], 4 * n);
            break;
        case GF_S_RECORD:
            need(st.arr[0], 8 * std::max<int64_t>(1, p.iters));
            break;
        default:
            break;
        }
    }
    // swapped slots hold buffers of the same size
    for (int round = 0; round < 2; ++round)
        for (int i = 0; i < p.n_steps; ++i)
            if (p.steps[i].kind == GF_S_SWAP) {
                const int a = p.steps[i].arr[0], b = p.steps[i].arr[1];
                need(a, bytes[b]), need(b, bytes[a]);
            }
    return GF_OK;
}

std::string fallback_key(const DProg &p, const gf_instance *inst, int n_inst, int mode)
{
    std::string k;
    k.append((const char *)p.steps, sizeof(DStep) * (size_t)p.n_steps);
    k.append((const char *)&p.n_pro, sizeof p.n_pro);
    k.append((const char *)&p.iters, sizeof p.iters);
    k.append((const char *)&mode, sizeof mode);
    for (int i = 0; i < n_inst; ++i)
        k.append((const char *)inst[i].ip, sizeof inst[i].ip);
    return k;
}

// The autotuner as the predictor's fallback: time every candidate shape on
// copies of the instances' arrays and scalars (the caller's data is only
// read), with the program's host calls and printfs left out (they do not
// depend on the launch shape and must not run more than once), pick the
// fastest and remember it for this program, sizes and mode. Per-region
// graph runs are tuned as per-region launches. Returns the candidate index,
// -1 if none could run, or a negative gf_status below -1 on failure.
int32_t tune_fallback(gf_ctx *ctx, const gf_program *prog, const DProg &p, const gf_instance *inst, int n_inst,
                      int mode, hipStream_t s, gf_launch *out, bool *cached, std::vector<gf_launch> *per)
{
    const std::string key = fallback_key(p, inst, n_inst, mode);
    auto hit = ctx->tuned.find(key);
    if (hit != ctx->tuned.end()) {
        *out = hit->second.launch;
        *per = hit->second.per;
        *cached = true;
        return hit->second.cand;
    }
    std::vector<gf_step> pro, body;
    for (int32_t i = 0; i < prog->n_prologue; ++i)
        if (prog->prologue[i].kind != GF_S_PRINTF && prog->prologue[i].kind != GF_S_CALL)
            pro.push_back(prog->prologue[i]);
    for (int32_t i = 0; i < prog->n_body; ++i)
        if (prog->body[i].kind != GF_S_PRINTF && prog->body[i].kind != GF_S_CALL)
            body.push_back(prog->body[i]);
    gf_program tp{(int32_t)pro.size(), pro.data(), (int32_t)body.size(), body.data(), prog->iters};
    // one device block per instance: its arrays (256-byte aligned) and scalars
    std::vector<gf_instance> tinst(inst, inst + n_inst);
    std::vector<void *> blocks(n_inst, nullptr);
    gf_status st = GF_OK;
    for (int i = 0; i < n_inst && st == GF_OK; ++i) {
        int64_t b[GF_MAX_ARRAYS];
        if ((st = slot_bytes(ctx, p, inst[i], s, b)) != GF_OK)
            break;
        int64_t total = 256 * (int64_t)(GF_MAX_SCALARS * sizeof(double) / 256 + 1);
        for (int k = 0; k < GF_MAX_ARRAYS; ++k)
            total += (b[k] + 255) / 256 * 256;
        if (hipMalloc(&blocks[i], (size_t)total) != hipSuccess) {
            st = fail(ctx, GF_ENOMEM, "autotuner fallback: copies of instance %d (%lld bytes)", i, (long long)total);
            break;
        }
        char *q = (char *)blocks[i];
        hipError_t e = hipMemcpyAsync(q, inst[i].scal, GF_MAX_SCALARS * sizeof(double), hipMemcpyDeviceToDevice, s);
        tinst[i].scal = (double *)q;
        q += 256 * (int64_t)(GF_MAX_SCALARS * sizeof(double) / 256 + 1);
        for (int k = 0; k < GF_MAX_ARRAYS && e == hipSuccess; ++k) {
            if (b[k] == 0 || !inst[i].arr[k]) {
                tinst[i].arr[k] = b[k] == 0 ? inst[i].arr[k] : nullptr;
                continue;
            }
            e = hipMemcpyAsync(q, inst[i].arr[k], (size_t)b[k], hipMemcpyDeviceToDevice, s);
            tinst[i].arr[k] = q;
            q += (b[k] + 255) / 256 * 256;
        }
        if (e != hipSuccess)
            st = hipfail(ctx, e, "autotuner fallback: copying the instance");
    }
    int32_t best = -1;
    if (st == GF_OK && n_inst > 1 && mode == GF_EXEC_PERSISTENT) {
        // batched persistent run: a shape per instance (gf_tune_batched)
        std::vector<gf_launch> outs(n_inst);
        float ms = 0.0f;
        const int32_t ran = gf_tune_batched(ctx, &tp, tinst.data(), n_inst, 3, outs.data(), &ms, s);
        if (ran < 0) {
            st = (gf_status)ran;
        } else {
            *out = outs[0];
            *per = outs;
            best = 0;
            ctx->tuned[key] = {outs[0], -1, outs};
        }
    } else if (st == GF_OK) {
        gf_launch cand[GF_NUM_CANDIDATES];
        float ms[GF_NUM_CANDIDATES];
        const int32_t nc = gf_tune_candidates(ctx, &tp, tinst.data(), cand);
        const int tmode = mode == GF_EXEC_PER_REGION_GRAPH ? GF_EXEC_PER_REGION : mode;
        if (nc < 0) {
            st = (gf_status)nc;
        } else {
            const int32_t ran = gf_tune(ctx, &tp, tinst.data(), n_inst, tmode, cand, nc, 3, ms, &best, s);
            if (ran < 0)
                st = (gf_status)ran;
            else if (best >= 0) {
                *out = cand[best];
                ctx->tuned[key] = {cand[best], best, {}};
            }
        }
    }
    hipStreamSynchronize(s);
    for (void *b : blocks)
        if (b)
            hipFree(b);
    if (st != GF_OK)
        return st < -1 ? st : GF_EHIP;
    *cached = false;
    return best;
}

}  // namespace

extern "C" {

gf_status gf_nest_features(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                           double *out, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!inst || !out || n_inst < 1)
        return fail(ctx, GF_EINVAL, "null instance or output, or n_inst < 1");
    DProg p;
    gf_status st = build_program(ctx, prog, &p);
    if (st != GF_OK)
        return st;
    hipSetDevice(ctx->device);
    return nest_features(ctx, p, inst[0], n_inst, (hipStream_t)hip_stream, out);
}

int32_t gf_predict_launch(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                          int32_t mode, gf_launch *out, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!inst || !out || n_inst < 1 || n_inst > GF_MAX_INSTANCES)
        return fail(ctx, GF_EINVAL, "null instance or output, or n_inst out of range");
    DProg p;
    gf_status st = build_program(ctx, prog, &p);
    if (st != GF_OK)
        return st;
    if (ctx->pred_params.empty())
        return -1;
    hipSetDevice(ctx->device);
    return predict_launch(ctx, p, inst, n_inst, mode, (hipStream_t)hip_stream, out);
}

int32_t gf_tune_pick(const float *ms, int32_t n)
{
    if (!ms || n <= 0)
        return -1;
    int32_t best = -1;
    for (int32_t i = 0; i < n; ++i)
        if (std::isfinite(ms[i]) && (best < 0 || ms[i] < ms[best]))
            best = i;
    return best;
}

int32_t gf_batch_plan(int32_t n_inst, const int64_t *items, const double *weights, int32_t budget, int32_t align,
                      int32_t *group, int32_t *xcd)
{
    if (n_inst < 1 || n_inst > GF_MAX_INSTANCES || !items || !group || !xcd || budget < n_inst || budget > 4096)
        return GF_EINVAL;
    std::vector<int64_t> it(items, items + n_inst);
    std::vector<double> w(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        if (it[i] < 1)
            return GF_EINVAL;
        w[i] = (weights && weights[i] > 0.0) ? weights[i] : (double)it[i];
    }
    std::vector<int> g(n_inst, 1), x(n_inst, -1);
    const int grid = plan_batch(n_inst, it, w, budget, align != 0, g, x);
    for (int i = 0; i < n_inst; ++i) {
        group[i] = g[i];
        xcd[i] = x[i];
    }
    return grid;
}

gf_status gf_region_run_batched(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                                int32_t mode, const gf_launch *launches, gf_run_stats *stats, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!launches || !inst || n_inst < 1 || n_inst > GF_MAX_INSTANCES)
        return fail(ctx, GF_EINVAL, "need 1..%d instances and as many launches", GF_MAX_INSTANCES);
    if (mode == GF_EXEC_KERNEL_SPLIT)
        return fail(ctx, GF_EUNSUPPORTED, "the kernel split runs one instance");
    std::vector<InstShape> sh(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        if (launches[i].tile_y < 0 || launches[i].num_wg < 0)
            return fail(ctx, GF_EINVAL, "instance %d: negative rows per tile or weight", i);
        sh[i].tile_y = launches[i].tile_y;
        sh[i].weight = (double)launches[i].num_wg;
    }
    gf_launch common = launches[0];
    common.num_wg = 0;
    common.tile_y = 0;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    gf_status st = order_before(ctx, s);
    if (st != GF_OK)
        return st;
    st = region_run(ctx, prog, inst, n_inst, mode, &common, stats, hip_stream, sh.data());
    if (st == GF_OK)
        mark_after(ctx, s);
    return st;
}

int32_t gf_tune_candidates(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, gf_launch *out)
{
    if (!ctx || !inst || !out)
        return GF_EINVAL;
    DProg p;
    gf_status st = build_program(ctx, prog, &p);
    if (st != GF_OK)
        return st;
    for (int c = 0; c < GF_NUM_CANDIDATES; ++c)
        out[c] = decode_candidate(p, *inst, c, ctx->num_cu);
    return GF_NUM_CANDIDATES;
}

int32_t gf_tune(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst, int32_t mode,
                const gf_launch *candidates, int32_t n_cand, int32_t reps, float *ms_out, int32_t *best_index,
                void *hip_stream)
{
    if (!ctx || !inst || n_inst < 1 || !ms_out || reps < 1)
        return GF_EINVAL;
    std::vector<gf_launch> cands;
    if (candidates) {
        if (n_cand < 1)
            return fail(ctx, GF_EINVAL, "no candidates");
        cands.assign(candidates, candidates + n_cand);
    } else {
        cands.resize(GF_NUM_CANDIDATES);
        int32_t k = gf_tune_candidates(ctx, prog, inst, cands.data());
        if (k < 0)
            return k;
    }
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, GF_EHIP, "event create");
    int32_t ran = 0;
    std::vector<float> t(reps);
    for (size_t i = 0; i < cands.size(); ++i) {
        ms_out[i] = INFINITY;
        if (gf_region_run(ctx, prog, inst, n_inst, mode, &cands[i], nullptr, hip_stream) != GF_OK)
            continue;
        bool ok = true;
        for (int r = 0; r < reps && ok; ++r) {
            hipEventRecord(e0, s);
            ok = gf_region_run(ctx, prog, inst, n_inst, mode, &cands[i], nullptr, hip_stream) == GF_OK;
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess)
                ok = false;
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            t[r] = ms;
        }
        if (gf_sync(ctx, hip_stream, nullptr) != GF_OK || !ok)
            continue;
        std::sort(t.begin(), t.end());
        ms_out[i] = t[reps / 2];
        ++ran;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best_index)
        *best_index = gf_tune_pick(ms_out, (int32_t)cands.size());
    ctx->err.clear();
    return ran;
}

int32_t gf_tune_batched(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst, int32_t reps,
                        gf_launch *out, float *best_ms, void *hip_stream)
{
    if (!ctx || !prog || !inst || !out || n_inst < 1 || n_inst > GF_MAX_INSTANCES || reps < 1)
        return GF_EINVAL;
    DProg p;
    gf_status st = build_program(ctx, prog, &p);
    if (st != GF_OK)
        return st;
    hipSetDevice(ctx->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int mode = GF_EXEC_PERSISTENT;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, GF_EHIP, "event create");
    int32_t timed = 0;
    // median of reps timed runs after one warm-up; +inf if the run fails
    auto time_run = [&](const std::vector<gf_instance> &in, const gf_launch &common,
                        const std::vector<gf_launch> &per, int *grid) -> float {
        gf_run_stats rs{};
        if (gf_region_run_batched(ctx, prog, in.data(), (int32_t)in.size(), mode, per.data(), &rs, hip_stream) !=
            GF_OK)
            return INFINITY;
        std::vector<float> t(reps);
        for (int r = 0; r < reps; ++r) {
            hipEventRecord(e0, s);
            if (gf_region_run_batched(ctx, prog, in.data(), (int32_t)in.size(), mode, per.data(), nullptr,
                                      hip_stream) != GF_OK)
                return INFINITY;
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess)
                return INFINITY;
            hipEventElapsedTime(&t[r], e0, e1);
        }
        if (gf_sync(ctx, hip_stream, nullptr) != GF_OK)
            return INFINITY;
        (void)common;
        ++timed;
        if (grid)
            *grid = rs.num_wg;
        std::sort(t.begin(), t.end());
        return t[reps / 2];
    };
    std::vector<gf_instance> all(inst, inst + n_inst);
    std::vector<gf_launch> best(n_inst);
    float best_t = INFINITY;
    const bool has2d = (program_region_mask(p) & (1u << GF_R_JACOBI2D)) != 0;
    if (!has2d) {
        // one common shape from the single-program candidates, item weights
        gf_launch cand[GF_NUM_CANDIDATES];
        if (gf_tune_candidates(ctx, prog, inst, cand) < 0) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return GF_EINVAL;
        }
        for (int c = 0; c < GF_NUM_CANDIDATES; ++c) {
            std::vector<gf_launch> per(n_inst, cand[c]);
            for (auto &l : per)
                l.num_wg = 0;
            const float ms = time_run(all, cand[c], per, nullptr);
            if (ms < best_t) {
                best_t = ms;
                best = per;
            }
        }
    } else {
        // size classes of the first stencil size
        std::vector<int> cls(n_inst);
        std::map<int, std::vector<int>> members;
        for (int i = 0; i < n_inst; ++i) {
            const int64_t n = std::max<int64_t>(1, first_stencil_size(p, inst[i]));
            int c = 0;
            while ((n >> (c + 1)) > 0)
                ++c;
            cls[i] = c;
            members[c].push_back(i);
        }
        static const int kWg[3] = {64, 128, 256};
        static const int kSeg[5] = {8, 16, 32, 64, 128};
        for (int wgs : kWg) {
            gf_launch common;
            std::memset(&common, 0, sizeof common);
            common.wg_size = wgs;
            common.xcd_remap = 1;
            std::map<int, int> seg_of;
            std::map<int, double> cost_of;
            for (auto &kv : members) {
                std::vector<gf_instance> sub;
                for (int i : kv.second)
                    sub.push_back(inst[i]);
                float bt = INFINITY;
                int bs = kSeg[2], bgrid = 0;
                for (int sg : kSeg) {
                    std::vector<gf_launch> per(sub.size(), common);
                    for (auto &l : per)
                        l.tile_y = sg;
                    int grid = 0;
                    const float ms = time_run(sub, common, per, &grid);
                    if (ms < bt) {
                        bt = ms;
                        bs = sg;
                        bgrid = grid;
                    }
                }
                seg_of[kv.first] = bs;
                // workgroup-milliseconds per work item at the chosen rows
                double items = 0.0;
                Tiling tt = choose_tiling(p, &common);
                tt.tile_y = bs;
                for (int i : kv.second)
                    items += (double)std::max<int64_t>(1, max_items(p, inst[i], tt));
                cost_of[kv.first] = std::isfinite(bt) ? (double)bt * std::max(1, bgrid) / items : 0.0;
            }
            for (int variant = 0; variant < 2; ++variant) {
                std::vector<gf_launch> per(n_inst, common);
                double wmax = 0.0;
                std::vector<double> wv(n_inst, 0.0);
                for (int i = 0; i < n_inst; ++i) {
                    per[i].tile_y = seg_of[cls[i]];
                    Tiling tt = choose_tiling(p, &common);
                    tt.tile_y = per[i].tile_y;
                    const double items = (double)std::max<int64_t>(1, max_items(p, inst[i], tt));
                    wv[i] = variant == 0 ? items * cost_of[cls[i]] : items;
                    wmax = std::max(wmax, wv[i]);
                }
                for (int i = 0; i < n_inst; ++i)
                    per[i].num_wg = wmax > 0.0 ? std::max(1, (int)std::lround(1e6 * wv[i] / wmax)) : 0;
                const float ms = time_run(all, common, per, nullptr);
                if (ms < best_t) {
                    best_t = ms;
                    best = per;
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!std::isfinite(best_t))
        return fail(ctx, GF_EINVAL, "no batched configuration could run");
    for (int i = 0; i < n_inst; ++i)
        out[i] = best[i];
    if (best_ms)
        *best_ms = best_t;
    ctx->err.clear();
    return timed;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Launch-config predictor
// ---------------------------------------------------------------------------

namespace {

constexpr int kMaxMlpBatch = 65536;

// Ensure the predictor scratch holds `floats` floats (grown by reallocation;
// the previous contents are not kept).
gf_status mlp_scratch(gf_ctx *ctx, size_t floats)
{
    if (ctx->d_mlp_floats >= floats)
        return GF_OK;
    if (ctx->d_mlp) {
        hipDeviceSynchronize();
        hipFree(ctx->d_mlp);
        ctx->d_mlp = nullptr;
        ctx->d_mlp_floats = 0;
    }
    if (hipMalloc((void **)&ctx->d_mlp, floats * sizeof(float)) != hipSuccess)
        return fail(ctx, GF_ENOMEM, "predictor scratch");
    ctx->d_mlp_floats = floats;
    return GF_OK;
}

size_t mlp_part_floats(int32_t batch) { return (size_t)mlp_blocks(batch) * GF_MLP_NPARAMS; }

}  // namespace

extern "C" {

gf_status gf_mlp_forward(gf_ctx *ctx, const float *d_params, const float *d_feats, int32_t batch, float *d_y,
                         float *d_z1, float *d_z2, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_params || (batch > 0 && (!d_feats || !d_y)) || batch < 0 || batch > kMaxMlpBatch)
        return fail(ctx, GF_EINVAL, "bad MLP forward arguments");
    hipSetDevice(ctx->device);
    hipError_t e = launch_mlp_forward(d_params, d_feats, batch, d_y, d_z1, d_z2, (hipStream_t)hip_stream);
    return e == hipSuccess ? GF_OK : hipfail(ctx, e, "MLP forward");
}

gf_status gf_mlp_backward(gf_ctx *ctx, const float *d_params, const float *d_feats, const float *d_z1,
                          const float *d_z2, const float *d_y, const float *d_target, const float *d_mask,
                          int32_t batch, float inv_norm, float *d_grads, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_params || !d_feats || !d_z1 || !d_z2 || !d_y || !d_target || !d_mask || !d_grads || batch < 1 ||
        batch > kMaxMlpBatch)
        return fail(ctx, GF_EINVAL, "bad MLP backward arguments");
    hipSetDevice(ctx->device);
    gf_status st = order_before(ctx, (hipStream_t)hip_stream);
    if (st == GF_OK)
        st = mlp_scratch(ctx, mlp_part_floats(batch));
    if (st != GF_OK)
        return st;
    hipError_t e = launch_mlp_backward(d_params, d_feats, d_z1, d_z2, d_y, d_target, d_mask, batch, inv_norm,
                                       ctx->d_mlp, d_grads, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hipfail(ctx, e, "MLP backward");
    mark_after(ctx, (hipStream_t)hip_stream);
    return GF_OK;
}

gf_status gf_mlp_loss(gf_ctx *ctx, const float *d_y, const float *d_target, const float *d_mask, int64_t count,
                      float inv_norm, float *d_loss, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_y || !d_target || !d_mask || !d_loss || count < 0)
        return fail(ctx, GF_EINVAL, "bad MLP loss arguments");
    hipSetDevice(ctx->device);
    gf_status st = order_before(ctx, (hipStream_t)hip_stream);
    if (st == GF_OK)
        st = mlp_scratch(ctx, 64);
    if (st != GF_OK)
        return st;
    hipError_t e = launch_mlp_loss(d_y, d_target, d_mask, count, inv_norm, ctx->d_mlp, d_loss,
                                   (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hipfail(ctx, e, "MLP loss");
    mark_after(ctx, (hipStream_t)hip_stream);
    return GF_OK;
}

gf_status gf_adam_step(gf_ctx *ctx, float *d_params, const float *d_grads, float *d_m, float *d_v, int32_t n,
                       float lr, float beta1, float beta2, float eps, int32_t t, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_params || !d_grads || !d_m || !d_v || n < 0 || t < 1)
        return fail(ctx, GF_EINVAL, "bad Adam arguments");
    hipSetDevice(ctx->device);
    hipError_t e = launch_adam(d_params, d_grads, d_m, d_v, n, lr, beta1, beta2, eps, t, (hipStream_t)hip_stream);
    return e == hipSuccess ? GF_OK : hipfail(ctx, e, "Adam step");
}

gf_status gf_train_predictor(gf_ctx *ctx, float *d_params, float *d_m, float *d_v, const float *d_feats,
                             const float *d_target, const float *d_mask, int32_t batch, float inv_norm,
                             int32_t epochs, float lr, float *d_loss_hist, void *hip_stream)
{
    if (!ctx)
        return GF_EINVAL;
    if (!d_params || !d_m || !d_v || !d_feats || !d_target || !d_mask || batch < 1 || batch > kMaxMlpBatch ||
        epochs < 0)
        return fail(ctx, GF_EINVAL, "bad training arguments");
    hipSetDevice(ctx->device);
    // scratch: gradient partials | grads | z1 | z2 | y | loss partials
    const size_t part = mlp_part_floats(batch);
    const size_t zsz = (size_t)batch * GF_MLP_HIDDEN, ysz = (size_t)batch * GF_MLP_OUT;
    gf_status st = order_before(ctx, (hipStream_t)hip_stream);
    if (st == GF_OK)
        st = mlp_scratch(ctx, part + GF_MLP_NPARAMS + 2 * zsz + ysz + 64);
    if (st != GF_OK)
        return st;
    float *dpart = ctx->d_mlp, *dg = dpart + part, *z1 = dg + GF_MLP_NPARAMS, *z2 = z1 + zsz, *y = z2 + zsz,
          *lpart = y + ysz;
    hipStream_t s = (hipStream_t)hip_stream;
    for (int32_t e = 0; e < epochs; ++e) {
        hipError_t r = launch_mlp_forward(d_params, d_feats, batch, y, z1, z2, s);
        if (r == hipSuccess && d_loss_hist)
            r = launch_mlp_loss(y, d_target, d_mask, (int64_t)ysz, inv_norm, lpart, d_loss_hist + e, s);
        if (r == hipSuccess)
            r = launch_mlp_backward(d_params, d_feats, z1, z2, y, d_target, d_mask, batch, inv_norm, dpart, dg, s);
        if (r == hipSuccess)
            r = launch_adam(d_params, dg, d_m, d_v, GF_MLP_NPARAMS, lr, 0.9f, 0.999f, 1e-8f, e + 1, s);
        if (r != hipSuccess)
            return hipfail(ctx, r, "training step");
    }
    mark_after(ctx, s);
    return GF_OK;
}

gf_status gf_predictor_set(gf_ctx *ctx, const float *h_params, const float *h_mean, const float *h_std)
{
    if (!ctx)
        return GF_EINVAL;
    if (!h_params || !h_mean || !h_std)
        return fail(ctx, GF_EINVAL, "null predictor arrays");
    ctx->pred_params.assign(h_params, h_params + GF_MLP_NPARAMS);
    ctx->pred_mean.assign(h_mean, h_mean + GF_MLP_IN);
    ctx->pred_std.assign(h_std, h_std + GF_MLP_IN);
    return GF_OK;
}

int32_t gf_predict(gf_ctx *ctx, const double *h_features, const uint8_t *valid, float *scores)
{
    if (!ctx || !h_features)
        return GF_EINVAL;
    if (ctx->pred_params.empty())
        return -1;
    float f[GF_MLP_IN];
    for (int k = 0; k < GF_MLP_IN; ++k) {
        const double x = std::log2(1.0 + std::max(0.0, h_features[k]));
        const double sd = ctx->pred_std[k] > 0.0f ? ctx->pred_std[k] : 1.0;
        const double z = (x - ctx->pred_mean[k]) / sd;
        if (!(std::fabs(z) <= 4.0))
            return -1;
        f[k] = (float)z;
    }
    float out[GF_MLP_OUT];
    mlp_forward_host(ctx->pred_params.data(), f, out);
    if (scores)
        std::memcpy(scores, out, sizeof out);
    int32_t best = -1;
    for (int c = 0; c < GF_MLP_OUT; ++c)
        if ((!valid || valid[c]) && (best < 0 || out[c] < out[best]))
            best = c;
    return best;
}

}  // extern "C"
