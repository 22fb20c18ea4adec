// gf_device.h -- device building blocks: wavefront/workgroup reductions,
// the cross-workgroup barrier, the static worksharing formula and the RPC
// client. Included only by gf_kernels.hip.
#pragma once

#include <math.h>

#include "gf_internal.h"

namespace gf {

// ---------------------------------------------------------------------------
// Reductions. The paper leaves reduction clauses unrewritten (Section 4.3);
// they follow OpenMP: identity-initialised private copies, combined with the
// original value. A butterfly over the wavefront gives every lane the same
// bits (each level adds the same two partials, commutatively), so the tree
// is deterministic for a fixed workgroup size.
// ---------------------------------------------------------------------------

template <int OP>
struct RedOp;
template <>
struct RedOp<GF_OP_SUM> {
    static __device__ __forceinline__ double identity() { return 0.0; }
    static __device__ __forceinline__ double apply(double a, double b) { return a + b; }
};
template <>
struct RedOp<GF_OP_MAX> {
    static __device__ __forceinline__ double identity() { return -INFINITY; }
    static __device__ __forceinline__ double apply(double a, double b) { return a > b ? a : b; }
};

__device__ __forceinline__ double red_identity(int op) { return op == GF_OP_MAX ? -INFINITY : 0.0; }

// Order-preserving map of doubles to unsigned 64-bit keys (negative values
// have every bit flipped, non-negative ones the sign bit set), so an
// unsigned atomic max over keys is the max over the doubles: exact, and the
// same bits in any order of arrival (NaN-free inputs; -0 sorts below +0).
__device__ __forceinline__ uint64_t max_key(double d)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double max_unkey(uint64_t k)
{
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k));
}
constexpr uint64_t kMaxKeyIdentity = 0x000FFFFFFFFFFFFFull;  // max_key(-infinity)
__device__ __forceinline__ double red_apply(int op, double a, double b)
{
    return op == GF_OP_MAX ? (a > b ? a : b) : a + b;
}

template <int OP>
__device__ __forceinline__ double wave_reduce(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v = RedOp<OP>::apply(v, __shfl_xor(v, off, kWave));
    return v;
}

// Workgroup reduction; the result is valid in thread 0. `lds` holds at least
// blockDim.x / 64 doubles. Every thread of the workgroup must call it.
template <int OP>
__device__ __forceinline__ double block_reduce(double v, double *lds)
{
    v = wave_reduce<OP>(v);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    if (lane == 0)
        lds[wid] = v;
    __syncthreads();
    if (wid == 0) {
        v = lane < nw ? lds[lane] : RedOp<OP>::identity();
        v = wave_reduce<OP>(v);
    }
    __syncthreads();
    return v;
}

__device__ __forceinline__ double block_reduce_rt(int op, double v, double *lds)
{
    return op == GF_OP_MAX ? block_reduce<GF_OP_MAX>(v, lds) : block_reduce<GF_OP_SUM>(v, lds);
}

// Reduce p[0..n) in a fixed order (strided per thread, then the workgroup
// tree). Every workgroup that calls this on the same data with the same
// blockDim gets the same bits; the result is valid in thread 0.
// COHERENT: read each partial with an agent-scope load, for partials that
// were stored at agent scope and never written back by a release.
template <bool COHERENT = false>
__device__ __forceinline__ double reduce_partials(int op, const double *p, int64_t n, double *lds)
{
    double acc = red_identity(op);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        acc = red_apply(op, acc,
                        COHERENT ? __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : p[i]);
    return block_reduce_rt(op, acc, lds);
}

// ---------------------------------------------------------------------------
// Sticky error word and time.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void set_error(int32_t *err, int32_t code)
{
    int32_t expected = kErrNone;
    __hip_atomic_compare_exchange_strong(err, &expected, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t read_error(const int32_t *err)
{
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Region operands may arrive as generic pointers (the persistent kernel
// reads them from LDS); casting them to the global address space lets the
// compiler emit global loads with scalar bases instead of flat loads with
// 64-bit per-lane addresses.
#define GF_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GF_GLOBAL T *gptr(T *p)
{
    return (GF_GLOBAL T *)p;
}

// Values every lane agrees on (read from LDS, say) moved to scalar registers.
__device__ __forceinline__ void *uniform_ptr(void *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (void *)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double uniform_f64(double d)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(d));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(d));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// ---------------------------------------------------------------------------
// Cross-workgroup barrier (paper, Section 3.3: an `omp barrier` inside a
// multi-team region becomes a barrier over all teams built on global atomic
// counters). Arrivals climb a tree of counters with fan-in 16, one 128-byte
// line each, so no line takes more than 16 atomics per barrier; the last
// arrival at the root bumps a generation word on which every workgroup
// waits. Each wavefront first publishes its own stores at agent scope (a
// plain __syncthreads does not wait for stores); the last arrival of every
// counter acquires before climbing, so the release of the generation orders
// every workgroup's writes before every waiter's acquire. A counter is reset
// by its last arrival before it climbs, hence before the generation moves
// and before anyone can arrive again. A watchdog turns a stuck barrier into
// a sticky error and a clean exit instead of a hang. Returns false if the
// kernel must stop.
// ---------------------------------------------------------------------------

struct BarrierState {
    uint32_t gen;
    int32_t ok;
};

__device__ __forceinline__ bool barrier_wait(uint32_t *genw, uint32_t g, int32_t *err, int64_t timeout_ticks)
{
    const uint64_t t0 = now_ticks();
    uint32_t spins = 0;
    while (__hip_atomic_load(genw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 63u) == 0) {
            if (read_error(err) != kErrNone)
                return false;
            if ((int64_t)(now_ticks() - t0) > timeout_ticks) {
                set_error(err, kErrBarrierTimeout);
                return false;
            }
        }
    }
    return true;
}

// member: this workgroup's index in the barrier's group of nmembers.
// genw: the generation word; tree: first counter line of this barrier.
// Publication of a workgroup's stores before it arrives: every wavefront
// waits until its own stores are acknowledged (s_waitcnt vmcnt(0)), then the
// workgroup barrier, then one agent-scope release by thread 0 (which writes
// the XCD's L2 back for the other XCDs). One release per workgroup instead of
// one per wavefront halves the barrier's cost at 256+ workgroups.
__device__ __forceinline__ void wg_publish()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt left at their maxima
    __syncthreads();
    if (threadIdx.x == 0)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// The cheap half of wg_publish: every wavefront's memory operations have
// completed (loads returned; stores acknowledged, which for agent-scope
// stores means they reached memory past the XCD's L2), then the workgroup
// barrier. No L2 write-back: plain stores stay in this XCD's L2.
__device__ __forceinline__ void wg_settle()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
}

__device__ __forceinline__ bool tree_barrier(uint32_t *genw, uint32_t *tree, uint32_t member, uint32_t nmembers,
                                             BarrierState *bs, int32_t *err, int64_t timeout_ticks)
{
    wg_publish();
    if (threadIdx.x == 0) {
        const uint32_t g = bs->gen;
        uint32_t idx = member, n = nmembers, base = 0;
        bool top = true;
        while (n > 1) {
            const uint32_t grp = idx / kTreeFanIn;
            const uint32_t size = (n - grp * kTreeFanIn) < (uint32_t)kTreeFanIn ? n - grp * kTreeFanIn : kTreeFanIn;
            uint32_t *c = tree + (base + grp) * kLineWords;
            const uint32_t a = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a != size - 1) {
                top = false;
                break;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            base += (n + kTreeFanIn - 1) / kTreeFanIn;
            n = (n + kTreeFanIn - 1) / kTreeFanIn;
            idx = grp;
        }
        int32_t ok = 1;
        if (top)
            __hip_atomic_store(genw, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        else
            ok = barrier_wait(genw, g, err, timeout_ticks) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        bs->gen = g + 1u;
        bs->ok = ok;
    }
    __syncthreads();
    return bs->ok != 0;
}

// Flat barrier for the small groups of a batched launch: one line, word 0
// counts arrivals, word 1 is the generation (same publication protocol as
// the tree barrier).
__device__ __forceinline__ bool flat_barrier(uint32_t *line, uint32_t nmembers, BarrierState *bs, int32_t *err,
                                             int64_t timeout_ticks)
{
    wg_publish();
    if (threadIdx.x == 0) {
        const uint32_t g = bs->gen;
        int32_t ok = 1;
        if (nmembers > 1) {
            const uint32_t a = __hip_atomic_fetch_add(&line[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a == nmembers - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&line[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&line[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = barrier_wait(&line[1], g, err, timeout_ticks) ? 1 : 0;
            }
        } else {
            __hip_atomic_store(&line[1], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        bs->gen = g + 1u;
        bs->ok = ok;
    }
    __syncthreads();
    return bs->ok != 0;
}

// Group barrier of a batched group whose members all run on one XCD (checked
// when the launch starts): the members share that XCD's L2, so a member's
// stores are visible to the others once acknowledged, and no L2 write-back
// is needed; waiters invalidate their own caches (agent-scope acquire). The
// last arrival resets the count before it moves the generation.
__device__ __forceinline__ bool local_group_barrier(uint32_t *line, uint32_t nmembers, BarrierState *bs, int32_t *err,
                                                    int64_t timeout_ticks)
{
    wg_settle();
    if (threadIdx.x == 0) {
        const uint32_t g = bs->gen;
        int32_t ok = 1;
        const uint32_t a = __hip_atomic_fetch_add(&line[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == nmembers - 1) {
            __hip_atomic_store(&line[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // the reset has landed before the generation moves
            __hip_atomic_store(&line[1], g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = barrier_wait(&line[1], g, err, timeout_ticks) ? 1 : 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        bs->gen = g + 1u;
        bs->ok = ok;
    }
    __syncthreads();
    return bs->ok != 0;
}

// ---------------------------------------------------------------------------
// XCD-aware grid barrier. The L2 is per XCD, so what the release and acquire
// fences of the tree barrier do per workgroup (write the XCD's L2 back,
// invalidate it) needs doing once per XCD: a workgroup's stores are in its
// XCD's L2 once acknowledged, so after the XCD's last arrival has counted
// every member it writes that L2 back for all of them. Every workgroup then
// waits for the global generation to move and acquires (invalidates) for
// itself. The write-backs (one per XCD instead of one per workgroup) are
// what the tree barrier pays most for.
// Membership is counted once per launch: each workgroup reads its XCD id
// from the hardware register and adds itself to that XCD's registration word
// (tagged with the launch's epoch so stale counts from earlier launches are
// ignored); a tree barrier then makes the counts final.
// ---------------------------------------------------------------------------

struct XcdState {
    uint32_t x;    // this workgroup's XCD
    uint32_t mx;   // members on that XCD
    uint32_t nx;   // XCDs with members
    int32_t use;   // 1: XCD barrier usable (every id was in range)
};

__device__ __forceinline__ uint32_t hw_xcc_id()
{
    // s_getreg_b32 of HW_REG_XCC_ID (id 20), bits [3:0]
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11));
}

// Thread 0 only: register this workgroup with its XCD for launch `epoch`.
__device__ __forceinline__ void xcd_register(uint32_t *lines, uint32_t epoch, XcdState *xs)
{
    const uint32_t id = hw_xcc_id();
    if (id >= (uint32_t)kNumXcd) {
        __hip_atomic_fetch_add(lines + kXcdBadLine * kLineWords, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        xs->x = 0;
        return;
    }
    xs->x = id;
    uint64_t *w = (uint64_t *)(lines + (kXcdRegLine0 + id) * kLineWords);
    uint64_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        const uint64_t nw = ((uint32_t)(old >> 32) == epoch) ? old + 1u : (((uint64_t)epoch << 32) | 1u);
        if (__hip_atomic_compare_exchange_strong(w, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            break;
    }
}

// Thread 0 only, after a full barrier that follows every registration.
// The bad-id counter is read by every workgroup after that barrier and reset
// by nobody: any non-zero value disables the XCD barrier for this context.
__device__ __forceinline__ void xcd_finalize(uint32_t *lines, uint32_t epoch, XcdState *xs)
{
    uint32_t nx = 0, mx = 0;
    for (int k = 0; k < kNumXcd; ++k) {
        const uint64_t v = __hip_atomic_load((uint64_t *)(lines + (kXcdRegLine0 + k) * kLineWords),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t c = ((uint32_t)(v >> 32) == epoch) ? (uint32_t)v : 0u;
        nx += c ? 1u : 0u;
        if ((uint32_t)k == xs->x)
            mx = c;
    }
    xs->mx = mx;
    xs->nx = nx;
    xs->use = __hip_atomic_load(lines + kXcdBadLine * kLineWords, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
              mx > 0;
}

__device__ __forceinline__ bool wait_equal(uint32_t *w, uint32_t want, int32_t *err, int64_t timeout_ticks)
{
    const uint64_t t0 = now_ticks();
    uint32_t spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 63u) == 0) {
            if (read_error(err) != kErrNone)
                return false;
            if ((int64_t)(now_ticks() - t0) > timeout_ticks) {
                set_error(err, kErrBarrierTimeout);
                return false;
            }
        }
    }
    return true;
}

// reset (nullable): a 64-bit word the last arrival sets to kMaxKeyIdentity
// before it releases the others -- every workgroup has then arrived, so none
// still reads it, and none writes it again before the release.
__device__ __forceinline__ bool xcd_barrier(uint32_t *lines, const XcdState &xs, BarrierState *bs, int32_t *err,
                                            int64_t timeout_ticks, uint64_t *reset = nullptr)
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's stores are in the XCD's L2
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t *genw = lines + 1;
        uint32_t *xcnt = lines + (kXcdCntLine0 + xs.x) * kLineWords;
        uint32_t *top = lines + kXcdTopLine * kLineWords;
        const uint32_t g = bs->gen;
        int32_t ok = 1;
        const uint32_t a = __hip_atomic_fetch_add(xcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == xs.mx - 1) {
            // leader of this XCD: every member's stores are in this L2
            __hip_atomic_store(xcnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write this XCD's L2 back
            const uint32_t b = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (b == xs.nx - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (reset)
                    __hip_atomic_store(reset, kMaxKeyIdentity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0x0F70);
                __hip_atomic_store(genw, g + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                ok = wait_equal(genw, g + 1u, err, timeout_ticks) ? 1 : 0;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // invalidate this XCD's L2 (and our L1)
        } else {
            // Members wait for the global generation themselves rather than
            // for a flag their leader sets after seeing it (one hop less),
            // and each invalidates at agent scope: measured, an L1-only
            // invalidate after the leader's L2 invalidate let stale lines
            // through.
            ok = wait_equal(genw, g + 1u, err, timeout_ticks) ? 1 : 0;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        bs->gen = g + 1u;
        bs->ok = ok;
    }
    __syncthreads();
    return bs->ok != 0;
}

// The XCD barrier with a finishing step: the workgroup whose XCD leader
// arrives last runs fin() with all its threads between the arrival and the
// release. It first invalidates its XCD's L2, so fin() reads what every
// other workgroup stored before arriving (their leaders wrote their L2s
// back); what fin() publishes it writes with agent-scope atomic stores,
// which the waiting workgroups read with agent-scope atomic loads once they
// are released. The arrival side is the same as in xcd_barrier.
template <class Fin>
__device__ __forceinline__ bool xcd_barrier_fin(uint32_t *lines, const XcdState &xs, BarrierState *bs, int32_t *err,
                                                int64_t timeout_ticks, Fin fin)
{
    __shared__ int32_t s_fin;
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    uint32_t *genw = lines + 1;
    if (threadIdx.x == 0) {
        uint32_t *xcnt = lines + (kXcdCntLine0 + xs.x) * kLineWords;
        uint32_t *top = lines + kXcdTopLine * kLineWords;
        const uint32_t g = bs->gen;
        int32_t ok = 1, last = 0;
        const uint32_t a = __hip_atomic_fetch_add(xcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == xs.mx - 1) {
            __hip_atomic_store(xcnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t b = __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (b == xs.nx - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = 1;  // releases the others after fin()
            } else {
                ok = wait_equal(genw, g + 1u, err, timeout_ticks) ? 1 : 0;
            }
        } else {
            ok = wait_equal(genw, g + 1u, err, timeout_ticks) ? 1 : 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        bs->gen = g + 1u;
        bs->ok = ok;
        s_fin = last;
    }
    __syncthreads();
    if (s_fin) {
        fin();
        __builtin_amdgcn_s_waitcnt(0x0F70);  // fin's stores are acknowledged
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(genw, bs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return bs->ok != 0;
}

// Logical worker id of workgroup `wg` among `nwg`: workgroups are dispatched
// round-robin over the 8 XCDs (each with its own L2), so with remapping the
// workers of one XCD get consecutive ids and hence neighbouring tiles.
__device__ __forceinline__ int64_t worker_id(int64_t wg, int64_t nwg, int remap)
{
    if (!remap || nwg < kNumXcd)
        return wg;
    const int64_t per = nwg / kNumXcd;
    const int64_t full = per * kNumXcd;
    if (wg >= full)
        return wg;
    return (wg % kNumXcd) * per + wg / kNumXcd;
}

// ---------------------------------------------------------------------------
// Static worksharing with continuous global thread ids (Section 3.3): thread
// t of T owns [t*q + min(t,r), (t+1)*q + min(t+1,r)) with q = n / T,
// r = n % T for schedule(static), or chunks c, c+T*c, ... for
// schedule(static, c).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void static_range(int64_t n, int64_t T, int64_t t, int64_t *lo, int64_t *hi)
{
    const int64_t q = n / T, r = n % T;
    *lo = t * q + (t < r ? t : r);
    *hi = (t + 1) * q + (t + 1 < r ? t + 1 : r);
}

// ---------------------------------------------------------------------------
// RPC client (Section 2.3 / 3.2). A ticket from a device-memory counter
// selects a slot; the client waits until the slot's previous use is done,
// fills the request and publishes it with a system-scope release store.
// Posted calls return at once; blocking calls wait for `done` (the paper's
// completion flag in shared memory) and return the host's value.
// ---------------------------------------------------------------------------

// Wait until a slot word (done or freed) reaches `want`.
__device__ __forceinline__ bool rpc_wait_word(const uint64_t *word, uint64_t want, const RpcRing &rpc, int32_t *err)
{
    const uint64_t t0 = now_ticks();
    uint32_t spins = 0;
    while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) < want) {
        __builtin_amdgcn_s_sleep(2);
        if ((++spins & 15u) == 0 && (int64_t)(now_ticks() - t0) > rpc.timeout_ticks) {
            set_error(err, kErrRpcTimeout);
            return false;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    return true;
}

// Called by a single thread. Returns false on timeout (error word set).
__device__ __forceinline__ bool rpc_call(const RpcRing &rpc, uint32_t callee, uint32_t fmt_id, uint32_t nargs,
                                         const uint64_t *args, uint32_t flags, int64_t *ret, int32_t *err)
{
    const uint64_t t = __hip_atomic_fetch_add(rpc.ticket, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    RpcSlot *slot = rpc.slots + (t & rpc.mask);
    const uint64_t nslots = (uint64_t)rpc.mask + 1;
    if (t >= nslots && !rpc_wait_word(&slot->freed, t - nslots + 1, rpc, err))
        return false;
    slot->callee = callee;
    slot->fmt_id = fmt_id;
    slot->nargs = nargs;
    slot->flags = flags;
    for (uint32_t i = 0; i < nargs && i < 8; ++i)
        slot->args[i] = args[i];
    __hip_atomic_store(&slot->seq, t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    if (flags & GF_STEP_BLOCKING) {
        if (!rpc_wait_word(&slot->done, t + 1, rpc, err))
            return false;
        if (ret)
            *ret = __hip_atomic_load(&slot->ret, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return true;
}

}  // namespace gf
