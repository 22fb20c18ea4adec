// gf_internal.h -- device-side program representation, scratch layout and
// the RPC slot format shared by the libgf translation units (not public).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf.h"
#include "gf_heap_dev.h"

namespace gf {

// Persistent kernels receive the whole program by value as a kernel
// argument (copied by the runtime at enqueue time, so the caller's structs
// are free on return). 24 steps keep the argument block under 4 KiB.
constexpr int kMaxDevSteps = GF_MAX_STEPS;
constexpr int kMaxGlue = 8;
constexpr int kWave = 64;
constexpr int kNumXcd = 8;

struct DStep {
    int32_t kind;
    int32_t arr[5];
    int32_t sc[3];
    int32_t red_op;
    int32_t np;
    int32_t every;
    int32_t fmt_id;
    int32_t nargs;
    uint32_t flags;
    uint32_t mask;
    int64_t chunk;
    double c;
};

struct DProg {
    int32_t n_pro;
    int32_t n_body;
    int32_t iters;
    int32_t n_steps;      // n_pro + n_body
    int64_t last_region;  // flattened step index of the last region executed (-1: none)
    int64_t barriers;     // grid barriers one run executes
    DStep steps[kMaxDevSteps];
};

struct DInst {
    void *arr[GF_MAX_ARRAYS];
    double *scal;
    int64_t ip[GF_MAX_IPARAMS];
};

// Batched persistent launch: workgroup b of the grid belongs to instance
// `inst` as member `member` of a group of `gsize` workgroups; the group's
// barrier lives on line kGroupLine0 + inst; its reduction partials start at
// `part_off` in each half of the partials buffer; `tile_y` (> 0) replaces the
// launch's rows per tile for this instance. inst < 0: an idle workgroup.
struct BatchEntry {
    int32_t inst;
    int32_t member;
    int32_t gsize;
    int32_t tile_y;
    int64_t part_off;
};

// aligned = 1: the table places every group on one XCD, assuming workgroup b
// runs on XCD b mod 8 (the round-robin dispatch); the kernel checks that at
// start and falls back to the cross-XCD group barrier if any workgroup is
// elsewhere.
struct BatchTable {
    const BatchEntry *wg;   // gridDim.x entries
    const DInst *inst;      // per-instance bindings
    int32_t aligned;
};

// Tiling chosen on the host; identical in every workgroup of a launch.
struct Tiling {
    int32_t wg_size;
    int32_t tile_y;
    int32_t tile_z;
    int32_t items;
    int32_t xcd_remap;
    int32_t prefetch;  // 3D stencil: planes requested ahead of the one computed (1 or 2)
};

// One RPC request slot in pinned, coherent host memory (cf. the paper's
// RPCInfo / RPCArgInfo records, Section 3.2): the device fills the body,
// then publishes `seq` = ticket + 1 with a system-scope release store; the
// host runs the landing pad, writes `ret` and publishes `done` = ticket + 1.
// `freed` = ticket + 1 says the slot and its payload may be reused: the host
// sets it with `done`, except for a blocking call that copies objects back
// from the payload, whose device side sets it after the copy.
struct alignas(128) RpcSlot {
    uint64_t seq;
    uint32_t callee;
    uint32_t fmt_id;
    uint32_t nargs;
    uint32_t flags;
    uint64_t args[8];
    int64_t ret;
    uint64_t done;
    uint64_t freed;
};
static_assert(sizeof(RpcSlot) == 128, "RPC slot is one 128-byte line");

enum : uint32_t { kCalleePrintf = 1, kCalleeRegion = 2, kCalleeCall = 3 };

// Device copy of a registered call site (gf_rpc_register_call): per
// argument its source and, for a reference, the object and where the
// object sits in the slot payload (`pos`, 16-byte aligned) and which
// reference it is (`ref`, the index into the caller's resolved objects).
struct DCallArg {
    int32_t kind;
    int32_t type;
    int32_t slot;
    int32_t mode;
    int64_t value;
    int64_t start;
    int64_t size;
    int64_t offset;
    int32_t pos;
    int32_t ref;
};

struct DCall {
    int32_t callee;
    int32_t nargs;
    int32_t nrefs;
    int32_t payload;  // payload bytes used
    DCallArg a[GF_CALL_MAX_ARGS];
};

// Slot flag bit (kHeapValueFlag0 << k): heap reference argument k was not
// found in the heap and travels as a plain value.
constexpr uint32_t kHeapValueFlag0 = 1u << 8;

// Device-side timing accumulators of one call site (GF_STEP_TIMED), in
// 100 MHz clock ticks: calls, args, copy-in, wait, copy-out.
constexpr int kCallStatWords = 5;

// Device error word codes (sticky; first writer wins).
enum : int32_t {
    kErrNone = 0,
    kErrBarrierTimeout = 1,
    kErrRpcTimeout = 2,
    kErrBadStep = 3,
    kErrRegionLaunch = 4,  // the host could not launch a region requested by the main kernel
};

struct RpcRing {
    RpcSlot *slots;      // host pinned (device-visible)
    uint64_t *ticket;    // device memory
    uint32_t mask;       // nslots - 1
    uint32_t payload;    // payload bytes per slot
    int64_t timeout_ticks;  // s_memrealtime ticks (100 MHz)
    char *payloads;      // host pinned: slot i's payload at i * payload
    const DCall *calls;  // device: registered call sites
    unsigned long long *call_stats;  // device: kCallStatWords per call site
    heapdev::DHeap heap;  // heap for GF_ARG_HEAPREF lookups (base NULL: none)
};

// Device scratch owned by a context. Each counter sits on its own 128-byte
// line so spinning workgroups do not share lines with unrelated atomics.
struct Scratch {
    double *partials;        // reduction partials, two halves (double buffer)
    int64_t partials_cap;    // doubles per half
    uint32_t *lines;         // counters: line i = lines + 32*i
    int32_t *error;          // sticky device error word
    int64_t barrier_timeout_ticks;
    uint32_t *hist_rows;     // histogram partial rows (kHistRowsMax rows of 65536 u16)
    uint32_t epoch;          // persistent-launch sequence number (XCD registration)
    int32_t barrier_kind;    // kBarrierTree or kBarrierXcd
};

constexpr int kBarrierTree = 0;  // every workgroup writes back and invalidates its L2
constexpr int kBarrierXcd = 1;   // one write-back and one L2 invalidate per XCD
// Below this grid size the tree barrier is cheaper (fewer serial hops).
constexpr int kXcdBarrierMinWg = 96;
// ... and for programs with fewer barriers than this (its per-launch
// registration costs one tree barrier).
constexpr int64_t kXcdBarrierMinBarriers = 8;

constexpr int kHistRowsMax = 512;

constexpr int kLineWords = 32;  // uint32 words per 128-byte line
// line 0: generation word of the grid barrier; lines kTreeLine0..: the
// arrival counters of the barrier's fan-in tree; lines kGroupLine0 + i:
// per-instance group barriers {count, gen}; lines kFinalizeLine0 + i:
// per-region last-workgroup counters, fed by the kNumXcd arrival counters
// at lines kFinalizeSubLine0 + i * kNumXcd + g. Words 4-5 of a group line
// carry the return value of a GF_S_CALL from the group's first workgroup to
// the others.
constexpr int kTreeFanIn = 16;
constexpr int kTreeLine0 = 1;
constexpr int kTreeLines = 512;  // >= 4096/16 + 4096/256 + 1
constexpr int kGroupLine0 = kTreeLine0 + kTreeLines;
constexpr int kFinalizeLine0 = kGroupLine0 + GF_MAX_INSTANCES;
// XCD barrier: per-XCD registration words (epoch << 32 | members), per-XCD
// arrival counters, the count of XCD leaders, and
// the count of workgroups that reported an unexpected XCD id.
constexpr int kXcdRegLine0 = kFinalizeLine0 + GF_MAX_INSTANCES;
constexpr int kXcdCntLine0 = kXcdRegLine0 + kNumXcd;
constexpr int kXcdTopLine = kXcdCntLine0 + kNumXcd;
constexpr int kXcdBadLine = kXcdTopLine + 1;
constexpr int kFinalizeSubLine0 = kXcdBadLine + 1;
// Two 64-bit slots (one line each) into which the persistent kernel's
// workgroups fold a MAX reduction with one atomic each; regions alternate
// between them.
constexpr int kMaxSlotLine0 = kFinalizeSubLine0 + GF_MAX_INSTANCES * kNumXcd;
// Placement check of a batched launch, 64-bit words tagged epoch << 32:
// word 0 counts the workgroups that found themselves on another XCD than the
// first workgroup of their residue class (blockIdx.x mod kNumXcd); word 1 + r
// holds that first workgroup's XCD id + 1 for class r.
constexpr int kBatchPlaceLine = kMaxSlotLine0 + 2;
// The value a reduction's last arriving workgroup publishes under the XCD
// barrier (the bits of a double).
constexpr int kRedSlotLine = kBatchPlaceLine + 1;
constexpr int kNumLines = kRedSlotLine + 1;

// A serial step attached to a per-region launch, with its array operand
// resolved on the host (SWAPs are applied by the host while it walks the
// step list).
struct Glue {
    int32_t kind;
    int32_t sc[3];
    int32_t every;
    int32_t fmt_id;
    int32_t nargs;
    int32_t iter;
    uint32_t flags;
    uint32_t pad_;
    double c;
    double *rec;  // GF_S_RECORD destination array
    void *obj[GF_CALL_MAX_REFS];  // GF_S_CALL: array slots of its references, resolved
};

struct RegionLaunch {
    DStep step;
    void *arr[5];          // resolved operands
    double *scal;          // the instance's scalar variables (device)
    int64_t n;             // size
    int32_t n_items;
    int32_t n_glue;
    int32_t inst;          // instance index (finalize counter line)
    int32_t publish;       // 1: the glue reads what the region wrote (a host call with references)
    Glue glue[kMaxGlue];
};

// Launch-config predictor (gf_mlp.hip).
hipError_t launch_mlp_forward(const float *P, const float *feats, int32_t batch, float *y, float *z1, float *z2,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float *P, const float *feats, const float *z1, const float *z2, const float *y,
                               const float *tgt, const float *mask, int32_t batch, float inv_norm, float *part,
                               float *grads, hipStream_t s);
hipError_t launch_mlp_loss(const float *y, const float *tgt, const float *mask, int64_t count, float inv_norm,
                           float *part, float *loss, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int32_t n, float lr, float b1, float b2,
                       float eps, int32_t t, hipStream_t s);
int mlp_blocks(int32_t batch);
void mlp_forward_host(const float *P, const float *f, float *out);

// Host-side launch helpers implemented in gf_kernels.hip.
hipError_t launch_persistent(const DProg &prog, const DInst &inst, const Tiling &t, int num_wg,
                             const Scratch &scr, const RpcRing &rpc, hipStream_t s,
                             const BatchTable *batch = nullptr);
int persistent_capacity(const DProg &prog, const Tiling &t, int num_cu);
// Co-resident workgroups of the per-region kernel that runs regions of `kind`.
int region_capacity(int kind, const Tiling &t, int num_cu);
hipError_t launch_main(const DProg &prog, const DInst &inst, const RpcRing &rpc, const Scratch &scr,
                       hipStream_t s);
hipError_t launch_region(const RegionLaunch &rl, const Tiling &t, int num_wg, const Scratch &scr,
                         const RpcRing &rpc, hipStream_t s);
hipError_t launch_reduce(int op, int dt, const void *in, int64_t n, void *out, const Scratch &scr,
                         int num_cu, hipStream_t s);
int64_t reduce_grid(int64_t n, int num_cu, int64_t max_wg);
hipError_t launch_reduce_into(int op, int dt, const void *in, int64_t n, void *out, void *part, uint32_t *cnt,
                              int64_t g, hipStream_t s);
hipError_t launch_clear_u32(uint32_t *p, int32_t n, hipStream_t s);
// gf_reduce_noalloc's static scratch (gf_noalloc.hip): set-up per device
// (device current), its address, and the reduction on it
hipError_t noalloc_setup(int device);
void *noalloc_ptr(int device);
size_t noalloc_scratch_bytes();
hipError_t noalloc_reduce(int device, int num_cu, int op, int dt, const void *in, int64_t n, void *out,
                          hipStream_t s, int64_t *grid_out);
hipError_t launch_copy(void *dst, const void *src, int64_t nbytes, int num_wg, hipStream_t s);

// Number of work items (tiles / chunks) a region splits into under tiling t.
int64_t region_items(const DStep &st, int64_t n, const Tiling &t);

// Histogram support: the histogram runs in its own kernel family (1024-thread
// workgroups, 128 KiB LDS); phase 1 writes one partial row per workgroup.
bool program_is_hist_family(const DProg &prog);
bool program_mixes_hist(const DProg &prog);
int64_t hist_parts(uint32_t mask);
hipError_t launch_phases(const RegionLaunch &rl, int wg_size, int num_wg, const Scratch &scr, const RpcRing &rpc,
                         hipStream_t s);
int phases_capacity(int wg_size, int num_cu);
hipError_t launch_hist_merge(const RegionLaunch &rl, int64_t rows_used, const Scratch &scr, const RpcRing &rpc,
                             int num_cu, hipStream_t s);

}  // namespace gf
