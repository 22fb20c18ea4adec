/*
 * gf.h -- C ABI of libgf: GPU-First execution of legacy OpenMP-style loop
 * programs on one MI355X (gfx950).
 *
 * Model (paper, Section 2.1 "OpenMP Execution Model" and Section 3.3
 * "Multi-Team Execution and Kernel Split"): a legacy program is serial code
 * run by one initial thread, interleaved with `parallel for` regions. Each
 * region's iterations are spread over every thread of every workgroup with
 * continuous global thread ids, and the implicit barrier at the end of a
 * region spans all workgroups. Host-only library calls (printf, fprintf,
 * snprintf, sscanf, fwrite, fread) made by the initial thread are forwarded
 * to the host by a synchronous client-server remote procedure call
 * (Section 2.3 "Host Remote Procedural Call", Section 3.2 "Generating Remote
 * Procedural Calls").
 *
 * A program is given as a step list (gf_program): a prologue run once and a
 * body run `iters` times. A step is either a REGION (a loop body from the
 * region catalogue below, optionally with one reduction clause into a scalar
 * variable) or a SERIAL op of the initial thread (scalar arithmetic, pointer
 * swap, history record, printf or another host call through RPC).
 *
 * Reductions: the paper does not rewrite reduction clauses (Section 4.3), so
 * they follow OpenMP semantics: private copies start at the operator's
 * identity; the variable ends as its original value combined with all
 * contributions. The combination order of floating-point sums is
 * unspecified; libgf fixes it per tile decomposition, so a given launch
 * configuration is bit-reproducible.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* or held in gf_instance are DEVICE pointers (HIP
 *    device memory, e.g. from torch tensors) owned by the caller; they must
 *    stay valid until the enqueued work has completed on `hip_stream`.
 *  - Host-side structs (gf_program, gf_instance, gf_launch) are copied
 *    during the call; the caller may free them on return.
 *  - `hip_stream` is a hipStream_t (NULL = the default stream). Runs and
 *    reductions are enqueued asynchronously on it.
 *  - Return value: GF_OK (0) or a negative gf_status. Argument errors are
 *    detected before anything is enqueued. Device-side failures (barrier or
 *    RPC watchdog, bad step) set a sticky error word that surfaces as
 *    GF_EDEVICE / GF_ETIMEOUT from the next gf_sync or gf_region_run.
 *  - gf_last_error(ctx) returns a message for the last failure on that ctx.
 *  - No C++ exception crosses the ABI. A ctx is not thread-safe, except that
 *    gf_rpc_poll may run concurrently on one server thread.
 *  - Work enqueued through one ctx shares its device scratch (reduction
 *    partials, counter lines, the batched-launch table, training buffers),
 *    so a ctx orders its own enqueues across streams: a gf_region_run,
 *    gf_reduce, gf_mlp_backward, gf_mlp_loss or gf_train_predictor call on a
 *    stream other than the previous such call's first makes that stream
 *    wait for the previous call's work. Work enqueued while the caller
 *    captures the stream into a graph is not tracked; two captured graphs of
 *    one ctx must not be replayed concurrently. Use one ctx per stream for
 *    concurrent execution.
 */
#ifndef GF_H
#define GF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx gf_ctx;

typedef enum {
    GF_OK = 0,
    GF_EINVAL = -1,       /* invalid argument or program; nothing enqueued */
    GF_ENOMEM = -2,       /* host or device allocation failed */
    GF_EHIP = -3,         /* a HIP runtime call failed */
    GF_ETIMEOUT = -4,     /* a device watchdog (barrier or RPC wait) expired */
    GF_ERPC = -5,         /* malformed RPC request */
    GF_EDEVICE = -6,      /* device reported an error (bad step, ring overflow) */
    GF_EUNSUPPORTED = -7  /* valid request the library does not implement */
} gf_status;

typedef enum { GF_OP_SUM = 0, GF_OP_MAX = 1, GF_OP_NONE = -1 } gf_op;
typedef enum { GF_F64 = 0, GF_U32 = 1, GF_U64 = 2, GF_I64 = 3 } gf_dtype;

typedef enum {
    GF_EXEC_PER_REGION = 0,       /* one kernel launch per region (host walks the steps) */
    GF_EXEC_PERSISTENT = 1,       /* one cooperative launch; grid barrier between regions */
    GF_EXEC_PER_REGION_GRAPH = 2, /* per-region launches captured once into a HIP graph */
    GF_EXEC_KERNEL_SPLIT = 3      /* the paper's kernel split (Section 3.3): a one-thread main
                                     kernel runs the serial steps and asks the host by RPC to
                                     launch each region, waiting for it; one instance; the call
                                     returns when the program has finished */
} gf_exec;

#define GF_MAX_ARRAYS 16
#define GF_MAX_SCALARS 16
#define GF_MAX_IPARAMS 8
#define GF_MAX_STEPS 24    /* prologue + body steps of one program */
#define GF_MAX_INSTANCES 4096

/* ---- step kinds --------------------------------------------------------
 * Region kinds: `parallel for` bodies. Operands are array slots (arr[]),
 * scalar slots (sc[]) and a size taken from the instance (ip[np]).
 *
 * GF_R_JACOBI2D  arr[0]=u (in, n x n f64 row-major), arr[1]=w (out).
 *                For every interior (j,i): v = ((W+E)+(S+N))*0.25, w = v,
 *                d = v-u. Reduction clause (optional, op SUM): d*d into sc[0].
 * GF_R_JACOBI3D  arr[0]=u (in, n^3 f64, x fastest), arr[1]=w (out).
 *                v = (((xm+xp)+(ym+yp))+(zm+zp))*(1/6). Reduction (optional,
 *                op MAX): |d| into sc[0].
 * GF_R_SPMV      arr[0]=rowptr (i32, n+1), arr[1]=col (i32), arr[2]=val (f64),
 *                arr[3]=x (f64), arr[4]=y (f64, out); y_i = sum_k val*x[col],
 *                summed serially in column order per row. n = rows.
 * GF_R_DOT       arr[0]=a, arr[1]=b (f64, n). Reduction SUM of a_i*b_i into sc[0].
 * GF_R_AXPBY     arr[0]=out, arr[1]=x, arr[2]=y (f64, n; out may alias x or y):
 *                out_i = x_i + s*y_i with s = scal[sc[1]] * c (c = +1 or -1
 *                for exactness; any double allowed).
 * GF_R_HIST      arr[0]=keys (u32, n), arr[1]=bins (u32); bins[key & mask] += 1.
 * GF_R_OWNER     arr[0]=owner (i32, n): owner[i] = continuous global thread
 *                id that executed iteration i under schedule(static[,chunk]).
 * GF_R_PHASES    a `parallel` region with manual worksharing and barriers
 *                (Section 3.3: thread-id queries and `omp barrier` rewritten
 *                to span all workgroups). Thread t of T (the global
 *                omp_get_thread_num / omp_get_num_threads, continuous across
 *                workgroups) owns the block [t*q + min(t,r), (t+1)*q +
 *                min(t+1,r)) of [0, n), q = n / T, r = n % T. For phase
 *                p = 0 .. P-1 (P = chunk >= 1) it computes, over its block,
 *                dst[i] = src[i] + src[(i + s) % n] with s = mask (< n), then
 *                all threads meet at an `omp barrier` before the next phase
 *                reads what other workgroups wrote. src and dst start as
 *                arr[0] and arr[1] (f64, n) and swap after every phase, so the
 *                result is in arr[P % 2]. arr[2] (optional, -1 for none; i32,
 *                n): owner[i] = t. No reduction clause. Per-region launches
 *                use at most one co-resident wave of workgroups (the in-region
 *                barrier needs all of them resident).
 *
 * Serial kinds (the initial thread; scal = the instance's scalar variables,
 * `iter` = 0-based body iteration, -1 in the prologue):
 * GF_S_SET       scal[sc[0]] = c
 * GF_S_COPY      scal[sc[0]] = scal[sc[1]]
 * GF_S_DIV       scal[sc[0]] = scal[sc[1]] / scal[sc[2]]
 * GF_S_SQRT      scal[sc[0]] = sqrt(scal[sc[1]])
 * GF_S_SWAP      swap array slots arr[0] and arr[1]
 * GF_S_RECORD    ((double*)arr-slot arr[0])[iter] = scal[sc[0]]
 * GF_S_PRINTF    if ((iter+1) % every == 0): printf(format fmt_id) through
 *                RPC with arguments (int)(iter+1), scal[sc[0]] .. scal[sc[nargs-2]]
 *                (nargs counts the iteration argument). Posted (fire and
 *                forget) unless flags & GF_STEP_BLOCKING.
 * GF_S_CALL      a host library call through RPC at call site fmt_id (from
 *                gf_rpc_register_call). It fires once in the prologue, and
 *                in the body when (iter+1) % every == 0. Reference arguments
 *                are copied into the request and back by their access mode.
 *                If sc[0] >= 0, scal[sc[0]] = the callee's return value (as a
 *                double). A call with write or read-write references or a
 *                return slot must be blocking (GF_STEP_BLOCKING).
 *                GF_STEP_TIMED adds per-stage timing (gf_rpc_call_stats).
 *                Persistent mode: the call runs on the first workgroup,
 *                then a grid barrier publishes its writes to every
 *                workgroup.
 */
typedef enum {
    GF_R_JACOBI2D = 1,
    GF_R_JACOBI3D = 2,
    GF_R_SPMV = 3,
    GF_R_DOT = 4,
    GF_R_AXPBY = 5,
    GF_R_HIST = 6,
    GF_R_OWNER = 7,
    GF_R_PHASES = 8,
    GF_S_SET = 32,
    GF_S_COPY = 33,
    GF_S_DIV = 34,
    GF_S_SQRT = 35,
    GF_S_SWAP = 36,
    GF_S_RECORD = 37,
    GF_S_PRINTF = 38,
    GF_S_CALL = 39
} gf_step_kind;

#define GF_STEP_BLOCKING 1u
#define GF_STEP_TIMED 2u   /* GF_S_CALL: accumulate per-stage times */
/* GF_STEP_NOWAIT on a region: OpenMP's nowait clause (Section 3.3: a
 * region's implicit barrier becomes a barrier across all workgroups in the
 * persistent modes; nowait removes it). Threads that finish their part go on
 * to the steps that follow without waiting for the others. The caller
 * guarantees, as an OpenMP programmer does, that nothing before the next
 * barrier reads or writes another thread's part of what the region
 * accessed. As with OpenMP's static schedule, GF_R_DOT and GF_R_AXPBY over
 * the same size in one launch give element i to the same thread, so an
 * axpby writing r may skip its barrier before a dot reading r. Rejected
 * (GF_EINVAL) with a reduction clause (its value needs the barrier), on
 * GF_R_HIST and GF_R_PHASES, and when a GF_S_CALL with reference arguments
 * follows before the next region (its copy-in would read data other
 * workgroups may still write).
 * The per-region and kernel-split modes end every region with its launch
 * and ignore the flag. */
#define GF_STEP_NOWAIT 4u

typedef struct {
    int32_t kind;      /* gf_step_kind */
    int32_t arr[5];    /* array slot indices (unused: -1) */
    int32_t sc[3];     /* scalar slot indices (unused: -1) */
    int32_t red_op;    /* reduction clause of a region: GF_OP_SUM / GF_OP_MAX / GF_OP_NONE */
    int32_t np;        /* index into gf_instance.ip of the region's size */
    int32_t every;     /* GF_S_PRINTF period (iterations) */
    int32_t fmt_id;    /* GF_S_PRINTF format id from gf_rpc_register_format;
                          GF_S_CALL call-site id from gf_rpc_register_call */
    int32_t nargs;     /* GF_S_PRINTF argument count incl. the iteration number */
    uint32_t flags;    /* GF_STEP_BLOCKING, GF_STEP_TIMED (serial); GF_STEP_NOWAIT (regions) */
    uint32_t mask;     /* GF_R_HIST bin mask (nbins - 1, nbins a power of two);
                          GF_R_PHASES shift s */
    int64_t chunk;     /* GF_R_OWNER schedule(static, chunk), 0 = schedule(static);
                          GF_R_PHASES phase count */
    double c;          /* constant of GF_S_SET / GF_R_AXPBY */
} gf_step;

typedef struct {
    int32_t n_prologue;
    const gf_step *prologue;
    int32_t n_body;
    const gf_step *body;
    int32_t iters;     /* body repetitions (the program's main loop) */
} gf_program;

/* Bindings of one program instance. arr[] are device pointers; scal is a
 * device array of GF_MAX_SCALARS doubles holding the scalar variables (read
 * at start, written back at the end); ip[] are sizes. */
typedef struct {
    void *arr[GF_MAX_ARRAYS];
    double *scal;
    int64_t ip[GF_MAX_IPARAMS];
} gf_instance;

/* Launch configuration. Zero fields mean "choose": the persistent grid is
 * sized from occupancy; tiles come from the tuning database, else defaults. */
typedef struct {
    int32_t wg_size;     /* threads per workgroup (multiple of 64, <= 1024) */
    int32_t num_wg;      /* workgroups (persistent: <= co-resident capacity);
                            0 = default: persistent, up to two per CU with
                            balanced rounds of work items; per region, one
                            per work item up to 16 per CU, SpMV up to the
                            region kernel's resident capacity */
    int32_t tile_y;      /* 3D stencil: rows per tile (1, 2, 4, 8 or 16); 2D stencil:
                          * rows per segment a workgroup marches through (>= 1) */
    int32_t tile_z;      /* 3D stencil z-segment length */
    int32_t items;       /* elements per thread for streaming regions (histogram:
                          * groups of four keys per thread per chunk, 1, 2, 4 or 8) */
    int32_t xcd_remap;   /* 1: map consecutive tiles to one XCD (8 XCDs) */
    int32_t prefetch;    /* 3D stencil: planes loaded ahead of the one computed, 1 or 2
                          * (2 needs tile_y <= 8); ignored by other regions */
} gf_launch;

typedef struct {
    int32_t regions;       /* region executions enqueued */
    int32_t launches;      /* kernel launches enqueued */
    int32_t barriers;      /* grid barriers executed per persistent launch */
    int32_t num_wg;        /* workgroups used (largest launch) */
    int32_t wg_size;
    int32_t rpc_posted;    /* filled by gf_sync: RPC requests serviced so far */
    int32_t candidate;     /* gf_region_run with launch NULL: the launch shape the
                              installed predictor or its autotuner fallback chose
                              (0..31), -1 if none */
    int32_t launch_source; /* where the launch shape came from: GF_LAUNCH_* */
} gf_run_stats;

#define GF_LAUNCH_GIVEN 0        /* the caller's launch, or the defaults */
#define GF_LAUNCH_PREDICTED 1    /* the installed predictor's choice */
#define GF_LAUNCH_TUNED 2        /* the autotuner, timed during this call (predictor deferred) */
#define GF_LAUNCH_TUNED_CACHED 3 /* the autotuner's earlier choice for this program, sizes and mode */

typedef struct {
    int32_t rpc_slots;        /* ring slots (power of two, 8..4096); 0 = 256 */
    int32_t rpc_capture;      /* 1: landing pads append output to a buffer read by
                                 gf_rpc_take_output instead of writing stdout (and,
                                 for GF_S_CALL fprintf / fwrite, stdout or stderr) */
    int32_t rpc_thread;       /* 1: libgf runs the RPC server thread itself */
    int64_t rpc_timeout_us;   /* device watchdog for RPC slot waits; 0 = 2 s */
    int64_t barrier_timeout_us; /* device watchdog for grid barriers; 0 = 10 s */
    int64_t rpc_payload;      /* payload bytes per ring slot for the objects of
                                 GF_S_CALL references (multiple of 16, 16..65536);
                                 0 = 1024 */
    int32_t tune_fallback;    /* gf_region_run with launch NULL when the installed
                                 predictor defers: 0 = run the autotuner (on copies of
                                 the instances' data) and cache its choice; -1 = use
                                 the default launch */
} gf_ctx_opts;

/* Create a context on HIP device `hip_device`: allocates the pinned RPC ring
 * (hipHostMalloc, coherent), device scratch (reduction partials, barrier
 * counters, error word, program copies). opts may be NULL (defaults). */
gf_status gf_ctx_create(int32_t hip_device, const gf_ctx_opts *opts, gf_ctx **out);
/* Waits for the device, stops the server thread, frees everything. NULL ok. */
gf_status gf_ctx_destroy(gf_ctx *ctx);
/* Message of the last failure on ctx (never NULL; "" if none). Valid until
 * the next call on ctx. */
const char *gf_last_error(const gf_ctx *ctx);

/* Run a legacy program (Section 3.3): enqueue n_inst instances of `prog` on
 * hip_stream in execution mode `mode`. With n_inst > 1 the instances run
 * concurrently in one persistent launch, each on its own group of
 * workgroups with group barriers (GF_EXEC_PERSISTENT), or as per-instance
 * launches (per-region modes). launch may be NULL: with an installed
 * predictor the predicted launch shape is used (gf_predict_launch; for SpMV
 * programs that call waits for hip_stream); when the predictor defers (the
 * program lies outside its training distribution, e.g. several instances)
 * the autotuner decides: every candidate shape is timed on copies of the
 * instances' arrays and scalars (allocated for the call and freed; the
 * program's printf and host-call steps left out), the fastest is used and
 * cached in the ctx for this program, sizes and mode (opts.tune_fallback).
 * Without a predictor, or with the fallback off, the defaults are used.
 * stats (nullable) receives counts. Asynchronous: results are valid after
 * the stream completes; call gf_sync to surface device errors. */
gf_status gf_region_run(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst,
                        int32_t n_inst, int32_t mode, const gf_launch *launch,
                        gf_run_stats *stats, void *hip_stream);

/* A single reduction region over a device array: d_out[0] = op over
 * d_in[0..n) (SUM: + ; MAX: max, F64 max starts from -infinity, unsigned
 * from 0, I64 from INT64_MIN). U32 inputs are widened: d_out is a u64 for
 * GF_U32 (sum and max) and of type dt otherwise. F64 sums use a fixed two-pass tree
 * (deterministic for a given n). n may be 0 (identity). */
gf_status gf_reduce(gf_ctx *ctx, int32_t op, int32_t dt, const void *d_in, int64_t n,
                    void *d_out, void *hip_stream);

/* gf_reduce without any allocation, for callers that cannot allocate
 * device memory at call time: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same arguments, semantics and
 * result bits as gf_reduce (same grid and summation order). Its scratch is
 * a static device array of 8,448 bytes per GPU (one counter line and 1,024
 * per-workgroup partials), held until the process ends; gf_ctx_create
 * resolves that GPU's copy once, and this call allocates nothing and calls
 * no allocating routine. The grid never exceeds the 1,024 partials the
 * array holds, so any n >= 0 fits; a grid that would not fit is rejected
 * with GF_EINVAL. The counter word is cleared by a small kernel at the start
 * of every call (no memset). All calls on one GPU share its array: calls
 * that overlap on one GPU (several streams or host threads, in any
 * context) race and give wrong results; the caller serialises them. Not
 * ordered against the context's other work on other streams. */
gf_status gf_reduce_noalloc(gf_ctx *ctx, int32_t op, int32_t dt, const void *d_in, int64_t n,
                            void *d_out, void *hip_stream);

/* Service pending RPC requests in ticket (FIFO) order (Section 2.3: the
 * host is the server of a synchronous client-server protocol): runs the
 * landing pad of each request, writes its return value and marks it done.
 * Waits up to timeout_us for the first request (0 = do not wait). Returns
 * the number of requests serviced (>= 0) or a negative gf_status. */
int32_t gf_rpc_poll(gf_ctx *ctx, int32_t max_requests, int32_t timeout_us);

/* Register a printf format for device-side calls; sig lists the argument
 * types: 'i' (64-bit int) or 'd' (double), e.g. "id". Returns id >= 0 or a
 * negative gf_status. The host landing pad is selected by (callee, sig). */
int32_t gf_rpc_register_format(gf_ctx *ctx, const char *fmt, const char *sig);

/* ---- general host calls (Section 3.2, "Generating Remote Procedural Calls")
 * A call site names a host callee and describes each argument the way the
 * device-side argument record of the paper does. Value arguments travel as
 * 64-bit words; an opaque host pointer (such as a FILE *) is a value and is
 * used by the host unchanged. A reference argument points into an object in
 * device memory: the object (start, size) inside array slot `slot` of the
 * instance, and the pointer's byte offset into it. Objects of read and
 * read-write references are copied into the request's payload before the
 * call; the host passes the callee a pointer at the same offset into its
 * copy; objects of write and read-write references are copied back after
 * the call (a write-only object is zero-filled on the host first, so bytes
 * the callee does not write come back as zero). The host wrapper that makes
 * the call is selected by (callee, argument types): one non-variadic landing
 * pad per type signature of a variadic callee. */
typedef enum {
    GF_CALLEE_FPRINTF = 1,  /* int fprintf(FILE *f, const char *fmt, ...);
                               fixed "pp", then up to 4 of 'i' 'd' 'p' */
    GF_CALLEE_SNPRINTF = 2, /* int snprintf(char *buf, size_t n, const char *fmt, ...);
                               fixed "pip", then up to 4 of 'i' 'd' 'p' */
    GF_CALLEE_SSCANF = 3,   /* int sscanf(const char *s, const char *fmt, ...);
                               fixed "pp", then up to 6 of 'p' */
    GF_CALLEE_FWRITE = 4,   /* size_t fwrite(const void *p, size_t size, size_t n, FILE *f); "piip" */
    GF_CALLEE_FREAD = 5     /* size_t fread(void *p, size_t size, size_t n, FILE *f); "piip" */
} gf_callee;

typedef enum {
    GF_ARG_CONST = 0,   /* value: the word `value` (an integer, a double's bits, or a host pointer) */
    GF_ARG_SCALAR = 1,  /* value: scal[slot] as a double ('d') or truncated to int64 ('i') */
    GF_ARG_ITER = 2,    /* value: iter + 1 (0 in the prologue), type 'i' */
    GF_ARG_REF = 3,     /* reference into array slot `slot`, type 'p' */
    GF_ARG_HEAPREF = 4  /* reference through a heap pointer, type 'p': the pointer is the
                           64-bit word at element `start` of array slot `slot`. At the call
                           the context's heap (gf_ctx_set_heap) looks up the live allocation
                           that holds it (the paper's run-time lookup of an object the
                           compiler cannot name); that whole object, at most `size` bytes,
                           is copied in and back by `mode`, and the callee gets the pointer
                           at the same offset into the copy. A pointer the heap does not
                           hold, or an object larger than `size`, is passed unchanged as a
                           value (Section 3.2) */
} gf_arg_kind;

typedef enum { GF_REF_READ = 1, GF_REF_WRITE = 2, GF_REF_READWRITE = 3 } gf_ref_mode;

#define GF_CALL_MAX_ARGS 8
#define GF_CALL_MAX_REFS 4
#define GF_CALL_MAX_SITES 64

typedef struct {
    int32_t kind;     /* gf_arg_kind */
    int32_t type;     /* 'i' (int64), 'd' (double) or 'p' (pointer) */
    int32_t slot;     /* GF_ARG_SCALAR: scalar slot; GF_ARG_REF, GF_ARG_HEAPREF: array slot */
    int32_t mode;     /* GF_ARG_REF, GF_ARG_HEAPREF: gf_ref_mode */
    int64_t value;    /* GF_ARG_CONST: the 64-bit word */
    int64_t start;    /* GF_ARG_REF: byte offset of the object in the array;
                         GF_ARG_HEAPREF: index of the pointer word in the array */
    int64_t size;     /* GF_ARG_REF: object bytes (>= 1); GF_ARG_HEAPREF: the largest
                         object shipped (>= 16) */
    int64_t offset;   /* GF_ARG_REF: byte offset of the pointer into the object (0..size) */
} gf_call_arg;

/* Register a call site: callee (gf_callee) and nargs argument records.
 * Checks the types against the callee's parameters, at most
 * GF_CALL_MAX_REFS references, and that the objects (each rounded up to 16
 * bytes) fit the slot payload. Returns the call-site id >= 0 or a negative
 * gf_status (GF_EINVAL; GF_EUNSUPPORTED for a signature without a landing
 * pad). The caller guarantees that each referenced object, and the pointer
 * word of each heap reference, lies inside its array, and that host pointer
 * values are valid on the host. */
int32_t gf_rpc_register_call(gf_ctx *ctx, int32_t callee, const gf_call_arg *args, int32_t nargs);

/* Average per-call stage times in microseconds of the GF_STEP_TIMED calls at
 * one call site (paper, Section 5, RPC performance). The device stages use
 * the GPU's 100 MHz constant clock; the host stages the host's monotonic
 * clock. Valid after gf_sync. */
typedef struct {
    int64_t calls;           /* timed calls */
    double dev_args_us;      /* device: take a ticket, wait for a free slot, build the argument words */
    double dev_copy_in_us;   /* device: copy read and read-write objects into the payload */
    double dev_wait_us;      /* device: publish the request until the completion flag is seen */
    double dev_copy_out_us;  /* device: copy write and read-write objects back */
    double host_decode_us;   /* host: read the request, translate references into payload pointers */
    double host_call_us;     /* host: the landing pad (the library call) */
    double host_reply_us;    /* host: store the return value and the completion flag */
    double transit_us;       /* dev_wait_us minus the host stages: request and reply in flight
                                plus the server's pickup delay */
} gf_call_stats;

/* Fill *out for call site `call_id`; reset != 0 clears its counters. */
gf_status gf_rpc_call_stats(gf_ctx *ctx, int32_t call_id, gf_call_stats *out, int32_t reset);

/* Copy captured landing-pad output (rpc_capture=1) into buf (NUL-terminated,
 * at most cap-1 bytes) and clear it. Returns bytes copied or gf_status. */
int64_t gf_rpc_take_output(gf_ctx *ctx, char *buf, int64_t cap);

/* Block until all work enqueued on hip_stream completes, service remaining
 * posted RPCs, and surface the sticky device error word. */
gf_status gf_sync(gf_ctx *ctx, void *hip_stream, gf_run_stats *stats);

/* Persistent-launch capacity: co-resident workgroups of wg_size threads for
 * the persistent kernel that would run `prog` (0 on error). */
int32_t gf_persistent_capacity(gf_ctx *ctx, const gf_program *prog, int32_t wg_size);

/* After the last batched persistent launch of ctx has completed: the number
 * of its workgroups that ran on another XCD than the first workgroup of their
 * residue class (blockIdx.x mod 8; the batched table keeps each group in one
 * class). 0: every group shared one XCD and used the group barrier without
 * L2 write-back; > 0: all groups used the cross-XCD one. -1 if that launch
 * made no placement check (groups laid out in order). Which XCD takes which
 * class varies between launches and is not checked. Synchronises with the
 * device. Diagnostic. */
int64_t gf_batch_misplaced(gf_ctx *ctx);

/* Device copy kernel (bandwidth probe for the HBM ceiling): d_dst = d_src,
 * nbytes a multiple of 16. num_wg > 0: a grid-stride loop over num_wg
 * workgroups; num_wg <= 0: one 4 x 16-byte tile per thread over the whole
 * array. */
gf_status gf_copy(gf_ctx *ctx, void *d_dst, const void *d_src, int64_t nbytes, int32_t num_wg,
                  void *hip_stream);

/* ---- autotuner -----------------------------------------------------------
 * The paper fixes team counts by hand and notes that matching them to the
 * loop matters (Section 5.3, "Parallel Region Modeling"); libgf instead
 * times a fixed list of GF_NUM_CANDIDATES launch shapes on the real run.
 * Candidate c (0..31) is decoded per kernel family of the program, with
 * a = c & 3, b = (c >> 2) & 3, h = c >> 4:
 *   3D stencil : tile_y = {1,2,4,8}[a], tile_z = ceil((n-2)/{2,3,4,6}[b]),
 *                num_wg = h ? 3 * CUs : default
 *   2D stencil : tile_y = {2,8,32,128}[a] rows per segment,
 *                wg_size = {64,128,192,256}[b], xcd_remap = 1 - h
 *   streaming (SpMV, dot, axpby): wg_size = {64,128,192,256}[a],
 *                items = {1,2,4,8}[b], num_wg = h ? 4 * CUs : default
 *   histogram  : wg_size = {256,512,768,1024}[a], items = {1,2,4,8}[b],
 *                num_wg = h ? CUs : CUs / 2
 * (n is the size of the program's first stencil region in `inst`). */
#define GF_NUM_CANDIDATES 32

/* Write the GF_NUM_CANDIDATES decoded launches for prog/inst into out.
 * Returns GF_NUM_CANDIDATES or a negative gf_status. */
int32_t gf_tune_candidates(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, gf_launch *out);

/* Time candidate launches by running the program for real on n_inst
 * instances in `mode` on hip_stream: one warm-up run, then `reps` runs timed
 * with HIP events; ms_out[i] receives the median (+infinity if candidate i
 * cannot run). The runs' side effects on the instances' data happen
 * (reps + 1) times per candidate. Blocks until done. candidates NULL uses
 * the built-in list (n_cand = GF_NUM_CANDIDATES). *best_index receives the
 * fastest candidate (gf_tune_pick). Returns the number of candidates that
 * ran, or a negative gf_status. */
int32_t gf_tune(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst, int32_t mode,
                const gf_launch *candidates, int32_t n_cand, int32_t reps, float *ms_out, int32_t *best_index,
                void *hip_stream);

/* Index of the smallest finite ms[i] (ties: lowest index), or -1 if none is
 * finite. Pure host function. */
int32_t gf_tune_pick(const float *ms, int32_t n);

/* ---- batched runs with a launch shape per instance -----------------------
 * Many uneven instances of one program (not in the paper): instance i runs
 * with launches[i].tile_y rows per tile (0: the default; a 3D stencil's rows
 * must be the same for all, being compiled into the kernel) and a share of
 * the persistent grid proportional to launches[i].num_wg (a relative weight;
 * 0: its number of work items). wg_size, items, xcd_remap and prefetch are
 * taken from launches[0]; the grid is the co-resident capacity. In the
 * persistent mode the instances are packed onto the eight XCDs and each
 * instance's workgroups stay on one XCD (see DESIGN of the batched launch);
 * the per-region modes launch each instance with its own rows per tile.
 * Same conventions as gf_region_run otherwise. */
gf_status gf_region_run_batched(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst,
                                int32_t n_inst, int32_t mode, const gf_launch *launches,
                                gf_run_stats *stats, void *hip_stream);

/* The plan of a batched persistent launch (pure host function, used by
 * gf_region_run_batched): instance i has items[i] >= 1 work items per region
 * and weight weights[i] (its total cost; NULL or <= 0: items[i]). With align,
 * instances are packed onto the 8 XCDs (xcd[i]; heaviest first onto the least
 * loaded XCD with room) and each XCD's budget / 8 workgroups are shared among
 * its instances; else xcd[i] = -1 and the whole budget is shared. A group of
 * g workgroups takes ceil(items / g) items each per region; group[i]
 * receives the sizes that minimise the slowest group's time (greedy: the
 * slowest group gets just enough workgroups to take one item less each,
 * while the budget lasts). Returns the grid (8 x the largest XCD's
 * workgroups when aligned, else the sum of the groups), or GF_EINVAL. */
int32_t gf_batch_plan(int32_t n_inst, const int64_t *items, const double *weights, int32_t budget,
                      int32_t align, int32_t *group, int32_t *xcd);

/* Autotuner for batched persistent runs: instances are grouped into size
 * classes (floor(log2 n) of the program's first stencil size); for each
 * common workgroup size in {64, 128, 256} every class is run alone with each
 * rows-per-segment candidate in {8, 16, 32, 64, 128} and keeps its fastest;
 * the class's cost per work item (median ms x workgroups / items) then
 * weights its instances' shares of the grid. The whole batch is timed with
 * those weights and with plain item-count weights; the fastest of all
 * becomes out[0..n_inst) (for gf_region_run_batched), and *best_ms its
 * median (nullable). Programs without a 2D stencil get one common shape from
 * gf_tune's candidates, weighted by items. Every timed run changes the
 * instances' data like a real run (reps + 1 runs per configuration). Blocks
 * until done. Returns the number of configurations timed, or a negative
 * gf_status. */
int32_t gf_tune_batched(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                        int32_t reps, gf_launch *out, float *best_ms, void *hip_stream);

/* ---- learned launch-config predictor --------------------------------------
 * Not in the paper (its team counts are chosen by hand): a small FP32 MLP
 * maps 8 loop features to a predicted log(t_c / t_best) for each of the
 * GF_NUM_CANDIDATES launch shapes; the argmin over valid shapes is used, and
 * inputs outside the training distribution defer to the autotuner.
 * Features (raw, before the log2(1+x) transform and standardisation): trip
 * count, algorithmic bytes per iteration, flops per iteration, stencil
 * radius, reduction count, nonzeros per row, instance count, element size.
 * Parameters are one float array of GF_MLP_NPARAMS values laid out as
 * W1[64][8] b1[64] W2[64][64] b2[64] W3[32][64] b3[32] (row-major). */
#define GF_MLP_IN 8
#define GF_MLP_HIDDEN 64
#define GF_MLP_OUT GF_NUM_CANDIDATES
#define GF_MLP_NPARAMS (64 * 8 + 64 + 64 * 64 + 64 + 32 * 64 + 32)

/* Forward pass on the device: d_y[b][32] for b < batch; d_z1/d_z2 (nullable,
 * batch x 64) receive the pre-activations the backward pass needs. */
gf_status gf_mlp_forward(gf_ctx *ctx, const float *d_params, const float *d_feats, int32_t batch, float *d_y,
                         float *d_z1, float *d_z2, void *hip_stream);

/* Gradients of L = inv_norm * sum over b,c of mask[b][c] (y - target)^2 into
 * d_grads (GF_MLP_NPARAMS floats, overwritten); relu'(0) = 0. Deterministic
 * (per-block partials summed in block order). batch <= 65536. */
gf_status gf_mlp_backward(gf_ctx *ctx, const float *d_params, const float *d_feats, const float *d_z1,
                          const float *d_z2, const float *d_y, const float *d_target, const float *d_mask,
                          int32_t batch, float inv_norm, float *d_grads, void *hip_stream);

/* d_loss[0] = inv_norm * sum mask * (y - target)^2 over count entries. */
gf_status gf_mlp_loss(gf_ctx *ctx, const float *d_y, const float *d_target, const float *d_mask, int64_t count,
                      float inv_norm, float *d_loss, void *hip_stream);

/* One Adam update (t >= 1 is the step number for bias correction). */
gf_status gf_adam_step(gf_ctx *ctx, float *d_params, const float *d_grads, float *d_m, float *d_v, int32_t n,
                       float lr, float beta1, float beta2, float eps, int32_t t, void *hip_stream);

/* Full-batch training on the device: `epochs` steps of forward, loss,
 * backward and Adam (beta1 0.9, beta2 0.999, eps 1e-8) starting from
 * d_params (updated in place; d_m, d_v Adam moments, zero them to start);
 * d_loss_hist[e] receives the loss before step e. inv_norm = 1 / sum(mask). */
gf_status gf_train_predictor(gf_ctx *ctx, float *d_params, float *d_m, float *d_v, const float *d_feats,
                             const float *d_target, const float *d_mask, int32_t batch, float inv_norm,
                             int32_t epochs, float lr, float *d_loss_hist, void *hip_stream);

/* Install a trained predictor for launch-time use: host copies of the
 * parameters and the per-feature mean and standard deviation of the
 * transformed training features. */
gf_status gf_predictor_set(gf_ctx *ctx, const float *h_params, const float *h_mean, const float *h_std);

/* Predict the launch shape for raw features (host FP32 forward). valid
 * (nullable, GF_NUM_CANDIDATES bytes) restricts the argmin; scores
 * (nullable) receives the 32 outputs. Returns the candidate index, -1 if no
 * predictor is installed or any standardised feature lies outside [-4, 4]
 * (the caller then tunes). */
int32_t gf_predict(gf_ctx *ctx, const double *h_features, const uint8_t *valid, float *scores);

/* The predictor's raw features of a program: those of its dominant region
 * (largest trip count x bytes per iteration) bound by inst[0], with the
 * instance count n_inst. Per region kind (trip count; bytes, flops per
 * iteration; stencil radius; reduction targets; nonzeros per row; element
 * size): 2D/3D stencil ((n-2)^d; 16, 2d+3; 1; 1 with a reduction clause
 * else 0; 0; 8), SpMV (rows; 12 nz + 20, 2 nz; 0; 0; nz = rowptr[n] / n; 8),
 * dot (n; 16, 2; 0; 1; 0; 8), axpby (n; 24, 2; 0; 0; 0; 8), histogram
 * (n; 4, 0; 0; bins, the array section reduced into; 0; 4). For SpMV the
 * row pointer's last entry is read from the device on hip_stream (this call
 * then waits for that stream). out receives GF_MLP_IN doubles. */
gf_status gf_nest_features(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                           double *out, void *hip_stream);

/* Launch-time choice: features (gf_nest_features), the candidates that can
 * run prog on inst in `mode` (tiling, instance and co-residency checks), and
 * gf_predict over them. On success writes the decoded launch to *out and
 * returns its index; returns -1 when no predictor is installed, the program
 * lies outside the training distribution or no candidate can run (the caller
 * then tunes or uses the defaults); argument errors also return a negative
 * status. gf_region_run does this by itself for launch == NULL and one
 * instance when a predictor is installed. */
int32_t gf_predict_launch(gf_ctx *ctx, const gf_program *prog, const gf_instance *inst, int32_t n_inst,
                          int32_t mode, gf_launch *out, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
