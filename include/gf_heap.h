/*
 * gf_heap.h -- C ABI of libgf's device heap: the "balanced" allocator of the
 * paper (Section 3.4, "Heap Allocators and Allocation Tracking"), which
 * malloc/free calls made inside regions use. Its allocation microbenchmark
 * follows Section 5.1, "Allocator Performance".
 *
 * The heap is cut into N x M chunks. A thread allocates from chunk
 * (thread id in its workgroup mod N, workgroup id mod M), under that chunk's
 * lock, so threads that map to different chunks never contend. Within each
 * team slot, the chunk of thread slot 0 is `first_ratio` times the size of
 * the others, because the initial thread allocates the serial code's large
 * objects. Inside a chunk an entry is a 16-byte header (link to the entry
 * below, size, in-use mark) followed by the user data. Allocations go on top
 * of the highest entry. Freeing marks an entry unused, and freeing the top
 * entry moves the watermark down over it and over every unused entry
 * directly below. When the space above the watermark is too small, the
 * entries are searched from the bottom for the first unused one that is
 * large enough, and that entry is reused whole. Otherwise the allocation
 * returns NULL.
 *
 * The allocator keeps a record of every live object, so the object that
 * holds a pointer can be found (the paper's run-time lookup of a reference
 * argument's object): see GF_HEAP_OP_FIND.
 *
 * Sizes: a request of b bytes takes max(1, ceil(b / 16)) 16-byte units. The
 * heap is split into M equal team shares of whole units, and each share into
 * (first_ratio + N - 1) equal parts, rounded down.
 *
 * Conventions as in gf.h: d_* pointers are device memory owned by the
 * caller; calls that take a hip_stream enqueue asynchronously on it.
 * Functions marked "synchronous" wait for the device. A heap may be used from
 * one host thread at a time.
 */
#ifndef GF_HEAP_H
#define GF_HEAP_H

#include <stdint.h>

#include "gf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_heap gf_heap;

typedef struct {
    int64_t bytes;            /* heap size in bytes (16 .. 2^35) */
    int32_t thread_slots;     /* N >= 1 */
    int32_t team_slots;       /* M >= 1 */
    int32_t first_ratio;      /* >= 1 */
    int32_t vendor;           /* 1: no heap of its own; gf_heap_bench uses the HIP
                                 runtime's device malloc/free with a heap of `bytes`
                                 (for comparison); script, tops: GF_EUNSUPPORTED */
    int64_t lock_timeout_us;  /* a chunk lock not obtained within this time makes
                                 the call fail (counted, returns NULL); 0 = 2 s */
} gf_heap_opts;

/* Create a heap on HIP device `hip_device` (device memory for the heap, the
 * chunk headers and four counters). Every chunk starts empty. */
gf_status gf_heap_create(int32_t hip_device, const gf_heap_opts *opts, gf_heap **out);
/* Wait for the device and free everything. NULL ok. */
gf_status gf_heap_destroy(gf_heap *heap);
/* Empty every chunk (enqueued on hip_stream); pointers from before are invalid. */
gf_status gf_heap_reset(gf_heap *heap, void *hip_stream);

/* A script of heap operations run by one device thread, in order. Operation i
 * is three int64 words at d_ops[3i]: {op, a, b}; its results are two int64
 * words at d_res[2i]:
 *   GF_HEAP_OP_MALLOC  a = bytes, b = thread id | (workgroup id << 32) for the
 *                      chunk choice; res = {byte offset of the user data from
 *                      the heap's start, or -1; 0}
 *   GF_HEAP_OP_FREE    frees the pointer returned by operation a (< i); a
 *                      NULL result is freed as NULL; res = {0, 0}
 *   GF_HEAP_OP_FIND    looks up the byte at offset b into the result of
 *                      operation a; res = {offset of the live allocation
 *                      that holds it, its size in bytes}, or {-1, 0}
 * Errors: GF_EINVAL for a bad operation (checked on the host first). */
#define GF_HEAP_OP_MALLOC 1
#define GF_HEAP_OP_FREE 2
#define GF_HEAP_OP_FIND 3
gf_status gf_heap_script(gf_heap *heap, const int64_t *d_ops, int32_t n_ops, int64_t *d_res, void *hip_stream);

/* The allocation microbenchmark: `teams` workgroups of `threads` threads
 * (1 .. 1024). Every thread allocates `bytes` bytes (a multiple of 8, >= 8),
 * writes a value derived from its global id into every 8-byte word, and
 * then, by mode:
 *   GF_HEAP_BENCH_ROUNDTRIP  checks the words and frees the block;
 *   GF_HEAP_BENCH_HOLD       stores the pointer in d_ptrs[global id] (device,
 *                            teams * threads entries) and keeps the block;
 *   GF_HEAP_BENCH_RELEASE    does not allocate: checks and frees d_ptrs[gid]
 *                            from an earlier HOLD with the same shape.
 * NULL allocations, blocks whose words were overwritten by someone else, lock
 * timeouts and frees of pointers outside the heap are counted
 * (gf_heap_counts). */
#define GF_HEAP_BENCH_ROUNDTRIP 0
#define GF_HEAP_BENCH_HOLD 1
#define GF_HEAP_BENCH_RELEASE 2
gf_status gf_heap_bench(gf_heap *heap, int32_t teams, int32_t threads, int64_t bytes, int32_t mode, void **d_ptrs,
                        void *hip_stream);

/* Synchronous: out[0] NULL allocations, out[1] corrupt blocks, out[2] lock
 * timeouts, out[3] bad frees, since creation or the last reset of the
 * counts; reset != 0 clears them. */
gf_status gf_heap_counts(gf_heap *heap, uint64_t out[4], int32_t reset);

/* Device address of the heap's first byte (NULL for a vendor heap): the
 * offsets of gf_heap_script are relative to it. */
void *gf_heap_base(const gf_heap *heap);

/* Let ctx's host calls look up GF_ARG_HEAPREF pointers in `heap` (NULL:
 * none; every such pointer then travels as a value). The heap must outlive
 * the runs that use it. Not a vendor heap. */
gf_status gf_ctx_set_heap(gf_ctx *ctx, gf_heap *heap);

/* Synchronous: the watermark (units above the chunk's start in use or
 * reserved) of each chunk, N*M values into tops (host), n >= N*M. */
gf_status gf_heap_tops(gf_heap *heap, uint32_t *tops, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
