/*
 * tstream.h -- C ABI of libtstream: the STREAM kernels (copy, scale, add,
 * triad) on AMD Instinct MI355X (gfx950), expressed the way Heller et al.,
 * "Closing the Performance Gap with Modern C++", frame data-parallel work:
 *
 *   target     a place: one GPU plus the HIP stream work is ordered on
 *              (Section 3.1; the GPU target of Section 4.2 is exactly the
 *              pair "device id + stream");
 *   allocator  arrays placed on a target's device, with bulk construction
 *              (fill) run on the device itself (Section 3.2, Listing 1, and
 *              the GPU allocator of Section 4.2);
 *   executor   the target again: every algorithm call is one bulk launch on
 *              the target's stream (Section 3.3, Listing 2; bulk execution
 *              is what makes GPUs fast, Sections 3.3 and 4.2);
 *   algorithms copy and transform over placed arrays (Section 3.4), here the
 *              four maps of the generic STREAM benchmark (Section 5,
 *              Listing 4).
 *
 * Conventions for every function:
 *   - Returns ts_status: TS_OK (0) or a negative error.  On error a message
 *     is available from ts_last_error() (thread-local); out-parameters are
 *     written only on success.  No C++ exception crosses the ABI.
 *   - Handles are opaque; objects made by *_create / *_alloc are owned by the
 *     caller and released by the matching *_destroy / *_free, which never
 *     fail on a valid handle (the allocator's bulk_destroy is noexcept,
 *     Listing 1) and accept NULL as a no-op.  Arrays, batches, transforms
 *     and graphs refer to the target they were made on: destroy them before
 *     that target.
 *   - "Device pointer" means memory of the target's device (from hipMalloc,
 *     or a torch CUDA/HIP tensor); "host pointer" means ordinary CPU memory.
 *   - Algorithm, fill and copy calls are asynchronous and ordered on the
 *     target's stream; ts_target_synchronize() is the blocking form
 *     (Listing 2's execute).  Calls that return values to the host
 *     (ts_checksum, ts_mismatch_count, ts_batch_mismatch_count, ts_time_op,
 *     ts_autotune*) block until their result is ready.
 *   - Arrays are contiguous, one-dimensional, of one storage type.  Storage
 *     types other than binary64 are evaluated in binary32 (the map in
 *     binary32, fmaf for triad) and rounded back to nearest-even; copy moves
 *     stored bits unchanged.
 *   - Overlapping calls on different host threads must use different
 *     targets (streams); handles are not internally locked.
 */
#ifndef TSTREAM_H
#define TSTREAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define TS_API __attribute__((visibility("default")))
#else
#define TS_API
#endif

#define TS_VERSION_MAJOR 2
#define TS_VERSION_MINOR 1

typedef enum {
    TS_OK = 0,
    TS_E_INVALID = -1,     /* NULL or unknown handle, bad argument value      */
    TS_E_SHAPE = -2,       /* an operand shorter than the element count       */
    TS_E_DTYPE = -3,       /* operands of different storage types             */
    TS_E_PLACEMENT = -4,   /* an array not placed on the executor's device    */
    TS_E_ALIAS = -5,       /* output partly overlaps an input; batch
                              instances share memory                       */
    TS_E_DEVICE = -6,      /* HIP runtime error (message has its text)        */
    TS_E_OOM = -7,         /* device or host allocation failed                */
    TS_E_UNSUPPORTED = -8  /* valid request the library cannot serve         */
} ts_status;

/* Storage types.  TS_U8 (bytes, e.g. characters) is accepted by the array,
 * host-copy and transform calls only; the STREAM maps, fills, checksums,
 * batches and tuning take the four floating-point types (TS_E_UNSUPPORTED
 * otherwise). */
typedef enum { TS_F64 = 0, TS_F32 = 1, TS_BF16 = 2, TS_F16 = 3, TS_U8 = 4 } ts_dtype;

/* The four maps of Listing 4, in the order the benchmark runs them. */
typedef enum { TS_COPY = 0, TS_SCALE = 1, TS_ADD = 2, TS_TRIAD = 3 } ts_op;

typedef struct ts_target_s *ts_target;
typedef struct ts_array_s *ts_array;
typedef struct ts_batch_s *ts_batch;
typedef struct ts_graph_s *ts_graph;
typedef struct ts_event_s *ts_event;
typedef struct ts_future_s *ts_future;
typedef struct ts_transform_s *ts_transform;

/* ------------------------------------------------------------------------ */
/* Errors and version                                                        */
/* ------------------------------------------------------------------------ */

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next ts_* call on the same thread. */
TS_API const char *ts_last_error(void);
TS_API int ts_version(int *major, int *minor);

/* ------------------------------------------------------------------------ */
/* Targets (Section 3.1; GPU target = device + stream, Section 4.2)         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int device;                 /* HIP device ordinal                        */
    int compute_units;          /* CUs reported by the device                */
    int wavefront_size;         /* 64 on CDNA                                */
    int max_threads_per_block;
    int clock_khz;
    int memory_clock_khz;
    int memory_bus_width_bits;
    uint64_t hbm_bytes;         /* device memory                             */
    uint64_t l2_bytes;          /* L2 per the runtime (per XCD on MI3xx)     */
    double peak_bytes_per_s;    /* denominator used for % of peak: 8.0e12   */
    char arch[64];              /* e.g. "gfx950:sramecc+:xnack-"             */
    char name[128];
} ts_device_info;

/* Create a target on `device` (Section 4.2: a GPU target is a device and a
 * stream).  `hip_stream`:
 *   NULL              a non-blocking stream the library creates and destroys
 *                     with the target (as ts_target_create_owned);
 *   hipStreamLegacy   ((void*)1) the device's legacy default stream, which
 *                     orders with every blocking stream (graph capture is
 *                     not available on it);
 *   any other         a hipStream_t of that device (e.g.
 *                     torch.cuda.Stream().cuda_stream), borrowed.
 * Errors: TS_E_INVALID (out NULL, device out of range), TS_E_DEVICE (no
 * usable GPU / HIP failure), TS_E_OOM. */
TS_API int ts_target_create(int device, void *hip_stream, ts_target *out);
/* Same, on a non-blocking stream the library creates and destroys with the
 * target. */
TS_API int ts_target_create_owned(int device, ts_target *out);
/* Host-CPU target (the paper's NUMA back-end, Section 4.1): a set of CPUs,
 * one worker thread pinned to each.  Arrays allocated on it live in host
 * memory and are divided into equal contiguous blocks over the workers in
 * the order of `cpus` (the block allocator); bulk construction and every
 * algorithm call run each block on its own worker (the pinned executor), so
 * the first touch places a block's pages on its worker's NUMA node.  `cpus`
 * NULL (or ncpus 0) takes every CPU the process may run on, grouped by NUMA
 * domain.  Calls on a host target complete before they return.  Its arrays
 * may hold any storage type and copy to and from host memory; the maps,
 * fills, checksums and mismatch counts take binary64 and binary32 storage,
 * transforms also bytes (TS_U8), TS_E_UNSUPPORTED otherwise.  Batches,
 * graphs, events and tuning are GPU-only (TS_E_UNSUPPORTED).  Its arrays and its
 * executor report device -1, so host and GPU arrays never mix
 * (TS_E_PLACEMENT). */
TS_API int ts_target_create_host(const int *cpus, int ncpus, ts_target *out);
/* NUMA domains of the CPUs this process may use (1 when the machine does
 * not expose its topology), and the CPU ids of one domain: writes up to
 * `cap` ids and the full count. */
TS_API int ts_host_numa_domains(int *count);
TS_API int ts_host_domain_cpus(int domain, int *cpus, int cap, int *count);
TS_API int ts_target_destroy(ts_target target);
/* Block until all work enqueued on the target's stream has finished. */
TS_API int ts_target_synchronize(ts_target target);
TS_API int ts_target_info(ts_target target, ts_device_info *out);
/* The hipStream_t the target orders its work on. */
TS_API int ts_target_stream(ts_target target, void **hip_stream_out);
/* Enqueue host callback fn(user) after all work enqueued so far on the
 * target (the continuation behind Listing 2's async_execute futures; the
 * GPU executor signals completion from a stream callback, Section 4.2).
 * fn runs on a runtime thread and must not call into the HIP runtime. */
TS_API int ts_target_then(ts_target target, void (*fn)(void *), void *user);

/* ------------------------------------------------------------------------ */
/* Arrays: placement and bulk construction (Section 3.2, Listing 1)          */
/* ------------------------------------------------------------------------ */

/* Allocate n elements of `dtype` on the target's device (owning).  The
 * allocation base is at least 256-byte aligned; the array starts
 * `offset_elems` elements past it (offset 1 makes a deliberately misaligned
 * array).  Contents are undefined until filled.
 * Errors: TS_E_INVALID, TS_E_OOM (hipMalloc out of memory), TS_E_DEVICE. */
TS_API int ts_array_alloc(ts_target target, ts_dtype dtype, size_t n,
                          size_t offset_elems, ts_array *out);
/* Borrow n elements at `dev_ptr` (device pointer of the target's device,
 * aligned to the element size).  ts_array_free releases only the handle.
 * The memory must outlive every enqueued use.  The n elements must lie in
 * the one device allocation that holds dev_ptr (as the runtime reports it:
 * for memory carved out of a larger allocation, as torch's caching allocator
 * does, that is the larger allocation).
 * Errors: TS_E_INVALID (NULL with n > 0, misaligned), TS_E_PLACEMENT
 * (pointer of another device, of host memory, or of no known allocation),
 * TS_E_SHAPE (the allocation ends before the n-th element). */
TS_API int ts_array_wrap(ts_target target, ts_dtype dtype, void *dev_ptr,
                         size_t n, ts_array *out);
/* Release the handle (and the memory, if the array owns it).  Work still
 * enqueued on the array must have finished (synchronize first). */
TS_API int ts_array_free(ts_array array);
TS_API int ts_array_info(ts_array array, void **dev_ptr, size_t *n,
                         ts_dtype *dtype);

/* bulk_construct on the device (Listing 1; the GPU allocator constructs on
 * the device, Section 4.2).  ts_fill stores `value` rounded to nearest-even
 * into the storage type (via binary32 for the 16-bit types).
 * ts_fill_uniform stores element j (j = 0..n-1) as
 *   u = (h >> 11) * 2^-52 - 1,  h = SplitMix64 output number
 *   (first_index + j + 1) from the state seed ^ (stream_id << 48),
 * an exact binary64 value in [-1, 1), narrowed to binary32 by RNE and then,
 * for bfloat16/binary16, to the storage type by RNE.  Asynchronous.
 * ts_fill_uniform_range stores lo + w * ((h >> 11) * 2^-53), w = hi - lo,
 * each operation rounded in binary64 (so values lie in [lo, hi], hi only
 * through rounding), then narrowed the same way; with
 * lo = -1, hi = 1 it equals ts_fill_uniform bit for bit.  lo < hi, both
 * finite with a finite difference, else TS_E_INVALID.  stream_id < 2^16.
 * Floating-point storage only (TS_E_UNSUPPORTED for TS_U8). */
TS_API int ts_fill(ts_array array, double value);
TS_API int ts_fill_uniform_range(ts_array array, uint64_t seed,
                                 uint64_t stream_id, uint64_t first_index,
                                 double lo, double hi);
TS_API int ts_fill_uniform(ts_array array, uint64_t seed, uint64_t stream_id,
                           uint64_t first_index);

/* Host <-> device copies (the parallel copy specialised to the runtime's
 * memcpy, Section 4.2).  n elements; enqueued on the array's target stream;
 * the host buffer must stay valid and untouched until the stream has
 * reached the copy (synchronize the target).  Errors: TS_E_SHAPE if n
 * exceeds the array, TS_E_INVALID on NULL. */
TS_API int ts_copy_from_host(ts_array dst, const void *host_src, size_t n);
TS_API int ts_copy_to_host(void *host_dst, ts_array src, size_t n);

/* ------------------------------------------------------------------------ */
/* Algorithms on an execution target (Section 3.4; maps of Listing 4)        */
/* ------------------------------------------------------------------------ */
/*
 * Element count = n of the first input (iterator-range semantics); every
 * other operand must hold at least that many elements (else TS_E_SHAPE).
 * All operands share one storage type (else TS_E_DTYPE) and live on the
 * executor's device (else TS_E_PLACEMENT).  dst may equal an input exactly
 * (in place); any other overlap between dst and an input is TS_E_ALIAS.
 * A zero count returns TS_OK without a launch.  For the non-binary64 types
 * q is rounded once to binary32.  One kernel launch per call, enqueued on
 * `exec`'s stream; launch parameters come from the tuning table.
 */
/* Listing 4 "Copy": dst[j] = src[j]. */
TS_API int ts_copy(ts_target exec, ts_array src, ts_array dst);
/* Listing 4 "Scale": dst[j] = q * src[j]. */
TS_API int ts_scale(ts_target exec, ts_array src, ts_array dst, double q);
/* Listing 4 "Add": dst[j] = x[j] + y[j]. */
TS_API int ts_add(ts_target exec, ts_array x, ts_array y, ts_array dst);
/* Listing 4 "Triad": dst[j] = x[j] + q * y[j] as one fused multiply-add,
 * fma(q, y[j], x[j]) (single rounding).  The benchmark's a = b + q*c is
 * ts_triad(exec, b, c, a, q). */
TS_API int ts_triad(ts_target exec, ts_array x, ts_array y, ts_array dst,
                    double q);
/* One benchmark iteration of Listing 4 over a, b, c:
 * c = a; b = q*c; c = a + b; a = b + q*c (four launches, in order).
 * a, b, c must not overlap; count = n of a. */
TS_API int ts_stream_iteration(ts_target exec, ts_array a, ts_array b,
                               ts_array c, double q);

/* ------------------------------------------------------------------------ */
/* Validation (the STREAM benchmark's own result check, done on the GPU)    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double sum;          /* sum of x[j] widened to binary64                      */
    double abs_dev_sum;  /* sum of |x[j] - expected|                             */
    double max_abs_dev;  /* max |x[j] - expected|, NaN terms ignored (fmax);
                            0 for an empty array                                */
    uint64_t mismatches; /* elements whose binary64 value differs in bits from
                            `expected` (NaN matches NaN)                       */
} ts_checksum_out;

/* Binary64 reductions over the whole array, in a fixed two-pass tree whose
 * shape depends only on n and on the array's address modulo 16 bytes (so
 * results are reproducible run to run for an array).
 * Blocking.  The sums differ from a sequential sum only by rounding order. */
TS_API int ts_checksum(ts_target exec, ts_array x, double expected,
                       ts_checksum_out *out);
/* Allocation-free form of ts_checksum, for callers that cannot allocate
 * device or pinned memory while they run (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same two kernels
 * and the same reduction tree as ts_checksum, so the four results are
 * bitwise identical to ts_checksum's for the same array.
 *   dev_out: device memory of the target's GPU (caller-owned, 8-byte
 *            aligned, room for one ts_checksum_out, not overlapping x); the
 *            result is written there in stream order on the target's
 *            stream.  The call does not wait: synchronise the target (or
 *            order later work on its stream) before reading dev_out.
 * The partial sums live in a fixed device array of 4096 parts of 32 bytes
 * (128 KiB) per GPU, loaded with the library and held until the process
 * ends; its address is resolved when a target is created on that GPU.  A
 * checksum of any length uses at most 4096 parts, so no n is refused for
 * scratch size (the check stays, TS_E_SHAPE).  The call makes no hipMalloc,
 * hipHostMalloc, hipFree or hipMemset and does not synchronise.  Every call on
 * one GPU shares that array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * GPU targets only (TS_E_UNSUPPORTED on a host target); TS_E_PLACEMENT if
 * dev_out is not device memory of the target's GPU; TS_E_ALIAS if it
 * overlaps x.  An empty array stores {0, 0, 0, 0}. */
TS_API int ts_checksum_noalloc(ts_target exec, ts_array x, double expected,
                               ts_checksum_out *dev_out);
/* Number of j < n(x) with stored bits of x[j] != ref[j] (NaN matches NaN).
 * ref must hold n(x) elements of the same type.  Blocking. */
TS_API int ts_mismatch_count(ts_target exec, ts_array x, ts_array ref,
                             uint64_t *out);

/* ------------------------------------------------------------------------ */
/* Launch configuration and tuning                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t block;       /* threads per workgroup: 64..1024, multiple of 64 */
    int32_t unroll;      /* vectors per lane per step: 1, 2, 4, 8           */
    int32_t vec_bytes;   /* bytes per lane access: 16 or 8 (the element size
                            selects the element-wise path)                  */
    int32_t nt_load;     /* 1: nontemporal loads                            */
    int32_t nt_store;    /* 1: nontemporal stores                           */
    int32_t grid_per_cu; /* workgroups per CU with a grid-stride loop; 0: one
                            pass, i.e. enough workgroups to cover the array
                            once (batched: one workgroup per tile)          */
    int64_t tile_elems;  /* batched: elements per tile, a multiple of 8;
                            0 = default.  Ignored by plain kernels          */
    int32_t tiles_per_wg; /* batched: consecutive tiles per workgroup, 1, 2,
                            4 or 8 (0 = 1); more than 1 needs unroll <= 2.
                            Plain kernels: 0 or 1                          */
    int32_t record_ahead; /* batched, one workgroup per tile (grid_per_cu 0,
                            tiles_per_wg 1): 1 = each workgroup also reads
                            the tile record 2048 workgroups ahead into its
                            XCD's L2; 0 = off.  Plain kernels: 0          */
    int32_t wgs_per_tile; /* batched: one-wave workgroups that share each
                            tile, 1 (0 = 1) or a power of two up to 128;
                            workgroup w takes piece w mod P of tile w / P
                            (one vector per lane, then every P-th), so
                            consecutive workgroups, spread over the CUs,
                            cover consecutive pieces of a tile.  More than 1
                            needs block 64, unroll 1, grid_per_cu 0,
                            tiles_per_wg 1 and record_ahead 0, and allows
                            vec_bytes 8 beside 16.  Plain kernels: 0 or 1 */
} ts_kernel_cfg;

/* Operand alignment classes (keys of the tuning table). */
enum { TS_ALIGN_16 = 0,     /* every operand 16-byte aligned                */
       TS_ALIGN_SHARED = 1, /* same misalignment: a short head is peeled    */
       TS_ALIGN_MIXED = 2   /* different misalignments: element-wise path   */
};

/* Launch configuration the library would use for this key.  `n` selects
 * the size bucket floor(log2(n)). */
TS_API int ts_get_kernel_cfg(ts_op op, ts_dtype dtype, size_t n,
                             int align_class, int batched, ts_kernel_cfg *out);
/* Force `cfg` for every call of (op, dtype) (plain if batched == 0, batched
 * otherwise), overriding the table; NULL removes the override.  Results are
 * bit-identical under every valid configuration.  TS_E_INVALID for an
 * invalid configuration. */
TS_API int ts_set_kernel_cfg(ts_op op, ts_dtype dtype, int batched,
                             const ts_kernel_cfg *cfg);
/* The candidate set the autotuner searches (plain or batched).  Writes up
 * to `cap` entries and the full count to *count. */
TS_API int ts_autotune_candidates(int batched, ts_kernel_cfg *out, size_t cap,
                                  size_t *count);
/* Time every candidate for (op, dtype) at n elements with the given offset
 * from a 256-byte aligned base (library-allocated scratch arrays, freed
 * before return), median of `reps` event-timed launches each after a
 * warm-up, store the fastest in the table and return it with its rate in
 * STREAM bytes per second (copy/scale count 2 arrays, add/triad 3).
 * Blocking.  TS_E_OOM if the scratch arrays do not fit. */
TS_API int ts_autotune(ts_target target, ts_op op, ts_dtype dtype, size_t n,
                       size_t offset_elems, int reps, ts_kernel_cfg *best,
                       double *best_bytes_per_s);
/* Same for the batched kernel of (op) over an existing batch (its arrays'
 * contents are overwritten). */
TS_API int ts_autotune_batch(ts_target target, ts_batch batch, ts_op op,
                             int reps, ts_kernel_cfg *best,
                             double *best_bytes_per_s);
/* Tuning table persistence (a small JSON file).  Load merges entries and
 * fails with TS_E_INVALID, leaving the table unchanged, on a malformed file
 * or another format version.  TS_TUNE_CACHE in the environment names a file
 * loaded at the first ts_target_create. */
TS_API int ts_tune_cache_load(const char *path);
TS_API int ts_tune_cache_save(const char *path);
TS_API int ts_tune_cache_clear(void);

/* Time `reps` back-to-back launches of one map between two events on the
 * executor's stream; *ms_total receives the elapsed milliseconds.  Operands
 * as for the algorithm calls (y ignored by copy/scale).  Blocking. */
TS_API int ts_time_op(ts_target exec, ts_op op, ts_array x, ts_array y,
                      ts_array dst, double q, int reps, float *ms_total);

/* Memory-system probe (a measurement tool, not one of the paper's
 * algorithms).  Section 5 reads STREAM as the memory bandwidth that the
 * implementation attains; this launch measures what the memory system
 * itself delivers for a given mix of traffic, so the maps can be judged
 * against it: a straight-line kernel over 16-byte vectors that reads
 * `reads` arrays (0, 1: x, or 2: x and y) and writes `writes` arrays
 * (0 or 1: dst), with no arithmetic beyond a bitwise fold.
 *   reads 1, writes 1: dst = x (bits);  reads 2, writes 1: dst = x XOR y;
 *   reads 0, writes 1: every 32-bit word of dst = `mark`;
 *   writes 0: each lane folds what it reads by XOR and stores the fold into
 *   dst only when its first word equals `mark`, so the first bytes/unroll
 *   bytes of dst are unspecified afterwards.
 * The first `bytes` bytes of each operand take part: `bytes` must be a
 * positive multiple of vec_bytes * cfg->block * cfg->unroll (TS_E_SHAPE), every
 * operand must start on a 16-byte boundary (TS_E_SHAPE), hold at least
 * `bytes` bytes (TS_E_SHAPE) and lie on the executor's device
 * (TS_E_PLACEMENT); operands of any storage type; dst must not overlap an
 * input (TS_E_ALIAS); y is ignored unless reads == 2, x unless reads >= 1.
 * One launch of bytes / (vec_bytes * block * unroll) workgroups, which must
 * hold at most 2^31 - 1 workgroups and 2^32 - 1 lanes (TS_E_SHAPE: the
 * probe has no loop to cover more), asynchronous on
 * the executor's stream; GPU targets only (TS_E_UNSUPPORTED on a host
 * target). */
typedef struct {
    int32_t reads;           /* 0, 1 or 2 (writes + reads >= 1)               */
    int32_t writes;          /* 0 or 1 (reads 0 needs writes 1)               */
    int32_t block;           /* lanes per workgroup: 64..1024, multiple of 64 */
    int32_t unroll;          /* vectors per lane: 1, 2 or 4                   */
    int32_t nt_load;         /* 1: nontemporal loads                          */
    int32_t nt_store;        /* 1: nontemporal stores                         */
    int32_t wave_contiguous; /* 1: each wave covers unroll*64 vectors in a
                                row; 0: a lane's vectors lie a workgroup
                                apart                                        */
    int32_t lds_bytes;       /* dynamic LDS per workgroup, 0..the device's
                                LDS per CU: caps the workgroups resident on
                                a CU (0: no cap)                             */
    int32_t vec_bytes;       /* bytes per lane access: 16 or 8 (0 means 16) */
} ts_probe_cfg;
TS_API int ts_probe_bandwidth(ts_target exec, const ts_probe_cfg *cfg,
                              ts_array x, ts_array y, ts_array dst,
                              size_t bytes, uint32_t mark);

/* ------------------------------------------------------------------------ */
/* Batched ragged instances: one launch per map over all instances          */
/* ------------------------------------------------------------------------ */

/* One instance: device pointers of its three arrays (len elements each) and
 * its scalar.  The maps keep Listing 4's roles inside every instance:
 * copy c = a, scale b = q*c, add c = a + b, triad a = b + q*c. */
typedef struct {
    void *a;
    void *b;
    void *c;
    uint64_t len;
    double q;
} ts_batch_desc;

/* Copy `count` descriptors (host memory), split every instance into tiles,
 * and upload the tile tables to the target's device.  The primary plan uses
 * the triad's tile size from the tuning table (or the forced configuration);
 * a map whose configuration asks for another tile size gets a plan of its
 * own, so each map runs on its tuned tiles.  Zero-length instances are
 * allowed and hold no memory.  One launch runs every instance at once, so
 * the rules are checked here, before anything is planned:
 *  - each of a_i, b_i, c_i (len_i elements) lies in one device allocation
 *    of the target's device (TS_E_PLACEMENT otherwise; TS_E_SHAPE when the
 *    allocation ends before element len_i - 1);
 *  - inside one instance two arrays are the very same pointer (in place) or
 *    share no byte; arrays of different instances share no byte
 *    (TS_E_ALIAS otherwise).
 * Errors: TS_E_INVALID (NULL pointer with len > 0, misaligned element),
 * TS_E_PLACEMENT, TS_E_SHAPE, TS_E_ALIAS, TS_E_OOM, TS_E_DEVICE.  Blocking
 * (uploads complete). */
TS_API int ts_batch_create(ts_target target, ts_dtype dtype,
                           const ts_batch_desc *host_descs, size_t count,
                           ts_batch *out);
/* Waits for the work enqueued on the batch's device, then frees its tile
 * tables. */
TS_API int ts_batch_destroy(ts_batch batch);
TS_API int ts_batch_info(ts_batch batch, size_t *count, uint64_t *total_elems,
                         uint64_t *tiles, int64_t *tile_elems);
/* Re-plan with tile_elems (multiple of 8, > 0) and pin it: every map then
 * runs on this one plan, whatever its configuration's tile size.  Blocking.
 * Re-planning (this call, ts_autotune_batch) frees the old tile tables;
 * graphs captured from the batch before it are then refused at launch
 * (TS_E_INVALID). */
TS_API int ts_batch_set_tile(ts_batch batch, int64_t tile_elems);
/* Apply map `op` to every instance in one launch (bulk
 * execution over all instances, Sections 3.3 and 4.2). */
TS_API int ts_batch_op(ts_target exec, ts_batch batch, ts_op op);
/* The same map as one plain launch per instance (the comparison form). */
TS_API int ts_batch_op_plain(ts_target exec, ts_batch batch, ts_op op);
/* Bulk construction of array `which` (0 = a, 1 = b, 2 = c) of every
 * instance: a constant, or uniform[-1,1) with stream 16 + 3*i + which for
 * instance i (same generator as ts_fill_uniform, first_index 0). */
TS_API int ts_batch_fill(ts_target exec, ts_batch batch, int which,
                         double value);
TS_API int ts_batch_fill_uniform(ts_target exec, ts_batch batch, int which,
                                 uint64_t seed);
/* Per-instance count of elements of array `which` whose binary64 value
 * differs in bits from expected[i] (host array of `count` values, NaN
 * matches NaN); counts[i] receives instance i's count.  Blocking. */
TS_API int ts_batch_mismatch_count(ts_target exec, ts_batch batch, int which,
                                   const double *expected, uint64_t *counts);

/* ------------------------------------------------------------------------ */
/* HIP graphs                                                                */
/* ------------------------------------------------------------------------ */

/* Capture the four batched maps of one benchmark iteration (copy, scale,
 * add, triad) on the target's stream into an instantiated graph.  The
 * target's stream must not be the legacy default stream
 * (TS_E_UNSUPPORTED).  A graph whose batch was re-planned or destroyed
 * after the capture is refused at launch (TS_E_INVALID). */
TS_API int ts_graph_capture_stream_iteration(ts_target target, ts_batch batch,
                                             ts_graph *out);
/* Capture a single batched map (one graph node). */
TS_API int ts_graph_capture_batch_op(ts_target target, ts_batch batch,
                                     ts_op op, ts_graph *out);
/* Capture one plain benchmark iteration over arrays a, b, c (four nodes). */
TS_API int ts_graph_capture_arrays_iteration(ts_target target, ts_array a,
                                             ts_array b, ts_array c, double q,
                                             ts_graph *out);
/* Capture `iterations` consecutive benchmark iterations into one graph
 * (4 x iterations nodes, in the order eager calls would run them).  A graph
 * launch has a fixed cost of several microseconds regardless of its size,
 * so small arrays gain from graphs only when one launch holds many
 * kernels.  1 <= iterations <= TS_GRAPH_MAX_ITERATIONS (TS_E_INVALID
 * otherwise); the other rules are those of the one-iteration calls. */
#define TS_GRAPH_MAX_ITERATIONS 4096
TS_API int ts_graph_capture_arrays_iterations(ts_target target, ts_array a,
                                              ts_array b, ts_array c, double q,
                                              int iterations, ts_graph *out);
TS_API int ts_graph_capture_stream_iterations(ts_target target, ts_batch batch,
                                              int iterations, ts_graph *out);
/* Enqueue the graph `repeats` times on the target's stream.  TS_E_INVALID
 * (nothing enqueued) when the graph's batch was re-planned or destroyed, or
 * one of its library-allocated arrays freed, after the capture; borrowed
 * memory must stay valid while the graph is in use. */
TS_API int ts_graph_launch(ts_target target, ts_graph graph, int repeats);
/* Waits for the work enqueued on the graph's device, then releases it. */
TS_API int ts_graph_destroy(ts_graph graph);

/* ------------------------------------------------------------------------ */
/* Events: completion and timing of enqueued work (Listing 2's futures)      */
/* ------------------------------------------------------------------------ */

TS_API int ts_event_create(ts_event *out);
/* An event for timing only: recording it makes no system-scope release, so
 * the runtime neither writes back nor invalidates caches around it and it
 * perturbs the work it brackets less.  Its completion does not make device
 * writes visible to the host: synchronize the target (or use an event from
 * ts_event_create) before the host reads results. */
TS_API int ts_event_create_timing(ts_event *out);
TS_API int ts_event_destroy(ts_event event);
/* Mark the current end of the target's stream. */
TS_API int ts_event_record(ts_event event, ts_target target);
TS_API int ts_event_synchronize(ts_event event);
/* TS_OK (0) if the recorded work has finished, 1 if it is still pending. */
TS_API int ts_event_query(ts_event event);
TS_API int ts_event_elapsed_ms(ts_event start, ts_event end, float *ms);

/* ------------------------------------------------------------------------ */
/* Futures: host-side completion of asynchronous work (Listing 2)            */
/* ------------------------------------------------------------------------ */
/* The paper's asynchronous executor functions (async_execute,
 * bulk_async_execute, Listing 2) return futures; its GPU executor makes them
 * ready from a callback attached to the stream (Section 4.2).  Here every
 * algorithm call is already asynchronous on the target's stream, and
 * ts_target_async returns the future of all work enqueued so far: a host
 * callback on the stream marks it ready.  Waiting does not synchronise the
 * device; it blocks the calling thread until the callback has run. */
TS_API int ts_target_async(ts_target target, ts_future *out);
/* Block until the future is ready. */
TS_API int ts_future_wait(ts_future future);
/* 1 if ready, 0 if still pending (never blocks). */
TS_API int ts_future_ready(ts_future future);
/* Release the future; waits for its callback first if it is still pending. */
TS_API int ts_future_destroy(ts_future future);

/* ------------------------------------------------------------------------ */
/* Generic transforms: a user expression compiled at run time               */
/* ------------------------------------------------------------------------ */
/* The paper's GPU executor runs any device callable (Section 4.2) and its
 * hello-world example transforms a vector of chars with to_upper (Section
 * 3.4, Listing 3).  Here the callable is the text of a C++ expression in the
 * element values `x` (and `y` when n_inputs == 2) and the scalar `q`, all of
 * the storage type's arithmetic type: double (TS_F64), float (TS_F32,
 * TS_BF16, TS_F16; 16-bit values widen exactly and the result is rounded to
 * nearest-even), int (TS_U8).  The result is converted to the storage type:
 * dst[j] = expr(x[j], y[j], q).  Nothing is contracted (-ffp-contract=off);
 * __builtin_fma(q, y, x) is a fused triad.  The expression is compiled once
 * per (expression, inputs, type, GPU architecture) and cached for the life
 * of the process.  The expression is compiled as C++ source and runs with
 * the caller's privileges: pass only trusted text.  GPU targets compile
 * with hipRTC.  Host-CPU targets
 * (Section 4.1) compile with the system C++ compiler (TS_HOST_CXX, default
 * "c++", run as a child process) into a shared object that their pinned
 * workers run over their blocks; they take TS_F64, TS_F32 and TS_U8, and
 * `fma` there is std::fma.  A transform runs on targets of the kind it was
 * made for (TS_E_PLACEMENT otherwise).  Errors: TS_E_INVALID with the
 * compiler's log when the expression does not compile; TS_E_UNSUPPORTED
 * without hipRTC (GPU) or a host compiler (host), or for 16-bit storage on
 * a host target.  ts_transform_apply follows the rules of the algorithm
 * calls (count = n of x; shapes, types, placement, aliasing) and is
 * asynchronous on the executor's stream (host targets: complete on
 * return).  ts_transform_destroy first waits for the work enqueued on its
 * device, so launches still in flight finish before the code is unloaded. */
TS_API int ts_transform_create(ts_target target, const char *expr, int n_inputs,
                               ts_dtype dtype, ts_transform *out);
TS_API int ts_transform_apply(ts_target exec, ts_transform transform,
                              ts_array x, ts_array y, ts_array dst, double q);
/* Compiler messages of the transform's compilation (may be empty). */
TS_API int ts_transform_log(ts_transform transform, const char **log);
TS_API int ts_transform_destroy(ts_transform transform);

#ifdef __cplusplus
}
#endif
#endif /* TSTREAM_H */
