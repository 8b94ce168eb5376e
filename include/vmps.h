/*
 * vmps: stable run-adaptive sorting on AMD MI355X (gfx950).
 *
 * C ABI of libvmps.so.  The operations follow "Virtual-Memory Powersort":
 *   - sort input[0,n) stably, result back in input (Algorithm 1, Abstract
 *     Powersort: NewBuffer takes the input, Copy hands it back);
 *   - runs are maximal non-decreasing runs forced to a minimum length by
 *     sorting (ExtractRun, Sections 2 and 3; minrun rule of Section 5);
 *   - merges follow Powersort's merge policy (Power theorem, Section 2) and
 *     keep equal keys in input order (StandardMerge, Algorithm 2);
 *   - runs live either in the input or in one n-element buffer, and every
 *     merge reads one buffer and writes the other (Pingpong Powersort,
 *     Section 3);
 *   - all extra memory is a caller-provided workspace allocated up front
 *     (pre-allocation of buffers, Section 4.1).
 *
 * Conventions for every call:
 *   - Keys are unsigned (VMPS_U32 or VMPS_U64) and ascend; values are 32-bit
 *     payloads moved with their keys.  Equal keys keep their input order.
 *   - All pointers except those marked "host" are device pointers of the
 *     current HIP device.  The caller owns every buffer; the library
 *     allocates no device memory and keeps no pointer after its stream work
 *     ends.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls only enqueue work: they never synchronise the host, and their
 *     results are ready when the stream reaches that point.
 *   - Lengths are limited to n < 2^32.  Keys must be aligned to their size.
 *   - Arguments are validated before anything is enqueued; on error nothing
 *     is written.  VMPS_ERR_DEVICE reports a failed HIP launch.
 */
#ifndef VMPS_H
#define VMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VMPS_OK = 0,
    VMPS_ERR_INVALID_ARG = 1,
    VMPS_ERR_WORKSPACE_TOO_SMALL = 2,
    VMPS_ERR_UNSUPPORTED = 3,
    VMPS_ERR_DEVICE = 4
} vmps_status;

typedef enum { VMPS_U32 = 0, VMPS_U64 = 1 } vmps_dtype;

/* vmps_sort flags */
#define VMPS_VALUES_IOTA 1u /* `values` is output only: receives the stable
                               permutation (original index of each output key) */

/* Human-readable name of a status code (static string). */
const char* vmps_status_string(vmps_status s);

/* Minimum run length for n elements: l = n, then l = ceil(l/2) while
 * l >= 64 (Section 5, "Algorithm variants"). */
int32_t vmps_minrun(int64_t n);

/* Workspace bytes vmps_sort needs for n keys of type kt, with or without
 * values.  bytes: host pointer.  n < 0 or bytes == NULL -> INVALID_ARG. */
vmps_status vmps_sort_workspace_size(int64_t n, vmps_dtype kt, int has_values, size_t* bytes);

/* Stable sort of keys[0,n) in place (Algorithm 1 with Pingpong buffers).
 *   keys   : n keys, sorted in place.
 *   values : NULL, or n payloads moved with the keys; with VMPS_VALUES_IOTA
 *            it is output only and receives the stable argsort.
 *   ws     : at least vmps_sort_workspace_size() bytes, 256-byte aligned;
 *            holds the second Pingpong buffer and the merge schedule.
 * n in {0,1} is a no-op.  Errors: INVALID_ARG (n<0, n>=2^32, NULL keys or ws
 * with n>1, misaligned keys, values aliasing keys, unknown flags),
 * WORKSPACE_TOO_SMALL, DEVICE. */
vmps_status vmps_sort(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                      void* ws, size_t ws_bytes, void* stream);

/* Workspace of vmps_merge. */
vmps_status vmps_merge_workspace_size(int64_t na, int64_t nb, vmps_dtype kt, size_t* bytes);

/* StandardMerge (Algorithm 2, right) of sorted a[0,na) and b[0,nb) into
 * out[0,na+nb): an element of a precedes an equal element of b.  va/vb/vout
 * are all NULL or all non-NULL.  out must not overlap a or b.
 * Errors: INVALID_ARG (negative or too large lengths, NULL pointers with
 * non-zero length, overlap), WORKSPACE_TOO_SMALL, DEVICE. */
vmps_status vmps_merge(const void* a, const uint32_t* va, int64_t na, const void* b,
                       const uint32_t* vb, int64_t nb, void* out, uint32_t* vout, vmps_dtype kt,
                       void* ws, size_t ws_bytes, void* stream);

/* Run decomposition of keys[0,n) (ExtractRun applied from the left until
 * the input is used up).  Each run is the maximal non-decreasing run from
 * its start, or minrun elements if that run is shorter (the last run may be
 * shorter still).  minrun <= 0 selects vmps_minrun(n); an explicit minrun
 * must be >= min(16, n) (INVALID_ARG otherwise).
 *   run_bounds : device, capacity vmps_max_runs(n, minrun)+1 u32; receives
 *                r+1 bounds (0 = b[0] < ... < b[r] = n).
 *   num_runs   : device int64 receiving r.
 *   ws         : vmps_sort_workspace_size(n, kt, 0) bytes suffice. */
vmps_status vmps_extract_runs(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun,
                              uint32_t* run_bounds, int64_t* num_runs, void* ws,
                              size_t ws_bytes, void* stream);

/* Upper bound on the number of runs for n elements and minimum run length
 * minrun (<= 0: vmps_minrun(n)). */
int64_t vmps_max_runs(int64_t n, int32_t minrun);

/* Power of every run boundary (theorem of Section 2): for runs [i,j),[j,k)
 * of an n-element input, the least p such that an integer c has
 * (i+j)/(2n) < c/2^p <= (j+k)/(2n).
 *   run_bounds : device, r+1 u32 bounds as produced by vmps_extract_runs.
 *   num_runs   : device int64 r.
 *   powers     : device, r-1 bytes (capacity max_runs) receive the powers. */
vmps_status vmps_run_powers(const uint32_t* run_bounds, const int64_t* num_runs, int64_t n,
                            int64_t max_runs, uint8_t* powers, void* stream);

/* The merge schedule vmps_sort executes, for inspection (host-visible
 * results after the stream is synchronised).  All output arrays are device
 * pointers with capacity vmps_max_runs(n, 0).
 *   node_l/node_m/node_r : merges longer than the LDS tile, as
 *                          [l,m) + [m,r), in position order
 *   node_level           : their power
 *   node_buf             : buffer they write (0 = keys, 1 = workspace)
 *   seg_start/seg_end/seg_buf : the LDS-sorted subtrees and long runs
 *   counts               : device int64[4] = {runs, merges in HBM, segments,
 *                          merge cost M}
 *   tile                 : host, receives the LDS tile length used */
vmps_status vmps_sort_schedule(const void* keys, int64_t n, vmps_dtype kt, int has_values,
                               uint32_t* node_l, uint32_t* node_m, uint32_t* node_r,
                               uint8_t* node_level, uint8_t* node_buf, uint32_t* seg_start,
                               uint32_t* seg_end, uint8_t* seg_buf, int64_t* counts,
                               int32_t* tile, void* ws, size_t ws_bytes, void* stream);

/* Workspace of vmps_segmented_sort. */
vmps_status vmps_segmented_sort_workspace_size(int64_t total, int64_t nseg, vmps_dtype kt,
                                               int has_values, size_t* bytes);

/* Independent stable sorts of keys[off[s], off[s+1]) for s < nseg, each a
 * Powersort instance of its own length (its own minrun and powers).
 *   seg_offsets : device int64[nseg+1], non-decreasing, off[0] = 0,
 *                 off[nseg] = total.  The table is checked on the device:
 *                 a bad table sorts nothing and leaves keys unchanged.
 *   values      : NULL or total payloads. */
vmps_status vmps_segmented_sort(void* keys, uint32_t* values, const int64_t* seg_offsets,
                                int64_t nseg, int64_t total, vmps_dtype kt, void* ws,
                                size_t ws_bytes, void* stream);

/* ---- launch timing (instrumentation) ----
 * When enabled, the library brackets its hot launches with HIP events on
 * the caller's stream.  vmps_trace_collect() waits for those events and
 * returns, per kind, the summed milliseconds and the number of bracketed
 * launches since the previous collect, then forgets them.  Host-side state
 * shared by all calls of the process (not for concurrent use). */
typedef enum {
    VMPS_TRACE_PLAN = 0,            /* whole planner (runs, powers, tree, placement) */
    VMPS_TRACE_TILESORT = 1,        /* LDS Powersort of subtrees / buckets */
    VMPS_TRACE_LEVEL_PARTITION = 2, /* merge-path splits of one tree level */
    VMPS_TRACE_LEVEL_MERGE = 3,     /* merges of one tree level */
    VMPS_TRACE_HISTOGRAM = 4,       /* learned partition: bucket histogram */
    VMPS_TRACE_SCATTER = 5,         /* learned partition: stable scatter */
    VMPS_TRACE_TRAIN = 6,           /* CDF model training + table */
    VMPS_TRACE_SAMPLE = 7,          /* sample gather + sample sort */
    VMPS_TRACE_KINDS = 8
} vmps_trace_kind;

vmps_status vmps_trace_enable(int on);
/* ms, launches: host arrays of nkinds entries. */
vmps_status vmps_trace_collect(double* ms, int64_t* launches, int32_t nkinds);

#ifdef __cplusplus
}
#endif
#endif /* VMPS_H */
