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
 *     ends.  (Only with the opt-in host_wait tuning: each host thread gets
 *     one 132-byte pinned host buffer and one event per device on its first
 *     such sort, kept until the process ends.)
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls enqueue work and their results are ready when the stream
 *     reaches that point; no call waits on the host.  The sorts that merge
 *     beyond the LDS tile launch one merge-level pair per possible power
 *     (at most ceil(log2 n)); a level the planner left empty returns at
 *     once on the GPU.  Opt-in (tuning field host_wait = 1): they copy the
 *     planner's per-level merge counts to a pinned host buffer, wait for
 *     that copy and launch only the non-empty levels (not under graph
 *     capture).
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
#define VMPS_DESCENDING_RUNS 2u /* ExtractRun also takes maximal strictly
                               decreasing runs and reverses them (the remark
                               on decreasing runs in Section 5); the output is
                               the same stable sort, runs and merges differ */

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
 *   flags  : VMPS_VALUES_IOTA, VMPS_DESCENDING_RUNS (or-ed).
 * n in {0,1} is a no-op.  Errors: INVALID_ARG (n<0, n>=2^32, NULL keys or ws
 * with n>1, misaligned keys, values aliasing keys, unknown flags),
 * WORKSPACE_TOO_SMALL, DEVICE. */
vmps_status vmps_sort(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                      void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vmps_sort with its workspace in a
 * fixed device array inside the library instead of `ws`.  Same arguments,
 * result and errors as vmps_sort; it calls no allocator, never waits on the
 * host (the host_wait tuning is ignored) and is asynchronous on `stream`.
 *   - The array holds vmps_noalloc_scratch_bytes() bytes (96 MiB) on every
 *     GPU the library runs on, from its first use there until the process
 *     ends.  A sort whose vmps_sort_workspace_size exceeds it (n above about
 *     6.9 million for 64-bit keys with values, 16.5 million for 32-bit keys
 *     alone) -> WORKSPACE_TOO_SMALL, with nothing enqueued.
 *   - All calls on one GPU share that GPU's array: calls that overlap in
 *     time on one GPU (two streams, two host threads) race and give wrong
 *     results; order them on one stream.  Each call overwrites what the last
 *     one left there, and nothing in it needs clearing between calls. */
vmps_status vmps_sort_noalloc(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                              void* stream);
size_t vmps_noalloc_scratch_bytes(void);

/* ---- Virtual-Memory Powersort (Section 4) ----------------------------
 * The same stable sort as vmps_sort without the second Pingpong buffer:
 * the merge levels write into pages (P elements, the merge output tile:
 * 4096, or 2048 for 64-bit keys with values) taken from a pool of
 * window + 9 extra pages and from input pages whose elements have all been
 * consumed (the paper's free list); a page table maps the array's pages to
 * where they are, and a final Copy permutes the pages into place.  A level
 * runs in rounds of `window` pages.  A page whose merge output is exactly
 * its own contents (a prefix of the left run below the right run, a suffix
 * of the right run above the left run) keeps its physical page: no fresh
 * page and no data movement (the remark on skipping whole pages in Sec. 2).  Memory beyond keys and values: the
 * pool, one page per 64 for the Copy, a few words per page, and the merge
 * schedule (as vmps_sort's).
 *   window_pages : pages per round (0: N/16, at least 64, N = ceil(n/P));
 *                  larger windows mean fewer launches and a larger pool. */
typedef struct {
    int64_t page_elems;    /* P */
    int64_t pages;         /* N = ceil(n / P) */
    int64_t window_pages;  /* W, after the default and the clamp to N */
    int64_t pool_pages;    /* W + 9 */
    int64_t copy_pages;    /* ceil(N / 64) pages saved by the Copy */
    size_t  buffer_bytes;  /* pool + copy pages, keys and values */
    size_t  workspace_bytes; /* all of ws, the merge schedule included */
} vmps_vm_layout;
vmps_status vmps_sort_vm_layout(int64_t n, vmps_dtype kt, int has_values, int64_t window_pages,
                                vmps_vm_layout* out);

/* Statistics of a vmps_sort_vm call (device array of 8 counts, written at
 * the end of the call when `stats` is not NULL):
 *   [0] schedule faults: 0 on every correct run (a fresh page handed out
 *       before its release, or a broken page permutation)
 *   [1] elements carried (copied into a fresh page without merging)
 *   [2] elements moved by the final Copy
 *   [3] elements written by the page merges
 *   [4] merge levels that touched pages, [5] fresh pages written by them
 *   [6] elements of pages a merge left in place (the page-skipping merge:
 *       the page's output tile is exactly its own contents, so it keeps
 *       its physical page; [3] + [6] is the merge cost of the nodes longer
 *       than the LDS tile). */
#define VMPS_VM_STATS 8

/* Stable sort of keys[0,n) in place with paged merge levels.
 *   keys, values, flags : as vmps_sort (VMPS_VALUES_IOTA, VMPS_DESCENDING_RUNS).
 *   window_pages        : see above (>= 0).
 *   ws                  : vmps_sort_vm_layout().workspace_bytes, 256-byte aligned.
 *   stats               : NULL or a device array of VMPS_VM_STATS uint64.
 * Asynchronous on `stream`; n in {0,1} is a no-op.  Errors as vmps_sort. */
vmps_status vmps_sort_vm(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                         int64_t window_pages, void* ws, size_t ws_bytes, uint64_t* stats, void* stream);

/* ---- Large records (the 30-word record types of Sec. 5; hypothesis H4) --
 * Stable sort of n records of record_bytes bytes by a key field (u32 or
 * u64, kt) at byte key_offset: the (key, index) pairs are sorted with
 * vmps_sort's path (runs, powers, Pingpong merges), then every record is
 * gathered once into `out`.  Each record is read and written once instead
 * of once per merge level it passes through.
 *   records, out : device, n * record_bytes bytes each, 4-byte aligned, not
 *                  overlapping (8-byte aligned with record_bytes % 8 == 0
 *                  moves 8-byte words).
 *   record_bytes : multiple of 4 (of 8, and records 8-byte aligned, with
 *                  u64 keys), at least the key size; key_offset a multiple
 *                  of the key size with key_offset + key size <=
 *                  record_bytes.
 *   flags        : 0 or VMPS_DESCENDING_RUNS.
 *   ws           : vmps_sort_records_workspace_size() bytes, 256-aligned.
 * Asynchronous on `stream`.  Errors: INVALID_ARG, WORKSPACE_TOO_SMALL,
 * DEVICE. */
vmps_status vmps_sort_records_workspace_size(int64_t n, vmps_dtype kt, size_t* bytes);
vmps_status vmps_sort_records(const void* records, void* out, int64_t n, int32_t record_bytes, int32_t key_offset,
                              vmps_dtype kt, uint32_t flags, void* ws, size_t ws_bytes, void* stream);

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

/* The chain of vmps_sort with VMPS_DESCENDING_RUNS: at a chain point s the
 * natural run is the maximal strictly decreasing one when x[s+1] < x[s] (it
 * is reversed by the sort), else the maximal non-decreasing one; shorter
 * than minrun, it is forced to minrun.  Arguments as vmps_extract_runs. */
vmps_status vmps_extract_runs_desc(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun,
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

/* ---- learned CDF partitioning ----
 * A small model of the keys' distribution routes every key to one of B
 * buckets that are increasing key ranges; a stable scatter groups the keys
 * by bucket and every bucket is then sorted by Powersort as an instance of
 * its own (vmps_segmented_sort), so the result is exactly the stable sort
 * whatever the model predicts: a poor model only makes buckets uneven, and
 * buckets longer than the LDS tile go through the merge levels.
 *
 * Model: feature z(key) = (bit length << F) | the F bits below the leading
 * one (integer, monotone); u = (z - z_lo) / (z_hi - z_lo) over the sorted
 * sample; f(u) = b2 + sum_h w2[h] relu(w1[h] u + b1[h]) trained on the
 * sample's empirical CDF (i + 1/2)/m with mean squared error and Adam,
 * starting from hinges at sample quantiles; the model is then compiled into
 * a monotone Q32 knot table every 2^shift feature units and a key's bucket
 * is (table interpolation * B) >> 32, all in integers. */
#define VMPS_CDF_MAX_HIDDEN 64
#define VMPS_CDF_MAX_KNOTS 4096
#define VMPS_CDF_MAX_BATCH 32768
#define VMPS_CDF_MAX_SAMPLE (1 << 24)
/* Buckets: ids of at most 18 bits (two scatter levels of at most 9 bits). */
#define VMPS_MAX_BUCKETS 262144
/* vmps_learned_config.flags: keep the parameters after the last Adam step
 * even when their loss exceeds the initial model's (the default keeps the
 * better of the two); for checking the training trajectory. */
#define VMPS_CDF_KEEP_TRAINED 1

typedef struct {
    int32_t num_buckets;  /* B: power of two in [2, VMPS_MAX_BUCKETS]; 0 = automatic */
    int32_t hidden;       /* H in {16, 32, 64} */
    int32_t steps;        /* Adam steps (>= 0) */
    int32_t batch;        /* minibatch points per step, multiple of 64, in
                             [64, VMPS_CDF_MAX_BATCH] */
    float lr;             /* Adam learning rate */
    int32_t knots;        /* K: at most this many table segments (1..4096) */
    int32_t feature_bits; /* F in [4, 24] */
    int32_t flags;        /* 0, or VMPS_CDF_KEEP_TRAINED */
    int64_t sample_size;  /* m: keys sampled at SplitMix64 positions, in
                             [2, min(n, VMPS_CDF_MAX_SAMPLE)] */
    uint64_t seed;        /* SplitMix64 seed of the sample positions */
} vmps_learned_config;

/* The compiled model (lives in device memory; 33 KiB). */
typedef struct {
    uint64_t z_lo, z_hi;         /* feature range of the sorted sample */
    int32_t key_bits, feature_bits, hidden;
    int32_t knots;               /* table has knots+1 entries */
    int32_t shift;               /* knot spacing 2^shift feature units */
    int32_t trained;             /* 1 if Adam improved on the initial model */
    float loss_init, loss_final; /* MSE on every 64th sample point */
    float w1[VMPS_CDF_MAX_HIDDEN], b1[VMPS_CDF_MAX_HIDDEN], w2[VMPS_CDF_MAX_HIDDEN];
    float b2, reserved;
    uint64_t table[VMPS_CDF_MAX_KNOTS + 1];
} vmps_cdf_model;

/* Bucket statistics and the model's error judge.  The judge runs over the
 * sorted sample x_0 <= ... <= x_{m-1} with targets y_i = (i + 1/2)/m and F
 * the compiled table (the function the partition uses):
 *   bucket error |bucket(x_i) - floor(B y_i)|, an integer;
 *   CDF error    |B F(x_i) - B y_i| in buckets, from exact 128-bit integer
 *                numerators rounded to double at the end.
 * All zero when the call took the plain path (judge_samples == 0). */
typedef struct {
    int64_t buckets, nonempty_buckets;
    int64_t fallback_buckets, fallback_keys; /* buckets longer than the LDS tile */
    int64_t max_bucket;
    float loss_init, loss_final;
    int64_t judge_samples;         /* m */
    int64_t judge_max_bucket_err;  /* max_i bucket error */
    double judge_mean_bucket_err;  /* mean bucket error */
    double judge_max_err;          /* max_i CDF error (buckets) */
    double judge_mean_err;         /* mean CDF error (buckets) */
    double overflow_fraction;      /* fallback_buckets / buckets */
} vmps_learned_stats;

/* Defaults for n keys of type kt (host struct): automatic B, H = 64,
 * 32 Adam steps of 8192 points at learning rate 5e-5, K = 4096 knots,
 * F = 20, m = n/256 sample keys clamped to [8192, 2^20] (and to n),
 * seed 55. */
vmps_status vmps_learned_default_config(int64_t n, vmps_dtype kt, vmps_learned_config* cfg);

vmps_status vmps_learned_workspace_size(int64_t n, vmps_dtype kt, int has_values,
                                        const vmps_learned_config* cfg, size_t* bytes);

/* Stable sort of keys[0,n) through the learned partition (sample, sort the
 * sample with vmps_sort, train, compile, partition, sort every bucket).
 * values as in vmps_sort (flags: VMPS_VALUES_IOTA).  model / stats: device,
 * nullable, receive the compiled model and bucket statistics.  cfg: host.
 * Inputs too small for the model (n < 4 * LDS tile or m < 1024) take the
 * plain vmps_sort path. */
vmps_status vmps_sort_learned(void* keys, uint32_t* values, int64_t n, vmps_dtype kt,
                              uint32_t flags, const vmps_learned_config* cfg,
                              vmps_cdf_model* model, vmps_learned_stats* stats, void* ws,
                              size_t ws_bytes, void* stream);

/* Keys at the sample positions: out[i] = keys[SplitMix64(seed, i) mod n],
 * i < m, where SplitMix64(seed, i) is output i (0-based) of the published
 * SplitMix64 generator seeded with seed. */
vmps_status vmps_sample(const void* keys, int64_t n, vmps_dtype kt, int64_t m, uint64_t seed,
                        void* out, void* stream);

/* Minibatch MSE gradient of the model (forward and backward kernels).
 *   params : device float[3H+1] = w1[H] b1[H] w2[H] b2
 *   u, y   : device float[nb] inputs and targets
 *   grad   : device float[3H+1]; loss: device float[1] */
vmps_status vmps_cdf_grad(const float* params, int32_t hidden, const float* u, const float* y,
                          int32_t nb, float* grad, float* loss, void* stream);

/* Workspace of vmps_cdf_train for m sample keys: the features and the
 * training state between Adam steps. */
vmps_status vmps_cdf_train_workspace_size(int64_t m, size_t* bytes);

/* Train on a sorted sample and compile (model: device).  Quantile
 * initialisation, cfg->steps Adam steps (minibatch j of step s is sample
 * point ((s*batch + j) * 0x9E3779B1) mod m; one launch per step, the
 * minibatch's gradient summed over workgroups in a fixed order), then the
 * better of the initial and the trained model by the MSE over every 64th
 * sample point (or the trained one with VMPS_CDF_KEEP_TRAINED).  ws: at
 * least vmps_cdf_train_workspace_size(m) bytes, 256-byte aligned; on return
 * its first m floats hold the normalised features u_i = (z_i - z_lo)/(z_hi -
 * z_lo) the model was trained on (fp32). */
vmps_status vmps_cdf_train(const void* sorted_sample, int64_t m, vmps_dtype kt,
                           const vmps_learned_config* cfg, vmps_cdf_model* model, void* ws,
                           size_t ws_bytes, void* stream);

/* Compile given parameters (device float[3H+1]) for a feature range. */
vmps_status vmps_cdf_compile(const float* params, int32_t hidden, uint64_t z_lo, uint64_t z_hi,
                             int32_t key_bits, int32_t feature_bits, int32_t knots,
                             vmps_cdf_model* model, void* stream);

/* Bucket id of every key under a compiled model (ids: device u32[n]). */
vmps_status vmps_bucket_ids(const void* keys, int64_t n, vmps_dtype kt, const vmps_cdf_model* model,
                            int32_t num_buckets, uint32_t* ids, void* stream);

vmps_status vmps_partition_workspace_size(int64_t n, vmps_dtype kt, int has_values,
                                          int32_t num_buckets, size_t* bytes);

/* Stable partition by bucket id (a stable counting sort by bucket): keys
 * with smaller bucket ids first, input order inside a bucket.
 * bucket_offsets: device int64[B+1].  keys_out must not overlap keys_in. */
vmps_status vmps_partition(const void* keys_in, const uint32_t* vals_in, int64_t n, vmps_dtype kt,
                           const vmps_cdf_model* model, int32_t num_buckets, void* keys_out,
                           uint32_t* vals_out, int64_t* bucket_offsets, void* ws, size_t ws_bytes,
                           void* stream);

/* ---- launch parameters (autotuning) ----
 * Parameters that change how the work is spread over the GPU, never the
 * result.  One table entry per key type and with/without values, shared by
 * every later call in the process (set it before sorting; not for use
 * concurrently with sorts).  A zero field keeps the built-in default. */
typedef struct {
    int32_t tile_wg_per_cu; /* workgroups per CU in the persistent LDS pass
                               (0: as many as LDS and registers allow) */
    int32_t merge_grid;     /* workgroups of one HBM merge level (0: 2048) */
    int32_t bucket_div;     /* learned path: buckets of about T/bucket_div
                               keys, T the LDS tile (0: 8) */
    int32_t host_wait;      /* 1: the sorts wait on the host for the
                               planner's merge-level counts and launch only
                               the non-empty levels; 0 (default): fully
                               asynchronous, every level launched (empty
                               ones return at once); 0 or 1 only */
    int32_t merge_ki;       /* outputs per thread of an HBM merge-level tile
                               (256 threads): 8 or 16 (0: 16, or 8 for 64-bit
                               keys with values); the workspace sizes allow
                               either.  The paged sort keeps the default. */
    int32_t tile_elems;     /* segmented sort (vmps_segmented_sort and its
                               graph), 32-bit keys without values only: the
                               LDS tile T, 16384 or 8192 elements (0: 16384);
                               other configurations accept 0 only.  The
                               segmented workspace size allows either. */
    int32_t tile_threads;   /* threads of a tile-pass workgroup with
                               tile_elems = 8192: 512 (16 keys per thread) or
                               256 (32 per thread); 0 keeps 512.  Must be 0
                               or 512 when tile_elems is 0 or 16384. */
} vmps_tuning;

/* t == NULL restores the defaults.  Negative fields, bucket_div > 64,
 * host_wait outside {0, 1}, merge_ki outside {0, 8, 16}, or a tile_elems /
 * tile_threads pair other than those listed above -> INVALID_ARG. */
vmps_status vmps_set_tuning(vmps_dtype kt, int has_values, const vmps_tuning* t);
vmps_status vmps_get_tuning(vmps_dtype kt, int has_values, vmps_tuning* t);

/* ---- graph capture ----
 * The whole enqueue sequence of one call captured into a HIP graph (on a
 * private capture stream, with launch tracing suspended), so that the same
 * sort of the same buffers can be replayed with one launch.  The buffers,
 * sizes and workspace are bound at capture time and must stay allocated
 * until vmps_graph_destroy; each replay sorts whatever the buffers then
 * hold.  Nothing is executed by the capture itself.  Argument errors are
 * those of the captured call. */
typedef struct vmps_graph_s* vmps_graph;

vmps_status vmps_segmented_sort_graph(void* keys, uint32_t* values, const int64_t* seg_offsets, int64_t nseg,
                                      int64_t total, vmps_dtype kt, void* ws, size_t ws_bytes,
                                      vmps_graph* graph);
vmps_status vmps_sort_learned_graph(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                                    const vmps_learned_config* cfg, vmps_learned_stats* stats, void* ws,
                                    size_t ws_bytes, vmps_graph* graph);
/* Replays a captured graph on `stream` (asynchronous). */
vmps_status vmps_graph_launch(vmps_graph graph, void* stream);
vmps_status vmps_graph_destroy(vmps_graph graph);

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
