// Internal declarations of the vmps HIP library (gfx950 / MI355X).
//
// The library sorts unsigned keys stably with Powersort's merge policy
// ("Virtual-Memory Powersort", Algorithm 1 and the Power theorem of Section 2,
// Pingpong buffers of Section 3), re-scheduled for a GPU:
//   * runs and powers are computed for all positions at once,
//   * the merge tree is executed level by level (a level = one power),
//   * subtrees no longer than an LDS tile are sorted inside one workgroup,
//   * longer merges are split into fixed-size output tiles by merge path.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vmps.h"

namespace vmps {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int WAVE = 64;
constexpr int MAX_LEVEL = 33;          // powers are 1..32 for n <= 2^32
constexpr uint32_t BITMAP_TILE = 4096; // positions per run-scan workgroup
constexpr uint32_t CHAIN_BLOCK = 2048; // long runs per chain-scan block

// ------------------------------------------------------------ helpers --
__host__ __device__ inline uint32_t minrun_of(uint64_t n)
{
    // minrun rule of Section 5: halve (rounding up) until below 64
    uint64_t l = n;
    while (l >= 64) l = (l + 1) >> 1;
    return (uint32_t)l;
}

__host__ __device__ inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Highest power a merge longer than T elements can have, in Powersort
// instances of at most n elements (the powers of Section 2, from 32-bit
// midpoint expansions).  Every boundary inside a node of power p has power
// at least p, so the runs on its two sides sum to less than il 2^(2-p) (plus
// one unit of the midpoints' rounding), and the node's run midpoints lie in
// a window of width il 2^(1-p): the node is shorter than 3 il 2^(1-p) plus
// rounding, under 4.5 il 2^(1-p).  So a node longer than T has 2^p < 9 n / T,
// and the levels above that power hold no merge in HBM.  Capped at
// ceil(log2 n), above which no power occurs.
inline uint32_t hbm_top_level(uint64_t n, uint32_t T)
{
    uint32_t top = 1;
    while (top < 32 && (1ull << top) < n) ++top;
    uint32_t p = 1;
    while (p < top && ((uint64_t)2 * T << p) < 9 * n) ++p;
    return p;
}

// Inclusive scan across the 64 lanes of a wave.
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over the workgroup; *total gets the workgroup sum.
// lds must hold blockDim/64 + 1 words.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* lds, uint32_t* total)
{
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    uint32_t inc = wave_incl_scan(v);
    if (lane == WAVE - 1) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < nw; ++w) { uint32_t t = lds[w]; lds[w] = acc; acc += t; }
        lds[nw] = acc;
    }
    __syncthreads();
    uint32_t res = lds[wave] + inc - v;
    if (total) *total = lds[nw];
    __syncthreads();
    return res;
}

// Position of the first set bit (0-based) of a non-zero word.
__device__ inline int ffs64(uint64_t w) { return __ffsll((unsigned long long)w) - 1; }

// One LDS-sort unit: a subtree of at most T elements (or a single sorted run
// longer than T), its Powersort instance, and the buffer it must end up in.
struct Seg {
    uint32_t start;  // global position
    uint32_t end;
    uint32_t inst;   // instance index
    uint32_t dst;    // 0 = keys (A), 1 = workspace copy (B)
};

// Device pointers of the planner, carved from the caller's workspace.
struct Plan {
    uint32_t n, k;                 // total length, number of instances
    uint32_t T;                    // LDS tile length (elements)
    uint32_t big_min;              // instances longer than this are planned here
    uint32_t T_out;                // merge output tile length
    uint32_t n_tiles_out;          // ceil(n / T_out)
    uint32_t lr_cap, run_cap, ent_cap, seg_cap, chain_blocks, bm_tiles, bm_words;
    uint32_t h_cap;                // nodes longer than T (HBM nodes)
    // instances
    const int64_t* inst_off64;     // caller offsets (k+1), may be null for k = 1
    bool off_trusted;              // offsets built by the library: valid by construction
    const uint32_t* k_dev;         // nullable: instances from this count on (device) are empty
    uint32_t* inst_start;          // k+1
    uint32_t* inst_big;            // k (0/1), scanned into inst_bigrank
    uint32_t* inst_bigrank;        // k
    uint32_t* inst_rfinal;         // k
    uint32_t* inst_run_lo;         // k
    uint32_t* inst_run_hi;         // k
    // run detection
    uint64_t* bitmap;              // bm_words
    uint32_t* tile_first;          // bm_tiles
    uint32_t* tile_next;           // bm_tiles
    // descending runs (vmps_sort with VMPS_DESCENDING_RUNS, one instance):
    // first position that is not a descent, per bitmap tile, and after it
    uint32_t desc;                 // 0 or 1
    uint32_t* tile_first0;         // bm_tiles
    uint32_t* tile_next0;          // bm_tiles
    uint32_t* tile_cnt;            // bm_tiles
    uint32_t* tile_off;            // bm_tiles
    uint32_t* lr_u;                // lr_cap
    uint32_t* lr_e;
    uint32_t* lr_inst;
    uint32_t* lr_cnt;
    uint32_t* lr_base;
    uint32_t* chain_val;           // chain_blocks * 64
    uint64_t* chain_known;         // chain_blocks
    uint32_t* chain_rin;           // chain_blocks
    uint32_t* ent_cnt;             // ent_cap
    uint32_t* ent_base;
    uint32_t* ent_inst;
    uint32_t* ent_off;
    // runs and boundaries
    uint32_t* run_start;           // run_cap + 1
    uint32_t* run_inst;            // run_cap
    uint32_t* run_q;               // run_cap
    uint8_t*  power;               // run_cap (boundary t between runs t, t+1)
    uint32_t* bnd_l;               // run_cap: left neighbour boundary (run index) or NONE
    uint32_t* bnd_r;               // run_cap
    uint32_t* bnd_lpos;            // run_cap: node start L
    uint32_t* bnd_rpos;            // run_cap: node end R
    uint32_t* hbm_flag;            // run_cap
    uint32_t* hbm_rank;            // run_cap
    uint32_t* hbm_idx;             // run_cap: boundary -> HBM list index
    uint32_t* hbm_list;            // h_cap
    uint32_t* hbm_par[2];          // h_cap each
    uint32_t* hbm_val[2];
    uint32_t* hbm_depth;           // points at the final hbm_val buffer
    uint32_t* hbm_tiles;           // run_cap + 1 : output tiles per HBM node, scanned
    uint32_t* hbm_tile_off;
    // LDS segments
    Seg* segs;                     // seg_cap
    // merge levels: (HBM node, output tile) pairs grouped by power level
    uint32_t pair_cap;
    uint32_t* level;               // 3 * MAX_LEVEL: pairs per level, first pair, fill position
    uint32_t* node_base;           // h_cap: first pair of every HBM node
    uint32_t* pairs;               // 2 * pair_cap
    uint32_t* splits;              // 2 * pair_cap: merge-path split at both ends of every pair
    // counters (device scalars)
    uint32_t* counters;            // see CNT_* below
    // scan scratch
    uint32_t* scan_tmp;            // scan_tmp_words
    uint64_t scan_tmp_words;
    // statistics
    unsigned long long* stats;     // [0] M, [1] M_hbm, [2] levels
};

enum {
    CNT_NBIG = 0, CNT_NLONG, CNT_NENT, CNT_NRUNS, CNT_NHBM, CNT_NSEG, CNT_NPAIRS,
    CNT_MAXPOW, CNT_BAD, CNT_TICKET, CNT_TICKET2, CNT_COUNT = 16
};

// ------------------------------------------------------------ tracing --
// Brackets the launches issued in its lifetime with HIP events when
// vmps_trace_enable(1) is in effect (kinds: vmps_trace_kind).
class TraceScope {
public:
    TraceScope(int kind, hipStream_t s);
    ~TraceScope();
    TraceScope(const TraceScope&) = delete;
    TraceScope& operator=(const TraceScope&) = delete;

private:
    int kind_;
    hipStream_t stream_;
    void* a_;
};

// ------------------------------------------------------------ tuning --
// Launch parameters that change speed, never results (vmps_set_tuning).
struct Tuning {
    int tile_wg_per_cu;  // workgroups per CU of the persistent LDS pass (0: as many as fit)
    int merge_grid;      // workgroups of a merge level (0: 2048)
    int bucket_div;      // learned buckets target the tile length / bucket_div (0: 2)
    int host_wait;       // 1: wait on the host for the level counts, launch the non-empty levels only
    int merge_ki;        // outputs per thread of a merge-level tile (0: default)
    int tile_elems;      // segmented sort, 32-bit keys without values: LDS tile (0: default)
    int tile_threads;    // workgroup size of that tile pass (0: 512)
};
const Tuning& tuning_for(int key_bits, bool has_values);

// Tracing is suspended while a graph is captured (events are not captured).
bool trace_suspend();
void trace_resume(bool was_on);

// ------------------------------------------------------------ host API --
// min_len: a lower bound on every run's length but each instance's last
// (16 for explicit minruns and several instances; a one-instance sort with
// the minrun rule passes minrun_of(n)), which sizes the run arrays.
size_t plan_workspace_bytes(uint64_t n, uint64_t k, uint32_t T, uint32_t T_out, uint32_t min_len = 16);
// Carve Plan arrays from ws; returns bytes used.
size_t plan_carve(Plan& P, void* ws, uint64_t n, uint64_t k, uint32_t T, uint32_t T_out, uint32_t min_len = 16);

// Re-lay every level's pairs in position order (nodes left to right, each
// node's tiles in order).  bsum, boff: MAX_LEVEL * plan_order_blocks(P)
// words each; tmp: scan_tmp_words of that count.
uint64_t plan_order_blocks(const Plan& P);
hipError_t plan_order_levels(Plan& P, uint32_t* bsum, uint32_t* boff, uint32_t* tmp, hipStream_t s);

// Enqueue run detection + powers + tree + placement for the instances.
// key_bits: 32 or 64. ell_override: 0 = minrun rule.
hipError_t plan_enqueue(Plan& P, const void* keys, int key_bits, uint32_t ell_override,
                        hipStream_t s);

// Device-wide exclusive scan of count u32 values (count read from device if
// count_dev != null, else count_host). total (device, nullable) gets the sum.
hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t count_host,
                              const uint32_t* count_dev, uint32_t* total, uint32_t* tmp,
                              hipStream_t s);
uint64_t scan_tmp_words(uint64_t count);

hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t count, hipStream_t s);

// LDS Powersort over the segment list (k_tilesort).
// narrow (64-bit keys without values): the tile pass variant that sorts
// segments whose keys span less than 2^32 on 32-bit offsets, with segments
// of up to 4096 keys in a launch of 256-thread workgroups (four per CU) and
// the longer ones in the 512-thread launch; worth it where most segments
// are short and narrow (the learned buckets).  32-bit keys without values
// also run plans made with T = 8192 (the segmented sort's tuned tile), in
// 512-thread or, with threads = 256, 256-thread workgroups; any other T
// for that configuration is an error.
hipError_t tilesort_enqueue(const Plan& P, void* keysA, void* keysB, uint32_t* valsA,
                            uint32_t* valsB, int key_bits, int vmode, uint32_t narrow,
                            hipStream_t s, int threads = 0);
uint32_t tilesort_capacity(int key_bits, int has_values);
size_t tilesort_lds_bytes(int key_bits, int has_values, uint32_t T);

// HBM merge levels.
// With the opt-in host_wait tuning (and allowed by the caller): copies the
// planner's per-level pair counts to pinned host memory (not while the
// stream is being captured); the next merge_levels_enqueue for the same plan
// waits for that copy only (the tile pass enqueued in between keeps the GPU
// busy meanwhile) and launches the non-empty levels alone.  Otherwise it
// disarms any earlier probe and every level is launched.
hipError_t level_probe_enqueue(const Plan& P, int key_bits, int has_values, hipStream_t s,
                               bool allowed = true);
// fused: every level is one launch whose workgroups search their own tile
// cuts (for plans whose levels are mostly empty).
hipError_t merge_levels_enqueue(const Plan& P, void* keysA, void* keysB, uint32_t* valsA,
                                uint32_t* valsB, int key_bits, int has_values, hipStream_t s,
                                bool fused = false);
// Merge-level output tile with the tuning's merge_ki; the built-in default
// (the paged sort's page); the smallest choice, which sizes workspaces.
uint32_t merge_tile_out(int key_bits, int has_values);
uint32_t merge_tile_default(int key_bits, int has_values);
constexpr uint32_t MERGE_TILE_MIN = 256 * 8;

// Standalone stable merge of two sorted arrays.
hipError_t merge_two_enqueue(const void* a, const uint32_t* va, uint32_t na, const void* b,
                             const uint32_t* vb, uint32_t nb, void* out, uint32_t* vout,
                             int key_bits, uint32_t* splits, hipStream_t s);

// Groups of consecutive learned buckets, at most C keys each (a bucket
// longer than C alone): goff[0, G] the group starts and n, goff(G, B] = n
// (empty instances).  Scratch: group_scratch_words(B) words.
// The group count G goes to *group_count(scratch) (device).
uint64_t group_scratch_words(uint32_t B);
hipError_t group_enqueue(const int64_t* boff, uint32_t B, uint32_t n, uint32_t C, int64_t* goff,
                         uint32_t* scratch, hipStream_t s);
const uint32_t* group_count(const uint32_t* scratch, uint32_t B);

// Learned partition (learned.hip).
uint64_t partition_arena_words(uint64_t n, uint32_t B);
hipError_t partition_enqueue(const void* kin, const uint32_t* vin, void* ktmp, uint32_t* vtmp, void* kout,
                             uint32_t* vout, uint32_t n, int key_bits, int vmode, const vmps_cdf_model* model,
                             uint32_t B, int64_t* bucket_off, uint32_t* arena, hipStream_t s);
hipError_t sample_enqueue(const void* keys, uint64_t n, int key_bits, uint64_t m, uint64_t seed, void* out,
                          hipStream_t s);
// Training: features into u (m floats), then initialisation, one launch per
// Adam step and the final choice and compilation, with their state in tb
// (train_buf_floats() floats).
uint64_t train_buf_floats();
hipError_t train_enqueue(const void* sorted, uint64_t m, int key_bits, const vmps_learned_config& c, float* u, float* tb,
                         vmps_cdf_model* model, hipStream_t s);
hipError_t grad_enqueue(const float* params, int H, const float* u, const float* y, int nb, float* grad,
                        float* loss, hipStream_t s);
hipError_t compile_enqueue(const float* params, int H, uint64_t z_lo, uint64_t z_hi, int key_bits, int fbits,
                           int K, vmps_cdf_model* model, hipStream_t s);
hipError_t bucket_ids_enqueue(const void* keys, uint64_t n, int key_bits, const vmps_cdf_model* model,
                              uint32_t B, uint32_t* ids, hipStream_t s);
// Error judge over the sorted sample (JUDGE_GRID workgroups, 6 partial
// words each in part), then the bucket statistics.
constexpr uint32_t JUDGE_GRID = 256;
hipError_t learned_stats_enqueue(const int64_t* off, uint32_t B, uint32_t T, const vmps_cdf_model* model,
                                 const void* sample, uint64_t m, int key_bits, uint64_t* part,
                                 vmps_learned_stats* st, hipStream_t s);

// Paged merge levels (vm.hip): workspace bytes, pool + copy page bytes,
// page length, and the sort (n > 1, arguments checked).
size_t vm_workspace_bytes(uint64_t n, int key_bits, int has_values, uint64_t window_pages);
size_t vm_buffer_bytes(uint64_t n, int key_bits, int has_values, uint64_t window_pages);
uint32_t vm_page_elems(int key_bits, int has_values);
uint64_t vm_window_pages(uint64_t n, int key_bits, int has_values, uint64_t window_pages);
hipError_t vm_sort_enqueue(void* keys, uint32_t* values, uint64_t n, int key_bits, int vmode, uint32_t desc,
                           uint64_t window_pages, void* ws, unsigned long long* stats, hipStream_t s);

// Large records (records.hip): key extraction, (key, index) sort in the
// workspace after the keys and indices, gather.  *st gets the sort's status.
size_t records_workspace_bytes(uint64_t n, int key_bits);
hipError_t records_enqueue(const void* in, void* out, uint64_t n, uint32_t rb, uint32_t off, int key_bits,
                           uint32_t flags, void* ws, size_t sort_ws_bytes, hipStream_t s, vmps_status* st);

// The whole stable sort of one array with a caller-provided workspace
// (vmps_sort's body after its argument checks; allow_host_wait = false never
// waits on the host and allocates nothing, whatever the tuning says;
// fused_levels: one launch per merge level, as merge_levels_enqueue's).
vmps_status sort_in_workspace(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags, void* ws,
                              size_t ws_bytes, hipStream_t s, bool allow_host_wait, bool fused_levels = false);
vmps_status check_sort_args(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags);

}  // namespace vmps

#define VMPS_HIP(x)                                  \
    do {                                             \
        hipError_t e__ = (x);                        \
        if (e__ != hipSuccess) return e__;           \
    } while (0)
