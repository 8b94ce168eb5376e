// Merges longer than an LDS tile, one tree level (one power) per launch.
//
// Every merge [L,Mid) + [Mid,R) of the level is cut into output tiles of
// T_out elements aligned to multiples of T_out in the array; the cut points
// of the two inputs come from a merge-path binary search (the output prefix
// of length d holds the first i elements of the left run and the first d-i
// of the right run).  This plays the role of PageMerge in Algorithm 2: a
// merge into a bounded output page whose trip count is fixed, so the inner
// loop needs no output bound check.  Ties go to the left run (StandardMerge).
#include "merge_tile.hpp"

namespace vmps {

struct LevelArgs {
    const uint32_t* level;   // pairs per level, then first pair of each level
    const uint32_t* pairs;   // (HBM node, output tile)
    const uint32_t* hbm_list;
    const uint32_t* lpos;
    const uint32_t* rpos;
    const uint32_t* run_start;
    const uint32_t* depth;
    uint32_t* splits;        // split at both ends of every pair
    uint32_t T_out;
    uint32_t lvl;
};

// Merge-path splits at both ends of every output tile of the level (one
// thread per end); an empty level returns at once.
template <typename K>
__global__ void k_level_partition(LevelArgs A, const K* __restrict__ keysA, const K* __restrict__ keysB)
{
    const uint32_t cnt = A.level[A.lvl], off = A.level[MAX_LEVEL + A.lvl];
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < 2ull * cnt;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = off + (uint32_t)(x >> 1), end = (uint32_t)(x & 1);
        const uint32_t q = A.pairs[2 * (uint64_t)i], tt = A.pairs[2 * (uint64_t)i + 1];
        const uint32_t t = A.hbm_list[q];
        const uint32_t L = A.lpos[t], Mid = A.run_start[t + 1], R = A.rpos[t];
        const K* src = (A.depth[q] & 1u) ? keysA : keysB;  // node writes to depth parity, reads the other
        const uint64_t t0 = (uint64_t)tt * A.T_out;
        const uint32_t o = end ? (uint32_t)(R < t0 + A.T_out ? R : t0 + A.T_out) : (uint32_t)(L > t0 ? L : t0);
        A.splits[2 * (uint64_t)i + end] = merge_path<K>(src + L, Mid - L, src + Mid, R - Mid, o - L);
    }
}

// One output tile per workgroup iteration, over the level's pairs.  FUSED:
// the tile cuts are searched here instead of read from k_level_partition's
// table, so a level is one launch (for levels that are mostly empty, as in
// the learned path, where only buckets longer than the tile reach them,
// that halves the launches).  The workgroup takes its tiles in chunks of
// up to NT / 2: all their cuts are searched at once, one thread each, then
// the chunk's tiles are merged in turn, so one search latency is spent per
// chunk rather than per tile.
template <typename K, bool VAL, int NT, int KI, bool FUSED>
__global__ __launch_bounds__(NT) void k_level_merge(LevelArgs A, K* __restrict__ keysA, K* __restrict__ keysB,
                                                    uint32_t* __restrict__ valsA, uint32_t* __restrict__ valsB)
{
    constexpr uint32_t TO = NT * KI;
    constexpr uint32_t SP = MergeLds<TO>::SP;
    constexpr uint32_t CH = FUSED ? NT / 2 : 1;  // tiles per chunk
    __shared__ uint32_t s_cut[2 * CH];
    extern __shared__ __align__(16) uint8_t smem[];
    K* S = (K*)smem;
    uint32_t* SV = (uint32_t*)(S + SP);
    const uint32_t cnt = A.level[A.lvl], off = A.level[MAX_LEVEL + A.lvl];
    for (uint64_t jb = blockIdx.x; jb < cnt; jb += (uint64_t)gridDim.x * CH) {
        if constexpr (FUSED) {
            // cut x: tile k = x / 2 of the chunk, its start (even x) or end
            const uint32_t x = threadIdx.x;
            const uint64_t j = jb + (uint64_t)(x >> 1) * gridDim.x;
            if (x < 2 * CH && j < cnt) {
                const uint32_t i = off + (uint32_t)j;
                const uint32_t q = A.pairs[2 * (uint64_t)i], tt = A.pairs[2 * (uint64_t)i + 1];
                const uint32_t t = A.hbm_list[q];
                const uint32_t L = A.lpos[t], Mid = A.run_start[t + 1], R = A.rpos[t];
                const K* src = (A.depth[q] & 1u) ? keysA : keysB;
                const uint64_t t0 = (uint64_t)tt * TO;
                const uint32_t o = (x & 1) ? (uint32_t)(R < t0 + TO ? R : t0 + TO) : (uint32_t)(L > t0 ? L : t0);
                s_cut[x] = merge_path<K>(src + L, Mid - L, src + Mid, R - Mid, o - L);
            }
            __syncthreads();
        }
        for (uint32_t k = 0; k < CH; ++k) {
            const uint64_t jj = jb + (uint64_t)k * gridDim.x;
            if (jj >= cnt) break;
            const uint32_t i = off + (uint32_t)jj;
            const uint32_t q = A.pairs[2 * (uint64_t)i], tt = A.pairs[2 * (uint64_t)i + 1];
            const uint32_t t = A.hbm_list[q];
            const uint32_t L = A.lpos[t], Mid = A.run_start[t + 1], R = A.rpos[t];
            const bool dstB = (A.depth[q] & 1u) != 0;
            K* src = dstB ? keysA : keysB;
            K* dst = dstB ? keysB : keysA;
            uint32_t* vsrc = dstB ? valsA : valsB;
            uint32_t* vdst = dstB ? valsB : valsA;
            const uint64_t t0 = (uint64_t)tt * TO;
            const uint32_t o0 = (uint32_t)(L > t0 ? L : t0);
            const uint32_t o1 = (uint32_t)(R < t0 + TO ? R : t0 + TO);
            const uint32_t i0 = FUSED ? s_cut[2 * k] : A.splits[2 * (uint64_t)i];
            const uint32_t i1 = FUSED ? s_cut[2 * k + 1] : A.splits[2 * (uint64_t)i + 1];
            const uint32_t j0 = (o0 - L) - i0, j1 = (o1 - L) - i1;
            merge_tile<K, VAL, NT, KI>(src + L, VAL ? vsrc + L : nullptr, i0, i1, src + Mid,
                                       VAL ? vsrc + Mid : nullptr, j0, j1, dst + o0, VAL ? vdst + o0 : nullptr, S,
                                       SV);
        }
        if constexpr (FUSED) __syncthreads();  // every cut read before the next chunk's are written
    }
}

// Opt-in host wait (tuning host_wait = 1).  Per host thread and device: a
// pinned copy of the level counts and the event that marks its arrival
// (allocated on first use, kept until exit).
struct LevelProbe {
    uint32_t* host = nullptr;
    hipEvent_t ev = nullptr;
    const uint32_t* src = nullptr;
    bool armed = false;
};

static LevelProbe& level_probe()
{
    thread_local LevelProbe pr[16];
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) d = 0;
    return pr[d & 15];
}

hipError_t level_probe_enqueue(const Plan& P, int key_bits, int has_values, hipStream_t s, bool allowed)
{
    LevelProbe& pr = level_probe();
    pr.armed = false;
    if (!allowed || !tuning_for(key_bits, has_values != 0).host_wait) return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    VMPS_HIP(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;  // a graph launches every level
    if (!pr.host) {
        VMPS_HIP(hipHostMalloc((void**)&pr.host, sizeof(uint32_t) * MAX_LEVEL, hipHostMallocDefault));
        VMPS_HIP(hipEventCreateWithFlags(&pr.ev, hipEventDisableTiming));
    }
    VMPS_HIP(hipMemcpyAsync(pr.host, P.level, sizeof(uint32_t) * MAX_LEVEL, hipMemcpyDeviceToHost, s));
    VMPS_HIP(hipEventRecord(pr.ev, s));
    pr.src = P.level;
    pr.armed = true;
    return hipSuccess;
}

template <typename K, bool VAL, int NT, int KI>
static hipError_t launch_levels(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                                hipStream_t s, bool fused)
{
    constexpr uint32_t TO = NT * KI;
    constexpr size_t lds = (sizeof(K) + (VAL ? sizeof(uint32_t) : 0)) * MergeLds<TO>::SP;
    static bool attr_set[16] = {};  // once per device
    int dev = 0;
    VMPS_HIP(hipGetDevice(&dev));
    if (!attr_set[dev & 15]) {
        VMPS_HIP(hipFuncSetAttribute((const void*)k_level_merge<K, VAL, NT, KI, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        VMPS_HIP(hipFuncSetAttribute((const void*)k_level_merge<K, VAL, NT, KI, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev & 15] = true;
    }
    LevelArgs A;
    A.level = P.level;
    A.pairs = P.pairs;
    A.hbm_list = P.hbm_list;
    A.lpos = P.bnd_lpos;
    A.rpos = P.bnd_rpos;
    A.run_start = P.run_start;
    A.depth = P.hbm_depth;
    A.splits = P.splits;
    A.T_out = TO;
    const uint32_t top = hbm_top_level(P.n, P.T);  // higher levels hold no merge longer than T
    const uint64_t most = (uint64_t)P.n_tiles_out + 2 * ((uint64_t)P.n / (P.T ? P.T : 1) + 1);  // pairs of one level
    const unsigned pgrid = (unsigned)(ceil_div(2 * most, 256) < 256 ? ceil_div(2 * most, 256) : 256);
    const int tg = tuning_for(sizeof(K) * 8, VAL).merge_grid;
    const uint64_t gcap = tg > 0 ? (uint64_t)tg : 2048u;
    const unsigned mgrid = (unsigned)(most < gcap ? most : gcap);
    uint32_t cnt[MAX_LEVEL];
    bool known = false;
    LevelProbe& pr = level_probe();
    if (pr.armed && pr.src == P.level) {
        pr.armed = false;
        VMPS_HIP(hipEventSynchronize(pr.ev));
        for (int l = 0; l < MAX_LEVEL; ++l) cnt[l] = pr.host[l];
        known = true;
    }
    for (int lvl = (int)top; lvl >= 1; --lvl) {
        A.lvl = (uint32_t)lvl;
        unsigned pg = pgrid, mg = mgrid;
        if (known) {
            if (cnt[lvl] == 0) continue;
            const uint64_t c = cnt[lvl];
            pg = (unsigned)(ceil_div(2 * c, 256) < pgrid ? ceil_div(2 * c, 256) : pgrid);
            mg = (unsigned)(c < mgrid ? c : mgrid);
        }
        if (fused) {
            TraceScope tr(VMPS_TRACE_LEVEL_MERGE, s);
            k_level_merge<K, VAL, NT, KI, true><<<mg, NT, lds, s>>>(A, (K*)keysA, (K*)keysB, valsA, valsB);
            continue;
        }
        {
            TraceScope tr(VMPS_TRACE_LEVEL_PARTITION, s);
            k_level_partition<K><<<pg, 256, 0, s>>>(A, (const K*)keysA, (const K*)keysB);
        }
        {
            TraceScope tr(VMPS_TRACE_LEVEL_MERGE, s);
            k_level_merge<K, VAL, NT, KI, false><<<mg, NT, lds, s>>>(A, (K*)keysA, (K*)keysB, valsA, valsB);
        }
    }
    return hipGetLastError();
}

uint32_t merge_tile_default(int key_bits, int has_values)
{
    if (key_bits == 64 && has_values) return 256 * 8;
    return 256 * 16;
}

uint32_t merge_tile_out(int key_bits, int has_values)
{
    const int ki = tuning_for(key_bits, has_values != 0).merge_ki;
    return ki ? 256u * (uint32_t)ki : merge_tile_default(key_bits, has_values);
}

// The level tiles are those the plan was made with (P.T_out).
hipError_t merge_levels_enqueue(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                                int key_bits, int has_values, hipStream_t s, bool fused)
{
    const bool k16 = P.T_out == 256 * 16;
    if (key_bits == 32) {
        if (has_values) {
            if (k16) return launch_levels<uint32_t, true, 256, 16>(P, keysA, keysB, valsA, valsB, s, fused);
            return launch_levels<uint32_t, true, 256, 8>(P, keysA, keysB, valsA, valsB, s, fused);
        }
        if (k16) return launch_levels<uint32_t, false, 256, 16>(P, keysA, keysB, valsA, valsB, s, fused);
        return launch_levels<uint32_t, false, 256, 8>(P, keysA, keysB, valsA, valsB, s, fused);
    }
    if (has_values) {
        if (k16) return launch_levels<uint64_t, true, 256, 16>(P, keysA, keysB, valsA, valsB, s, fused);
        return launch_levels<uint64_t, true, 256, 8>(P, keysA, keysB, valsA, valsB, s, fused);
    }
    if (k16) return launch_levels<uint64_t, false, 256, 16>(P, keysA, keysB, valsA, valsB, s, fused);
    return launch_levels<uint64_t, false, 256, 8>(P, keysA, keysB, valsA, valsB, s, fused);
}

// ------------------------------------------------- merge of two arrays --
template <typename K>
__global__ void k_merge2_partition(const K* __restrict__ a, uint32_t na, const K* __restrict__ b, uint32_t nb,
                                   uint32_t TO, uint32_t ntiles, uint32_t* __restrict__ splits)
{
    const uint32_t tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile > ntiles) return;
    const uint64_t d = (uint64_t)tile * TO;
    const uint32_t dd = (uint32_t)(d < (uint64_t)na + nb ? d : (uint64_t)na + nb);
    splits[tile] = merge_path<K>(a, na, b, nb, dd);
}

template <typename K, bool VAL, int NT, int KI>
__global__ __launch_bounds__(NT) void k_merge2(const K* __restrict__ a, const uint32_t* __restrict__ va, uint32_t na,
                                               const K* __restrict__ b, const uint32_t* __restrict__ vb,
                                               uint32_t nb, K* __restrict__ out, uint32_t* __restrict__ vout,
                                               uint32_t ntiles, const uint32_t* __restrict__ splits)
{
    constexpr uint32_t TO = NT * KI;
    constexpr uint32_t SP = MergeLds<TO>::SP;
    extern __shared__ __align__(16) uint8_t smem[];
    K* S = (K*)smem;
    uint32_t* SV = (uint32_t*)(S + SP);
    const uint64_t ntot = (uint64_t)na + nb;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t o0 = (uint64_t)tile * TO;
        const uint64_t o1 = o0 + TO < ntot ? o0 + TO : ntot;
        const uint32_t i0 = splits[tile], i1 = splits[tile + 1];
        const uint32_t j0 = (uint32_t)(o0 - i0), j1 = (uint32_t)(o1 - i1);
        merge_tile<K, VAL, NT, KI>(a, va, i0, i1, b, vb, j0, j1, out + o0, VAL ? vout + o0 : nullptr, S, SV);
    }
}

template <typename K, bool VAL>
static hipError_t merge2_t(const K* a, const uint32_t* va, uint32_t na, const K* b, const uint32_t* vb,
                           uint32_t nb, K* out, uint32_t* vout, uint32_t* splits, hipStream_t s)
{
    constexpr int NT = 256, KI = 16;
    constexpr uint32_t TO = NT * KI;
    constexpr size_t lds = (sizeof(K) + (VAL ? sizeof(uint32_t) : 0)) * MergeLds<TO>::SP;
    static bool attr_set[16] = {};  // once per device
    int dev = 0;
    VMPS_HIP(hipGetDevice(&dev));
    if (!attr_set[dev & 15]) {
        VMPS_HIP(hipFuncSetAttribute((const void*)k_merge2<K, VAL, NT, KI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
        attr_set[dev & 15] = true;
    }
    const uint64_t ntot = (uint64_t)na + nb;
    const uint32_t ntiles = (uint32_t)ceil_div(ntot, TO);
    k_merge2_partition<K><<<(unsigned)ceil_div(ntiles + 1, 256), 256, 0, s>>>(a, na, b, nb, TO, ntiles, splits);
    const unsigned grid = ntiles < 4096 ? ntiles : 4096;
    k_merge2<K, VAL, NT, KI><<<grid, NT, lds, s>>>(a, va, na, b, vb, nb, out, vout, ntiles, splits);
    return hipGetLastError();
}

hipError_t merge_two_enqueue(const void* a, const uint32_t* va, uint32_t na, const void* b, const uint32_t* vb,
                             uint32_t nb, void* out, uint32_t* vout, int key_bits, uint32_t* splits,
                             hipStream_t s)
{
    if ((uint64_t)na + nb == 0) return hipSuccess;
    const bool vals = vout != nullptr;  // va or vb may be null when its run is empty
    if (key_bits == 32) {
        if (vals) return merge2_t<uint32_t, true>((const uint32_t*)a, va, na, (const uint32_t*)b, vb, nb,
                                                (uint32_t*)out, vout, splits, s);
        return merge2_t<uint32_t, false>((const uint32_t*)a, va, na, (const uint32_t*)b, vb, nb, (uint32_t*)out,
                                         vout, splits, s);
    }
    if (vals) return merge2_t<uint64_t, true>((const uint64_t*)a, va, na, (const uint64_t*)b, vb, nb,
                                            (uint64_t*)out, vout, splits, s);
    return merge2_t<uint64_t, false>((const uint64_t*)a, va, na, (const uint64_t*)b, vb, nb, (uint64_t*)out, vout,
                                     splits, s);
}

}  // namespace vmps
