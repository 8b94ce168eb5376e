// LDS Powersort of one segment per workgroup.
//
// A segment is either a whole small Powersort instance or a subtree of a
// large instance's merge tree that fits the tile (the planner guarantees the
// segment starts and ends on run boundaries).  Inside LDS the workgroup
// repeats the method on the segment:
//   ExtractRun with the minrun extension (Sections 2, 3 and 5): descent
//     bitmap by ballot, long natural runs, the chain of run starts;
//   Power of every boundary (theorem of Section 2) from the 32-bit midpoint
//     expansions, with positions taken in the instance's coordinates so the
//     powers equal those of the whole instance;
//   forced runs sorted stably (rank of (key, position) inside the run,
//     which yields exactly the straight insertion sort's result);
//   merges of Algorithm 1 by decreasing power, each level split over the
//     threads by merge path, StandardMerge semantics (Algorithm 2): on ties
//     the left run goes first.
// The result is written once, to the buffer the planner chose (Pingpong).
#include "vmps_internal.hpp"

namespace vmps {

template <typename K>
__device__ inline K bcast_lane(K x, int j);

template <>
__device__ inline uint32_t bcast_lane<uint32_t>(uint32_t x, int j)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, j);
}

template <>
__device__ inline uint64_t bcast_lane<uint64_t>(uint64_t x, int j)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

template <int TCAP>
struct TileMeta {
    static constexpr uint32_t RC = TCAP / 32 + 3;  // runs (each >= 32 long but the last)
    static constexpr uint32_t BW = TCAP / 64 + 2;  // bitmap words
};

template <typename K, int NT, int TCAP, int VMODE>
constexpr size_t tile_lds_bytes()
{
    using M = TileMeta<TCAP>;
    size_t b = 2 * sizeof(K) * TCAP;
    if (VMODE) b += 2 * sizeof(uint32_t) * TCAP;
    b += 8 * M::BW;                    // bitmap
    b += 4 * (2 * M::RC);              // long runs (u, e)
    b += 4 * (2 * (M::RC + 1));        // progressions (base, prefix)
    b += 4 * (M::RC + 1);              // run starts
    b += 4 * M::RC;                    // Q
    b += 4 * (2 * M::RC);              // node L, R per boundary
    b += 4 * M::RC;                    // node list of a level
    b += M::RC;                        // powers
    b += 4 * (NT / 64 + 1) + 64;       // scan scratch + scalars
    return (b + 15) & ~(size_t)15;
}

template <typename K, int NT, int TCAP, int VMODE>
__global__ __launch_bounds__(NT) void k_tilesort(K* __restrict__ keysA, K* __restrict__ keysB,
                                                 uint32_t* __restrict__ valsA, uint32_t* __restrict__ valsB,
                                                 const Seg* __restrict__ segs,
                                                 const uint32_t* __restrict__ nseg_dev, uint32_t nseg_host,
                                                 const uint32_t* __restrict__ inst_start, uint32_t ell_ovr)
{
    using M = TileMeta<TCAP>;
    constexpr int NW = NT / 64;
    constexpr uint32_t KI = TCAP / NT;
    static_assert(TCAP % NT == 0, "tile must split evenly");
    static_assert(TCAP / 64 + 1 <= NT, "one thread per bitmap word");

    extern __shared__ __align__(16) uint8_t smem[];
    uint8_t* sp = smem;
    K* KA = (K*)sp; sp += sizeof(K) * TCAP;
    K* KB = (K*)sp; sp += sizeof(K) * TCAP;
    uint32_t* VA = nullptr;
    uint32_t* VB = nullptr;
    if (VMODE) { VA = (uint32_t*)sp; sp += 4 * TCAP; VB = (uint32_t*)sp; sp += 4 * TCAP; }
    uint64_t* bm = (uint64_t*)sp; sp += 8 * M::BW;
    uint32_t* LRu = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* LRe = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* PGb = (uint32_t*)sp; sp += 4 * (M::RC + 1);
    uint32_t* PGc = (uint32_t*)sp; sp += 4 * (M::RC + 1);
    uint32_t* RS = (uint32_t*)sp; sp += 4 * (M::RC + 1);
    uint32_t* Qv = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* BL = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* BR = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* NLi = (uint32_t*)sp; sp += 4 * M::RC;
    uint32_t* scan_lds = (uint32_t*)sp; sp += 4 * (NW + 1);
    uint32_t* scal = (uint32_t*)sp; sp += 4 * 8;  // [0] progressions [1] runs [2] power mask [3] nodes
    uint8_t* PW = sp;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nseg = nseg_dev ? *nseg_dev : nseg_host;

    for (uint32_t si = blockIdx.x; si < nseg; si += gridDim.x) {
        const Seg sg = segs[si];
        const uint32_t a = sg.start;
        const uint32_t len = sg.end - sg.start;
        if (len == 0) continue;
        if (len > TCAP) {
            // a single natural run longer than the tile: already sorted
            if (sg.dst == 1) {
                for (uint32_t i = tid; i < len; i += NT) {
                    keysB[a + i] = keysA[a + i];
                    if (VMODE == 1) valsB[a + i] = valsA[a + i];
                    if (VMODE == 2) valsB[a + i] = a + i;
                }
            } else if (VMODE == 2) {
                for (uint32_t i = tid; i < len; i += NT) valsA[a + i] = a + i;
            }
            continue;
        }
        const uint32_t ib = inst_start[sg.inst];
        const uint32_t il = inst_start[sg.inst + 1] - ib;
        const uint32_t ell = ell_ovr ? ell_ovr : minrun_of(il);
        const uint32_t g = a - ib;

        // 1. load
        for (uint32_t i = tid; i < len; i += NT) {
            KA[i] = keysA[a + i];
            if (VMODE == 1) VA[i] = valsA[a + i];
            if (VMODE == 2) VA[i] = a + i;
        }
        __syncthreads();

        // 2. descent bitmap (positions >= len count as boundaries)
        const uint32_t W = len / 64 + 1;
        for (uint32_t w = wave; w < W; w += NW) {
            const uint32_t p = w * 64 + lane;
            const bool bit = (p >= len) || (p == 0) || (KA[p - 1] > KA[p]);
            const uint64_t word = __ballot(bit);
            if (lane == 0) bm[w] = word;
        }
        __syncthreads();

        // 3. long natural runs (length >= minrun), one thread per word
        uint32_t cnt = 0, lu0 = 0, le0 = 0, lu1 = 0, le1 = 0;
        if ((uint32_t)tid < W) {
            const uint64_t word = bm[tid];
            const uint32_t p0 = tid * 64;
            uint64_t bits = word;
            while (bits) {
                const int b = ffs64(bits);
                bits &= bits - 1;
                const uint32_t u = p0 + b;
                if (u >= len) break;
                const uint64_t above = (b == 63) ? 0ull : ((word >> (b + 1)) << (b + 1));
                uint32_t next = len;
                if (above) {
                    next = p0 + ffs64(above);
                } else {
                    for (uint32_t ww = tid + 1; ww < W; ++ww) {
                        const uint64_t x = bm[ww];
                        if (x) { next = ww * 64 + ffs64(x); break; }
                    }
                }
                if (next > len) next = len;
                if (next - u >= ell) {
                    if (cnt == 0) { lu0 = u; le0 = next; } else { lu1 = u; le1 = next; }
                    ++cnt;
                }
            }
        }
        if (cnt > 2) cnt = 2;  // runs of >= 32 elements: at most two start in a word
        uint32_t nlr;
        const uint32_t lro = block_excl_scan(cnt, scan_lds, &nlr);
        if (cnt > 0) { LRu[lro] = lu0; LRe[lro] = le0; }
        if (cnt > 1) { LRu[lro + 1] = lu1; LRe[lro + 1] = le1; }
        __syncthreads();

        // 4. chain of run starts: progressions of step minrun between jumps
        if (tid == 0) {
            uint32_t r = 0, np = 0, acc = 0;
            for (uint32_t j = 0; j < nlr; ++j) {
                const uint32_t u = LRu[j], e = LRe[j];
                const uint32_t sf = u + ((r % ell) + ell - u % ell) % ell;
                if (e - sf >= ell) {
                    PGb[np] = r; PGc[np] = acc;
                    acc += (sf - r) / ell + 1;
                    ++np;
                    r = e;
                }
            }
            PGb[np] = r; PGc[np] = acc;
            acc += (r < len) ? (len - r + ell - 1) / ell : 0u;
            ++np;
            PGc[np] = acc;
            scal[0] = np;
            scal[1] = acc < M::RC - 1 ? acc : M::RC - 1;  // runs >= 32 long: never clamps
            scal[2] = 0;
        }
        __syncthreads();
        const uint32_t np = scal[0], kr = scal[1];

        // 5. run starts
        for (uint32_t t = tid; t < kr; t += NT) {
            uint32_t lo = 0, hi = np;
            while (hi - lo > 1) {
                const uint32_t m = (lo + hi) >> 1;
                if (PGc[m] <= t) lo = m; else hi = m;
            }
            RS[t] = PGb[lo] + (t - PGc[lo]) * ell;
        }
        if (tid == 0) RS[kr] = len;
        __syncthreads();

        // 6. midpoint expansions and powers
        for (uint32_t t = tid; t < kr; t += NT) {
            const uint64_t s2 = 2ull * g + RS[t] + RS[t + 1];
            Qv[t] = (uint32_t)((s2 << 31) / il);
        }
        __syncthreads();
        for (uint32_t t = tid; t + 1 < kr; t += NT) {
            const uint32_t p = __clz(Qv[t] ^ Qv[t + 1]) + 1;
            PW[t] = (uint8_t)p;
            atomicOr(&scal[2], 1u << (p - 1));
        }
        __syncthreads();
        // node extents: nearest boundaries of smaller power inside the segment
        for (uint32_t t = tid; t + 1 < kr; t += NT) {
            const uint32_t p = PW[t], sh = 32 - p;
            const uint64_t c = (uint64_t)Qv[t + 1] >> sh;
            const uint64_t V = (c - 1) << sh, Wd = (c + 1) << sh;
            int lo = -1, hi = (int)t;
            while (hi - lo > 1) {
                const int m = (lo + hi) >> 1;
                if (Qv[m] < V) lo = m; else hi = m;
            }
            BL[t] = lo < 0 ? 0u : RS[lo + 1];
            int lo2 = (int)t + 1, hi2 = (int)kr;
            while (hi2 - lo2 > 1) {
                const int m = (lo2 + hi2) >> 1;
                if (Qv[m] < Wd) lo2 = m; else hi2 = m;
            }
            BR[t] = (lo2 == (int)kr - 1) ? len : RS[lo2 + 1];
        }

        // 7. forced runs: stable rank sort inside each run (one wave per run)
        K* cur = KA;
        K* oth = KB;
        uint32_t* vcur = VA;
        uint32_t* voth = VB;
        for (uint32_t t = wave; t < kr; t += NW) {
            const uint32_t s = RS[t], rl = RS[t + 1] - RS[t];
            bool sorted = true;
            K x = 0;
            uint32_t v = 0;
            if (rl <= 64) {
                if ((uint32_t)lane < rl) {
                    x = cur[s + lane];
                    if (VMODE) v = vcur[s + lane];
                }
                const bool desc = lane > 0 && (uint32_t)lane < rl && cur[s + lane - 1] > x;
                sorted = __ballot(desc) == 0;
            }
            if (sorted) {
                for (uint32_t i = lane; i < rl; i += 64) {
                    oth[s + i] = cur[s + i];
                    if (VMODE) voth[s + i] = vcur[s + i];
                }
            } else {
                uint32_t rank = 0;
                for (uint32_t j = 0; j < rl; ++j) {
                    const K y = bcast_lane<K>(x, (int)j);
                    rank += (y < x || (y == x && j < (uint32_t)lane)) ? 1u : 0u;
                }
                if ((uint32_t)lane < rl) {
                    oth[s + rank] = x;
                    if (VMODE) voth[s + rank] = v;
                }
            }
        }
        __syncthreads();
        { K* tk = cur; cur = oth; oth = tk; uint32_t* tv = vcur; vcur = voth; voth = tv; }

        // 8. merges by decreasing power
        uint32_t mask = scal[2];
        while (mask) {
            const uint32_t p = 32 - __clz(mask);
            mask &= ~(1u << (p - 1));
            if (wave == 0) {
                uint32_t base = 0;
                for (uint32_t c0 = 0; c0 + 1 < kr; c0 += 64) {
                    const uint32_t t = c0 + lane;
                    const bool f = (t + 1 < kr) && PW[t] == p;
                    const uint64_t bal = __ballot(f);
                    if (f) NLi[base + __popcll(bal & ((1ull << lane) - 1))] = t;
                    base += __popcll(bal);
                }
                if (lane == 0) scal[3] = base;
            }
            __syncthreads();
            const int nn = (int)scal[3];
            uint32_t pos = tid * KI;
            const uint32_t end = min(len, pos + KI);
            if (pos < end) {
                int ni = -1;
                {
                    int lo = -1, hi = nn;
                    while (hi - lo > 1) {
                        const int m = (lo + hi) >> 1;
                        if (BL[NLi[m]] <= pos) lo = m; else hi = m;
                    }
                    ni = lo;
                }
                while (pos < end) {
                    while (ni + 1 < nn && BL[NLi[ni + 1]] <= pos) ++ni;
                    const bool inside = ni >= 0 && pos < BR[NLi[ni]];
                    if (inside) {
                        const uint32_t t = NLi[ni];
                        const uint32_t L = BL[t], Mid = RS[t + 1], R = BR[t];
                        const uint32_t stop = min(end, R);
                        const uint32_t na = Mid - L, nb = R - Mid, d = pos - L;
                        uint32_t lo = d > nb ? d - nb : 0u, hi = min(d, na);
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (cur[L + mid] <= cur[Mid + d - 1 - mid]) lo = mid + 1; else hi = mid;
                        }
                        uint32_t ia = L + lo, jb = Mid + (d - lo);
                        for (; pos < stop; ++pos) {
                            const bool takeA = ia < Mid && (jb >= R || cur[ia] <= cur[jb]);
                            if (takeA) {
                                oth[pos] = cur[ia];
                                if (VMODE) voth[pos] = vcur[ia];
                                ++ia;
                            } else {
                                oth[pos] = cur[jb];
                                if (VMODE) voth[pos] = vcur[jb];
                                ++jb;
                            }
                        }
                    } else {
                        const uint32_t nextL = (ni + 1 < nn) ? BL[NLi[ni + 1]] : len;
                        const uint32_t stop = min(end, nextL);
                        for (; pos < stop; ++pos) {
                            oth[pos] = cur[pos];
                            if (VMODE) voth[pos] = vcur[pos];
                        }
                    }
                }
            }
            __syncthreads();
            { K* tk = cur; cur = oth; oth = tk; uint32_t* tv = vcur; vcur = voth; voth = tv; }
        }

        // 9. one write to the planned buffer
        K* outK = sg.dst ? keysB : keysA;
        uint32_t* outV = sg.dst ? valsB : valsA;
        for (uint32_t i = tid; i < len; i += NT) {
            outK[a + i] = cur[i];
            if (VMODE) outV[a + i] = vcur[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- host --
template <typename K, int NT, int TCAP, int VMODE>
static hipError_t launch_tilesort(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                                  const uint32_t* nseg_dev, uint32_t nseg_host, uint32_t grid,
                                  uint32_t ell_ovr, hipStream_t s)
{
    constexpr size_t lds = tile_lds_bytes<K, NT, TCAP, VMODE>();
    static bool attr_set = false;
    if (!attr_set) {
        VMPS_HIP(hipFuncSetAttribute((const void*)k_tilesort<K, NT, TCAP, VMODE>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set = true;
    }
    TraceScope tr(VMPS_TRACE_TILESORT, s);
    k_tilesort<K, NT, TCAP, VMODE><<<grid, NT, lds, s>>>((K*)keysA, (K*)keysB, valsA, valsB, P.segs, nseg_dev,
                                                        nseg_host, P.inst_start, ell_ovr);
    return hipGetLastError();
}

uint32_t tilesort_capacity(int key_bits, int has_values)
{
    if (key_bits == 32) return has_values ? 8192u : 16384u;
    return has_values ? 4096u : 8192u;
}

size_t tilesort_lds_bytes(int key_bits, int has_values, uint32_t)
{
    if (key_bits == 32)
        return has_values ? tile_lds_bytes<uint32_t, 1024, 8192, 1>() : tile_lds_bytes<uint32_t, 1024, 16384, 0>();
    return has_values ? tile_lds_bytes<uint64_t, 512, 4096, 1>() : tile_lds_bytes<uint64_t, 1024, 8192, 0>();
}

hipError_t tilesort_enqueue(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                            int key_bits, int vmode, uint32_t ell_override, hipStream_t s)
{
    const uint32_t grid = P.seg_cap < 4096u ? P.seg_cap : 4096u;
    const uint32_t* nseg_dev = P.counters + CNT_NSEG;
    if (key_bits == 32) {
        if (vmode == 0) return launch_tilesort<uint32_t, 1024, 16384, 0>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
        if (vmode == 1) return launch_tilesort<uint32_t, 1024, 8192, 1>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
        return launch_tilesort<uint32_t, 1024, 8192, 2>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
    }
    if (vmode == 0) return launch_tilesort<uint64_t, 1024, 8192, 0>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
    if (vmode == 1) return launch_tilesort<uint64_t, 512, 4096, 1>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
    return launch_tilesort<uint64_t, 512, 4096, 2>(P, keysA, keysB, valsA, valsB, nseg_dev, 0, grid, ell_override, s);
}

}  // namespace vmps
