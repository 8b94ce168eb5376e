// LDS Powersort of one segment per workgroup.
//
// A segment is either a whole small Powersort instance or a subtree of a
// large instance's merge tree that fits the tile (the planner guarantees it
// starts and ends on run boundaries).  Inside LDS the workgroup repeats the
// method on the segment:
//   ExtractRun with the minrun extension (Sections 2, 3 and 5): descent
//     bitmap by ballot, long natural runs, the chain of run starts;
//   Power of every boundary (theorem of Section 2) from the 32-bit midpoint
//     expansions, with positions in the instance's coordinates so the powers
//     equal those of the whole instance;
//   forced runs sorted stably: bottom-up merges of aligned blocks inside the
//     run, which gives exactly the insertion sort's result;
//   merges of Algorithm 1 by decreasing power (StandardMerge: on ties the
//     left run goes first).
// Every merge pass is split over the threads by merge path: thread i owns
// outputs [i*KI, (i+1)*KI), computes them into registers, and writes them
// back into the single LDS buffer after a barrier.  The segment is written
// once, to the buffer the planner chose (Pingpong).
#include <type_traits>

#include "merge_tile.hpp"

namespace vmps {

// One spare LDS slot after every 32 elements: threads write KI = 16
// consecutive outputs, and the padding spreads simultaneous writes of a wave
// over distinct banks.
__device__ __forceinline__ uint32_t px(uint32_t i) { return i + (i >> 5); }

// The layout of a tile's elements (LAY): 0 plain; 1 one spare slot after
// every 32 elements (px); 2 one spare slot after every 16.  In a merge pass
// lane t reads near position t * KI / 2 of each run and writes KI outputs
// from t * KI, so in the plain layout lanes a few apart meet in one LDS
// bank; a spare slot per 16 32-bit elements spreads both patterns over the
// banks (the 16 outputs of a lane start 17 words after the previous lane's).
template <int LAY>
__device__ __forceinline__ uint32_t pxp(uint32_t i) { return LAY == 1 ? px(i) : (LAY == 2 ? i + (i >> 4) : i); }

// Length of the blocks the spare slots separate (elements).
template <int LAY>
constexpr uint32_t lay_block() { return LAY == 2 ? 16u : 32u; }

// S[pxp<LAY>(i)] read with its byte offset formed as (i + i / block) scaled
// by the key size: one shift and one v_add_lshl_u32 (plain VGPR arithmetic),
// with the buffer's base left to the LDS instruction's offset field.  Left
// to itself the compiler splits the scaled sum into two scaled terms, two
// more instructions on every merge step.
template <int LAY, typename K>
__device__ __forceinline__ K lds_get(const K* __restrict__ S, uint32_t i)
{
    if constexpr (LAY == 0) {
        return S[i];
    } else {
        const uint32_t q = i >> (LAY == 1 ? 5 : 4);
        uint32_t off;
        if constexpr (sizeof(K) == 8)
            asm("v_add_lshl_u32 %0, %1, %2, 3" : "=v"(off) : "v"(i), "v"(q));
        else
            asm("v_add_lshl_u32 %0, %1, %2, 2" : "=v"(off) : "v"(i), "v"(q));
        return *(const K*)((const uint8_t*)S + off);
    }
}

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
// (the step number is a constant expression inside f).
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// The B cursor of a merge step from the A cursor: inside one node every
// output advances exactly one cursor, so before output j the cursors sum to
// s0 + j, and jb = (s0 - ia) + j with s0 >= ia.  One v_sad_u32 (|a - b| + c,
// plain VGPR arithmetic) instead of advancing jb by the complement of the
// comparison's lane mask (a select and an add).
template <int J>
__device__ __forceinline__ uint32_t b_cursor(uint32_t s0, uint32_t ia)
{
    uint32_t jb;
    asm("v_sad_u32 %0, %1, %2, %3" : "=v"(jb) : "v"(s0), "v"(ia), "i"(J));
    return jb;
}

template <int TCAP>
struct TileMeta {
    static constexpr uint32_t RC = TCAP / 32 + 3;  // runs: each >= 32 long except the last
    static constexpr uint32_t BW = TCAP / 64 + 2;  // bitmap words
    static constexpr uint32_t SP = TCAP + TCAP / 32 + 1;  // padded element slots
};

// Whether a tile configuration declares its LDS statically (see k_tilesort).
template <typename K, int VMODE>
constexpr bool tile_lds_static() { return !(sizeof(K) == 4 && VMODE != 0); }

template <typename K, int NT, int TCAP, int VMODE>
constexpr size_t tile_lds_bytes()
{
    using M = TileMeta<TCAP>;
    // every section starts 16-byte aligned
    size_t b = (sizeof(K) * M::SP + 15) & ~(size_t)15;
    if (VMODE) b += (4 * M::SP + 15) & ~(size_t)15;
    b += 8 * M::BW;                   // bitmap
    b += 4 * 2 * M::RC;               // long runs (u, e), later Q and the node list
    b += 4 * 2 * (M::RC + 1);         // progressions (base, prefix), later node L, R
    b += 4 * (M::RC + 1);             // run starts
    b += 4 * M::RC;                   // node starts in level order
    b += 2 * M::RC;                   // powers, sorted-run flags
    b += 4 * 2 * 34;                  // level start / count
    b += 4 * (NT / 64) * 33;          // per-wave power counts
    b += 4 * (NT / 64 + 1) + 64;      // scan scratch + scalars
    return (b + 15) & ~(size_t)15;
}

// One merge pass.  Every output position belongs to one node of the pass:
// a merge node [L,M)+[M,R) or a copy node (M == R: the range stays as it
// is).  Thread i produces outputs [i*KI, (i+1)*KI) into registers: the first
// node is found by nd.first (with a merge-path search when the thread starts
// inside a merge node), every later node starts exactly where the previous one
// ended, so nd.next needs no search.  The single static loop keeps the
// register staging arrays indexed by constants.  After a barrier the outputs
// go back into the same LDS buffer.
template <typename K, int KI, int TCAP, int VMODE, int LAY, typename Nodes>
__device__ __forceinline__ void merge_pass(K* __restrict__ S, uint32_t* __restrict__ SV, uint32_t len, uint32_t tid,
                                           Nodes nd)
{
    // KI dividing the padding block keeps a thread's outputs inside one
    // block (affine write-back); other KI compute each output's slot
    constexpr bool AFFINE = lay_block<LAY>() % KI == 0;
    const uint32_t p0 = tid * KI;
    K rk[KI];
    uint32_t rv[KI];
    if (p0 < len) {
        uint32_t L, M, R;
        nd.first(p0, L, M, R);
        uint32_t ia = p0, jb = R;
        if (M < R) {
            const uint32_t na = M - L, nb = R - M, d = p0 - L;
            uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (S[pxp<LAY>(L + mid)] <= S[pxp<LAY>(M + d - 1 - mid)]) lo = mid + 1; else hi = mid;
            }
            ia = L + lo;
            jb = M + (d - lo);
        }
        K ha = S[pxp<LAY>(ia)], hb = S[pxp<LAY>(jb)];
        // the lane's outputs that land in the segment: [p0, pe)
        const uint32_t pe = min(p0 + KI, len);
        uint32_t M2 = R, R2 = R;  // the node starting at R, when the outputs reach it
        Nodes n2 = nd;
        if (R < pe) n2.next(R, M2, R2);
        if (__all(pe <= R)) {
            // Every lane's outputs lie in its first node: no node changes.
            // Indices stay <= max(R, p0 + KI) <= TCAP.  Wave-uniform, so a
            // wave runs one of the three loops only.
            const uint32_t s0 = ia + jb;
            static_for<KI>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                const bool takeA = ia < M && (jb >= R || ha <= hb);
                rk[j] = takeA ? ha : hb;
                if (VMODE) rv[j] = SV[pxp<LAY>(takeA ? ia : jb)];
                // the A cursor advances by the comparison's bit, the B
                // cursor follows from the sum
                ia += takeA ? 1u : 0u;
                // kept opaque, so that the compiler does not re-associate
                // the chain of increments (it would rebuild each step's
                // bit as a 0/1 value: one more instruction per step)
                asm("" : "+v"(ia));
                if constexpr (j + 1 < KI) {
                    jb = b_cursor<j + 1>(s0, ia);
                    const K nv = lds_get<LAY>(S, takeA ? ia : jb);
                    ha = takeA ? nv : ha;
                    hb = takeA ? hb : nv;
                }
            });
        } else if (__all(pe <= R2)) {
            // At most one node change per lane, at output R (nodes at least
            // KI long, the usual case): the second node's state is set up
            // in advance and swapped in by selects, without a branch.
            const K ha2 = S[pxp<LAY>(R)], hb2 = S[pxp<LAY>(M2)];
            uint32_t Mc = M, Rc = R;
            // the change happens at step R - p0 (> 0): compared with the
            // unrolled step number, no per-step position is kept live
            const uint32_t jsw = R - p0;
            // cursor sums: s0 + j in the first node, s1 + j in the second
            // (both cursors of the first node end exactly at M and R)
            uint32_t s0 = ia + jb;
            const uint32_t s1 = R + M2 - jsw;
            static_for<KI>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                if constexpr (j > 0) {
                    const bool sw = jsw == (uint32_t)j;
                    ia = sw ? R : ia;
                    jb = sw ? M2 : jb;
                    s0 = sw ? s1 : s0;
                    Mc = sw ? M2 : Mc;
                    Rc = sw ? R2 : Rc;
                    ha = sw ? ha2 : ha;
                    hb = sw ? hb2 : hb;
                }
                const bool takeA = ia < Mc && (jb >= Rc || ha <= hb);
                rk[j] = takeA ? ha : hb;
                if (VMODE) rv[j] = SV[pxp<LAY>(takeA ? ia : jb)];
                ia += takeA ? 1u : 0u;
                // kept opaque, so that the compiler does not re-associate
                // the chain of increments (it would rebuild each step's
                // bit as a 0/1 value: one more instruction per step)
                asm("" : "+v"(ia));
                if constexpr (j + 1 < KI) {
                    jb = b_cursor<j + 1>(s0, ia);
                    const K nv = lds_get<LAY>(S, takeA ? ia : jb);
                    ha = takeA ? nv : ha;
                    hb = takeA ? hb : nv;
                }
            });
        } else {
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const uint32_t q = p0 + j;
            if (j > 0 && q == R) {
                nd.next(q, M, R);
                ia = q;
                jb = M;
                ha = S[pxp<LAY>(ia)];
                hb = S[pxp<LAY>(jb)];
            }
            // StandardMerge: the left run wins ties; a copy node only has a left run
            const bool takeA = ia < M && (jb >= R || ha <= hb);
            rk[j] = takeA ? ha : hb;
            if (VMODE) rv[j] = SV[pxp<LAY>(takeA ? ia : jb)];
            ia += takeA ? 1u : 0u;
            jb += takeA ? 0u : 1u;
            const uint32_t nx = takeA ? ia : jb;
            const K nv = lds_get<LAY>(S, nx < (uint32_t)TCAP ? nx : (uint32_t)TCAP);
            ha = takeA ? nv : ha;
            hb = takeA ? hb : nv;
        }
        }
    }
    __syncthreads();
    if constexpr (!AFFINE) {
        if (p0 < len) {
            const uint32_t cnt = len - p0;
#pragma unroll
            for (int j = 0; j < KI; ++j) {
                if ((uint32_t)j < cnt) {
                    S[pxp<LAY>(p0 + j)] = rk[j];
                    if (VMODE) SV[pxp<LAY>(p0 + j)] = rv[j];
                }
            }
        }
    } else if (p0 < len) {
        // KI divides the block length and p0 is a multiple of KI: the
        // outputs share one padding block, pxp<LAY>(p0 + j) = pxp<LAY>(p0) + j
        const uint32_t cnt = len - p0, w0 = pxp<LAY>(p0);
        if constexpr (LAY == 0 && sizeof(K) == 4 && KI % 4 == 0) {
            if (cnt >= (uint32_t)KI) {
                // plain layout: 16-byte stores (p0 is a multiple of KI)
#pragma unroll
                for (int q = 0; q < KI / 4; ++q) {
                    *(uint4*)(S + w0 + 4 * q) = make_uint4(rk[4 * q], rk[4 * q + 1], rk[4 * q + 2], rk[4 * q + 3]);
                    if (VMODE)
                        *(uint4*)(SV + w0 + 4 * q) = make_uint4(rv[4 * q], rv[4 * q + 1], rv[4 * q + 2], rv[4 * q + 3]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < KI; ++j) {
                    if ((uint32_t)j < cnt) {
                        S[w0 + j] = rk[j];
                        if (VMODE) SV[w0 + j] = rv[j];
                    }
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < KI; ++j) {
                if ((uint32_t)j < cnt) {
                    S[w0 + j] = rk[j];
                    if (VMODE) SV[w0 + j] = rv[j];
                }
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v |= (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// Stable sort of S[s, s+cnt), cnt <= 16, in registers: odd-even
// transposition network.  It only exchanges adjacent elements that are
// strictly inverted, so equal keys keep their order (the result of the
// insertion sort); the unused slots hold the largest key and stay last.
template <typename K, int VMODE, int LAY>
__device__ __forceinline__ void chunk_sort16(K* __restrict__ S, uint32_t* __restrict__ SV, uint32_t s, uint32_t cnt)
{
    K x[16];
    uint32_t v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const bool in = (uint32_t)j < cnt;
        x[j] = in ? S[pxp<LAY>(s + j)] : ~K(0);
        v[j] = (VMODE && in) ? SV[pxp<LAY>(s + j)] : 0u;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
        for (int i = r & 1; i + 1 < 16; i += 2) {
            const bool sw = x[i] > x[i + 1];
            const K lo = sw ? x[i + 1] : x[i], hi = sw ? x[i] : x[i + 1];
            x[i] = lo;
            x[i + 1] = hi;
            if (VMODE) {
                const uint32_t vl = sw ? v[i + 1] : v[i], vh = sw ? v[i] : v[i + 1];
                v[i] = vl;
                v[i + 1] = vh;
            }
        }
    }
    asm volatile("" : "+v"(s));  // recompute the addresses rather than keep 16 of them live
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if ((uint32_t)j < cnt) {
            S[pxp<LAY>(s + j)] = x[j];
            if (VMODE) SV[pxp<LAY>(s + j)] = v[j];
        }
    }
}

// Batcher's merge-exchange network for N inputs (N a power of two), as a
// list of comparators (a, b), a < b: Knuth's Algorithm M (The Art of
// Computer Programming, Vol. 3, 5.2.2), 191 comparators for N = 32.
template <int N>
struct BatcherNet {
    static constexpr int count()
    {
        int c = 0;
        for (int p = N / 2; p >= 1; p >>= 1) {
            int q = N / 2, r = 0, d = p;
            for (;;) {
                for (int i = 0; i + d < N; ++i)
                    if ((i & p) == r) ++c;
                if (q == p) break;
                d = q - p;
                q >>= 1;
                r = p;
            }
        }
        return c;
    }
    uint8_t a[count()], b[count()];
    constexpr BatcherNet() : a(), b()
    {
        int c = 0;
        for (int p = N / 2; p >= 1; p >>= 1) {
            int q = N / 2, r = 0, d = p;
            for (;;) {
                for (int i = 0; i + d < N; ++i)
                    if ((i & p) == r) {
                        a[c] = (uint8_t)i;
                        b[c] = (uint8_t)(i + d);
                        ++c;
                    }
                if (q == p) break;
                d = q - p;
                q >>= 1;
                r = p;
            }
        }
    }
};

// Sort of S[s, s+cnt), cnt <= N (32 or 64), keys without values: equal keys
// cannot be told apart, so the result of any sorting network is the stable
// sort (the result of the insertion sort).  Min/max comparators on the
// registers; unused slots hold the largest key and stay last.  With N = 64
// a whole forced run (minrun is below 64) is sorted by one lane, and no
// bottom-up merge pass over the tile is needed to join two 32-key halves.
template <int N>
constexpr BatcherNet<N> batcher_net{};

template <int N, typename K, int LAY>
__device__ __forceinline__ void chunk_sort_net(K* __restrict__ S, uint32_t s, uint32_t cnt)
{
    K x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = (uint32_t)j < cnt ? S[pxp<LAY>(s + j)] : ~K(0);
    // every comparator's register indices are compile-time constants (a
    // loop the compiler does not unroll fully would put x in scratch memory)
    static_for<BatcherNet<N>::count()>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        constexpr int ia = batcher_net<N>.a[c], ib = batcher_net<N>.b[c];
        const K u = x[ia], v = x[ib];
        x[ia] = u < v ? u : v;
        x[ib] = u < v ? v : u;
    });
    asm volatile("" : "+v"(s));  // recompute the addresses rather than keep N of them live
#pragma unroll
    for (int j = 0; j < N; ++j)
        if ((uint32_t)j < cnt) S[pxp<LAY>(s + j)] = x[j];
}

// Nodes of one bottom-up level inside the forced runs: aligned blocks of 2w
// from each unsorted run's start are merged as [ps, ps+w) + [ps+w, ps+2w);
// already sorted runs and runs of at most w elements are copy nodes.
struct RunLevel {
    const uint32_t* RS;
    const uint8_t* SR;
    uint32_t len, w, wlog, rt, rs, re;
    bool srt;
    __device__ void node_at(uint32_t q, uint32_t& M, uint32_t& R) const
    {
        if (srt || re - rs <= w) { M = re; R = re; return; }
        M = min(q + w, re);
        R = min(q + 2 * w, re);
    }
    __device__ void first(uint32_t q, uint32_t& L, uint32_t& M, uint32_t& R)
    {
        rs = RS[rt]; re = RS[rt + 1]; srt = SR[rt] != 0;
        L = rs + (((q - rs) >> (wlog + 1)) << (wlog + 1));
        node_at(L, M, R);
    }
    __device__ void next(uint32_t q, uint32_t& M, uint32_t& R)
    {
        if (q >= len) { M = len; R = len; return; }
        if (q == re) { ++rt; rs = q; re = RS[rt + 1]; srt = SR[rt] != 0; }
        node_at(q, M, R);
    }
};

// Nodes of one power level of the merge tree, in position order in
// NL[b0, b0+cn) (their starts in BLs): node t merges [BL[t], RS[t+1]) with
// [RS[t+1], BR[t]); the gaps between them are copy nodes.
struct TreeLevel {
    const uint32_t* NL;
    const uint32_t* BLs;
    const uint32_t* BR;
    const uint32_t* RS;
    uint32_t len, b0, cn, ni;
    __device__ void first(uint32_t q, uint32_t& L, uint32_t& M, uint32_t& R)
    {
        int lo = -1, hi = (int)cn;  // last node starting at or before q
        while (hi - lo > 1) {
            const int m = (lo + hi) >> 1;
            if (BLs[b0 + m] <= q) lo = m; else hi = m;
        }
        ni = (uint32_t)(lo + 1);
        if (lo >= 0) {
            const uint32_t t = NL[b0 + lo];
            if (q < BR[t]) { L = BLs[b0 + lo]; M = RS[t + 1]; R = BR[t]; return; }
        }
        L = q;
        M = R = ni < cn ? BLs[b0 + ni] : len;
    }
    __device__ void next(uint32_t q, uint32_t& M, uint32_t& R)
    {
        if (ni < cn) {
            const uint32_t bl = BLs[b0 + ni];
            if (bl == q) {
                const uint32_t t = NL[b0 + ni];
                ++ni;
                M = RS[t + 1];
                R = BR[t];
                return;
            }
            M = R = bl;
            return;
        }
        M = R = len;
    }
};

// All merges of one segment with KI outputs per thread: the bottom-up
// levels inside the forced runs above the sorted chunks of 2^cwl elements,
// then Algorithm 1's merges by decreasing power.
template <typename K, int KI, int TCAP, int VMODE, int LAY>
__device__ __forceinline__ void tile_merges(K* __restrict__ S, uint32_t* __restrict__ SV, uint32_t len, uint32_t tid,
                                            uint32_t kr,
                                            const uint32_t* RS, const uint8_t* SR, const uint32_t* NL,
                                            const uint32_t* BLs, const uint32_t* BR, const uint32_t* LVs,
                                            const uint32_t* LVc, uint32_t maxf, uint32_t mask, uint32_t cwl)
{
    uint32_t myrun = 0;  // run holding this thread's first output
    {
        const uint32_t q0 = tid * KI;
        uint32_t lo = 0, hi = kr;
        while (hi - lo > 1) {
            const uint32_t m = (lo + hi) >> 1;
            if (RS[m] <= q0) lo = m; else hi = m;
        }
        myrun = lo;
    }
    for (uint32_t wlog = cwl; (1u << wlog) < maxf; ++wlog) {
        RunLevel nd{RS, SR, len, 1u << wlog, wlog, myrun, 0, 0, false};
        merge_pass<K, KI, TCAP, VMODE, LAY>(S, SV, len, tid, nd);
    }
    while (mask) {
        const uint32_t p = 32 - __clz(mask);
        mask &= ~(1u << (p - 1));
        TreeLevel nd{NL, BLs, BR, RS, len, LVs[p], LVc[p], 0};
        merge_pass<K, KI, TCAP, VMODE, LAY>(S, SV, len, tid, nd);
    }
}

// HBM -> LDS, batches of loads in flight before their LDS stores.
template <typename K, int NT, int TCAP, int VMODE>
__device__ __forceinline__ void tile_load(K* __restrict__ S, uint32_t* __restrict__ SV, const K* __restrict__ src,
                                          const uint32_t* __restrict__ vsrc, uint32_t a, uint32_t len, uint32_t tid)
{
    static_assert(NT % 32 == 0, "affine padded index");
    constexpr int CH = TCAP / NT;
    constexpr int BT = CH < 8 ? CH : 8;
    const uint32_t pt = px(tid);
#pragma unroll
    for (int c = 0; c < CH; c += BT) {
        K r[BT];
        uint32_t v[BT];
#pragma unroll
        for (int j = 0; j < BT; ++j) {
            // unmasked loads (positions past the end read the last element
            // and are not stored), so that all of them are in flight at once
            const uint32_t i = (uint32_t)((c + j) * NT) + tid;
            const uint32_t ic = i < len ? i : len - 1;
            r[j] = src[a + ic];
            v[j] = VMODE == 1 ? vsrc[a + ic] : 0u;
        }
#pragma unroll
        for (int j = 0; j < BT; ++j) {
            const uint32_t i = (uint32_t)((c + j) * NT) + tid;
            const uint32_t pi = pt + (uint32_t)((c + j) * (NT + NT / 32));  // px(i), NT a multiple of 32
            if (i < len) {
                S[pi] = r[j];
                if (VMODE == 1) SV[pi] = v[j];
                if (VMODE == 2) SV[pi] = a + i;
            }
        }
    }
}

// LDS -> HBM, the reverse of tile_load; element x of the LDS copy goes out
// as base + x (base = 0 for a full-width copy).
template <typename KT, typename K, int NT, int TCAP, int VMODE, int LAY>
__device__ __forceinline__ void tile_store(const KT* __restrict__ S, const uint32_t* __restrict__ SV,
                                           K* __restrict__ dst, uint32_t* __restrict__ vdst, uint32_t a, uint32_t len,
                                           uint32_t tid, K base)
{
    static_assert(NT % 32 == 0, "affine padded index");
    constexpr int CH = TCAP / NT;
    constexpr int BT = CH < 8 ? CH : 8;
#pragma unroll
    for (int c = 0; c < CH; c += BT) {
        K r[BT];
        uint32_t v[BT];
#pragma unroll
        for (int j = 0; j < BT; ++j) {
            const uint32_t i = (uint32_t)((c + j) * NT) + tid;
            // pxp(i) = pxp(tid) + (c + j) * pxp(NT), NT a multiple of 32
            const uint32_t pi = LAY == 0 ? i : pxp<LAY>(tid) + (uint32_t)((c + j) * pxp<LAY>(NT));
            r[j] = i < len ? base + (K)S[pi] : K(0);
            v[j] = (VMODE && i < len) ? SV[pi] : 0u;
        }
#pragma unroll
        for (int j = 0; j < BT; ++j) {
            const uint32_t i = (uint32_t)((c + j) * NT) + tid;
            if (i < len) {
                dst[a + i] = r[j];
                if (VMODE) vdst[a + i] = v[j];
            }
        }
    }
}

// One load per 128-byte line of the keys (and values) of the workgroup's
// next segment, issued before the current segment's store: the lines come
// into the XCD's L2 while the store runs, and the next segment's own loads
// then find them there.  The loaded words are folded into one register
// that the next segment consumes as a dependence only (a single register
// carried around the loop, where the keys themselves would be 16).
template <typename K, int NT, int TCAP, int VMODE>
__device__ __forceinline__ uint32_t tile_touch(const K* __restrict__ src, const uint32_t* __restrict__ vsrc,
                                               const Seg nx, bool nok, uint32_t tid)
{
    constexpr uint32_t KL = 128 / sizeof(K);  // keys per line
    uint32_t t = 0;
    if (nok) {
        const uint32_t n = nx.end - nx.start;
        for (uint32_t i = tid * KL; i < n; i += NT * KL) t |= (uint32_t)src[nx.start + i];
        if (VMODE == 1)
            for (uint32_t i = tid * 32; i < n; i += NT * 32) t |= vsrc[nx.start + i];
    }
    return t;
}

// One step of a wave reduction of 64-bit values by DPP: each lane combines
// its value with the one CTRL names (lanes without a source, or in rows
// outside RM, combine with the identity).
template <bool MAX, int CTRL, int RM>
__device__ __forceinline__ uint64_t dpp_minmax_step(uint64_t v)
{
    constexpr uint64_t id = MAX ? 0ull : ~0ull;
    const uint32_t l = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)id, (int)(uint32_t)v, CTRL, RM, 0xf, false);
    const uint32_t h =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(id >> 32), (int)(uint32_t)(v >> 32), CTRL, RM, 0xf, false);
    const uint64_t t = ((uint64_t)h << 32) | l;
    return MAX ? (t > v ? t : v) : (t < v ? t : v);
}

// Minimum (or maximum) of a 64-bit value over the 64 lanes of a wave (all
// active), in scalar registers: prefix steps inside each row of 16 lanes
// (shifts 1, 2, 4, 8), then row 0's last lane into row 1 and row 2's into
// row 3, then lane 31 into rows 2 and 3; lane 63 holds the result.  No LDS
// traffic, where lane shuffles would take six LDS permute rounds per half.
template <bool MAX>
__device__ __forceinline__ uint64_t wave_minmax_u64(uint64_t v)
{
    v = dpp_minmax_step<MAX, 0x111, 0xf>(v);  // row_shr:1
    v = dpp_minmax_step<MAX, 0x112, 0xf>(v);  // row_shr:2
    v = dpp_minmax_step<MAX, 0x114, 0xf>(v);  // row_shr:4
    v = dpp_minmax_step<MAX, 0x118, 0xf>(v);  // row_shr:8
    v = dpp_minmax_step<MAX, 0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_minmax_step<MAX, 0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)h << 32) | l;
}

// HBM -> LDS for 64-bit keys: all CH keys of a thread in registers, the
// segment's minimum and maximum by a block reduction (red: 4 * NT/64 words
// of LDS), then either 32-bit offsets from the minimum (returns true, kmin
// = the minimum) when the range spans less than 2^32, or the keys.
template <int NT, int TCAP, int VMODE>
__device__ __forceinline__ bool tile_load_narrow(uint64_t* __restrict__ S, uint32_t* __restrict__ SV,
                                                 const uint64_t* __restrict__ src, const uint32_t* __restrict__ vsrc,
                                                 uint32_t a, uint32_t len, uint32_t tid, uint32_t* red,
                                                 uint64_t& kmin)
{
    static_assert(NT % 32 == 0, "affine padded index");
    constexpr int CH = TCAP / NT;
    constexpr int NW = NT / 64;
    const uint32_t pt = px(tid);
    uint64_t r[CH];
    uint32_t v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        // unmasked loads (positions past the end read the last element and
        // are excluded below), so that all of them are in flight at once
        const uint32_t i = (uint32_t)(c * NT) + tid;
        const uint32_t ic = i < len ? i : len - 1;
        r[c] = src[a + ic];
        v[c] = VMODE == 1 ? vsrc[a + ic] : 0u;
    }
    uint64_t lo = ~0ull, hi = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if ((uint32_t)(c * NT) + tid < len) {
            lo = r[c] < lo ? r[c] : lo;
            hi = r[c] > hi ? r[c] : hi;
        }
    }
    lo = wave_minmax_u64<false>(lo);
    hi = wave_minmax_u64<true>(hi);
    const uint32_t wave = tid >> 6;
    if ((tid & 63) == 0) {
        red[4 * wave + 0] = (uint32_t)lo;
        red[4 * wave + 1] = (uint32_t)(lo >> 32);
        red[4 * wave + 2] = (uint32_t)hi;
        red[4 * wave + 3] = (uint32_t)(hi >> 32);
    }
    __syncthreads();
    lo = ~0ull;
    hi = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t wl = ((uint64_t)red[4 * w + 1] << 32) | red[4 * w + 0];
        const uint64_t wh = ((uint64_t)red[4 * w + 3] << 32) | red[4 * w + 2];
        lo = wl < lo ? wl : lo;
        hi = wh > hi ? wh : hi;
    }
    // every lane holds the same minimum and maximum: keep them in scalar
    // registers (the decision and the minimum live across the whole segment)
    lo = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(lo >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)lo);
    hi = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(hi >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)hi);
    const bool narrow = hi - lo <= 0xffffffffull;  // len >= 1, so lo <= hi
    kmin = lo;
    uint32_t* S32 = (uint32_t*)S;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const uint32_t i = (uint32_t)(c * NT) + tid;
        const uint32_t pi = pt + (uint32_t)(c * (NT + NT / 32));  // px(i), NT a multiple of 32
        if (i < len) {
            // the narrow copy uses the one-per-16 padded layout (pxp<2>),
            // keys and values alike
            const uint32_t si = narrow ? pxp<2>(tid) + (uint32_t)(c * pxp<2>(NT)) : pi;
            if (narrow) S32[si] = (uint32_t)(r[c] - lo); else S[si] = r[c];
            if (VMODE == 1) SV[si] = v[c];
            if (VMODE == 2) SV[si] = a + i;
        }
    }
    return narrow;
}

// Pointers into the tile's LDS besides the elements and values.
struct TileLds {
    uint64_t* bm;
    uint32_t *R1, *R2, *RS, *LVs, *LVc, *wcnt, *scan_lds, *scal, *BLs;
    uint8_t *PW, *SR;
};

// Steps 2-8 of one segment on the LDS copy S (element type KT): ExtractRun,
// powers, node lists, the forced runs' sort and the merges.
template <typename KT, int NT, int TCAP, int VMODE, int LAY>
__device__ __forceinline__ void tile_body(KT* __restrict__ S, uint32_t* __restrict__ SV, const TileLds& T,
                                          uint32_t len, uint32_t ell, uint32_t g, uint32_t il, int tid, bool desc)
{
    using MT = TileMeta<TCAP>;
    constexpr int NW = NT / 64;
    constexpr int KI = TCAP / NT;
    constexpr uint32_t RC = MT::RC;
    const int lane = tid & 63, wave = tid >> 6;
    uint64_t* bm = T.bm;
    uint32_t *RS = T.RS, *LVs = T.LVs, *LVc = T.LVc, *wcnt = T.wcnt, *scan_lds = T.scan_lds, *scal = T.scal,
             *BLs = T.BLs;
    uint8_t *PW = T.PW, *SR = T.SR;
    // aliases: long runs -> (Q, node list); progressions -> (node L, node R)
    uint32_t* LRu = T.R1;
    uint32_t* LRe = T.R1 + RC;
    uint32_t* Qv = T.R1;
    uint32_t* NL = T.R1 + RC;
    uint32_t* PGb = T.R2;
    uint32_t* PGc = T.R2 + RC + 1;
    uint32_t* BL = T.R2;
    uint32_t* BR = T.R2 + RC + 1;

    // 2. descent bitmap (positions >= len count as boundaries)
    const uint32_t W = len / 64 + 1;
    for (uint32_t w = wave; w < W; w += NW) {
        const uint32_t p = w * 64 + lane;
        const bool bit = (p >= len) || (p == 0) || (S[pxp<LAY>(p - 1)] > S[pxp<LAY>(p)]);
        const uint64_t word = __ballot(bit);
        if (lane == 0) bm[w] = word;
    }
    __syncthreads();

    // 3. long natural runs (length >= minrun), one thread per word: maximal
    // non-decreasing runs start at a set bit and end at the next one; with
    // desc, maximal strictly decreasing runs start at a clear bit (or 0),
    // hold set bits only and end at the next clear bit (or len)
    constexpr int LRW = 4;  // runs of >= 32 elements, overlapping by at most one: at most 3 start in a word
    uint32_t cnt = 0, lu[LRW] = {}, le[LRW] = {};
    if ((uint32_t)tid < W) {
        const uint64_t word = bm[tid];
        const uint32_t p0 = tid * 64;
        for (int kind = 0; kind < (desc ? 2 : 1); ++kind) {
            const uint64_t ends = kind == 0 ? word : ~word;
            const uint64_t starts = kind == 0 ? word : (~word | (p0 == 0 ? 1ull : 0ull));
            // a long run starting at bit b has no end in (b, b+31]: only such
            // bits are examined
            uint64_t o = ends >> 1;
            o |= o >> 1;
            o |= o >> 2;
            o |= o >> 4;
            o |= o >> 8;
            o |= o >> 15;
            uint64_t bits = starts & ~o;
            while (bits) {
                const int b = ffs64(bits);
                bits &= bits - 1;
                const uint32_t u = p0 + b;
                if (u >= len) break;
                const uint64_t above = (b == 63) ? 0ull : ((ends >> (b + 1)) << (b + 1));
                uint32_t next = len;
                if (above) {
                    next = p0 + ffs64(above);
                } else {
                    for (uint32_t ww = tid + 1; ww < W; ++ww) {
                        const uint64_t x = kind == 0 ? bm[ww] : ~bm[ww];
                        if (x) { next = ww * 64 + ffs64(x); break; }
                    }
                }
                if (next > len) next = len;
                if (next - u >= ell && cnt < (uint32_t)LRW) {
                    uint32_t at = cnt;  // position order
                    while (at > 0 && lu[at - 1] > u) { lu[at] = lu[at - 1]; le[at] = le[at - 1]; --at; }
                    lu[at] = u;
                    le[at] = next;
                    ++cnt;
                }
            }
        }
    }
    uint32_t nlr;
    const uint32_t lro = block_excl_scan(cnt, scan_lds, &nlr);
#pragma unroll
    for (int c = 0; c < LRW; ++c)
        if ((uint32_t)c < cnt) { LRu[lro + c] = lu[c]; LRe[lro + c] = le[c]; }
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
        scal[1] = acc < RC - 1 ? acc : RC - 1;  // runs >= 32 long: never clamps
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

    // 6. sorted-run flags, midpoint expansions and powers
    uint32_t unsorted_max = 0, pmask = 0;
    for (uint32_t t = tid; t < kr; t += NT) {
        const uint32_t s = RS[t], e = RS[t + 1];
        bool sorted = true;     // no descent strictly inside (s, e)
        bool reversed = desc && s + 1 < e;  // with desc: only descents inside (s, e)
        if (s + 1 < e) {
            for (uint32_t w = (s + 1) >> 6; w <= ((e - 1) >> 6); ++w) {
                const uint32_t base = w * 64;
                uint64_t m = ~0ull;
                if (s + 1 > base) m &= ~0ull << (s + 1 - base);
                if (e - base < 64) m &= (1ull << (e - base)) - 1;
                const uint64_t word = bm[w] & m;
                if (word) sorted = false;
                if (word != m) reversed = false;
                if (!sorted && !reversed) break;
            }
        }
        // 1: already sorted; 2: strictly decreasing, reversed below, then
        // sorted (no equal keys inside, so the reversal is its stable sort)
        sorted = sorted || reversed;
        SR[t] = reversed ? 2 : (sorted ? 1 : 0);
        if (!sorted) unsorted_max = max(unsorted_max, e - s);
        const uint64_t s2 = 2ull * g + s + e;
        Qv[t] = (uint32_t)((s2 << 31) / il);
    }
    unsorted_max = wave_max(unsorted_max);
    if (lane == 0 && unsorted_max) atomicMax(&scal[3], unsorted_max);
    __syncthreads();
    for (uint32_t t = tid; t + 1 < kr; t += NT) {
        const uint32_t p = __clz(Qv[t] ^ Qv[t + 1]) + 1;
        PW[t] = (uint8_t)p;
        pmask |= 1u << (p - 1);
    }
    pmask = wave_or(pmask);
    if (lane == 0 && pmask) atomicOr(&scal[2], pmask);
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
    // node list: boundaries ordered by (power descending, position), one
    // thread per boundary, ranks from wave ballots on the power value
    {
        const uint32_t t = tid;
        const bool valid = t + 1 < kr;
        const uint32_t p = valid ? PW[t] : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const bool bit = (p >> k) & 1u;
            const uint64_t bk = __ballot(bit);
            peers &= bit ? bk : ~bk;
        }
        const uint32_t rw = __popcll(peers & ((1ull << lane) - 1));
        if (lane < 33) wcnt[wave * 33 + lane] = 0;
        __syncthreads();
        if (valid && rw == 0) wcnt[wave * 33 + p] = __popcll(peers);
        __syncthreads();
        if (tid <= 32) {
            uint32_t tot = 0;
            for (int w = 0; w < NW; ++w) tot += wcnt[w * 33 + tid];
            LVc[tid] = tot;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            for (int q = 32; q >= 1; --q) { LVs[q] = acc; acc += LVc[q]; }
        }
        __syncthreads();
        if (valid) {
            uint32_t r = LVs[p] + rw;
            for (int w = 0; w < wave; ++w) r += wcnt[w * 33 + p];
            NL[r] = t;
            BLs[r] = BL[t];
        }
    }
    __syncthreads();

    // 6b. with desc: reverse the strictly decreasing runs in place
    if (desc) {
        for (uint32_t t = 0; t < kr; ++t) {
            if (SR[t] != 2) continue;  // the same for every thread
            const uint32_t s = RS[t], e = RS[t + 1];
            for (uint32_t i = tid; i < (e - s) / 2; i += NT) {
                const uint32_t pa = pxp<LAY>(s + i), pb = pxp<LAY>(e - 1 - i);
                const KT ka = S[pa];
                S[pa] = S[pb];
                S[pb] = ka;
                if (VMODE) {
                    const uint32_t va = SV[pa];
                    SV[pa] = SV[pb];
                    SV[pb] = va;
                }
            }
            __syncthreads();
        }
    }
    // 7./8. forced runs, then the merges of Algorithm 1
    const uint32_t maxf = scal[3], mask = scal[2];
    // 7a. the first bottom-up levels of every forced run: chunks of 2^CWL
    // elements from the run start, sorted in registers (unsorted runs are
    // forced runs, shorter than 64).  Keys without values: 32-element chunks
    // by a sorting network, and in the 32-bit key kernels (plain layout,
    // registers to spare) whole forced runs of up to 64 keys when some
    // forced run is longer than 32 (the narrow kernels, at 128 registers,
    // spilled inside the 64-key network and ran 10% slower).  64-bit keys
    // without values: 16-element chunks by a sorting network (32 of them
    // spilled).  With values: 16-element chunks by the stable transposition
    // network.
    constexpr bool NET = VMODE == 0;  // keys without values: any network gives the stable sort
    constexpr bool NET32 = NET && sizeof(KT) == 4;
    constexpr bool NET64 = NET32 && LAY == 1;
    const uint32_t CWL = NET32 ? ((NET64 && maxf > 32) ? 6u : 5u) : 4u;
    if (maxf > 1) {
        const uint32_t cpr = (maxf + (1u << CWL) - 1) >> CWL;
        for (uint32_t x = tid; x < cpr * kr; x += NT) {
            const uint32_t r = x / cpr, c = x - r * cpr;
            const uint32_t cs = RS[r] + (c << CWL), ce = RS[r + 1];
            if (!SR[r] && cs + 1 < ce) {
                if constexpr (NET64) {
                    if (CWL == 6)
                        chunk_sort_net<64, KT, LAY>(S, cs, min(64u, ce - cs));
                    else
                        chunk_sort_net<32, KT, LAY>(S, cs, min(32u, ce - cs));
                } else if constexpr (NET32) {
                    chunk_sort_net<32, KT, LAY>(S, cs, min(32u, ce - cs));
                } else if constexpr (NET) {
                    chunk_sort_net<16, KT, LAY>(S, cs, min(16u, ce - cs));
                } else {
                    chunk_sort16<KT, VMODE, LAY>(S, SV, cs, min(16u, ce - cs));
                }
            }
        }
        __syncthreads();
    }
    // outputs per thread: the least of KI/2, 3KI/4 and KI that covers the
    // segment, so that at least two thirds of the threads have work
    if (len <= (uint32_t)(NT * (KI / 2)))
        tile_merges<KT, KI / 2, TCAP, VMODE, LAY>(S, SV, len, tid, kr, RS, SR, NL, BLs, BR, LVs, LVc, maxf, mask, CWL);
    else if (len <= (uint32_t)(NT * (3 * KI / 4)))
        tile_merges<KT, 3 * KI / 4, TCAP, VMODE, LAY>(S, SV, len, tid, kr, RS, SR, NL, BLs, BR, LVs, LVc, maxf, mask,
                                                      CWL);
    else
        tile_merges<KT, KI, TCAP, VMODE, LAY>(S, SV, len, tid, kr, RS, SR, NL, BLs, BR, LVs, LVc, maxf, mask, CWL);
}

// One segment of the LDS pass, by all NT threads of the calling workgroup.
// smem: tile_lds_bytes<K, NT, TCAP, VMODE>() bytes of LDS.  NARROW (64-bit
// keys without values): segments whose keys span less than 2^32 run on
// 32-bit offsets.
//   touch: the folded words of this segment's lines, loaded ahead by the
// previous segment (consumed at the start); before this segment's store the
// lines of the next segment nx are loaded ahead when nok is set.
template <typename K, int NT, int TCAP, int VMODE, bool NARROW>
__device__ __forceinline__ void tile_segment(uint8_t* smem, K* __restrict__ keysA, K* __restrict__ keysB,
                                             uint32_t* __restrict__ valsA, uint32_t* __restrict__ valsB,
                                             const Seg sg, const uint32_t* __restrict__ inst_start, bool desc,
                                             uint32_t& touch, const Seg nx, bool nok)
{
    using MT = TileMeta<TCAP>;
    constexpr int NW = NT / 64;
    constexpr int KI = TCAP / NT;
    constexpr uint32_t RC = MT::RC;
    static_assert(TCAP % NT == 0 && KI <= 32, "tile must split evenly, at most 32 outputs per thread");
    static_assert(TCAP / 64 + 1 <= NT, "one thread per bitmap word");
    // every run but an instance's last is at least 32 long, so a tile holds
    // fewer than TCAP / 32 boundaries
    static_assert(TCAP / 32 <= 64 * NW, "one thread per boundary in the power ranking");

    uint8_t* sp = smem;
    K* S = (K*)sp; sp += (sizeof(K) * MT::SP + 15) & ~(size_t)15;
    uint32_t* SV = nullptr;
    if (VMODE) { SV = (uint32_t*)sp; sp += (4 * MT::SP + 15) & ~(size_t)15; }
    uint64_t* bm = (uint64_t*)sp; sp += 8 * MT::BW;
    uint32_t* R1 = (uint32_t*)sp; sp += 4 * 2 * RC;
    uint32_t* R2 = (uint32_t*)sp; sp += 4 * 2 * (RC + 1);
    uint32_t* RS = (uint32_t*)sp; sp += 4 * (RC + 1);
    uint32_t* LVs = (uint32_t*)sp; sp += 4 * 34;
    uint32_t* LVc = (uint32_t*)sp; sp += 4 * 34;
    uint32_t* wcnt = (uint32_t*)sp; sp += 4 * NW * 33;
    uint32_t* scan_lds = (uint32_t*)sp; sp += 4 * (NW + 1);
    uint32_t* scal = (uint32_t*)sp; sp += 4 * 16;  // [0] progressions [1] runs [2] power mask [3] max unsorted run
    uint32_t* BLs = (uint32_t*)sp; sp += 4 * RC;  // BL of NL[i]: node starts in level order
    uint8_t* PW = sp; sp += RC;
    uint8_t* SR = sp;

    // the thread index is made opaque per segment so that the compiler
    // does not keep every unrolled address live across the whole loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t a = sg.start;
    const uint32_t len = sg.end - sg.start;
    if (len == 0) return;
    if (len > TCAP) {
        // a single natural run longer than the tile: already sorted, or
        // (with desc) strictly decreasing, which its first two keys tell;
        // every thread reads them before any thread swaps in place
        const bool rev = desc && keysA[a] > keysA[a + 1];
        __syncthreads();
        if (rev) {
            // reversed: position i takes element len - 1 - i (in place, or
            // into B); values follow, iota values are the source positions
            const uint32_t half = sg.dst == 1 ? len : len / 2;
            for (uint32_t i = tid; i < half; i += NT) {
                const uint32_t j = len - 1 - i;
                const K ki = keysA[a + i], kj = keysA[a + j];
                uint32_t vi = 0, vj = 0;
                if (VMODE == 1) { vi = valsA[a + i]; vj = valsA[a + j]; }
                if (VMODE == 2) { vi = a + i; vj = a + j; }
                if (sg.dst == 1) {
                    keysB[a + i] = kj;
                    if (VMODE) valsB[a + i] = vj;
                } else {
                    keysA[a + i] = kj;
                    keysA[a + j] = ki;
                    if (VMODE) { valsA[a + i] = vj; valsA[a + j] = vi; }
                }
            }
            if (VMODE == 2 && sg.dst != 1 && (len & 1) && tid == 0) valsA[a + len / 2] = a + len / 2;
            return;
        }
        if (sg.dst == 1) {
            for (uint32_t i = tid; i < len; i += NT) {
                keysB[a + i] = keysA[a + i];
                if (VMODE == 1) valsB[a + i] = valsA[a + i];
                if (VMODE == 2) valsB[a + i] = a + i;
            }
        } else if (VMODE == 2) {
            for (uint32_t i = tid; i < len; i += NT) valsA[a + i] = a + i;
        }
        return;
    }
    // the lines loaded ahead have arrived (a dependence only; the value
    // is not used)
    asm volatile("" ::"v"(touch));
    const uint32_t ib = inst_start[sg.inst];
    const uint32_t il = inst_start[sg.inst + 1] - ib;
    const uint32_t ell = minrun_of(il);
    const uint32_t g = a - ib;

    // 1. load; with NARROW, keys whose range in the segment spans less than
    // 2^32 are kept as 32-bit offsets from the segment's minimum (an order-
    // and equality-preserving map, so every step below gives the same result)
    bool narrow = false;
    K kmin = 0;
    if constexpr (NARROW)
        narrow = tile_load_narrow<NT, TCAP, VMODE>(S, SV, keysA, valsA, a, len, tid, wcnt, kmin);
    else
        tile_load<K, NT, TCAP, VMODE>(S, SV, keysA, valsA, a, len, tid);
    if (tid < 16) scal[tid] = 0;
    __syncthreads();

    // 2.-8. on the narrow or the full-width copy; 9. one write to the
    // planned buffer
    const TileLds T{bm, R1, R2, RS, LVs, LVc, wcnt, scan_lds, scal, BLs, PW, SR};
    int tid_st = tid;
    asm volatile("" : "+v"(tid_st));
    if constexpr (NARROW) {
        if (narrow) {
            tile_body<uint32_t, NT, TCAP, VMODE, 2>((uint32_t*)S, SV, T, len, ell, g, il, tid, desc);
            asm volatile("" : "+v"(tid_st));
            touch = tile_touch<K, NT, TCAP, VMODE>(keysA, valsA, nx, nok, tid_st);
            tile_store<uint32_t, K, NT, TCAP, VMODE, 2>((const uint32_t*)S, SV, sg.dst ? keysB : keysA,
                                                    sg.dst ? valsB : valsA, a, len, tid_st, kmin);
            __syncthreads();
            return;
        }
    }
    tile_body<K, NT, TCAP, VMODE, 1>(S, SV, T, len, ell, g, il, tid, desc);
    asm volatile("" : "+v"(tid_st));
    touch = tile_touch<K, NT, TCAP, VMODE>(keysA, valsA, nx, nok, tid_st);
    tile_store<K, K, NT, TCAP, VMODE, 1>(S, SV, sg.dst ? keysB : keysA, sg.dst ? valsB : valsA, a, len, tid_st, K(0));
    __syncthreads();
}


// The LDS pass as one persistent launch: as many workgroups as can be
// resident, each claiming the next segments from an atomic ticket (segments
// differ in length by orders of magnitude in a batch, so a fixed assignment
// would leave workgroups idle).  No workgroup ever waits for another.
// The ticket is broadcast through LDS and made wave-uniform, so the segment
// index lives in scalar registers as a block index would.
// MINW: waves per SIMD that the LDS footprint lets run at once, which
// bounds the registers a wave may use.
template <typename K, int NT, int TCAP, int VMODE, int MINW, bool NARROW>
__global__ __launch_bounds__(NT, MINW) void k_tilesort(K* __restrict__ keysA, K* __restrict__ keysB,
                                                       uint32_t* __restrict__ valsA, uint32_t* __restrict__ valsB,
                                                       const Seg* __restrict__ segs, uint32_t* __restrict__ counters,
                                                       const uint32_t* __restrict__ inst_start,
                                                       uint32_t len_lo, uint32_t len_hi, int ticket, int desc)
{
    // segments of length in (len_lo, len_hi] only, so that two launches of
    // different workgroup sizes can share one segment list (each with its
    // own ticket counter)
    // static LDS of the configuration's size: its address is a compile-time
    // constant, so an element's LDS offset needs no base register added
    // (the ticket word follows the tile's sections).  32-bit keys with values
    // take it as dynamic LDS instead: at their register limit the static
    // form spills more registers.
    constexpr bool STATIC_LDS = tile_lds_static<K, VMODE>();
    __shared__ __align__(16) uint8_t smem_s[STATIC_LDS ? tile_lds_bytes<K, NT, TCAP, VMODE>() + 16 : 16];
    extern __shared__ __align__(16) uint8_t smem_d[];
    uint8_t* smem = STATIC_LDS ? smem_s : smem_d;
    uint32_t& s_next = *(uint32_t*)(smem + tile_lds_bytes<K, NT, TCAP, VMODE>());
    const uint32_t nseg = counters[CNT_NSEG];
    uint32_t touch = 0;
    // a ticket claims sb consecutive segments: every claim is an atomic on
    // one counter shared by the whole grid, so claims are kept to about 16
    // per workgroup (at most 16 segments each) when segments are many
    uint32_t sb = nseg / (gridDim.x * 16u);
    sb = sb < 1u ? 1u : (sb > 16u ? 16u : sb);
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(&counters[ticket], 1u);
        __syncthreads();
        const uint32_t b0 = __builtin_amdgcn_readfirstlane(s_next) * sb;
        __syncthreads();
        if (b0 >= nseg) break;
        const uint32_t b1 = min(b0 + sb, nseg);
        for (uint32_t si = b0; si < b1; ++si) {
            const Seg sg = segs[si];
            const uint32_t len = sg.end - sg.start;
            if (len <= len_lo || len > len_hi) continue;
            // the next segment of the batch, when this launch sorts it in
            // LDS: its lines are loaded ahead
            Seg nx = sg;
            bool nok = false;
            if (si + 1 < b1) {
                nx = segs[si + 1];
                const uint32_t nl = nx.end - nx.start;
                nok = nl > len_lo && nl <= len_hi && nl > 0 && nl <= (uint32_t)TCAP;
            }
            tile_segment<K, NT, TCAP, VMODE, NARROW>(smem, keysA, keysB, valsA, valsB, sg, inst_start, desc != 0,
                                                     touch, nx, nok);
        }
    }
}

// ------------------------------------------------------------- host --
template <typename K, int NT, int TCAP, int VMODE, int MINW, bool NARROW = false>
static hipError_t launch_tilesort(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                                  int wg_per_cu, hipStream_t s, uint32_t len_lo = 0, uint32_t len_hi = 0xffffffffu,
                                  int ticket = CNT_TICKET)
{
    auto kern = k_tilesort<K, NT, TCAP, VMODE, MINW, NARROW>;
    // dynamic LDS bytes at launch: none when the kernel declares its LDS
    constexpr size_t lds = tile_lds_static<K, VMODE>() ? 0 : tile_lds_bytes<K, NT, TCAP, VMODE>() + 16;
    // the LDS limit and the occupancy, once per device
    static bool attr_set[16] = {};
    static int resident[16] = {};
    static int cus[16] = {};
    int dev = 0;
    VMPS_HIP(hipGetDevice(&dev));
    const int d = dev & 15;
    if (!attr_set[d]) {
        if (lds) VMPS_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        VMPS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident[d], (const void*)kern, NT, lds));
        VMPS_HIP(hipDeviceGetAttribute(&cus[d], hipDeviceAttributeMultiprocessorCount, dev));
        attr_set[d] = true;
    }
    int per_cu = resident[d] > 0 ? resident[d] : 1;
    if (wg_per_cu > 0 && wg_per_cu < per_cu) per_cu = wg_per_cu;
    uint64_t grid = (uint64_t)per_cu * (uint64_t)(cus[d] > 0 ? cus[d] : 1);
    if (grid > P.seg_cap) grid = P.seg_cap;
    TraceScope tr(VMPS_TRACE_TILESORT, s);
    kern<<<(unsigned)(grid ? grid : 1), NT, lds, s>>>((K*)keysA, (K*)keysB, valsA, valsB, P.segs, P.counters,
                                                     P.inst_start, len_lo, len_hi, ticket, (int)P.desc);
    return hipGetLastError();
}

uint32_t tilesort_capacity(int key_bits, int has_values)
{
    if (key_bits == 32) return has_values ? 8192u : 16384u;
    return has_values ? 4096u : 8192u;
}

// Tile configurations (threads, elements, values mode, waves per SIMD):
//   u32 keys          512 x 16384: 2 workgroups of 8 waves per CU (LDS)
//   u32 keys + values 512 x  8192: 2 per CU
//   u64 keys          512 x  8192: 2 per CU
//   u64 keys + values 256 x  4096: 3 per CU of 4 waves
size_t tilesort_lds_bytes(int key_bits, int has_values, uint32_t)
{
    if (key_bits == 32)
        return 16 + (has_values ? tile_lds_bytes<uint32_t, 512, 8192, 1>() : tile_lds_bytes<uint32_t, 512, 16384, 0>());
    return 16 + (has_values ? tile_lds_bytes<uint64_t, 256, 4096, 1>() : tile_lds_bytes<uint64_t, 512, 8192, 0>());
}

hipError_t tilesort_enqueue(const Plan& P, void* keysA, void* keysB, uint32_t* valsA, uint32_t* valsB,
                            int key_bits, int vmode, uint32_t narrow, hipStream_t s, int threads)
{
    const int w = tuning_for(key_bits, vmode != 0).tile_wg_per_cu;
    if (key_bits == 32) {
        if (vmode == 0) {
            // the plan's segments are at most P.T long: the kernel's tile
            // must hold them
            if (P.T == 8192) {
                if (threads == 256)
                    return launch_tilesort<uint32_t, 256, 8192, 0, 4>(P, keysA, keysB, valsA, valsB, w, s);
                return launch_tilesort<uint32_t, 512, 8192, 0, 4>(P, keysA, keysB, valsA, valsB, w, s);
            }
            if (P.T != 16384) return hipErrorInvalidValue;
            return launch_tilesort<uint32_t, 512, 16384, 0, 4>(P, keysA, keysB, valsA, valsB, w, s);
        }
        if (vmode == 1) return launch_tilesort<uint32_t, 512, 8192, 1, 4>(P, keysA, keysB, valsA, valsB, w, s);
        return launch_tilesort<uint32_t, 512, 8192, 2, 4>(P, keysA, keysB, valsA, valsB, w, s);
    }
    if (vmode == 0) {
        if (narrow) {
            // segments up to 4096 keys: 256-thread workgroups, four per CU
            VMPS_HIP((launch_tilesort<uint64_t, 256, 4096, 0, 4, true>(P, keysA, keysB, valsA, valsB, w, s, 0, 4096,
                                                                      CNT_TICKET2)));
            return launch_tilesort<uint64_t, 512, 8192, 0, 4, true>(P, keysA, keysB, valsA, valsB, w, s, 4096);
        }
        return launch_tilesort<uint64_t, 512, 8192, 0, 4>(P, keysA, keysB, valsA, valsB, w, s);
    }
    if (vmode == 1) return launch_tilesort<uint64_t, 256, 4096, 1, 3>(P, keysA, keysB, valsA, valsB, w, s);
    return launch_tilesort<uint64_t, 256, 4096, 2, 3>(P, keysA, keysB, valsA, valsB, w, s);
}

}  // namespace vmps
