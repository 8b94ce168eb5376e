// Merge-schedule planner: runs, powers, tree, Pingpong placement.
//
// Input: keys[0,n) split into k independent Powersort instances.  Instances
// no longer than the LDS tile T are left whole to the tile sorter; the rest
// are planned here, entirely on the device (no host round trip):
//
//  1. descent bitmap: bit p set iff keys[p-1] > keys[p] or p starts an
//     instance (boundaries of maximal non-decreasing runs, ExtractRun of
//     Sections 2 and 3);
//  2. long natural runs: runs of at least minrun elements (Section 5);
//  3. run starts: ExtractRun from s returns max(s + l, natural end) capped
//     at the instance end.  Between long natural runs the starts step by l;
//     inside a long run [u,e) the chain jumps to e iff it lands at a point
//     s with e - s >= l.  The state carried along is the last jump target,
//     so each long run acts as a map on phases mod l; the maps are composed
//     block by block and applied with a scan;
//  4. powers (theorem of Section 2) in closed form from the 32-bit
//     expansions Q of the run midpoints;
//  5. tree: the merge of Algorithm 1 at boundary t spans [L,R) where L, R are
//     the nearest boundaries of smaller power.  The nearest smaller boundary
//     on the left is the one whose midpoint interval holds (c-1)/2^p, with
//     c/2^p the witness of t (and (c+1)/2^p on the right), so it is found by
//     a galloping search over Q;
//  6. Pingpong placement (Section 3 as a tree): the root writes the input
//     buffer A and every node writes the buffer opposite its parent; node
//     depths of the merges longer than T come from pointer jumping;
//  7. LDS segments: the pieces between consecutive long merges, each with
//     the buffer its subtree must be written to; and a table of output tiles
//     per level for the HBM merges.
#include "vmps_internal.hpp"

namespace vmps {

// ------------------------------------------------------------------ util --
__device__ inline uint32_t inst_of(const uint32_t* inst_start, uint32_t k, uint32_t p)
{
    // largest i < k with inst_start[i] <= p
    uint32_t lo = 0, hi = k;  // answer in [lo, hi)
    while (hi - lo > 1) {
        uint32_t m = (lo + hi) >> 1;
        if (inst_start[m] <= p) lo = m; else hi = m;
    }
    return lo;
}

__device__ inline uint32_t inst_ell(const uint32_t* inst_start, uint32_t i, uint32_t ovr)
{
    return ovr ? ovr : minrun_of(inst_start[i + 1] - inst_start[i]);
}

// --------------------------------------------------------- instances --
// Offsets are validated; a bad table (not starting at 0, decreasing, or not
// ending at n) turns into one instance [0,n) marked "not to be sorted",
// which the tile sorter leaves untouched.
__global__ __launch_bounds__(1024) void k_inst_prep(const int64_t* __restrict__ off64, uint32_t k, uint32_t n,
                                                   uint32_t big_min, uint32_t* inst_start, uint32_t* inst_big,
                                                   uint32_t* inst_rfinal, uint32_t* inst_run_lo,
                                                   uint32_t* inst_run_hi, uint32_t* counters)
{
    constexpr int U = 8;  // entries per thread per round (i = round + u * 1024 + tid), loads in flight together
    constexpr uint32_t NTH = 1024;
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    // one workgroup validates the whole table
    if (off64) {
        int my_bad = 0;
        for (uint32_t r0 = 0; r0 <= k; r0 += U * NTH) {
            int64_t v[U], w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t i = r0 + u * NTH + threadIdx.x;
                v[u] = i <= k ? off64[i] : 0;
                w[u] = i < k ? off64[i + 1] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t i = r0 + u * NTH + threadIdx.x;
                if (i > k) continue;
                if (v[u] < 0 || v[u] > (int64_t)n) my_bad = 1;
                if (i == 0 && v[u] != 0) my_bad = 1;
                if (i == k && v[u] != (int64_t)n) my_bad = 1;
                if (i < k && w[u] < v[u]) my_bad = 1;
            }
        }
        if (my_bad) bad = 1;
    }
    __syncthreads();
    const bool bd = bad != 0;
    for (uint32_t r0 = 0; r0 <= k; r0 += U * NTH) {
        uint32_t a[U], e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = r0 + u * NTH + threadIdx.x;
            if (bd || !off64) {
                a[u] = i == 0 ? 0u : n;
                e[u] = n;
            } else {
                a[u] = i <= k ? (uint32_t)off64[i] : n;
                e[u] = i < k ? (uint32_t)off64[i + 1] : n;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = r0 + u * NTH + threadIdx.x;
            if (i > k) continue;
            inst_start[i] = a[u];
            if (i < k) {
                inst_big[i] = (!bd && e[u] - a[u] > big_min) ? 1u : 0u;
                inst_rfinal[i] = 0;
                inst_run_lo[i] = NONE;
                inst_run_hi[i] = NONE;
            }
        }
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < CNT_COUNT; ++c) counters[c] = 0;
        counters[CNT_BAD] = bad;
    }
}

// Instance table from offsets the library built itself (valid by
// construction, so no check): one thread per entry over the whole grid.
__global__ void k_inst_prep_trusted(const int64_t* __restrict__ off64, uint32_t k, uint32_t big_min,
                                    uint32_t* inst_start, uint32_t* inst_big, uint32_t* inst_rfinal,
                                    uint32_t* inst_run_lo, uint32_t* inst_run_hi, uint32_t* counters)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0)
        for (int c = 0; c < CNT_COUNT; ++c) counters[c] = 0;
    if (i > k) return;
    const uint32_t a = (uint32_t)off64[i];
    inst_start[i] = a;
    if (i < k) {
        inst_big[i] = (uint32_t)off64[i + 1] - a > big_min ? 1u : 0u;
        inst_rfinal[i] = 0;
        inst_run_lo[i] = NONE;
        inst_run_hi[i] = NONE;
    }
}

// The instance holding the first position of every bitmap tile, and
// whether the tile meets an instance the planner handles (one thread per
// tile, all searches in flight together; a tile crossing more than 64
// instance starts is counted as meeting one, which only costs time).
__global__ void k_tile_inst(const uint32_t* __restrict__ inst_start, const uint32_t* __restrict__ inst_big,
                            uint32_t k, uint32_t n, uint32_t ntile, uint32_t* __restrict__ tile_inst,
                            uint32_t* __restrict__ tile_big)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    const uint64_t p = (uint64_t)t * BITMAP_TILE;
    uint32_t my = 0, big = 0;
    if (p < n) {
        my = inst_of(inst_start, k, (uint32_t)p);
        const uint64_t end = p + BITMAP_TILE < n ? p + BITMAP_TILE : n;
        for (uint32_t i = my; i < k && inst_start[i] < end; ++i) {
            if (inst_big[i] || i - my >= 64) { big = 1; break; }
        }
    }
    tile_inst[t] = my;
    tile_big[t] = big;
}

// ------------------------------------------------------------ bitmap --
template <typename K>
__global__ __launch_bounds__(256) void k_bitmap(const K* __restrict__ keys, uint32_t n,
                                                const uint32_t* __restrict__ inst_start,
                                                const uint32_t* __restrict__ inst_big, uint32_t k,
                                                const uint32_t* __restrict__ tile_inst,
                                                const uint32_t* __restrict__ tile_big,
                                                uint64_t* __restrict__ bitmap,
                                                uint32_t* __restrict__ tile_first,
                                                uint32_t* __restrict__ tile_first0)
{
    constexpr int WPW = (int)(BITMAP_TILE / 64 / 4);  // words per wave
    constexpr uint32_t IW = 255;                     // instances staged in LDS
    __shared__ uint32_t s_first[4], s_first0[4];
    __shared__ uint32_t s_start[IW + 1];
    __shared__ uint32_t s_big[IW];
    const uint32_t tile = blockIdx.x;
    const uint64_t base = (uint64_t)tile * BITMAP_TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (k > 1 && tile_big[tile] == 0) {
        // only instances the tile pass sorts whole (or positions past n):
        // every position is a boundary
        if (lane < WPW) bitmap[(uint64_t)tile * 64 + wave + 4 * lane] = ~0ull;
        if (threadIdx.x == 0) tile_first[tile] = (uint32_t)base;
        if (threadIdx.x == 0 && tile_first0) tile_first0[tile] = NONE;
        return;
    }
    // instances overlapping the tile, from the one holding its first position
    const uint32_t my0 = (k > 1 && base < n) ? tile_inst[tile] : 0u;
    if (k > 1) {
        const uint32_t i = my0 + threadIdx.x;
        if (threadIdx.x <= IW) s_start[threadIdx.x] = i <= k ? inst_start[i] : n;
        if (threadIdx.x < IW) s_big[threadIdx.x] = i < k ? inst_big[i] : 0u;
        __syncthreads();
    }
    // the window holds every instance that overlaps the tile unless the tile
    // crosses more than IW instance starts (then the table is read directly)
    const bool window = k > 1 && (my0 + IW >= k || s_start[IW] >= base + BITMAP_TILE);
    uint32_t my = my0;
    // load[j]: the position lies in an instance the planner handles;
    // cmp[j]: and it is not that instance's first element
    bool load[WPW], cmp[WPW];
#pragma unroll
    for (int j = 0; j < WPW; ++j) {
        const uint64_t p = base + (uint64_t)(wave + 4 * j) * 64 + lane;
        load[j] = false;
        cmp[j] = false;
        if (p < n) {
            if (window) {
                while (my + 1 < k && s_start[my + 1 - my0] <= p) ++my;
                load[j] = s_big[my - my0] != 0;
                cmp[j] = load[j] && p != s_start[my - my0];
            } else if (k > 1) {
                while (my + 1 < k && inst_start[my + 1] <= p) ++my;
                load[j] = inst_big[my] != 0;
                cmp[j] = load[j] && p != inst_start[my];
            } else {
                load[j] = inst_big[0] != 0;
                cmp[j] = load[j] && p != 0;
            }
        }
    }
    // every key once; the predecessor comes from the next lower lane (lane 0
    // loads its own)
    K y[WPW], x0[WPW];
#pragma unroll
    for (int j = 0; j < WPW; ++j) {
        const uint64_t p = base + (uint64_t)(wave + 4 * j) * 64 + lane;
        y[j] = load[j] ? keys[p] : K(0);
        x0[j] = (lane == 0 && cmp[j]) ? keys[p - 1] : K(0);
    }
    uint32_t first = NONE, first0 = NONE;
#pragma unroll
    for (int j = 0; j < WPW; ++j) {
        const int w = wave + 4 * j;
        K x = (K)__shfl_up((unsigned long long)y[j], 1, 64);
        if (lane == 0) x = x0[j];
        // positions past n and instance heads are boundaries; so is every
        // position of an instance the tile pass sorts whole
        const bool bit = cmp[j] ? (x > y[j]) : true;
        const uint64_t word = __ballot(bit);
        if (lane == 0) bitmap[(uint64_t)tile * 64 + w] = word;
        if (word && first == NONE) first = (uint32_t)(base + (uint64_t)w * 64 + ffs64(word));
        // positions that end a strictly decreasing run: compared, not a descent
        const uint64_t word0 = __ballot(cmp[j] && !(x > y[j]));
        if (word0 && first0 == NONE) first0 = (uint32_t)(base + (uint64_t)w * 64 + ffs64(word0));
    }
    if (lane == 0) { s_first[wave] = first; s_first0[wave] = first0; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = s_first[0], m0 = s_first0[0];
        for (int w = 1; w < 4; ++w) { m = min(m, s_first[w]); m0 = min(m0, s_first0[w]); }
        tile_first[tile] = m;
        if (tile_first0) tile_first0[tile] = m0;
    }
}

// tile_next[t] = first set bit in tiles after t (one workgroup)
__global__ __launch_bounds__(1024) void k_suffix_min(const uint32_t* __restrict__ first,
                                                     uint32_t* __restrict__ next, uint32_t ntile)
{
    // rounds of R = 1024 * U entries from the right; the round passes through
    // LDS so that global reads and writes are coalesced, thread t owning the
    // U consecutive entries [U t, U t + U) of the round
    constexpr uint32_t U = 16, R = 1024 * U;
    __shared__ uint32_t buf[R];
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    uint32_t carry = NONE;  // minimum of everything right of the round
    const uint32_t rounds = (ntile + R - 1) / R;
    for (uint32_t rr = rounds; rr-- > 0;) {
        const uint32_t r0 = rr * R;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = r0 + u * 1024 + t;
            buf[u * 1024 + t] = i < ntile ? first[i] : NONE;
        }
        __syncthreads();
        uint32_t m = NONE;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) m = min(m, buf[U * t + u]);
        part[t] = m;
        __syncthreads();
        for (uint32_t d = 1; d < 1024; d <<= 1) {
            const uint32_t o = t + d < 1024 ? part[t + d] : NONE;
            __syncthreads();
            part[t] = min(part[t], o);
            __syncthreads();
        }
        uint32_t run = min(carry, t + 1 < 1024 ? part[t + 1] : NONE);
        const uint32_t all = part[0];
#pragma unroll
        for (int u = (int)U - 1; u >= 0; --u) {
            const uint32_t v = buf[U * t + u];
            buf[U * t + u] = run;
            run = min(run, v);
        }
        __syncthreads();
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = r0 + u * 1024 + t;
            if (i < ntile) next[i] = buf[u * 1024 + t];
        }
        carry = min(carry, all);
        __syncthreads();
    }
}

// Run-start candidates of a word: bits of `ends` (positions that end a run of
// the kind) whose next `span` positions hold no such end; the window past
// the word reads as "no end", so the last starts of a word stay candidates.
__device__ inline uint64_t run_start_candidates(uint64_t starts, uint64_t ends, uint32_t span)
{
    uint64_t o = span ? ends >> 1 : 0ull;
    uint32_t covered = 1;
    while (span && 2 * covered <= span) {
        o |= o >> covered;
        covered *= 2;
    }
    if (covered < span) o |= o >> (span - covered);
    return starts & ~o;
}

// Long natural runs: count (EMIT=false) or write (EMIT=true).  One wave
// per bitmap tile, one lane per 64-bit word.  Maximal non-decreasing runs
// start at a set bit (a descent, an instance head) and end at the next one.
// With tile_next0 (descending runs, one instance): maximal strictly
// decreasing runs start at a clear bit or at position 0, hold only set bits
// after their start and end at the next clear bit (or n); both kinds go to
// one list in position order.
template <bool EMIT>
__global__ __launch_bounds__(64) void k_long_runs(const uint64_t* __restrict__ bitmap, uint32_t n,
                                                  const uint32_t* __restrict__ tile_next,
                                                  const uint32_t* __restrict__ tile_next0,
                                                  const uint32_t* __restrict__ inst_start,
                                                  const uint32_t* __restrict__ inst_big, uint32_t k,
                                                  uint32_t ell_ovr, uint32_t cand_min, uint32_t lr_cap,
                                                  uint32_t* __restrict__ tile_cnt,
                                                  const uint32_t* __restrict__ tile_off,
                                                  uint32_t* __restrict__ lr_u, uint32_t* __restrict__ lr_e,
                                                  uint32_t* __restrict__ lr_inst)
{
    const uint32_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    const uint64_t w = (uint64_t)tile * 64 + lane;
    const uint64_t word = bitmap[w];
    const uint64_t p0 = w * 64;
    // a word holds at most 4 starts of increasing runs of length >= 16, and
    // with descending runs at most 4 more
    constexpr int CAP = 8;
    uint32_t cnt = 0;
    uint32_t ru[CAP] = {}, re[CAP] = {}, ri[CAP] = {};
    // a run of length >= cand_min starting at bit b has no end in
    // (b, b + cand_min)
    const uint32_t span = (cand_min < 33u ? (cand_min > 0u ? cand_min : 1u) : 33u) - 1u;
    for (int kind = 0; kind < (tile_next0 ? 2 : 1); ++kind) {
        const uint64_t ends = kind == 0 ? word : ~word;
        const uint64_t starts = kind == 0 ? word : (~word | (p0 == 0 ? 1ull : 0ull));
        uint64_t bits = run_start_candidates(starts, ends, span);
        while (bits) {
            const int b = ffs64(bits);
            bits &= bits - 1;
            const uint64_t u = p0 + b;
            if (u >= n) break;
            const uint64_t above = (b == 63) ? 0ull : ((ends >> (b + 1)) << (b + 1));
            uint64_t next;
            if (above) {
                next = p0 + ffs64(above);
            } else {
                next = NONE;
                for (uint64_t ww = w + 1; ww < (uint64_t)(tile + 1) * 64; ++ww) {
                    const uint64_t x = kind == 0 ? bitmap[ww] : ~bitmap[ww];
                    if (x) { next = ww * 64 + ffs64(x); break; }
                }
                if (next == NONE) next = kind == 0 ? tile_next[tile] : tile_next0[tile];
            }
            if (next > n) next = n;
            if (next - u < cand_min) continue;
            const uint32_t inst = k > 1 ? inst_of(inst_start, k, (uint32_t)u) : 0;
            if (!inst_big[inst]) continue;
            if (next - u < inst_ell(inst_start, inst, ell_ovr)) continue;
            if (cnt < CAP) {
                // keep the lane's runs in position order
                uint32_t at = cnt;
                while (at > 0 && ru[at - 1] > (uint32_t)u) {
                    ru[at] = ru[at - 1]; re[at] = re[at - 1]; ri[at] = ri[at - 1];
                    --at;
                }
                ru[at] = (uint32_t)u; re[at] = (uint32_t)next; ri[at] = inst;
            }
            ++cnt;
        }
    }
    if (cnt > CAP) cnt = CAP;
    const uint32_t inc = wave_incl_scan(cnt);
    if (!EMIT) {
        if (lane == 63) tile_cnt[tile] = inc;
    } else {
        uint32_t o = tile_off[tile] + inc - cnt;
        for (uint32_t c = 0; c < cnt && o + c < lr_cap; ++c) {
            lr_u[o + c] = ru[c];
            lr_e[o + c] = re[c];
            lr_inst[o + c] = ri[c];
        }
    }
}

// ------------------------------------------------------------- chain --
// x mod d and x / d for 32-bit x and a divisor d >= 1 from one 64-bit
// constant c = floor((2^64 - 1) / d) + 1, after Lemire, Kaser and Kurz,
// "Faster remainder by direct computation" (2019): x mod d is the high
// word of ((c x) mod 2^64) d, x / d the high word of c x.  c wraps to 0 for
// d = 1 (remainder 0, quotient x).  The chain walks below are sequential
// per lane, and a division by a variable costs several times more.
struct DivBy {
    uint64_t c;
    uint32_t d;
};
__device__ inline DivBy div_by(uint32_t d) { return DivBy{~0ull / d + 1, d}; }
__device__ inline uint32_t mod_by(uint32_t x, const DivBy& v) { return (uint32_t)__umul64hi(v.c * x, v.d); }
__device__ inline uint32_t quot_by(uint32_t x, const DivBy& v)
{
    return v.d == 1 ? x : (uint32_t)__umul64hi(v.c, x);
}

// Smallest x >= u with x == ph (mod l), ph < l, written from u's residue.
__device__ inline uint32_t chain_land(uint32_t u, uint32_t ph, const DivBy& l)
{
    uint32_t t = ph + l.d - mod_by(u, l);  // in [1, 2l - 1]
    if (t >= l.d) t -= l.d;
    return u + t;
}

// A block of long runs is walked as CHAIN_SUBS sub-blocks of CHAIN_SUB runs
// in parallel (one wave each, lane phi following the chain that enters the
// sub-block at phase phi), and the sub-block maps are then composed in
// order; the walks stay short although the blocks are long.
constexpr uint32_t CHAIN_SUBS = 16;
constexpr uint32_t CHAIN_SUB = CHAIN_BLOCK / CHAIN_SUBS;
constexpr uint32_t CHAIN_NT = 64 * CHAIN_SUBS;

struct ChainLds {
    uint32_t u[CHAIN_BLOCK], e[CHAIN_BLOCK], inst[CHAIN_BLOCK];
    uint32_t val[CHAIN_SUBS][64];
    uint64_t known[CHAIN_SUBS];
    uint32_t rin[CHAIN_SUBS];
};

// Instance of long run j (of block [j0, j1) staged in S), NONE before 0.
__device__ inline uint32_t chain_inst_at(const ChainLds& S, const uint32_t* __restrict__ lr_inst, uint32_t j0,
                                         uint32_t j)
{
    if (j + 1 == 0) return NONE;
    return j >= j0 ? S.inst[j - j0] : lr_inst[j];
}

// Stages the block's runs and computes the map of every sub-block: after
// the walk, lane phi of wave w holds the last jump target of the chain that
// enters sub-block w at phase phi, or 0 with its known bit clear (no jump
// and no instance change: the chain passes unchanged).
__device__ void chain_sub_maps(ChainLds& S, const uint32_t* __restrict__ lr_u, const uint32_t* __restrict__ lr_e,
                               const uint32_t* __restrict__ lr_inst, const uint32_t* __restrict__ inst_start,
                               uint32_t ell_ovr, uint32_t j0, uint32_t j1)
{
    const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (uint32_t j = j0 + tid; j < j1; j += CHAIN_NT) {
        S.u[j - j0] = lr_u[j]; S.e[j - j0] = lr_e[j]; S.inst[j - j0] = lr_inst[j];
    }
    __syncthreads();
    const uint32_t s0 = j0 + w * CHAIN_SUB, s1 = min(j1, s0 + CHAIN_SUB);
    bool known = false;
    uint32_t r = 0;
    if (s0 < j1) {
        uint32_t prev = chain_inst_at(S, lr_inst, j0, s0 - 1), ib = 0;
        DivBy ell = div_by(1);
        if (prev != NONE) { ell = div_by(inst_ell(inst_start, prev, ell_ovr)); ib = inst_start[prev]; }
        for (uint32_t j = s0; j < s1; ++j) {
            const uint32_t inst = S.inst[j - j0];
            if (inst != prev) {
                known = true; r = 0; prev = inst;
                ell = div_by(inst_ell(inst_start, inst, ell_ovr));
                ib = inst_start[inst];
            }
            const uint32_t u = S.u[j - j0] - ib, e = S.e[j - j0] - ib;
            const uint32_t ph = mod_by(known ? r : lane, ell);
            const uint32_t sf = chain_land(u, ph, ell);
            if (e - sf >= ell.d) { known = true; r = e; }
        }
    }
    S.val[w][lane] = r;
    const uint64_t m = __ballot(known);
    if (lane == 0) S.known[w] = m;
    __syncthreads();
}

// Map of a block of long runs: lane phi follows the chain entering the
// block at phase phi; afterwards it holds the last jump target (known) or
// is still the identity.
__global__ __launch_bounds__(CHAIN_NT) void k_chain_blocks(const uint32_t* __restrict__ lr_u,
                                                           const uint32_t* __restrict__ lr_e,
                                                           const uint32_t* __restrict__ lr_inst,
                                                           const uint32_t* __restrict__ inst_start,
                                                           uint32_t ell_ovr, const uint32_t* counters,
                                                           uint32_t* __restrict__ chain_val,
                                                           uint64_t* __restrict__ chain_known)
{
    __shared__ ChainLds S;
    const uint32_t nl = counters[CNT_NLONG];
    // a capped grid loops over the blocks (most of the capacity is unused)
    for (uint32_t b = blockIdx.x; (uint64_t)b * CHAIN_BLOCK < nl; b += gridDim.x) {
        const uint32_t j0 = b * CHAIN_BLOCK;
        const uint32_t j1 = min(nl, j0 + CHAIN_BLOCK);
        chain_sub_maps(S, lr_u, lr_e, lr_inst, inst_start, ell_ovr, j0, j1);
        if (threadIdx.x < 64) {
            // compose the sub-block maps: lane phi enters the block at phase phi
            const uint32_t lane = threadIdx.x;
            bool known = false;
            uint32_t r = 0;
            for (uint32_t v = 0; v < CHAIN_SUBS; ++v) {
                const uint32_t t0 = j0 + v * CHAIN_SUB;
                if (t0 >= j1) break;
                // known only after a first sub-block (v > 0): t0 - 1 is in the block
                const uint32_t ph = known ? r % inst_ell(inst_start, S.inst[t0 - 1 - j0], ell_ovr) : lane;
                if ((S.known[v] >> ph) & 1ull) { known = true; r = S.val[v][ph]; }
            }
            chain_val[(uint64_t)b * 64 + lane] = r;
            const uint64_t m = __ballot(known);
            if (lane == 0) chain_known[b] = m;
        }
        __syncthreads();  // LDS is staged again for the next block
    }
}

// Sequential composition over blocks: incoming chain state of every block.
// The block maps, instances and divisors are staged in LDS by the
// workgroup, SCAN_CHUNK blocks at a time, so that the sequential walk of
// thread 0 reads only LDS.
constexpr uint32_t SCAN_CHUNK = 64;

__global__ __launch_bounds__(256) void k_chain_scan(const uint32_t* __restrict__ lr_inst,
                                                    const uint32_t* __restrict__ inst_start, uint32_t ell_ovr,
                                                    const uint32_t* counters, const uint32_t* __restrict__ chain_val,
                                                    const uint64_t* __restrict__ chain_known,
                                                    uint32_t* __restrict__ chain_rin)
{
    __shared__ uint32_t sval[SCAN_CHUNK][64];
    __shared__ uint64_t sknown[SCAN_CHUNK];
    __shared__ uint32_t sfirst[SCAN_CHUNK], slast[SCAN_CHUNK];
    __shared__ DivBy sell[SCAN_CHUNK];
    const uint32_t nl = counters[CNT_NLONG];
    const uint32_t nb = (uint32_t)ceil_div(nl, CHAIN_BLOCK);
    uint32_t r = 0, prev_last = NONE;  // thread 0's chain state
    for (uint32_t c0 = 0; c0 < nb; c0 += SCAN_CHUNK) {
        const uint32_t cn = min(SCAN_CHUNK, nb - c0);
        for (uint32_t x = threadIdx.x; x < cn * 64; x += blockDim.x)
            sval[x >> 6][x & 63] = chain_val[(uint64_t)(c0 + (x >> 6)) * 64 + (x & 63)];
        for (uint32_t x = threadIdx.x; x < cn; x += blockDim.x) {
            const uint32_t j0 = (c0 + x) * CHAIN_BLOCK;
            const uint32_t first = lr_inst[j0];
            sknown[x] = chain_known[c0 + x];
            sfirst[x] = first;
            slast[x] = lr_inst[min(nl, j0 + CHAIN_BLOCK) - 1];
            sell[x] = div_by(inst_ell(inst_start, first, ell_ovr));
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (uint32_t x = 0; x < cn; ++x) {
                if (sfirst[x] != prev_last) r = 0;
                chain_rin[c0 + x] = r;
                const uint32_t ph = mod_by(r, sell[x]);
                if ((sknown[x] >> ph) & 1ull) r = sval[x][ph];
                prev_last = slast[x];
            }
        }
        __syncthreads();
    }
}

// One block of k_chain_apply, by the whole workgroup.
__device__ void chain_apply_block(ChainLds& S, const uint32_t* __restrict__ lr_u, const uint32_t* __restrict__ lr_e,
                                  const uint32_t* __restrict__ lr_inst, const uint32_t* __restrict__ inst_start,
                                  uint32_t ell_ovr, uint32_t nl, uint32_t b, uint32_t j0, uint32_t j1,
                                  const uint32_t* __restrict__ chain_rin, uint32_t* __restrict__ lr_cnt,
                                  uint32_t* __restrict__ lr_base, uint32_t* __restrict__ inst_rfinal)
{
    chain_sub_maps(S, lr_u, lr_e, lr_inst, inst_start, ell_ovr, j0, j1);
    if (threadIdx.x == 0) {
        // state entering every sub-block (before its first run's instance
        // check, as in one sequential walk)
        uint32_t r = chain_rin[b];
        for (uint32_t v = 0; v < CHAIN_SUBS; ++v) {
            const uint32_t t0 = j0 + v * CHAIN_SUB;
            if (t0 >= j1) break;
            S.rin[v] = r;
            const uint32_t pi = chain_inst_at(S, lr_inst, j0, t0 - 1);
            // a sub-block that opens an instance restarts from 0: its map is
            // known at every phase
            const uint32_t ph = (pi == NONE || S.inst[t0 - j0] != pi) ? 0u : r % inst_ell(inst_start, pi, ell_ovr);
            if ((S.known[v] >> ph) & 1ull) r = S.val[v][ph];
        }
    }
    __syncthreads();
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t s0 = j0 + w * CHAIN_SUB;
    if ((threadIdx.x & 63) != 0 || s0 >= j1) return;
    const uint32_t s1 = min(j1, s0 + CHAIN_SUB);
    uint32_t prev = chain_inst_at(S, lr_inst, j0, s0 - 1);
    uint32_t r = S.rin[w], ib = 0;
    DivBy ell = div_by(1);
    if (prev != NONE) { ell = div_by(inst_ell(inst_start, prev, ell_ovr)); ib = inst_start[prev]; }
    const uint32_t next_inst = s1 < j1 ? S.inst[s1 - j0] : (j1 < nl ? lr_inst[j1] : NONE);
    for (uint32_t j = s0; j < s1; ++j) {
        const uint32_t inst = S.inst[j - j0];
        if (inst != prev) {
            r = 0; prev = inst;
            ell = div_by(inst_ell(inst_start, inst, ell_ovr));
            ib = inst_start[inst];
        }
        const uint32_t u = S.u[j - j0] - ib, e = S.e[j - j0] - ib;
        const uint32_t sf = chain_land(u, mod_by(r, ell), ell);
        if (e - sf >= ell.d) {
            lr_cnt[j] = quot_by(sf - r, ell) + 1;
            lr_base[j] = r;
            r = e;
        } else {
            lr_cnt[j] = 0;
            lr_base[j] = 0;
        }
        const uint32_t nxt = (j + 1 < s1) ? S.inst[j + 1 - j0] : next_inst;
        if (nxt != inst) inst_rfinal[inst] = r;
    }
}

// Apply: walk each block with its real incoming state, recording for every
// long run where the chain jumps (run count of the progression it closes).
// The sub-block maps give each sub-block's incoming state, and the
// sub-blocks are then walked in parallel, one lane each.
__global__ __launch_bounds__(CHAIN_NT) void k_chain_apply(const uint32_t* __restrict__ lr_u,
                                                          const uint32_t* __restrict__ lr_e,
                                                          const uint32_t* __restrict__ lr_inst,
                                                          const uint32_t* __restrict__ inst_start,
                                                          uint32_t ell_ovr, const uint32_t* counters,
                                                          const uint32_t* __restrict__ chain_rin,
                                                          uint32_t* __restrict__ lr_cnt,
                                                          uint32_t* __restrict__ lr_base,
                                                          uint32_t* __restrict__ inst_rfinal)
{
    __shared__ ChainLds S;
    const uint32_t nl = counters[CNT_NLONG];
    // a capped grid loops over the blocks (most of the capacity is unused)
    for (uint32_t b = blockIdx.x; (uint64_t)b * CHAIN_BLOCK < nl; b += gridDim.x) {
        const uint32_t j0 = b * CHAIN_BLOCK;
        const uint32_t j1 = min(nl, j0 + CHAIN_BLOCK);
        chain_apply_block(S, lr_u, lr_e, lr_inst, inst_start, ell_ovr, nl, b, j0, j1, chain_rin, lr_cnt, lr_base,
                          inst_rfinal);
        __syncthreads();  // LDS is staged again for the next block
    }
}

// ----------------------------------------------------------- entries --
// Progressions of run starts: one per jumping long run (closing at it) and
// one tail per planned instance, laid out in position order.
__global__ void k_entries_lr(const uint32_t* __restrict__ lr_inst, const uint32_t* __restrict__ lr_cnt,
                             const uint32_t* __restrict__ lr_base,
                             const uint32_t* __restrict__ inst_bigrank, const uint32_t* counters,
                             uint32_t* __restrict__ ent_cnt, uint32_t* __restrict__ ent_base,
                             uint32_t* __restrict__ ent_inst)
{
    const uint32_t nl = counters[CNT_NLONG];
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nl; j += gridDim.x * blockDim.x) {
        const uint32_t inst = lr_inst[j];
        const uint32_t idx = j + inst_bigrank[inst];
        ent_cnt[idx] = lr_cnt[j];
        ent_base[idx] = lr_base[j];
        ent_inst[idx] = inst;
    }
}

__global__ void k_entries_tail(const uint32_t* __restrict__ lr_inst, const uint32_t* __restrict__ inst_start,
                               const uint32_t* __restrict__ inst_big,
                               const uint32_t* __restrict__ inst_bigrank,
                               const uint32_t* __restrict__ inst_rfinal, uint32_t k, uint32_t ell_ovr,
                               uint32_t* counters, uint32_t* __restrict__ ent_cnt,
                               uint32_t* __restrict__ ent_base, uint32_t* __restrict__ ent_inst)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nl = counters[CNT_NLONG];
    if (i == 0) counters[CNT_NENT] = nl + counters[CNT_NBIG];
    if (i >= k || !inst_big[i]) return;
    // number of long runs in instances <= i
    uint32_t lo = 0, hi = nl;
    while (lo < hi) {
        uint32_t m = (lo + hi) >> 1;
        if (lr_inst[m] <= i) lo = m + 1; else hi = m;
    }
    const uint32_t idx = lo + inst_bigrank[i];
    const uint32_t len = inst_start[i + 1] - inst_start[i];
    const uint32_t ell = inst_ell(inst_start, i, ell_ovr);
    const uint32_t rf = inst_rfinal[i];
    ent_cnt[idx] = rf < len ? (uint32_t)ceil_div(len - rf, ell) : 0u;
    ent_base[idx] = rf;
    ent_inst[idx] = i;
}

// -------------------------------------------------------------- runs --
__global__ void k_runs_emit(const uint32_t* __restrict__ ent_off, const uint32_t* __restrict__ ent_base,
                            const uint32_t* __restrict__ ent_inst, const uint32_t* __restrict__ inst_start,
                            uint32_t n, uint32_t ell_ovr, const uint32_t* counters,
                            uint32_t* __restrict__ run_start, uint32_t* __restrict__ run_inst)
{
    const uint32_t nr = counters[CNT_NRUNS], ne = counters[CNT_NENT];
    if (blockIdx.x == 0 && threadIdx.x == 0) run_start[nr] = n;
    if (ne == 0) return;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
        // largest entry e with ent_off[e] <= t (it has a non-zero count)
        uint32_t lo = 0, hi = ne;
        while (hi - lo > 1) {
            uint32_t m = (lo + hi) >> 1;
            if (ent_off[m] <= t) lo = m; else hi = m;
        }
        const uint32_t inst = ent_inst[lo];
        const uint32_t ell = inst_ell(inst_start, inst, ell_ovr);
        run_start[t] = inst_start[inst] + ent_base[lo] + (t - ent_off[lo]) * ell;
        run_inst[t] = inst;
    }
}

// Q[t] = floor(2^31 (s_t + e_t) / len): the first 32 bits of the binary
// expansion of the run midpoint over the instance length.
__global__ void k_run_q(const uint32_t* __restrict__ run_start, const uint32_t* __restrict__ run_inst,
                        const uint32_t* __restrict__ inst_start, const uint32_t* counters,
                        uint32_t* __restrict__ run_q, uint32_t* __restrict__ inst_run_lo,
                        uint32_t* __restrict__ inst_run_hi)
{
    const uint32_t nr = counters[CNT_NRUNS];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
        const uint32_t inst = run_inst[t];
        const uint32_t ib = inst_start[inst], il = inst_start[inst + 1] - ib;
        const bool last = (t + 1 == nr) || run_inst[t + 1] != inst;
        const uint64_t s = run_start[t] - ib;
        const uint64_t e = last ? il : run_start[t + 1] - ib;
        run_q[t] = (uint32_t)(((s + e) << 31) / il);
        if (t == 0 || run_inst[t - 1] != inst) inst_run_lo[inst] = t;
        if (last) inst_run_hi[inst] = t;
    }
}

// Power, witness, and the node [L,R) of every boundary.
__global__ void k_boundaries(const uint32_t* __restrict__ run_start, const uint32_t* __restrict__ run_inst,
                             const uint32_t* __restrict__ run_q, const uint32_t* __restrict__ inst_start,
                             const uint32_t* __restrict__ inst_run_lo,
                             const uint32_t* __restrict__ inst_run_hi, uint32_t T,
                             uint32_t* counters, uint8_t* __restrict__ power,
                             uint32_t* __restrict__ bnd_l, uint32_t* __restrict__ bnd_r,
                             uint32_t* __restrict__ bnd_lpos, uint32_t* __restrict__ bnd_rpos,
                             uint32_t* __restrict__ hbm_flag, unsigned long long* stats)
{
    const uint32_t nr = counters[CNT_NRUNS];
    uint64_t cost = 0, cost_hbm = 0;
    uint32_t pmax = 0;
    // grid-stride over the boundaries with a capped grid, so that the merge
    // cost sums end in one atomic per workgroup
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
        uint32_t p = 0;
        const uint32_t inst = run_inst[t];
        const uint32_t lo = inst_run_lo[inst], hi = inst_run_hi[inst];
        if (t == hi || lo == NONE || hi == NONE || t < lo || t > hi) {
            power[t] = 0;
            hbm_flag[t] = 0;
            bnd_l[t] = NONE; bnd_r[t] = NONE;
        } else {
            const uint32_t ib = inst_start[inst], ie = inst_start[inst + 1];
            const uint32_t qt = run_q[t], qn = run_q[t + 1];
            p = __clz(qt ^ qn) + 1;
            const uint32_t sh = 32 - p;
            const uint64_t c = (uint64_t)qn >> sh;
            const uint64_t V = (c - 1) << sh, W = (c + 1) << sh;
            // left: largest u in [lo, t) with Q[u] < V
            int64_t b = t, a, d = 1;
            for (;;) {
                a = (int64_t)b - d;
                if (a < (int64_t)lo) { a = (int64_t)lo - 1; break; }
                if (run_q[a] < V) break;
                b = a; d <<= 1;
            }
            while (b - a > 1) {
                int64_t m = (a + b) >> 1;
                if (run_q[m] < V) a = m; else b = m;
            }
            const uint32_t uL = a < (int64_t)lo ? NONE : (uint32_t)a;
            // right: largest u in (t, hi] with Q[u] < W
            a = (int64_t)t + 1; d = 1;
            for (;;) {
                b = a + d;
                if (b > (int64_t)hi) { b = (int64_t)hi + 1; break; }
                if (run_q[b] >= W) break;
                a = b; d <<= 1;
            }
            while (b - a > 1) {
                int64_t m = (a + b) >> 1;
                if (run_q[m] < W) a = m; else b = m;
            }
            const uint32_t uR = (a == (int64_t)hi) ? NONE : (uint32_t)a;
            const uint32_t L = uL == NONE ? ib : run_start[uL + 1];
            const uint32_t R = uR == NONE ? ie : run_start[uR + 1];
            power[t] = (uint8_t)p;
            bnd_l[t] = uL; bnd_r[t] = uR;
            bnd_lpos[t] = L; bnd_rpos[t] = R;
            hbm_flag[t] = (R - L > T) ? 1u : 0u;
            cost += R - L;
            if (R - L > T) cost_hbm += R - L;
        }
        pmax = max(pmax, p);
    }
    // wave sums, then workgroup sums, then one atomic per workgroup
    for (int d = 32; d >= 1; d >>= 1) {
        cost += __shfl_down(cost, d, 64);
        cost_hbm += __shfl_down(cost_hbm, d, 64);
        pmax = max(pmax, (uint32_t)__shfl_down((int)pmax, d, 64));
    }
    __shared__ unsigned long long s_cost[4], s_hbm[4];
    __shared__ uint32_t s_p[4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { s_cost[wave] = cost; s_hbm[wave] = cost_hbm; s_p[wave] = pmax; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long c = 0, ch = 0;
        uint32_t pm = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { c += s_cost[w]; ch += s_hbm[w]; pm = max(pm, s_p[w]); }
        if (c) atomicAdd(&stats[0], c);
        if (ch) atomicAdd(&stats[1], ch);
        if (pm) atomicMax(&counters[CNT_MAXPOW], pm);
    }
}

// --------------------------------------------------------- HBM nodes --
__global__ void k_hbm_emit(const uint32_t* __restrict__ hbm_flag, const uint32_t* __restrict__ hbm_rank,
                           const uint32_t* counters, uint32_t h_cap, uint32_t* __restrict__ hbm_list,
                           uint32_t* __restrict__ hbm_idx)
{
    const uint32_t nr = counters[CNT_NRUNS];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
        if (hbm_flag[t]) {
            const uint32_t r = hbm_rank[t];
            if (r < h_cap) hbm_list[r] = t;  // more only from an inconsistent plan
            hbm_idx[t] = r;
        }
    }
}

// parent of an HBM node: the nearer-in-tree of its two smaller-power
// neighbours, i.e. the one with the larger power.
__global__ void k_depth_init(const uint32_t* __restrict__ hbm_list, const uint32_t* __restrict__ hbm_idx,
                             const uint32_t* __restrict__ bnd_l, const uint32_t* __restrict__ bnd_r,
                             const uint8_t* __restrict__ power, const uint32_t* __restrict__ hbm_flag,
                             const uint32_t* counters, uint32_t* __restrict__ par, uint32_t* __restrict__ val)
{
    const uint32_t h = counters[CNT_NHBM];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < h; q += gridDim.x * blockDim.x) {
        const uint32_t t = hbm_list[q];
        const uint32_t l = bnd_l[t], r = bnd_r[t];
        uint32_t parent;
        if (l == NONE) parent = r;
        else if (r == NONE) parent = l;
        else parent = power[l] > power[r] ? l : r;
        const bool ok = parent != NONE && hbm_flag[parent] && hbm_idx[parent] < h;
        par[q] = ok ? hbm_idx[parent] : q;
        val[q] = ok ? 1u : 0u;
    }
}

__global__ void k_depth_jump(const uint32_t* __restrict__ par_in, const uint32_t* __restrict__ val_in,
                             const uint32_t* counters, uint32_t* __restrict__ par_out,
                             uint32_t* __restrict__ val_out)
{
    const uint32_t h = counters[CNT_NHBM];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < h; q += gridDim.x * blockDim.x) {
        const uint32_t p = par_in[q];
        val_out[q] = val_in[q] + val_in[p];
        par_out[q] = par_in[p];
    }
}

// ------------------------------------------------------ LDS segments --
__device__ inline uint32_t seg_dst(uint32_t depth_parent) { return (depth_parent + 1) & 1u; }

__global__ void k_segs_hbm(const uint32_t* __restrict__ hbm_list, const uint32_t* __restrict__ run_start,
                           const uint32_t* __restrict__ run_inst, const uint8_t* __restrict__ power,
                           const uint32_t* __restrict__ depth, const uint32_t* __restrict__ inst_start,
                           const uint32_t* counters, Seg* __restrict__ segs)
{
    const uint32_t h = counters[CNT_NHBM];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < h; q += gridDim.x * blockDim.x) {
        const uint32_t t = hbm_list[q];
        const uint32_t inst = run_inst[t];
        uint32_t a = inst_start[inst], par = q;
        if (q > 0) {
            const uint32_t tp = hbm_list[q - 1];
            if (run_inst[tp] == inst) {
                a = run_start[tp + 1];
                if (power[tp] > power[t]) par = q - 1;
            }
        }
        Seg s;
        s.start = a; s.end = run_start[t + 1]; s.inst = inst; s.dst = seg_dst(depth[par]);
        segs[q] = s;
    }
}

__global__ void k_segs_inst(const uint32_t* __restrict__ hbm_list, const uint32_t* __restrict__ run_start,
                            const uint32_t* __restrict__ run_inst, const uint32_t* __restrict__ depth,
                            const uint32_t* __restrict__ inst_start, const uint32_t* __restrict__ inst_big,
                            const uint32_t* __restrict__ inst_bigrank, uint32_t k,
                            const uint32_t* __restrict__ k_dev, uint32_t* counters, Seg* __restrict__ segs)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t h = counters[CNT_NHBM], nbig = counters[CNT_NBIG];
    // trailing empty instances (from *k_dev on) get no segment to visit
    if (i == 0) counters[CNT_NSEG] = h + (k_dev ? min(k, *k_dev) : k);
    if (i >= k) return;
    const uint32_t ib = inst_start[i], ie = inst_start[i + 1];
    Seg s;
    s.end = ie; s.inst = i;
    if (inst_big[i]) {
        // last HBM node with position < ie
        uint32_t lo = 0, hi = h;  // count of nodes with pos < ie
        while (lo < hi) {
            uint32_t m = (lo + hi) >> 1;
            if (run_start[hbm_list[m] + 1] < ie) lo = m + 1; else hi = m;
        }
        if (lo > 0 && run_inst[hbm_list[lo - 1]] == i) {
            s.start = run_start[hbm_list[lo - 1] + 1];
            s.dst = seg_dst(depth[lo - 1]);
        } else {
            s.start = ib; s.dst = 0;
        }
        segs[h + inst_bigrank[i]] = s;
    } else {
        s.start = ib; s.dst = 0;
        segs[h + nbig + (i - inst_bigrank[i])] = s;
    }
}

// ------------------------------------------------------- level table --
// Output tiles of every HBM node (T_out-aligned tiles of [L, R)), summed per
// power level.  level[0, MAX_LEVEL): tiles of each level; level[MAX_LEVEL,
// 2*MAX_LEVEL): their start in the level-ordered pair list; level[2*MAX_LEVEL,
// 3*MAX_LEVEL): fill positions.
// The counters of a level take one atomic per wave and power present in the
// wave (the lanes of one power summed first): one atomic per node put tens
// of thousands of updates on a handful of addresses.  p = MAX_LEVEL marks a
// lane without a node.  Returns, for the lane's power, the sum of v over the
// lanes of that power before it, and the value the level's counter held
// before the wave's atomic.
__device__ inline uint32_t wave_level_add(uint32_t p, uint32_t v, uint32_t* __restrict__ ctr, uint32_t& before)
{
    const int lane = threadIdx.x & (WAVE - 1);
    uint64_t todo = __ballot(p < MAX_LEVEL);
    uint32_t old = 0;
    before = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t pl = (uint32_t)__shfl((int)p, leader, WAVE);
        const bool mine = p == pl;
        const uint32_t inc = wave_incl_scan(mine ? v : 0u);
        const uint32_t tot = (uint32_t)__shfl((int)inc, WAVE - 1, WAVE);
        uint32_t o = 0;
        if (lane == leader) o = atomicAdd(&ctr[pl], tot);
        o = (uint32_t)__shfl((int)o, leader, WAVE);
        if (mine) {
            before = inc - v;
            old = o;
        }
        todo &= ~__ballot(mine);
    }
    return old;
}

__global__ void k_level_count(const uint32_t* __restrict__ hbm_list, const uint32_t* __restrict__ bnd_lpos,
                              const uint32_t* __restrict__ bnd_rpos, const uint8_t* __restrict__ power,
                              uint32_t T_out, const uint32_t* counters, uint32_t* __restrict__ tiles,
                              uint32_t* __restrict__ level)
{
    const uint32_t h = counters[CNT_NHBM];
    // whole workgroups step together, so that every lane of a wave takes
    // part in the wave's sums
    for (uint32_t b = blockIdx.x * blockDim.x; b < h; b += gridDim.x * blockDim.x) {
        const uint32_t q = b + threadIdx.x;
        uint32_t p = MAX_LEVEL, nt = 0;
        if (q < h) {
            const uint32_t t = hbm_list[q];
            const uint32_t L = bnd_lpos[t], R = bnd_rpos[t];
            nt = (R - 1) / T_out - L / T_out + 1;
            tiles[q] = nt;
            p = power[t] < MAX_LEVEL ? power[t] : MAX_LEVEL;
        }
        uint32_t before;
        wave_level_add(p, nt, level, before);
    }
}

__global__ void k_level_offsets(uint32_t* __restrict__ level, uint32_t pair_cap)
{
    if (threadIdx.x != 0) return;
    uint32_t acc = 0;
    for (int p = 0; p < (int)MAX_LEVEL; ++p) {
        // a count beyond the capacity cannot come from a consistent plan;
        // clamping keeps every write of k_level_fill in range
        const uint32_t c = acc + level[p] <= pair_cap ? level[p] : pair_cap - acc;
        level[p] = c;
        level[MAX_LEVEL + p] = acc;
        level[2 * MAX_LEVEL + p] = 0;
        acc += c;
    }
}

// Every HBM node reserves the slots of its output tiles in its level: the
// nodes of one power in a wave take consecutive slots from one atomic.
__global__ void k_level_reserve(const uint32_t* __restrict__ hbm_list, const uint8_t* __restrict__ power,
                                const uint32_t* __restrict__ tiles, const uint32_t* counters,
                                uint32_t* __restrict__ level, uint32_t* __restrict__ node_base)
{
    const uint32_t h = counters[CNT_NHBM];
    for (uint32_t b = blockIdx.x * blockDim.x; b < h; b += gridDim.x * blockDim.x) {
        const uint32_t q = b + threadIdx.x;
        uint32_t p = MAX_LEVEL, nt = 0;
        if (q < h) {
            p = power[hbm_list[q]];
            if (p < MAX_LEVEL) nt = tiles[q]; else p = MAX_LEVEL;
        }
        uint32_t before;
        const uint32_t old = wave_level_add(p, nt, level + 2 * MAX_LEVEL, before);
        if (q < h) node_base[q] = p < MAX_LEVEL ? level[MAX_LEVEL + p] + old + before : NONE;
    }
}

// Pair list by level: (HBM node, output tile) for every output tile.
__global__ void k_level_fill(const uint32_t* __restrict__ hbm_list, const uint32_t* __restrict__ bnd_lpos,
                             const uint8_t* __restrict__ power, const uint32_t* __restrict__ tile_off,
                             const uint32_t* __restrict__ node_base, uint32_t T_out, const uint32_t* counters,
                             const uint32_t* __restrict__ level, uint32_t* __restrict__ pairs)
{
    const uint32_t h = counters[CNT_NHBM], np = counters[CNT_NPAIRS];
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < np; x += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = h;
        while (hi - lo > 1) {
            uint32_t m = (lo + hi) >> 1;
            if (tile_off[m] <= x) lo = m; else hi = m;
        }
        const uint32_t t = hbm_list[lo];
        const uint32_t p = power[t];
        if (p >= MAX_LEVEL || node_base[lo] == NONE) continue;
        const uint32_t pos = node_base[lo] + (x - tile_off[lo]);
        if (pos >= level[MAX_LEVEL + p] + level[p]) continue;  // only past a clamped count
        pairs[2 * (uint64_t)pos] = lo;
        pairs[2 * (uint64_t)pos + 1] = bnd_lpos[t] / T_out + (x - tile_off[lo]);
    }
}

// ------------------------------------------------------------- host --
// Grid of the per-element planner kernels: they loop over a count known
// only on the device, and a grid sized for the capacity would mostly launch
// workgroups that find nothing to do.
static inline unsigned stride_grid(uint64_t cap)
{
    const uint64_t g = (cap + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g < 2048 ? g : 2048));
}

namespace {
struct Carver {
    uint8_t* base;
    size_t off;
    template <typename T>
    T* take(uint64_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (size_t)(count ? count : 1);
        return p;
    }
};

inline unsigned grid_for(uint64_t threads, unsigned block) { return (unsigned)ceil_div(threads ? threads : 1, block); }
}  // namespace

size_t plan_carve(Plan& P, void* ws, uint64_t n, uint64_t k, uint32_t T, uint32_t T_out, uint32_t min_len)
{
    Carver c{(uint8_t*)ws, 0};
    P.n = (uint32_t)n;
    P.k = (uint32_t)k;
    P.T = T;
    P.big_min = T;
    P.T_out = T_out;
    P.n_tiles_out = (uint32_t)ceil_div(n ? n : 1, T_out);
    // runs are at least min_len >= 16 long (explicit minrun >= 16, rule >=
    // 32) except the last of each instance
    // long runs are >= min_len long; an increasing and a decreasing one
    // share at most one element
    const uint64_t ml = min_len < 16 ? 16 : min_len;
    P.lr_cap = (uint32_t)(n / (ml - 1) + 3);
    P.run_cap = (uint32_t)(n / ml + k + 2);
    P.ent_cap = P.lr_cap + (uint32_t)k + 1;
    // nodes longer than T: those of one power level are disjoint, so fewer
    // than n / T + 1 per level
    {
        const uint64_t hc = (uint64_t)MAX_LEVEL * (n / (T ? T : 1) + 1) + 1;
        P.h_cap = (uint32_t)(hc < P.run_cap ? hc : P.run_cap);
    }
    P.seg_cap = P.h_cap + (uint32_t)k + 1;
    P.chain_blocks = (uint32_t)ceil_div(P.lr_cap, CHAIN_BLOCK);
    P.bm_tiles = (uint32_t)ceil_div(n / 64 + 2, 64);
    P.bm_words = P.bm_tiles * 64;
    P.inst_start = c.take<uint32_t>(k + 1);
    P.inst_big = c.take<uint32_t>(k);
    P.inst_bigrank = c.take<uint32_t>(k);
    P.inst_rfinal = c.take<uint32_t>(k);
    P.inst_run_lo = c.take<uint32_t>(k);
    P.inst_run_hi = c.take<uint32_t>(k);
    P.bitmap = c.take<uint64_t>(P.bm_words);
    P.tile_first = c.take<uint32_t>(P.bm_tiles);
    P.tile_next = c.take<uint32_t>(P.bm_tiles);
    P.tile_first0 = c.take<uint32_t>(P.bm_tiles);
    P.tile_next0 = c.take<uint32_t>(P.bm_tiles);
    P.desc = 0;
    P.tile_cnt = c.take<uint32_t>(P.bm_tiles);
    P.tile_off = c.take<uint32_t>(P.bm_tiles);
    P.lr_u = c.take<uint32_t>(P.lr_cap);
    P.lr_e = c.take<uint32_t>(P.lr_cap);
    P.lr_inst = c.take<uint32_t>(P.lr_cap);
    P.lr_cnt = c.take<uint32_t>(P.lr_cap);
    P.lr_base = c.take<uint32_t>(P.lr_cap);
    P.chain_val = c.take<uint32_t>((uint64_t)P.chain_blocks * 64);
    P.chain_known = c.take<uint64_t>(P.chain_blocks);
    P.chain_rin = c.take<uint32_t>(P.chain_blocks);
    P.ent_cnt = c.take<uint32_t>(P.ent_cap);
    P.ent_base = c.take<uint32_t>(P.ent_cap);
    P.ent_inst = c.take<uint32_t>(P.ent_cap);
    P.ent_off = c.take<uint32_t>(P.ent_cap);
    P.run_start = c.take<uint32_t>(P.run_cap + 1);
    P.run_inst = c.take<uint32_t>(P.run_cap);
    P.run_q = c.take<uint32_t>(P.run_cap);
    P.power = c.take<uint8_t>(P.run_cap);
    P.bnd_l = c.take<uint32_t>(P.run_cap);
    P.bnd_r = c.take<uint32_t>(P.run_cap);
    P.bnd_lpos = c.take<uint32_t>(P.run_cap);
    P.bnd_rpos = c.take<uint32_t>(P.run_cap);
    P.hbm_flag = c.take<uint32_t>(P.run_cap);
    P.hbm_rank = c.take<uint32_t>(P.run_cap);
    P.hbm_idx = c.take<uint32_t>(P.run_cap);
    P.hbm_list = c.take<uint32_t>(P.h_cap);
    P.hbm_par[0] = c.take<uint32_t>(P.h_cap);
    P.hbm_par[1] = c.take<uint32_t>(P.h_cap);
    P.hbm_val[0] = c.take<uint32_t>(P.h_cap);
    P.hbm_val[1] = c.take<uint32_t>(P.h_cap);
    P.hbm_tiles = c.take<uint32_t>(P.h_cap + 1);
    P.hbm_tile_off = c.take<uint32_t>(P.h_cap + 1);
    P.segs = c.take<Seg>(P.seg_cap);
    // output tiles of all HBM nodes: per level at most n_tiles_out plus two
    // per node, and a level holds fewer than n / T + 1 nodes longer than T;
    // sized for the smallest merge tile, so the tuning may pick any
    {
        const uint64_t per_level = ceil_div(n ? n : 1, MERGE_TILE_MIN) + 2 * (n / (T ? T : 1) + 1);
        const uint64_t cap = (uint64_t)MAX_LEVEL * per_level;
        P.pair_cap = (uint32_t)(cap < 0xffffffffull ? cap : 0xffffffffull);
    }
    P.level = c.take<uint32_t>(3 * MAX_LEVEL);
    P.node_base = c.take<uint32_t>(P.h_cap);
    P.pairs = c.take<uint32_t>(2 * (uint64_t)P.pair_cap);
    P.splits = c.take<uint32_t>(2 * (uint64_t)P.pair_cap);
    P.counters = c.take<uint32_t>(CNT_COUNT);
    P.stats = c.take<unsigned long long>(8);
    uint64_t cap = P.bm_tiles;
    if (P.run_cap + 1 > cap) cap = P.run_cap + 1;
    if (P.ent_cap > cap) cap = P.ent_cap;
    if (k > cap) cap = k;
    P.scan_tmp_words = scan_tmp_words(cap);
    P.scan_tmp = c.take<uint32_t>(P.scan_tmp_words);
    P.hbm_depth = nullptr;
    P.inst_off64 = nullptr;
    P.off_trusted = false;
    P.k_dev = nullptr;
    return c.off + 256;
}

size_t plan_workspace_bytes(uint64_t n, uint64_t k, uint32_t T, uint32_t T_out, uint32_t min_len)
{
    Plan P;
    return plan_carve(P, nullptr, n, k, T, T_out, min_len);
}

// Counts are clamped to the capacities the arrays were carved for, so a
// wrong count can only give a wrong schedule, never an access out of range.
__global__ void k_clamp(uint32_t* counters, int which, uint32_t cap)
{
    if (threadIdx.x == 0 && counters[which] > cap) {
        counters[which] = cap;
        counters[CNT_BAD] |= 2u;
    }
}

__global__ void k_zero_stats(unsigned long long* stats)
{
    if (threadIdx.x < 8) stats[threadIdx.x] = 0;
}

template <typename K>
static hipError_t plan_enqueue_t(Plan& P, const K* keys, uint32_t ell_ovr, hipStream_t s)
{
    const uint32_t n = P.n, k = P.k;
    uint32_t* C = P.counters;
    // tile_off and tile_cnt hold each bitmap tile's first instance and
    // whether it meets an instance the planner handles, until the long-run
    // counts take them over
    if (P.off_trusted && P.inst_off64)
        k_inst_prep_trusted<<<grid_for((uint64_t)k + 1, 256), 256, 0, s>>>(P.inst_off64, k, P.big_min, P.inst_start,
                                                                         P.inst_big, P.inst_rfinal, P.inst_run_lo,
                                                                         P.inst_run_hi, C);
    else
        k_inst_prep<<<1, 1024, 0, s>>>(P.inst_off64, k, n, P.big_min, P.inst_start, P.inst_big, P.inst_rfinal,
                                       P.inst_run_lo, P.inst_run_hi, C);
    if (k > 1)
        k_tile_inst<<<grid_for(P.bm_tiles, 256), 256, 0, s>>>(P.inst_start, P.inst_big, k, n, P.bm_tiles, P.tile_off,
                                                              P.tile_cnt);
    k_zero_stats<<<1, 64, 0, s>>>(P.stats);
    VMPS_HIP(scan_exclusive_u32(P.inst_big, P.inst_bigrank, k, nullptr, C + CNT_NBIG, P.scan_tmp, s));
    // 1. bitmap
    const bool desc = P.desc && k == 1;
    k_bitmap<K><<<P.bm_tiles, 256, 0, s>>>(keys, n, P.inst_start, P.inst_big, k, P.tile_off, P.tile_cnt,
                                           P.bitmap, P.tile_first, desc ? P.tile_first0 : nullptr);
    k_suffix_min<<<1, 1024, 0, s>>>(P.tile_first, P.tile_next, P.bm_tiles);
    if (desc) k_suffix_min<<<1, 1024, 0, s>>>(P.tile_first0, P.tile_next0, P.bm_tiles);
    // 2. long natural runs
    const uint32_t cand_min = (k == 1) ? (ell_ovr ? ell_ovr : minrun_of(n)) : 32u;
    k_long_runs<false><<<P.bm_tiles, 64, 0, s>>>(P.bitmap, n, P.tile_next, desc ? P.tile_next0 : nullptr,
                                                 P.inst_start, P.inst_big, k, ell_ovr, cand_min, P.lr_cap, P.tile_cnt,
                                                 nullptr, nullptr, nullptr, nullptr);
    VMPS_HIP(scan_exclusive_u32(P.tile_cnt, P.tile_off, P.bm_tiles, nullptr, C + CNT_NLONG, P.scan_tmp, s));
    k_clamp<<<1, 64, 0, s>>>(C, CNT_NLONG, P.lr_cap);
    k_long_runs<true><<<P.bm_tiles, 64, 0, s>>>(P.bitmap, n, P.tile_next, desc ? P.tile_next0 : nullptr,
                                                P.inst_start, P.inst_big, k, ell_ovr, cand_min, P.lr_cap, nullptr,
                                                P.tile_off, P.lr_u, P.lr_e, P.lr_inst);
    // 3. chain of run starts
    const unsigned chain_grid = P.chain_blocks < 512u ? P.chain_blocks : 512u;  // two workgroups per CU
    k_chain_blocks<<<chain_grid ? chain_grid : 1, CHAIN_NT, 0, s>>>(P.lr_u, P.lr_e, P.lr_inst, P.inst_start, ell_ovr, C,
                                                 P.chain_val, P.chain_known);
    k_chain_scan<<<1, 256, 0, s>>>(P.lr_inst, P.inst_start, ell_ovr, C, P.chain_val, P.chain_known, P.chain_rin);
    k_chain_apply<<<chain_grid ? chain_grid : 1, CHAIN_NT, 0, s>>>(P.lr_u, P.lr_e, P.lr_inst, P.inst_start, ell_ovr, C, P.chain_rin,
                                                P.lr_cnt, P.lr_base, P.inst_rfinal);
    k_entries_lr<<<stride_grid(P.lr_cap), 256, 0, s>>>(P.lr_inst, P.lr_cnt, P.lr_base, P.inst_bigrank, C,
                                                         P.ent_cnt, P.ent_base, P.ent_inst);
    k_entries_tail<<<grid_for(k, 256), 256, 0, s>>>(P.lr_inst, P.inst_start, P.inst_big, P.inst_bigrank,
                                                    P.inst_rfinal, k, ell_ovr, C, P.ent_cnt, P.ent_base,
                                                    P.ent_inst);
    VMPS_HIP(scan_exclusive_u32(P.ent_cnt, P.ent_off, P.ent_cap, C + CNT_NENT, C + CNT_NRUNS, P.scan_tmp, s));
    k_clamp<<<1, 64, 0, s>>>(C, CNT_NRUNS, P.run_cap);
    k_runs_emit<<<stride_grid(P.run_cap + 1), 256, 0, s>>>(P.ent_off, P.ent_base, P.ent_inst, P.inst_start, n,
                                                             ell_ovr, C, P.run_start, P.run_inst);
    // 4-5. powers and tree
    k_run_q<<<stride_grid(P.run_cap), 256, 0, s>>>(P.run_start, P.run_inst, P.inst_start, C, P.run_q,
                                                     P.inst_run_lo, P.inst_run_hi);
    const unsigned bgrid = grid_for(P.run_cap, 256) < 4096u ? grid_for(P.run_cap, 256) : 4096u;
    k_boundaries<<<bgrid, 256, 0, s>>>(P.run_start, P.run_inst, P.run_q, P.inst_start, P.inst_run_lo,
                                       P.inst_run_hi, P.T, C, P.power, P.bnd_l, P.bnd_r, P.bnd_lpos, P.bnd_rpos,
                                       P.hbm_flag, P.stats);
    // 6. nodes longer than T and their depths
    VMPS_HIP(scan_exclusive_u32(P.hbm_flag, P.hbm_rank, P.run_cap, C + CNT_NRUNS, C + CNT_NHBM, P.scan_tmp, s));
    k_clamp<<<1, 64, 0, s>>>(C, CNT_NHBM, P.h_cap);
    k_hbm_emit<<<stride_grid(P.run_cap), 256, 0, s>>>(P.hbm_flag, P.hbm_rank, C, P.h_cap, P.hbm_list, P.hbm_idx);
    k_depth_init<<<stride_grid(P.h_cap), 256, 0, s>>>(P.hbm_list, P.hbm_idx, P.bnd_l, P.bnd_r, P.power,
                                                          P.hbm_flag, C,
                                                          P.hbm_par[0], P.hbm_val[0]);
    int cur = 0;
    for (int round = 0; round < 6; ++round) {
        k_depth_jump<<<stride_grid(P.h_cap), 256, 0, s>>>(P.hbm_par[cur], P.hbm_val[cur], C,
                                                              P.hbm_par[cur ^ 1], P.hbm_val[cur ^ 1]);
        cur ^= 1;
    }
    P.hbm_depth = P.hbm_val[cur];
    // 7. LDS segments and the level table
    k_segs_hbm<<<stride_grid(P.h_cap), 256, 0, s>>>(P.hbm_list, P.run_start, P.run_inst, P.power,
                                                        P.hbm_depth, P.inst_start, C, P.segs);
    k_segs_inst<<<grid_for(k, 256), 256, 0, s>>>(P.hbm_list, P.run_start, P.run_inst, P.hbm_depth,
                                                 P.inst_start, P.inst_big, P.inst_bigrank, k, P.k_dev, C, P.segs);
    VMPS_HIP(fill_u32(P.level, 0, 3 * MAX_LEVEL, s));
    k_level_count<<<stride_grid(P.h_cap), 256, 0, s>>>(P.hbm_list, P.bnd_lpos, P.bnd_rpos, P.power, P.T_out,
                                                           C, P.hbm_tiles, P.level);
    VMPS_HIP(scan_exclusive_u32(P.hbm_tiles, P.hbm_tile_off, P.h_cap, C + CNT_NHBM, C + CNT_NPAIRS,
                                P.scan_tmp, s));
    k_clamp<<<1, 64, 0, s>>>(C, CNT_NPAIRS, P.pair_cap);
    k_level_offsets<<<1, 64, 0, s>>>(P.level, P.pair_cap);
    k_level_reserve<<<stride_grid(P.h_cap), 256, 0, s>>>(P.hbm_list, P.power, P.hbm_tiles, C, P.level,
                                                             P.node_base);
    k_level_fill<<<stride_grid(P.pair_cap), 256, 0, s>>>(P.hbm_list, P.bnd_lpos, P.power, P.hbm_tile_off,
                                                           P.node_base, P.T_out, C, P.level, P.pairs);
    return hipGetLastError();
}

// ------------------------------------------- position-ordered levels --
// The level table above reserves each node's pair slots with an atomic, so
// the nodes of a level appear in any order.  The paged merge levels need
// them in position order (a round takes consecutive pages).  Nodes q are in
// position order already, so the slot of node q is: the level's offset,
// plus the tiles of the same-level nodes before q.  Per block of
// ORDER_BLOCK nodes: the tiles of each level (level-major, so one flat scan
// gives level offset + earlier blocks), then the rank inside the block.
constexpr uint32_t ORDER_BLOCK = 256;

__global__ void k_order_sums(const uint32_t* __restrict__ hbm_list, const uint8_t* __restrict__ power,
                             const uint32_t* __restrict__ tiles, const uint32_t* counters, uint32_t nblocks,
                             uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t lv[MAX_LEVEL];
    const uint32_t h = counters[CNT_NHBM], b = blockIdx.x;
    if (threadIdx.x < MAX_LEVEL) lv[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t q = b * ORDER_BLOCK + threadIdx.x;
    if (q < h) {
        const uint32_t p = power[hbm_list[q]];
        if (p < MAX_LEVEL) atomicAdd(&lv[p], tiles[q]);
    }
    __syncthreads();
    if (threadIdx.x < MAX_LEVEL) bsum[(uint64_t)threadIdx.x * nblocks + b] = lv[threadIdx.x];
}

__global__ void k_order_apply(const uint32_t* __restrict__ hbm_list, const uint8_t* __restrict__ power,
                              const uint32_t* __restrict__ tiles, const uint32_t* counters, uint32_t nblocks,
                              const uint32_t* __restrict__ boff, uint32_t* __restrict__ node_base)
{
    __shared__ uint32_t lp[ORDER_BLOCK], lt[ORDER_BLOCK];
    const uint32_t h = counters[CNT_NHBM], b = blockIdx.x;
    const uint32_t q = b * ORDER_BLOCK + threadIdx.x;
    uint32_t p = MAX_LEVEL, t = 0;
    if (q < h) {
        p = power[hbm_list[q]];
        t = tiles[q];
    }
    lp[threadIdx.x] = p;
    lt[threadIdx.x] = t;
    __syncthreads();
    if (q >= h) return;
    if (p >= MAX_LEVEL) {
        node_base[q] = NONE;
        return;
    }
    uint32_t before = 0;
    for (uint32_t j = 0; j < threadIdx.x; ++j) before += lp[j] == p ? lt[j] : 0u;
    node_base[q] = boff[(uint64_t)p * nblocks + b] + before;
}

uint64_t plan_order_blocks(const Plan& P) { return ceil_div(P.h_cap, ORDER_BLOCK); }

hipError_t plan_order_levels(Plan& P, uint32_t* bsum, uint32_t* boff, uint32_t* tmp, hipStream_t s)
{
    const uint64_t nb = plan_order_blocks(P);
    uint32_t* C = P.counters;
    k_order_sums<<<(unsigned)nb, ORDER_BLOCK, 0, s>>>(P.hbm_list, P.power, P.hbm_tiles, C, (uint32_t)nb, bsum);
    VMPS_HIP(scan_exclusive_u32(bsum, boff, (uint64_t)MAX_LEVEL * nb, nullptr, nullptr, tmp, s));
    k_order_apply<<<(unsigned)nb, ORDER_BLOCK, 0, s>>>(P.hbm_list, P.power, P.hbm_tiles, C, (uint32_t)nb, boff,
                                                       P.node_base);
    k_level_fill<<<stride_grid(P.pair_cap), 256, 0, s>>>(P.hbm_list, P.bnd_lpos, P.power, P.hbm_tile_off,
                                                           P.node_base, P.T_out, C, P.level, P.pairs);
    return hipGetLastError();
}

hipError_t plan_enqueue(Plan& P, const void* keys, int key_bits, uint32_t ell_override, hipStream_t s)
{
    TraceScope tr(VMPS_TRACE_PLAN, s);
    if (key_bits == 32) return plan_enqueue_t<uint32_t>(P, (const uint32_t*)keys, ell_override, s);
    return plan_enqueue_t<uint64_t>(P, (const uint64_t*)keys, ell_override, s);
}

}  // namespace vmps
