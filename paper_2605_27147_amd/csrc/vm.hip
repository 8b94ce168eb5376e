// Virtual-Memory Powersort on the GPU (Section 4 of the paper): the merge
// levels run over pages instead of a second array.
//
// Memory is cut into pages of P elements (P = the merge output tile, a power
// of two): the input array's pages 0..N-1 and a small pool of extra pages.
// A page table pt maps every virtual page v (positions [vP, (v+1)P) of the
// array being sorted) to the physical page that holds it.  After the LDS
// tile pass (which sorts in place, so pt starts as the identity), each merge
// level writes every page it touches into a fresh physical page:
//
//  * the level's pages are taken in position order and cut into rounds of W
//    pages, one launch per round;
//  * an input page is released (joins the free sequence) once the last
//    round that reads any of its elements has run: the free list of the
//    paper, consumed input pages becoming output pages;
//  * the fresh page of the u-th touched page is entry u of the sequence
//    "pool, then released pages in release-round order"; it is free before
//    its round starts as long as the pool holds W + 4 pages (a round's W
//    outputs consume W pages' worth of elements, which leaves at most three
//    input pages partly consumed: the two merge-path frontiers and the page
//    holding the split between the two runs; one more for the array's
//    partial last page).  The schedule is checked on the device anyway;
//  * the pages left over at the end of a level are the next level's pool.
//  * Parts of a touched page that no merge of the level writes (the ends of
//    runs that are merged later) are copied into the fresh page ("carries").
//
// The input's partial last page is never reused for another page (it could
// not hold a full one), as in the paper.  At the end, Copy moves every page
// to its place in the array: the page permutation is cut into segments at
// heads (every 64th page index, the start of every path, the least page of
// a cycle with no such index); the contents of the heads that other segments
// end on are saved first, then every segment's pages move one after the
// other, each thread moving the same columns of every page, so no
// workgroup waits for another.
#include "merge_tile.hpp"

namespace vmps {

constexpr uint32_t VM_HEAD = 64;  // page indices that are multiples of this head a copy segment
constexpr uint32_t VM_NT = 256;   // threads of the copy workgroups

enum {
    VC_E = 0,     // pool pages at the start of the level
    VC_E_NEXT,    // pool pages after it
    VC_PARKED,    // pages of this level not released (the input's partial page)
    VC_U,         // pages the level touches
    VC_ROUNDS,    // rounds of the level
    VC_F,         // touched pages that need a fresh page (not kept in place)
    VC_COUNT = 8
};
enum { VS_BAD = 0, VS_CARRY, VS_COPY, VS_MERGED, VS_LEVELS, VS_PAGE_WRITES, VS_KEPT, VS_COUNT = 8 };
constexpr uint32_t KEPT = 0xFFFFFFFEu;  // release round of a page kept in place

struct VmArgs {
    // level table (position-ordered pairs)
    const uint32_t* level;
    const uint32_t* pairs;
    const uint32_t* hbm_list;
    const uint32_t* lpos;
    const uint32_t* rpos;
    const uint32_t* run_start;
    const uint32_t* node_base;
    const uint32_t* tiles;
    uint32_t* splits;
    const uint32_t* upage;  // per pair: index of its page among the level's touched pages
    // pages
    void* keys;             // the array (pages 0 .. nin-1)
    void* kpool;            // extra pages nin .. nin+emax-1
    uint32_t* vals;
    uint32_t* vpool;
    uint32_t* pt;           // N: virtual page -> physical page
    uint32_t* S;            // N + emax: free sequence of the level
    uint32_t* pool;         // emax: pool pages
    uint32_t* rel;          // N: release round of each touched page (NONE: parked, KEPT: kept in place)
    uint32_t* need;         // N: 1 when the touched page needs a fresh page
    uint32_t* fidx;         // N: its index among those (exclusive scan of need)
    uint32_t* oldp;         // N: its physical page before the level
    uint32_t* bins;         // rmax + 2: released pages per round, then (boff) their offsets
    uint32_t* boff;
    uint32_t* cursor;
    uint32_t* rfirst;       // rmax + 2: first pair of every round
    uint64_t* mark_start;   // N: (level << 32) | L of a level node starting inside page v
    uint64_t* mark_end;     // N: (level << 32) | R of a level node ending inside page v
    uint32_t* vc;           // VC_COUNT
    unsigned long long* vs; // VS_COUNT statistics
    uint32_t n, N, nin, logp, W, rmax, emax;
};

template <typename K>
struct Pages {
    K* keys;
    K* pool;
    uint32_t* vals;
    uint32_t* vpool;
    uint32_t nin, logp;
    __device__ K* kp(uint32_t p) const
    {
        return p < nin ? keys + ((uint64_t)p << logp) : pool + ((uint64_t)(p - nin) << logp);
    }
    __device__ uint32_t* vp(uint32_t p) const
    {
        return p < nin ? vals + ((uint64_t)p << logp) : vpool + ((uint64_t)(p - nin) << logp);
    }
    // key at virtual position x
    __device__ K key(const uint32_t* pt, uint32_t x) const { return kp(pt[x >> logp])[x & ((1u << logp) - 1)]; }
};

// ctr[key] += 1 for every lane that calls it, one atomic per distinct key
// in the wave (neighbouring pages mostly share a release round, and one
// atomic per page on a handful of counters serialises); returns the lane's
// slot among those counted for its key.
__device__ inline uint32_t wave_count(uint32_t* ctr, uint32_t key)
{
    const int lane = threadIdx.x & (WAVE - 1);
    uint64_t todo = __ballot(1);
    uint32_t slot = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t k0 = __shfl(key, leader, WAVE);
        const uint64_t same = __ballot(key == k0) & todo;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k0], (uint32_t)__popcll(same));
        base = __shfl(base, leader, WAVE);
        if ((same >> lane) & 1) slot = base + (uint32_t)__popcll(same & ((1ull << lane) - 1));
        todo &= ~same;
    }
    return slot;
}

template <typename K>
__device__ inline Pages<K> pages_of(const VmArgs& A)
{
    return Pages<K>{(K*)A.keys, (K*)A.kpool, A.vals, A.vpool, A.nin, A.logp};
}

// ------------------------------------------------------------ set-up --
__global__ void k_vm_init(VmArgs A, uint32_t e0)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.N; i += stride) {
        A.pt[i] = (uint32_t)i;
        A.mark_start[i] = ~0ull;
        A.mark_end[i] = ~0ull;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e0; i += stride)
        A.pool[i] = A.nin + (uint32_t)i;
    if (blockIdx.x == 0 && threadIdx.x < VC_COUNT) A.vc[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x < VS_COUNT) A.vs[threadIdx.x] = 0;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.vc[VC_E] = e0;
        A.vc[VC_E_NEXT] = e0;
    }
}

// Every LDS segment is sorted in place (no second array to alternate with).
__global__ void k_vm_segs_in_place(Seg* segs, const uint32_t* counters, uint32_t cap)
{
    const uint32_t ns = min(counters[CNT_NSEG], cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) segs[i].dst = 0;
}

// First pair of every level and of every new page starts a touched page.
__global__ void k_vm_page_flags(const uint32_t* __restrict__ pairs, const uint32_t* __restrict__ hbm_list,
                                const uint8_t* __restrict__ power, const uint32_t* counters, uint32_t cap,
                                uint32_t* __restrict__ flag)
{
    const uint32_t np = min(counters[CNT_NPAIRS], cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        uint32_t f = 1;
        if (i > 0) {
            const uint32_t p0 = power[hbm_list[pairs[2 * (uint64_t)(i - 1)]]];
            const uint32_t p1 = power[hbm_list[pairs[2 * (uint64_t)i]]];
            f = (p0 != p1 || pairs[2 * (uint64_t)(i - 1) + 1] != pairs[2 * (uint64_t)i + 1]) ? 1u : 0u;
        }
        flag[i] = f;
    }
}

// upage: the pair's page among its level's pages.  gpage is the exclusive
// scan of the flags, so the page that pair i starts or continues has global
// index gpage[i] + flag[i] - 1; the level's first pair starts its page 0.
__global__ void k_vm_upage(const uint32_t* __restrict__ pairs, const uint32_t* __restrict__ hbm_list,
                           const uint8_t* __restrict__ power, const uint32_t* __restrict__ level,
                           const uint32_t* counters, uint32_t cap, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ gpage, uint32_t* __restrict__ upage)
{
    const uint32_t np = min(counters[CNT_NPAIRS], cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        const uint32_t p = power[hbm_list[pairs[2 * (uint64_t)i]]];
        uint32_t first = p < MAX_LEVEL ? level[MAX_LEVEL + p] : i;
        first = first < np ? first : i;
        upage[i] = gpage[i] + flag[i] - 1u - gpage[first];
    }
}

// ------------------------------------------------------ one level --
// Merge-path splits at both ends of every pair, read through the page table
// (as k_level_partition on one array).  Block 0 also resets the level's
// round bins and commits the pool size left by the previous level.
template <typename K>
__global__ void k_vm_partition(VmArgs A, uint32_t lvl)
{
    const Pages<K> pg = pages_of<K>(A);
    if (blockIdx.x == 0) {
        for (uint32_t i = threadIdx.x; i < A.rmax + 2; i += blockDim.x) {
            A.bins[i] = 0;
            A.cursor[i] = 0;
        }
        if (threadIdx.x == 0) {
            A.vc[VC_E] = A.vc[VC_E_NEXT];
            A.vc[VC_U] = 0;
            A.vc[VC_ROUNDS] = 0;
            A.vc[VC_PARKED] = 0;
            A.vc[VC_F] = 0;
        }
    }
    const uint32_t cnt = A.level[lvl], off = A.level[MAX_LEVEL + lvl];
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < 2ull * cnt;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t i = off + (uint32_t)(x >> 1), end = (uint32_t)(x & 1);
        const uint32_t q = A.pairs[2 * (uint64_t)i], tt = A.pairs[2 * (uint64_t)i + 1];
        const uint32_t t = A.hbm_list[q];
        const uint32_t L = A.lpos[t], Mid = A.run_start[t + 1], R = A.rpos[t];
        const uint64_t t0 = (uint64_t)tt << A.logp, P = 1ull << A.logp;
        const uint32_t o = end ? (uint32_t)(R < t0 + P ? R : t0 + P) : (uint32_t)(L > t0 ? L : t0);
        const uint32_t d = o - L, na = Mid - L, nb = R - Mid;
        uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (pg.key(A.pt, L + mid) <= pg.key(A.pt, Mid + d - 1 - mid)) lo = mid + 1; else hi = mid;
        }
        A.splits[2 * (uint64_t)i + end] = lo;
    }
}

// Pair (of node q) whose output range holds element ia of the node's left
// run (a) or element jb of its right run (b): the last pair whose start
// split is at most that element.
__device__ inline uint32_t dest_pair_a(const VmArgs& A, uint32_t base, uint32_t cnt, uint32_t ia)
{
    uint32_t lo = base, hi = base + cnt - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (A.splits[2 * (uint64_t)mid] <= ia) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline uint32_t dest_pair_b(const VmArgs& A, uint32_t base, uint32_t cnt, uint32_t L, uint32_t jb)
{
    uint32_t lo = base, hi = base + cnt - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        const uint32_t t0 = A.pairs[2 * (uint64_t)mid + 1] << A.logp;
        const uint32_t o0 = L > t0 ? L : t0;
        const uint32_t j0 = (o0 - L) - A.splits[2 * (uint64_t)mid];
        if (j0 <= jb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pages a merge leaves where they are (the page-skipping merge of the
// remark on galloping in Sec. 2): a page where every output tile of the
// level takes exactly the elements at its own positions — a prefix of a
// left run that precedes every element of the right run, or a suffix of a
// right run that follows every element of the left run — and the rest is
// carried (stays anyway).  Every element of such a page stays, so nothing
// else reads it: it keeps its physical page and is neither written nor
// released.  Also the carry marks of the level's nodes and the number of
// touched pages.
__global__ void k_vm_keep(VmArgs A, uint32_t lvl)
{
    const uint32_t cnt = A.level[lvl], off = A.level[MAX_LEVEL + lvl];
    const uint32_t P = 1u << A.logp;
    uint32_t kept = 0;  // merge outputs left in place
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < cnt; x += gridDim.x * blockDim.x) {
        const uint32_t i = off + x;
        const uint32_t q = A.pairs[2 * (uint64_t)i], v = A.pairs[2 * (uint64_t)i + 1];
        const uint32_t t = A.hbm_list[q];
        const uint32_t L = A.lpos[t], R = A.rpos[t];
        if (v == (L >> A.logp) && (L & (P - 1))) A.mark_start[v] = ((uint64_t)lvl << 32) | L;
        if (v == ((R - 1) >> A.logp) && (R & (P - 1))) A.mark_end[v] = ((uint64_t)lvl << 32) | R;
        const uint32_t u = A.upage[i];
        if (x == cnt - 1) A.vc[VC_U] = min(u + 1, A.N);
        if (x > 0 && A.pairs[2 * (uint64_t)(i - 1) + 1] == v) continue;  // not the page's first pair
        if (u >= A.N) continue;  // only from a level table out of position order (counted below)
        const uint32_t vlo = v << A.logp;
        bool keep = true;
        uint32_t covered = 0;
        for (uint32_t j = i; j < off + cnt && j <= i + 1; ++j) {
            if (A.pairs[2 * (uint64_t)j + 1] != v) break;
            const uint32_t tj = A.hbm_list[A.pairs[2 * (uint64_t)j]];
            const uint32_t Lj = A.lpos[tj], Mj = A.run_start[tj + 1], Rj = A.rpos[tj];
            const uint32_t o0 = Lj > vlo ? Lj : vlo, o1 = Rj < vlo + P ? Rj : vlo + P;
            const uint32_t i0 = A.splits[2 * (uint64_t)j], i1 = A.splits[2 * (uint64_t)j + 1];
            const uint32_t j0 = (o0 - Lj) - i0, j1 = (o1 - Lj) - i1;
            keep = keep && ((j0 == 0 && j1 == 0) || (i0 == Mj - Lj && i1 == Mj - Lj));
            covered += o1 - o0;
        }
        A.need[u] = keep ? 0u : 1u;
        if (keep) kept += covered;
    }
    if (kept) atomicAdd(&A.vs[VS_KEPT], (unsigned long long)kept);
}

// For every touched page that is not kept: the round after which its old
// contents are no longer read (the latest round of a pair that takes one of
// its elements: the last element of each run part in the page decides,
// since a merge consumes each run in order).  Rounds count fresh pages.
__global__ void k_vm_release(VmArgs A, uint32_t lvl)
{
    const uint32_t cnt = A.level[lvl], off = A.level[MAX_LEVEL + lvl];
    const uint32_t P = 1u << A.logp;
    const uint32_t F = A.vc[VC_F];
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < cnt; x += gridDim.x * blockDim.x) {
        const uint32_t i = off + x;
        const uint32_t v = A.pairs[2 * (uint64_t)i + 1];
        const uint32_t u = A.upage[i];
        if (x == cnt - 1) {
            const uint32_t rounds = (F + A.W - 1) / A.W;
            A.vc[VC_ROUNDS] = rounds;
            A.rfirst[rounds] = off + cnt;
        }
        if (x > 0 && A.pairs[2 * (uint64_t)(i - 1) + 1] == v) continue;  // not the page's first pair
        if (u >= A.N) {  // only from a level table out of position order
            atomicAdd(&A.vs[VS_BAD], 1ull);
            continue;
        }
        if (!A.need[u]) {
            A.rel[u] = KEPT;
            continue;
        }
        const uint32_t f = A.fidx[u];
        if (f % A.W == 0) A.rfirst[f / A.W] = i;
        // the page's own round reads it only when part of it is carried
        // (covered by no node of the level)
        uint32_t last = 0, covered = 0;
        for (uint32_t j = i; j < off + cnt && j <= i + 1; ++j) {
            if (A.pairs[2 * (uint64_t)j + 1] != v) break;
            const uint32_t qj = A.pairs[2 * (uint64_t)j];
            const uint32_t tj = A.hbm_list[qj];
            const uint32_t Lj = A.lpos[tj], Mj = A.run_start[tj + 1], Rj = A.rpos[tj];
            const uint32_t vlo = v << A.logp, vhi = vlo + P;
            const uint32_t lo = Lj > vlo ? Lj : vlo, hi = Rj < vhi ? Rj : vhi;
            covered += hi - lo;
            const uint32_t base = A.node_base[qj], nt = A.tiles[qj];
            // an element's destination page is never a kept one (a kept
            // page's elements are its own)
            if (lo < Mj) {  // part of the left run: its last element
                const uint32_t ea = (hi < Mj ? hi : Mj) - 1;
                const uint32_t d = dest_pair_a(A, base, nt, ea - Lj);
                last = max(last, A.fidx[A.upage[d]]);
            }
            if (hi > Mj) {  // part of the right run
                const uint32_t d = dest_pair_b(A, base, nt, Lj, hi - 1 - Mj);
                last = max(last, A.fidx[A.upage[d]]);
            }
        }
        const uint32_t vlen = min(P, A.n - (v << A.logp));
        if (covered < vlen) last = max(last, f);
        const uint32_t old = A.pt[v];
        A.oldp[u] = old;
        if (old == A.nin - 1 && (A.n & (P - 1))) {
            A.rel[u] = NONE;  // the input's partial page holds no other page
            atomicAdd(&A.vc[VC_PARKED], 1u);
        } else {
            const uint32_t r = last / A.W;
            A.rel[u] = r;
            wave_count(A.bins, r);
        }
    }
}

// Offsets of the release rounds in the free sequence; pool size after the
// level.  One workgroup.
__global__ void k_vm_bins(VmArgs A)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const uint32_t nr = A.rmax + 1;
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nr; b += blockDim.x) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < nr ? A.bins[i] : 0u;
        uint32_t tot = 0;
        const uint32_t ex = block_excl_scan(v, lds, &tot);
        if (i < nr) A.boff[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) A.vc[VC_E_NEXT] = A.vc[VC_E] - A.vc[VC_PARKED];
}

// The free sequence S: the pool, then the released pages by round.  Entry
// f < F is the fresh page of the f-th page that needs one, written in round
// f / W: a released page there must have been released in an earlier round.
__global__ void k_vm_fill(VmArgs A)
{
    const uint32_t E = A.vc[VC_E], U = min(A.vc[VC_U], A.N), F = A.vc[VC_F];
    const uint32_t m = E > U ? E : U;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < m; u += gridDim.x * blockDim.x) {
        if (u < E) A.S[u] = A.pool[u];
        if (u < U && A.rel[u] < KEPT) {
            const uint32_t r = A.rel[u];
            const uint32_t idx = E + A.boff[r] + wave_count(A.cursor, r);
            A.S[idx] = A.oldp[u];
            if (idx < F && r >= idx / A.W) atomicAdd(&A.vs[VS_BAD], 1ull);
        }
    }
}

// One round: every pair whose page is among the round's W pages, merged
// through LDS from the old pages into the page's fresh one, plus the
// page's carried parts.
template <typename K, bool VAL, int NT, int KI>
__global__ __launch_bounds__(NT) void k_vm_round(VmArgs A, uint32_t lvl, uint32_t round)
{
    constexpr uint32_t SP = MergeLds<(uint32_t)(NT * KI)>::SP;
    extern __shared__ __align__(16) uint8_t smem[];
    K* S = (K*)smem;
    uint32_t* SV = (uint32_t*)(S + SP);
    if (round >= A.vc[VC_ROUNDS]) return;
    const Pages<K> pg = pages_of<K>(A);
    const uint32_t P = 1u << A.logp, mask = P - 1;
    const uint32_t cnt = A.level[lvl], off = A.level[MAX_LEVEL + lvl];
    const uint32_t p0 = max(A.rfirst[round], off), p1 = min(A.rfirst[round + 1], off + cnt);
    uint32_t moved = 0, merged = 0;
    for (uint32_t j = p0 + blockIdx.x; j < p1; j += gridDim.x) {
        const uint32_t q = A.pairs[2 * (uint64_t)j], v = A.pairs[2 * (uint64_t)j + 1];
        const uint32_t t = A.hbm_list[q];
        const uint32_t L = A.lpos[t], Mid = A.run_start[t + 1], R = A.rpos[t];
        const uint32_t vlo = v << A.logp;
        const uint32_t o0 = L > vlo ? L : vlo, o1 = R < vlo + P ? R : vlo + P;
        const uint32_t i0 = A.splits[2 * (uint64_t)j], i1 = A.splits[2 * (uint64_t)j + 1];
        const uint32_t j0 = (o0 - L) - i0, j1 = (o1 - L) - i1;
        const uint32_t up = A.upage[j];
        if (up >= A.N || !A.need[up]) continue;  // kept in place (or counted by k_vm_release)
        const uint32_t np = A.S[A.fidx[up]];
        K* dk = pg.kp(np) + (o0 - vlo);
        uint32_t* dv = VAL ? pg.vp(np) + (o0 - vlo) : nullptr;
        // a range of at most P elements spans at most two pages
        const uint32_t xa = L + i0, xb = Mid + j0;
        const uint32_t pa = xa >> A.logp, pb = xb >> A.logp;
        const uint32_t pa1 = pa + 1 < A.N ? pa + 1 : pa, pb1 = pb + 1 < A.N ? pb + 1 : pb;
        const uint32_t qa0 = A.pt[pa], qa1 = A.pt[pa1], qb0 = A.pt[pb], qb1 = A.pt[pb1];
        const K* ka0 = pg.kp(qa0);
        const K* ka1 = pg.kp(qa1);
        const K* kb0 = pg.kp(qb0);
        const K* kb1 = pg.kp(qb1);
        const uint32_t* va0 = VAL ? pg.vp(qa0) : nullptr;
        const uint32_t* va1 = VAL ? pg.vp(qa1) : nullptr;
        const uint32_t* vb0 = VAL ? pg.vp(qb0) : nullptr;
        const uint32_t* vb1 = VAL ? pg.vp(qb1) : nullptr;
        const uint32_t na = i1 - i0, logp = A.logp;
        merge_tile_io<K, VAL, NT, KI>(
            na, j1 - j0,
            [=](uint32_t e) {
                const uint32_t x = xa + e;
                return ((x >> logp) == pa ? ka0 : ka1)[x & mask];
            },
            [=](uint32_t e) {
                const uint32_t x = xa + e;
                return ((x >> logp) == pa ? va0 : va1)[x & mask];
            },
            [=](uint32_t e) {
                const uint32_t x = xb + (e - na);
                return ((x >> logp) == pb ? kb0 : kb1)[x & mask];
            },
            [=](uint32_t e) {
                const uint32_t x = xb + (e - na);
                return ((x >> logp) == pb ? vb0 : vb1)[x & mask];
            },
            [=](uint32_t e, K k, uint32_t val) {
                dk[e] = k;
                if (VAL) dv[e] = val;
            },
            S, SV);
        merged += o1 - o0;
        // carried parts of the page: the gap before the node's start (up to
        // the end of a level node ending in the page) and, when no level
        // node starts after it in the page, the rest after its end
        uint32_t g0 = 0, g1 = 0, h0 = 0, h1 = 0;
        if (v == (L >> A.logp) && (L & mask)) {
            const uint64_t me = A.mark_end[v];
            g0 = (uint32_t)(me >> 32) == lvl ? (uint32_t)me : vlo;
            g1 = L;
        }
        if (v == ((R - 1) >> A.logp) && (R & mask)) {
            const uint64_t ms = A.mark_start[v];
            if ((uint32_t)(ms >> 32) != lvl) {
                h0 = R;
                h1 = vlo + P < A.n ? vlo + P : A.n;
            }
        }
        if (g1 > g0 || h1 > h0) {
            const uint32_t op = A.pt[v];
            const K* sk = pg.kp(op);
            const uint32_t* sv = VAL ? pg.vp(op) : nullptr;
            K* nk = pg.kp(np);
            uint32_t* nv = VAL ? pg.vp(np) : nullptr;
            for (uint32_t x = g0 + threadIdx.x; x < g1; x += NT) {
                nk[x - vlo] = sk[x - vlo];
                if (VAL) nv[x - vlo] = sv[x - vlo];
            }
            for (uint32_t x = h0 + threadIdx.x; x < h1; x += NT) {
                nk[x - vlo] = sk[x - vlo];
                if (VAL) nv[x - vlo] = sv[x - vlo];
            }
            moved += (g1 - g0) + (h1 - h0);
        }
    }
    if (threadIdx.x == 0 && moved) atomicAdd(&A.vs[VS_CARRY], (unsigned long long)moved);
    if (threadIdx.x == 0 && merged) atomicAdd(&A.vs[VS_MERGED], (unsigned long long)merged);
}

// The touched pages now live in their fresh pages; the free sequence's
// leftover is the next pool.
__global__ void k_vm_level_end(VmArgs A, uint32_t lvl)
{
    const uint32_t cnt = A.level[lvl], off = A.level[MAX_LEVEL + lvl];
    const uint32_t F = A.vc[VC_F], En = A.vc[VC_E_NEXT];
    const uint32_t m = cnt > En ? cnt : En;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < m; x += gridDim.x * blockDim.x) {
        if (x < cnt) {
            const uint32_t i = off + x;
            const uint32_t v = A.pairs[2 * (uint64_t)i + 1];
            const uint32_t up = A.upage[i];
            if ((x == 0 || A.pairs[2 * (uint64_t)(i - 1) + 1] != v) && up < A.N && A.need[up])
                A.pt[v] = A.S[A.fidx[up]];
        }
        if (x < En && F <= A.N) A.pool[x] = A.S[F + x];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && cnt) {
        atomicAdd(&A.vs[VS_LEVELS], 1ull);
        atomicAdd(&A.vs[VS_PAGE_WRITES], (unsigned long long)F);
    }
}

// ------------------------------------------------------------- Copy --
// head[v]: 0 none, 1 a multiple of VM_HEAD that holds a page (saved to
// tmp first), 2 start of a path (keys page v holds nothing), 3 least page of
// a cycle without a multiple of VM_HEAD (saved in registers).
__global__ void k_vm_inverse(const uint32_t* __restrict__ pt, uint32_t N, uint32_t nin, uint32_t* __restrict__ inv)
{
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < N; v += gridDim.x * blockDim.x) {
        const uint32_t p = pt[v];
        if (p < nin) inv[p] = v;
    }
}

template <typename K, bool VAL>
__global__ __launch_bounds__(VM_NT) void k_vm_copy_heads(VmArgs A, const uint32_t* __restrict__ inv,
                                                         uint8_t* __restrict__ head, K* __restrict__ tk,
                                                         uint32_t* __restrict__ tv)
{
    __shared__ uint32_t ty;
    const Pages<K> pg = pages_of<K>(A);
    const uint32_t P = 1u << A.logp;
    for (uint32_t v = blockIdx.x; v < A.N; v += gridDim.x) {
        if (threadIdx.x == 0) {
            const uint32_t p = A.pt[v];
            uint32_t type = 0;
            if (p == v) {
                type = 0;
            } else if (inv[v] == NONE) {
                type = 2;
            } else if (v % VM_HEAD == 0) {
                type = 1;
            } else {
                // follow the chain of sources: a multiple of VM_HEAD or a
                // pool page ends it; coming back to v means a cycle with
                // no multiple of VM_HEAD, headed by its least page
                // (the page table is one-to-one, so the walk ends within
                // N steps; the bound only keeps a broken table from
                // looping, and is counted as a schedule fault)
                uint32_t x = p, least = v, steps = 0;
                while (true) {
                    if (x >= A.nin || x % VM_HEAD == 0) break;
                    if (x == v) {
                        type = least == v ? 3u : 0u;
                        break;
                    }
                    if (++steps > A.N) {
                        atomicAdd(&A.vs[VS_BAD], 1ull);
                        break;
                    }
                    least = x < least ? x : least;
                    x = A.pt[x];
                }
            }
            head[v] = (uint8_t)type;
            ty = type;
        }
        __syncthreads();
        if (ty == 1) {
            // page v holds virtual page inv[v]; its length
            const uint32_t w = inv[v];
            const uint32_t len = w == A.N - 1 ? A.n - (w << A.logp) : P;
            const K* sk = pg.kp(v);
            K* dk = tk + (uint64_t)(v / VM_HEAD) * P;
            for (uint32_t i = threadIdx.x; i < len; i += VM_NT) {
                dk[i] = sk[i];
                if (VAL) tv[(uint64_t)(v / VM_HEAD) * P + i] = pg.vp(v)[i];
            }
        }
        __syncthreads();
    }
}

// Every head walks its segment: page x takes the contents of page pt[x],
// then x = pt[x], until the source is a pool page, a saved head or the
// segment's own head.  The next page's contents are loaded before the
// current one is stored (the next source is never the page being stored:
// that would close a two-page cycle, which a walk from its head does not
// run into), so each step's load latency overlaps the previous store.
template <typename K, bool VAL, int PER>
__global__ __launch_bounds__(VM_NT) void k_vm_copy_move(VmArgs A, const uint32_t* __restrict__ inv,
                                                        const uint8_t* __restrict__ head, const K* __restrict__ tk,
                                                        const uint32_t* __restrict__ tv)
{
    const Pages<K> pg = pages_of<K>(A);
    const uint32_t P = 1u << A.logp;
    const uint32_t tid = threadIdx.x;
    uint32_t moved = 0;
    for (uint32_t v = blockIdx.x; v < A.N; v += gridDim.x) {
        const uint32_t type = head[v];
        if (type == 0) continue;
        K hk[PER], ck[PER], nk[PER];
        uint32_t hv[PER], cv[PER], nv[PER];
        // contents destined for page x, from page s (or its saved copy)
        auto fetch = [&](uint32_t s, uint32_t x, K* rk, uint32_t* rv) {
            const uint32_t len = x == A.N - 1 ? A.n - (x << A.logp) : P;
            if (s == v && type == 3) {
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    rk[j] = hk[j];
                    if (VAL) rv[j] = hv[j];
                }
                return;
            }
            const bool saved = s < A.nin && head[s] == 1;
            const K* sk = saved ? tk + (uint64_t)(s / VM_HEAD) * P : pg.kp(s);
            const uint32_t* sv = VAL ? (saved ? tv + (uint64_t)(s / VM_HEAD) * P : pg.vp(s)) : nullptr;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const uint32_t i = tid + (uint32_t)j * VM_NT;
                rk[j] = i < len ? sk[i] : K(0);
                if (VAL) rv[j] = i < len ? sv[i] : 0u;
            }
        };
        auto put = [&](uint32_t x, const K* rk, const uint32_t* rv) {
            const uint32_t len = x == A.N - 1 ? A.n - (x << A.logp) : P;
            K* dk = pg.kp(x);
            uint32_t* dv = VAL ? pg.vp(x) : nullptr;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const uint32_t i = tid + (uint32_t)j * VM_NT;
                if (i < len) {
                    dk[i] = rk[j];
                    if (VAL) dv[i] = rv[j];
                }
            }
            moved += len;
        };
        if (type == 3) {
            // page v holds the page that ends this cycle: keep it in
            // registers (every thread its columns)
            const uint32_t w = inv[v];
            const uint32_t wl = w == A.N - 1 ? A.n - (w << A.logp) : P;
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const uint32_t i = tid + (uint32_t)j * VM_NT;
                hk[j] = i < wl ? pg.kp(v)[i] : K(0);
                if (VAL) hv[j] = i < wl ? pg.vp(v)[i] : 0u;
            }
        }
        uint32_t x = v, s = A.pt[v], steps = 0;
        fetch(s, x, ck, cv);
        while (++steps <= A.N + 1) {
            const bool end = s >= A.nin || s == v || head[s] == 1;
            if (end) {
                put(x, ck, cv);
                break;
            }
            const uint32_t s2 = A.pt[s];
            fetch(s2, s, nk, nv);
            put(x, ck, cv);
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                ck[j] = nk[j];
                if (VAL) cv[j] = nv[j];
            }
            x = s;
            s = s2;
        }
    }
    if (tid == 0 && moved) atomicAdd(&A.vs[VS_COPY], (unsigned long long)moved);
}

__global__ void k_vm_zero_stats(VmArgs A)
{
    if (threadIdx.x < VS_COUNT) A.vs[threadIdx.x] = 0;
}

__global__ void k_vm_stats_out(const VmArgs A, unsigned long long* out)
{
    if (threadIdx.x < VS_COUNT) out[threadIdx.x] = A.vs[threadIdx.x];
}

// ------------------------------------------------------------ layout --
struct VmLayout {
    uint32_t P, logp, N, nin, W, emax, ntmp, rmax;
    uint64_t order_blocks, pair_cap;
    size_t plan, kpool, vpool, ktmp, vtmp, pt, inv, S, pool, rel, need, fidx, oldp, bins, boff, cursor, rfirst, mstart,
        mend,
        head, bsum, bscan, pflag, gpage, upage, scan, vc, vs, total;
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

static VmLayout vm_layout(uint64_t n, int kb, int has_values, uint64_t window_pages)
{
    VmLayout L{};
    const uint32_t T = tilesort_capacity(kb, has_values);
    L.P = merge_tile_default(kb, has_values);
    L.logp = 0;
    while ((1u << L.logp) < L.P) ++L.logp;
    L.N = (uint32_t)ceil_div(n ? n : 1, L.P);
    L.nin = L.N;
    uint64_t W = window_pages ? window_pages : (L.N / 16 > 64 ? L.N / 16 : 64);
    if (W > L.N) W = L.N;
    if (W < 1) W = 1;
    L.W = (uint32_t)W;
    L.emax = L.W + 9;
    L.ntmp = (uint32_t)ceil_div(L.N, VM_HEAD);
    L.rmax = (uint32_t)ceil_div(L.N, L.W) + 1;
    const size_t kbytes = kb / 8;
    Plan probe;
    const uint32_t ml = n > 0 ? minrun_of(n) : 1u;
    const size_t plan_bytes = plan_workspace_bytes(n, 1, T, L.P, ml);
    plan_carve(probe, nullptr, n, 1, T, L.P, ml);
    L.pair_cap = probe.pair_cap;
    L.order_blocks = plan_order_blocks(probe);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = a256(o + bytes); return at; };
    L.plan = take(plan_bytes);
    L.kpool = take(kbytes * L.emax * L.P);
    L.vpool = has_values ? take(4ull * L.emax * L.P) : 0;
    L.ktmp = take(kbytes * L.ntmp * L.P);
    L.vtmp = has_values ? take(4ull * L.ntmp * L.P) : 0;
    L.pt = take(4ull * L.N);
    L.inv = take(4ull * L.nin);
    L.S = take(4ull * (L.N + L.emax));
    L.pool = take(4ull * L.emax);
    L.rel = take(4ull * L.N);
    L.need = take(4ull * L.N);
    L.fidx = take(4ull * L.N);
    L.oldp = take(4ull * L.N);
    L.bins = take(4ull * (L.rmax + 2));
    L.boff = take(4ull * (L.rmax + 2));
    L.cursor = take(4ull * (L.rmax + 2));
    L.rfirst = take(4ull * (L.rmax + 2));
    L.mstart = take(8ull * L.N);
    L.mend = take(8ull * L.N);
    L.head = take(L.N);
    L.bsum = take(4ull * MAX_LEVEL * L.order_blocks);
    L.bscan = take(4ull * MAX_LEVEL * L.order_blocks);
    L.pflag = take(4ull * L.pair_cap);
    L.gpage = take(4ull * L.pair_cap);
    L.upage = take(4ull * L.pair_cap);
    const uint64_t sc = (uint64_t)MAX_LEVEL * L.order_blocks > L.pair_cap ? (uint64_t)MAX_LEVEL * L.order_blocks
                                                                          : L.pair_cap;
    L.scan = take(4ull * scan_tmp_words(sc));
    L.vc = take(4ull * VC_COUNT);
    L.vs = take(8ull * VS_COUNT);
    L.total = o;
    return L;
}

size_t vm_workspace_bytes(uint64_t n, int key_bits, int has_values, uint64_t window_pages)
{
    return vm_layout(n, key_bits, has_values, window_pages).total;
}

size_t vm_buffer_bytes(uint64_t n, int key_bits, int has_values, uint64_t window_pages)
{
    const VmLayout L = vm_layout(n, key_bits, has_values, window_pages);
    return L.pt - L.kpool;  // pool and copy pages (keys and values)
}

uint32_t vm_page_elems(int key_bits, int has_values) { return merge_tile_default(key_bits, has_values); }

uint64_t vm_window_pages(uint64_t n, int key_bits, int has_values, uint64_t window_pages)
{
    return vm_layout(n, key_bits, has_values, window_pages).W;
}

// ------------------------------------------------------------ driver --
template <typename K, bool VAL, int NT, int KI>
static hipError_t vm_levels(const Plan& P, const VmArgs& A, uint32_t* scan, hipStream_t s)
{
    constexpr uint32_t TO = NT * KI;
    constexpr size_t lds = (sizeof(K) + (VAL ? sizeof(uint32_t) : 0)) * MergeLds<TO>::SP;
    static bool attr_set[16] = {};
    int dev = 0;
    VMPS_HIP(hipGetDevice(&dev));
    if (!attr_set[dev & 15]) {
        VMPS_HIP(hipFuncSetAttribute((const void*)k_vm_round<K, VAL, NT, KI>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev & 15] = true;
    }
    // higher levels hold no merge longer than T: no pair, no page touched
    const uint32_t top = hbm_top_level(P.n, P.T);
    const uint64_t most = (uint64_t)P.n_tiles_out + 2 * ((uint64_t)P.n / (P.T ? P.T : 1) + 1);
    const unsigned pgrid = (unsigned)(ceil_div(2 * most, 256) < 256 ? ceil_div(2 * most, 256) : 256);
    const unsigned lgrid = (unsigned)(ceil_div(most + A.emax, 256) < 1024 ? ceil_div(most + A.emax, 256) : 1024);
    const unsigned rgrid = (unsigned)(2ull * A.W < 4096 ? 2ull * A.W : 4096);
    for (int lvl = (int)top; lvl >= 1; --lvl) {
        k_vm_partition<K><<<pgrid, 256, 0, s>>>(A, (uint32_t)lvl);
        k_vm_keep<<<lgrid, 256, 0, s>>>(A, (uint32_t)lvl);
        VMPS_HIP(scan_exclusive_u32(A.need, A.fidx, A.N, A.vc + VC_U, A.vc + VC_F, scan, s));
        k_vm_release<<<lgrid, 256, 0, s>>>(A, (uint32_t)lvl);
        k_vm_bins<<<1, 1024, 0, s>>>(A);
        k_vm_fill<<<lgrid, 256, 0, s>>>(A);
        for (uint32_t r = 0; r + 1 < A.rmax; ++r)
            k_vm_round<K, VAL, NT, KI><<<rgrid, NT, lds, s>>>(A, (uint32_t)lvl, r);
        k_vm_level_end<<<lgrid, 256, 0, s>>>(A, (uint32_t)lvl);
    }
    return hipGetLastError();
}

template <typename K, bool VAL>
static hipError_t vm_copy(const VmArgs& A, uint32_t* inv, uint8_t* head, void* tk, uint32_t* tv, hipStream_t s)
{
    VMPS_HIP(fill_u32(inv, NONE, A.nin, s));
    k_vm_inverse<<<(unsigned)ceil_div(A.N, 256), 256, 0, s>>>(A.pt, A.N, A.nin, inv);
    const unsigned g = A.N < 65536 ? A.N : 65536;
    k_vm_copy_heads<K, VAL><<<g, VM_NT, 0, s>>>(A, inv, head, (K*)tk, tv);
    const uint32_t P = 1u << A.logp;
    if (P / VM_NT == 16) k_vm_copy_move<K, VAL, 16><<<g, VM_NT, 0, s>>>(A, inv, head, (const K*)tk, tv);
    else k_vm_copy_move<K, VAL, 8><<<g, VM_NT, 0, s>>>(A, inv, head, (const K*)tk, tv);
    return hipGetLastError();
}

__global__ void k_vm_single_segment(uint32_t* inst_start, uint32_t n, Seg* segs, uint32_t* counters)
{
    inst_start[0] = 0;
    inst_start[1] = n;
    Seg sg;
    sg.start = 0; sg.end = n; sg.inst = 0; sg.dst = 0;
    segs[0] = sg;
    for (int c = 0; c < CNT_COUNT; ++c) counters[c] = 0;
    counters[CNT_NSEG] = 1;
}

template <typename K, bool VAL, int NT, int KI>
static hipError_t vm_sort_t(void* keys, uint32_t* values, uint64_t n, int vmode, uint32_t desc,
                            uint64_t window_pages, uint8_t* w, unsigned long long* stats, hipStream_t s)
{
    const int kb = (int)sizeof(K) * 8;
    const VmLayout L = vm_layout(n, kb, VAL ? 1 : 0, window_pages);
    Plan P;
    const uint32_t T = tilesort_capacity(kb, VAL ? 1 : 0);
    plan_carve(P, w + L.plan, n, 1, T, L.P, minrun_of(n));
    P.big_min = T;
    P.desc = desc;
    VmArgs A{};
    A.vc = (uint32_t*)(w + L.vc);
    A.vs = (unsigned long long*)(w + L.vs);
    A.n = (uint32_t)n;
    A.N = L.N;
    A.nin = L.nin;
    A.logp = L.logp;
    A.W = L.W;
    A.rmax = L.rmax;
    if (n <= T) {
        // one LDS segment, sorted in place; no page is ever touched
        k_vm_single_segment<<<1, 1, 0, s>>>(P.inst_start, (uint32_t)n, P.segs, P.counters);
        VMPS_HIP(tilesort_enqueue(P, keys, keys, values, values, kb, vmode, 0, s));
        if (stats) {
            k_vm_zero_stats<<<1, 64, 0, s>>>(A);
            k_vm_stats_out<<<1, 64, 0, s>>>(A, stats);
        }
        return hipGetLastError();
    }
    A.level = P.level;
    A.pairs = P.pairs;
    A.hbm_list = P.hbm_list;
    A.lpos = P.bnd_lpos;
    A.rpos = P.bnd_rpos;
    A.run_start = P.run_start;
    A.node_base = P.node_base;
    A.tiles = P.hbm_tiles;
    A.splits = P.splits;
    A.upage = (const uint32_t*)(w + L.upage);
    A.keys = keys;
    A.kpool = w + L.kpool;
    A.vals = values;
    A.vpool = VAL ? (uint32_t*)(w + L.vpool) : nullptr;
    A.pt = (uint32_t*)(w + L.pt);
    A.S = (uint32_t*)(w + L.S);
    A.pool = (uint32_t*)(w + L.pool);
    A.rel = (uint32_t*)(w + L.rel);
    A.need = (uint32_t*)(w + L.need);
    A.fidx = (uint32_t*)(w + L.fidx);
    A.oldp = (uint32_t*)(w + L.oldp);
    A.bins = (uint32_t*)(w + L.bins);
    A.boff = (uint32_t*)(w + L.boff);
    A.cursor = (uint32_t*)(w + L.cursor);
    A.rfirst = (uint32_t*)(w + L.rfirst);
    A.mark_start = (uint64_t*)(w + L.mstart);
    A.mark_end = (uint64_t*)(w + L.mend);
    uint32_t* C = P.counters;
    uint32_t* scan = (uint32_t*)(w + L.scan);
    uint32_t* pflag = (uint32_t*)(w + L.pflag);
    uint32_t* gpage = (uint32_t*)(w + L.gpage);

    VMPS_HIP(plan_enqueue(P, keys, kb, 0, s));
    k_vm_segs_in_place<<<(unsigned)(ceil_div(P.seg_cap, 256) < 2048 ? ceil_div(P.seg_cap, 256) : 2048), 256, 0, s>>>(
        P.segs, C, P.seg_cap);
    VMPS_HIP(tilesort_enqueue(P, keys, keys, values, values, kb, vmode, 0, s));
    VMPS_HIP(plan_order_levels(P, (uint32_t*)(w + L.bsum), (uint32_t*)(w + L.bscan), scan, s));
    const unsigned pg = (unsigned)(ceil_div(P.pair_cap, 256) < 2048 ? ceil_div(P.pair_cap, 256) : 2048);
    k_vm_page_flags<<<pg, 256, 0, s>>>(P.pairs, P.hbm_list, P.power, C, P.pair_cap, pflag);
    VMPS_HIP(scan_exclusive_u32(pflag, gpage, P.pair_cap, C + CNT_NPAIRS, nullptr, scan, s));
    k_vm_upage<<<pg, 256, 0, s>>>(P.pairs, P.hbm_list, P.power, P.level, C, P.pair_cap, pflag, gpage,
                                  (uint32_t*)(w + L.upage));
    A.emax = L.emax;
    k_vm_init<<<(unsigned)(ceil_div(L.N, 256) < 2048 ? ceil_div(L.N, 256) : 2048), 256, 0, s>>>(A, L.emax);
    VMPS_HIP((vm_levels<K, VAL, NT, KI>(P, A, scan, s)));
    VMPS_HIP((vm_copy<K, VAL>(A, (uint32_t*)(w + L.inv), w + L.head, w + L.ktmp,
                               VAL ? (uint32_t*)(w + L.vtmp) : nullptr, s)));
    if (stats) k_vm_stats_out<<<1, 64, 0, s>>>(A, stats);
    return hipGetLastError();
}

hipError_t vm_sort_enqueue(void* keys, uint32_t* values, uint64_t n, int key_bits, int vmode, uint32_t desc,
                           uint64_t window_pages, void* ws, unsigned long long* stats, hipStream_t s)
{
    uint8_t* w = (uint8_t*)ws;
    if (key_bits == 32) {
        if (values) return vm_sort_t<uint32_t, true, 256, 16>(keys, values, n, vmode, desc, window_pages, w, stats, s);
        return vm_sort_t<uint32_t, false, 256, 16>(keys, values, n, vmode, desc, window_pages, w, stats, s);
    }
    if (values) return vm_sort_t<uint64_t, true, 256, 8>(keys, values, n, vmode, desc, window_pages, w, stats, s);
    return vm_sort_t<uint64_t, false, 256, 16>(keys, values, n, vmode, desc, window_pages, w, stats, s);
}

}  // namespace vmps
