// Stable merge of two sorted ranges through LDS (StandardMerge of
// Algorithm 2: an element of the left range precedes an equal element of the
// right one), shared by the merge levels, the paged merge levels, the
// two-array merge and the LDS tile pass.
#pragma once
#include "vmps_internal.hpp"

namespace vmps {

// Number of elements of a among the first d outputs of the stable merge.
template <typename K>
__device__ inline uint32_t merge_path(const K* __restrict__ a, uint32_t na, const K* __restrict__ b,
                                      uint32_t nb, uint32_t d)
{
    uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= b[d - 1 - mid]) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// LDS slot of element i: one spare slot after every 32 elements, so that a
// wave writing KI consecutive elements per lane spreads over the banks.
__device__ __forceinline__ uint32_t mpx(uint32_t i) { return i + (i >> 5); }

// LDS slots for a tile of TO elements (with slack for the reads one past the
// end of the merge).
template <uint32_t TO>
struct MergeLds {
    static constexpr uint32_t SP = TO + TO / 32 + 64;
};

// Merge na elements of a and nb of b into out[0, na + nb) through LDS:
// all loads of the tile in flight at once, a merge-path split per thread,
// KI outputs per thread into registers (ties to a), then back through the
// same LDS buffer for coalesced stores (merge_tile below, with its inputs
// and output reached through functors instead of pointers; the paged merge
// levels use it): for a tile index e (a's elements first, then b's), ka(e) /
// kb(e) give the key of element e of a / element e - na of b, va(e) / vb(e)
// its value (called only when VAL); store(e, k, v) writes output e.
template <typename K, bool VAL, int NT, int KI, typename KA, typename VA, typename KB, typename VB, typename ST>
__device__ inline void merge_tile_io(uint32_t na, uint32_t nb, KA ka, VA va, KB kb, VB vb, ST store, K* S,
                                     uint32_t* SV)
{
    static_assert(NT % 32 == 0 && 32 % KI == 0, "affine padded indices");
    const uint32_t nt = na + nb;
    const uint32_t tid = threadIdx.x, pt = mpx(tid);
    {
        K r[KI];
        uint32_t v[KI];
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const uint32_t e = (uint32_t)j * NT + tid;
            r[j] = e < na ? ka(e) : (e < nt ? kb(e) : K(0));
            if (VAL) v[j] = e < na ? va(e) : (e < nt ? vb(e) : 0u);
        }
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const uint32_t e = (uint32_t)j * NT + tid, pe = pt + (uint32_t)j * (NT + NT / 32);
            if (e < nt) {
                S[pe] = r[j];
                if (VAL) SV[pe] = v[j];
            }
        }
    }
    __syncthreads();
    const uint32_t d = tid * KI;
    K rk[KI];
    uint32_t rv[KI];
    if (d < nt) {
        uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (S[mpx(mid)] <= S[mpx(na + d - 1 - mid)]) lo = mid + 1; else hi = mid;
        }
        uint32_t pa = lo, pb = na + (d - lo);
        K ha = S[mpx(pa)], hb = S[mpx(pb)];
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const bool takeA = pa < na && (pb >= nt || ha <= hb);
            const uint32_t cur = takeA ? pa : pb;
            rk[j] = takeA ? ha : hb;
            if (VAL) rv[j] = SV[mpx(cur)];
            const uint32_t nx = cur + 1;  // at most nt + KI: inside the slack
            pa = takeA ? nx : pa;
            pb = takeA ? pb : nx;
            const K nv = S[mpx(nx)];
            ha = takeA ? nv : ha;
            hb = takeA ? hb : nv;
        }
    }
    __syncthreads();
    if (d < nt) {
        const uint32_t w0 = mpx(d);  // the KI outputs share one padding block
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            if (d + j < nt) {
                S[w0 + j] = rk[j];
                if (VAL) SV[w0 + j] = rv[j];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KI; ++j) {
        const uint32_t e = (uint32_t)j * NT + tid, pe = pt + (uint32_t)j * (NT + NT / 32);
        if (e < nt) store(e, S[pe], VAL ? SV[pe] : 0u);
    }
    __syncthreads();
}

// Merge a[i0,i1) and b[j0,j1) into out[0, (i1-i0)+(j1-j0)) through LDS:
// all loads of the tile in flight at once, a merge-path split per thread,
// KI outputs per thread into registers (ties to a), then back through the
// same LDS buffer for coalesced stores.
template <typename K, bool VAL, int NT, int KI>
__device__ inline void merge_tile(const K* __restrict__ a, const uint32_t* __restrict__ va, uint32_t i0,
                                  uint32_t i1, const K* __restrict__ b, const uint32_t* __restrict__ vb,
                                  uint32_t j0, uint32_t j1, K* __restrict__ out, uint32_t* __restrict__ vout,
                                  K* S, uint32_t* SV)
{
    static_assert(NT % 32 == 0 && 32 % KI == 0, "affine padded indices");
    const uint32_t na = i1 - i0, nb = j1 - j0, nt = na + nb;
    const uint32_t tid = threadIdx.x, pt = mpx(tid);
    {
        K r[KI];
        uint32_t v[KI];
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const uint32_t e = (uint32_t)j * NT + tid;
            r[j] = e < na ? a[i0 + e] : (e < nt ? b[j0 + e - na] : K(0));
            if (VAL) v[j] = e < na ? va[i0 + e] : (e < nt ? vb[j0 + e - na] : 0u);
        }
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const uint32_t e = (uint32_t)j * NT + tid, pe = pt + (uint32_t)j * (NT + NT / 32);
            if (e < nt) {
                S[pe] = r[j];
                if (VAL) SV[pe] = v[j];
            }
        }
    }
    __syncthreads();
    const uint32_t d = tid * KI;
    K rk[KI];
    uint32_t rv[KI];
    if (d < nt) {
        uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (S[mpx(mid)] <= S[mpx(na + d - 1 - mid)]) lo = mid + 1; else hi = mid;
        }
        uint32_t pa = lo, pb = na + (d - lo);
        K ha = S[mpx(pa)], hb = S[mpx(pb)];
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            const bool takeA = pa < na && (pb >= nt || ha <= hb);
            const uint32_t cur = takeA ? pa : pb;
            rk[j] = takeA ? ha : hb;
            if (VAL) rv[j] = SV[mpx(cur)];
            const uint32_t nx = cur + 1;  // at most nt + KI: inside the slack
            pa = takeA ? nx : pa;
            pb = takeA ? pb : nx;
            const K nv = S[mpx(nx)];
            ha = takeA ? nv : ha;
            hb = takeA ? hb : nv;
        }
    }
    __syncthreads();
    if (d < nt) {
        const uint32_t w0 = mpx(d);  // the KI outputs share one padding block
#pragma unroll
        for (int j = 0; j < KI; ++j) {
            if (d + j < nt) {
                S[w0 + j] = rk[j];
                if (VAL) SV[w0 + j] = rv[j];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KI; ++j) {
        const uint32_t e = (uint32_t)j * NT + tid, pe = pt + (uint32_t)j * (NT + NT / 32);
        if (e < nt) {
            out[e] = S[pe];
            if (VAL) vout[e] = SV[pe];
        }
    }
    __syncthreads();
}

}  // namespace vmps
