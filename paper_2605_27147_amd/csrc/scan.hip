// Device-wide exclusive scan of u32 counts and a fill kernel.
//
// Per-block sums, then per-block scan plus offset.  Up to SCAN_FUSED
// blocks, each block of the second launch sums the block sums before it
// (and block 0 all of them, for the total); beyond that a single workgroup
// scans the block sums in a launch of its own.  The element count may live
// in device memory (written by an earlier kernel), so no host round trip is
// needed.
#include "vmps_internal.hpp"

namespace vmps {

constexpr int SCAN_NT = 256;
constexpr int SCAN_PER = 16;
constexpr uint32_t SCAN_BLOCK = SCAN_NT * SCAN_PER;  // 4096 elements per block

// The count is clamped to the capacity the launch was sized for.
__device__ inline uint64_t scan_count(uint64_t host, const uint32_t* dev)
{
    if (!dev) return host;
    const uint64_t c = *dev;
    return c < host ? c : host;
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_reduce(const uint32_t* in, uint64_t count_host,
                                                         const uint32_t* count_dev, uint32_t* sums)
{
    __shared__ uint32_t lds[SCAN_NT / WAVE + 1];
    const uint64_t count = scan_count(count_host, count_dev);
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK;
    if (base >= count) {
        if (threadIdx.x == 0) sums[blockIdx.x] = 0;
        return;
    }
    uint32_t acc = 0;
    for (int j = 0; j < SCAN_PER; ++j) {
        uint64_t i = base + (uint64_t)j * SCAN_NT + threadIdx.x;
        if (i < count) acc += in[i];
    }
    uint32_t tot;
    block_excl_scan(acc, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One workgroup scans nblocks block sums in place.
__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* sums, uint64_t nblocks, uint32_t* total)
{
    __shared__ uint32_t lds[1024 / WAVE + 1];
    uint32_t carry = 0;
    for (uint64_t b0 = 0; b0 < nblocks; b0 += 1024) {
        uint64_t i = b0 + threadIdx.x;
        uint32_t v = i < nblocks ? sums[i] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, lds, &tot);
        if (i < nblocks) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

constexpr uint64_t SCAN_FUSED = 2048;  // block sums read by each block at most

// Sum of a[0, m) by the whole block.
__device__ inline uint32_t block_sum(const uint32_t* a, uint32_t m, uint32_t* lds)
{
    uint32_t acc = 0;
    for (uint32_t i = threadIdx.x; i < m; i += SCAN_NT) acc += a[i];
    uint32_t tot;
    block_excl_scan(acc, lds, &tot);
    return tot;
}

// FUSED: sums holds the block sums (the offset of a block is the sum of
// those before it); otherwise their exclusive scan.
template <bool FUSED>
__global__ __launch_bounds__(SCAN_NT) void k_scan_down(const uint32_t* in, uint32_t* out,
                                                       uint64_t count_host, const uint32_t* count_dev,
                                                       const uint32_t* sums, uint32_t nblocks, uint32_t* total)
{
    __shared__ uint32_t lds[SCAN_NT / WAVE + 1];
    __shared__ uint32_t buf[SCAN_BLOCK];
    const uint64_t count = scan_count(count_host, count_dev);
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK;
    if (FUSED && blockIdx.x == 0) {
        const uint32_t all = block_sum(sums, nblocks, lds);
        if (threadIdx.x == 0 && total) *total = all;
    }
    if (base >= count) return;
    const uint32_t offset = FUSED ? block_sum(sums, blockIdx.x, lds) : sums[blockIdx.x];
    // coalesced load of the block into LDS; thread t then owns the SCAN_PER
    // consecutive elements [SCAN_PER t, SCAN_PER t + SCAN_PER)
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const uint64_t i = base + (uint64_t)j * SCAN_NT + threadIdx.x;
        buf[j * SCAN_NT + threadIdx.x] = i < count ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[SCAN_PER];
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        v[j] = buf[threadIdx.x * SCAN_PER + j];
        acc += v[j];
    }
    uint32_t ex = block_excl_scan(acc, lds, nullptr) + offset;
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        buf[threadIdx.x * SCAN_PER + j] = ex;
        ex += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SCAN_PER; ++j) {
        const uint64_t i = base + (uint64_t)j * SCAN_NT + threadIdx.x;
        if (i < count) out[i] = buf[j * SCAN_NT + threadIdx.x];
    }
}

uint64_t scan_tmp_words(uint64_t count) { return ceil_div(count > 0 ? count : 1, SCAN_BLOCK) + 1; }

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t count_host,
                              const uint32_t* count_dev, uint32_t* total, uint32_t* tmp,
                              hipStream_t s)
{
    // count_host is the capacity when count_dev is given
    const uint64_t nblocks = ceil_div(count_host > 0 ? count_host : 1, SCAN_BLOCK);
    k_scan_reduce<<<(unsigned)nblocks, SCAN_NT, 0, s>>>(in, count_host, count_dev, tmp);
    if (nblocks <= SCAN_FUSED) {
        k_scan_down<true><<<(unsigned)nblocks, SCAN_NT, 0, s>>>(in, out, count_host, count_dev, tmp,
                                                                (uint32_t)nblocks, total);
    } else {
        k_scan_top<<<1, 1024, 0, s>>>(tmp, nblocks, total);
        k_scan_down<false><<<(unsigned)nblocks, SCAN_NT, 0, s>>>(in, out, count_host, count_dev, tmp,
                                                                 (uint32_t)nblocks, nullptr);
    }
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    uint64_t blocks = ceil_div(count, 256);
    if (blocks > 8192) blocks = 8192;
    k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}

}  // namespace vmps
