// Large records (the record types of the paper's experiments, Sec. 5: 30
// 32-bit words moved as one element): a stable sort of records by a key
// field, done as a sort of (key, index) pairs followed by one gather of the
// records, so each record moves twice (read, write) instead of once per
// merge it takes part in (hypothesis H4: avoiding moves helps large
// objects).
#include "vmps_internal.hpp"

namespace vmps {

// keys[i] = the key field of record i (records of `rb` bytes, the key at
// byte `off`, aligned to its size).
template <typename K>
__global__ void k_rec_keys(const uint8_t* __restrict__ in, uint64_t n, uint32_t rb, uint32_t off,
                           K* __restrict__ keys)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        keys[i] = *(const K*)(in + i * rb + off);
}

// out record i = in record perm[i], word by word (W words of type Wd per
// record): consecutive threads take consecutive words, so each record is
// read and written as one contiguous run.
template <typename Wd>
__global__ void k_rec_gather(const Wd* __restrict__ in, const uint32_t* __restrict__ perm, uint64_t n, uint32_t W,
                             Wd* __restrict__ out)
{
    const uint64_t total = n * W;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = g / W;
        const uint32_t w = (uint32_t)(g - i * W);
        out[g] = in[(uint64_t)perm[i] * W + w];
    }
}

size_t records_workspace_bytes(uint64_t n, int key_bits)
{
    const size_t a = ((size_t)(key_bits / 8) * n + 255) & ~(size_t)255;
    const size_t b = (4 * (size_t)n + 255) & ~(size_t)255;
    return a + b;
}

hipError_t records_enqueue(const void* in, void* out, uint64_t n, uint32_t rb, uint32_t off, int key_bits,
                           uint32_t flags, void* ws, size_t sort_ws_bytes, hipStream_t s, vmps_status* st)
{
    uint8_t* w = (uint8_t*)ws;
    const size_t a = ((size_t)(key_bits / 8) * n + 255) & ~(size_t)255;
    void* keys = w;
    uint32_t* perm = (uint32_t*)(w + a);
    uint8_t* sort_ws = w + records_workspace_bytes(n, key_bits);
    const unsigned g = (unsigned)(ceil_div(n, 256) < 8192 ? ceil_div(n, 256) : 8192);
    if (key_bits == 32) k_rec_keys<uint32_t><<<g, 256, 0, s>>>((const uint8_t*)in, n, rb, off, (uint32_t*)keys);
    else k_rec_keys<uint64_t><<<g, 256, 0, s>>>((const uint8_t*)in, n, rb, off, (uint64_t*)keys);
    VMPS_HIP(hipGetLastError());
    *st = sort_in_workspace(keys, perm, (int64_t)n, key_bits == 32 ? VMPS_U32 : VMPS_U64,
                            VMPS_VALUES_IOTA | (flags & VMPS_DESCENDING_RUNS), sort_ws, sort_ws_bytes, s, false);
    if (*st != VMPS_OK) return hipSuccess;
    const uint64_t words8 = rb % 8 == 0 && ((uintptr_t)in & 7) == 0 && ((uintptr_t)out & 7) == 0;
    const uint64_t total = words8 ? n * (rb / 8) : n * (rb / 4);
    const unsigned gg = (unsigned)(ceil_div(total, 256) < 16384 ? ceil_div(total, 256) : 16384);
    if (words8) k_rec_gather<uint64_t><<<gg, 256, 0, s>>>((const uint64_t*)in, perm, n, rb / 8, (uint64_t*)out);
    else k_rec_gather<uint32_t><<<gg, 256, 0, s>>>((const uint32_t*)in, perm, n, rb / 4, (uint32_t*)out);
    return hipGetLastError();
}

}  // namespace vmps
