// vmps_sort_noalloc: the stable sort of vmps_sort with the workspace taken
// from a fixed device array of the library instead of the caller, for
// callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid hipMalloc).  Nothing here allocates: the array is
// part of the library's code object, one copy per GPU, held until the
// process ends.
#include <mutex>

#include "vmps_internal.hpp"

namespace {

// 96 MiB: every key type up to n = 2^22 (u64 keys with values need 82 MiB).
constexpr size_t SCRATCH_BYTES = 96ull << 20;

__device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

// Device address of `scratch` per device.  In host code the array's name is
// only a stand-in for the symbol, never a usable device address.
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

// Looks the address up once per device, with that device current.
hipError_t scratch_of(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t vmps_noalloc_scratch_bytes(void) { return SCRATCH_BYTES; }

vmps_status vmps_sort_noalloc(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags, void* stream)
{
    using namespace vmps;
    const vmps_status st = check_sort_args(keys, values, n, kt, flags);
    if (st != VMPS_OK) return st;
    size_t need = 0;
    if (vmps_sort_workspace_size(n, kt, values ? 1 : 0, &need) != VMPS_OK) return VMPS_ERR_INVALID_ARG;
    if (need > SCRATCH_BYTES) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return VMPS_ERR_DEVICE;
    void* ws = nullptr;
    if (scratch_of(dev, &ws) != hipSuccess) return VMPS_ERR_DEVICE;
    return sort_in_workspace(keys, values, n, kt, flags, ws, SCRATCH_BYTES, (hipStream_t)stream, false);
}

}  // extern "C"
