// C ABI of libvmps.so: argument checks, workspace carving, launch order.
#include <string.h>

#include "vmps_internal.hpp"

using namespace vmps;

struct vmps_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {
Tuning (&tuning_table())[2][2]
{
    static Tuning t[2][2] = {};
    return t;
}

// Captures what `enqueue` puts on a private stream into an instantiated graph.
template <typename F>
vmps_status capture_graph(vmps_graph* out, F enqueue)
{
    *out = nullptr;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return VMPS_ERR_DEVICE;
    const bool tracing = trace_suspend();
    vmps_status st = VMPS_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
        st = VMPS_ERR_DEVICE;
    } else {
        st = enqueue(cs);
        const hipError_t e = hipStreamEndCapture(cs, &g);
        if (st == VMPS_OK && e != hipSuccess) st = VMPS_ERR_DEVICE;
    }
    trace_resume(tracing);
    hipGraphExec_t ex = nullptr;
    if (st == VMPS_OK && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) st = VMPS_ERR_DEVICE;
    if (st != VMPS_OK) {
        if (g) (void)hipGraphDestroy(g);
    } else {
        *out = new vmps_graph_s{g, ex};
    }
    (void)hipStreamDestroy(cs);
    return st;
}


inline int key_bits_of(vmps_dtype kt) { return kt == VMPS_U64 ? 64 : 32; }
inline size_t key_bytes(vmps_dtype kt) { return kt == VMPS_U64 ? 8 : 4; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

inline vmps_status dev_status(hipError_t e) { return e == hipSuccess ? VMPS_OK : VMPS_ERR_DEVICE; }

// Workspace layout of a sort: [B keys][B values][plan]
struct SortLayout {
    size_t keys_b, vals_b, plan, total;
};

// One-array sorts with the minrun rule: every run but the last is at least
// minrun_of(n) long, which sizes the planner's run arrays.
static uint32_t rule_min_len(uint64_t n) { return n > 0 ? minrun_of(n) : 1u; }

SortLayout sort_layout(uint64_t n, uint64_t k, vmps_dtype kt, int has_values, uint32_t min_len, uint32_t T = 0)
{
    const int kb = key_bits_of(kt);
    SortLayout L;
    L.keys_b = 0;
    L.vals_b = align256(key_bytes(kt) * n);
    L.plan = L.vals_b + (has_values ? align256(4 * n) : 0);
    if (!T) T = tilesort_capacity(kb, has_values);
    const uint32_t TO = merge_tile_out(kb, has_values);
    L.total = L.plan + plan_workspace_bytes(n, k, T, TO, min_len);
    return L;
}

__global__ void k_single_segment(uint32_t* inst_start, uint32_t n, Seg* segs, uint32_t* counters)
{
    inst_start[0] = 0;
    inst_start[1] = n;
    Seg s;
    s.start = 0; s.end = n; s.inst = 0; s.dst = 0;
    segs[0] = s;
    for (int c = 0; c < CNT_COUNT; ++c) counters[c] = 0;
    counters[CNT_NSEG] = 1;
}

__global__ void k_write_zero_u32(uint32_t* p) { *p = 0; }
__global__ void k_write_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_powers(const uint32_t* __restrict__ bounds, const int64_t* __restrict__ num_runs, uint64_t n,
                         uint8_t* __restrict__ powers, uint64_t cap)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = *num_runs;
    if (r < 2 || t + 1 >= (uint64_t)r || t >= cap) return;
    const uint64_t i = bounds[t], j = bounds[t + 1], k = bounds[t + 2];
    const uint64_t A = ((i + j) << 31) / n, B = ((j + k) << 31) / n;
    powers[t] = (uint8_t)(__clz((uint32_t)(A ^ B)) + 1);
}

__global__ void k_export_runs(const uint32_t* __restrict__ run_start, const uint32_t* counters,
                              uint32_t* __restrict__ out, int64_t* num_runs, uint64_t cap)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nr = counters[CNT_NRUNS];
    if (t == 0) *num_runs = nr;
    if (t <= nr && t <= cap) out[t] = run_start[t];
}

__global__ void k_export_schedule(Plan P, uint32_t* node_l, uint32_t* node_m, uint32_t* node_r,
                                  uint8_t* node_level, uint8_t* node_buf, uint32_t* seg_start, uint32_t* seg_end,
                                  uint8_t* seg_buf, int64_t* counts)
{
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t h = P.counters[CNT_NHBM], ns = P.counters[CNT_NSEG];
    if (x == 0) {
        counts[0] = P.counters[CNT_NRUNS];
        counts[1] = h;
        counts[2] = ns;
        counts[3] = (int64_t)P.stats[0];
    }
    if (x < h) {
        const uint32_t t = P.hbm_list[x];
        node_l[x] = P.bnd_lpos[t];
        node_m[x] = P.run_start[t + 1];
        node_r[x] = P.bnd_rpos[t];
        node_level[x] = P.power[t];
        node_buf[x] = (uint8_t)(P.hbm_depth[x] & 1u);
    }
    if (x < ns) {
        seg_start[x] = P.segs[x].start;
        seg_end[x] = P.segs[x].end;
        seg_buf[x] = (uint8_t)P.segs[x].dst;
    }
}

template <typename F>
vmps_status guarded(F f)
{
    hipError_t e = f();
    if (e != hipSuccess) return VMPS_ERR_DEVICE;
    return dev_status(hipGetLastError());
}

vmps_status check_keys(const void* keys, int64_t n, vmps_dtype kt)
{
    if (n < 0 || (uint64_t)n >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    if (n > 0 && !keys) return VMPS_ERR_INVALID_ARG;
    if (keys && ((uintptr_t)keys % key_bytes(kt))) return VMPS_ERR_INVALID_ARG;
    return VMPS_OK;
}

}  // namespace

extern "C" {

const char* vmps_status_string(vmps_status s)
{
    switch (s) {
    case VMPS_OK: return "ok";
    case VMPS_ERR_INVALID_ARG: return "invalid argument";
    case VMPS_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case VMPS_ERR_UNSUPPORTED: return "unsupported";
    case VMPS_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

int32_t vmps_minrun(int64_t n) { return n <= 0 ? 0 : (int32_t)minrun_of((uint64_t)n); }

int64_t vmps_max_runs(int64_t n, int32_t minrun)
{
    if (n <= 0) return 0;
    (void)minrun;  // runs are at least 16 long except the last one
    return (int64_t)((uint64_t)n / 16 + 3);
}

vmps_status vmps_sort_workspace_size(int64_t n, vmps_dtype kt, int has_values, size_t* bytes)
{
    if (!bytes || n < 0 || (uint64_t)n >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    *bytes = sort_layout((uint64_t)n, 1, kt, has_values ? 1 : 0, rule_min_len((uint64_t)n)).total;
    return VMPS_OK;
}

vmps_status vmps_sort(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags, void* ws,
                      size_t ws_bytes, void* stream)
{
    const vmps_status st = check_sort_args(keys, values, n, kt, flags);
    if (st != VMPS_OK) return st;
    return sort_in_workspace(keys, values, n, kt, flags, ws, ws_bytes, (hipStream_t)stream, true);
}

vmps_status vmps_sort_records_workspace_size(int64_t n, vmps_dtype kt, size_t* bytes)
{
    if (!bytes || n < 0 || (uint64_t)n >= (1ull << 32) || (kt != VMPS_U32 && kt != VMPS_U64))
        return VMPS_ERR_INVALID_ARG;
    *bytes = records_workspace_bytes((uint64_t)n, key_bits_of(kt)) +
             sort_layout((uint64_t)n, 1, kt, 1, rule_min_len((uint64_t)n)).total;
    return VMPS_OK;
}

vmps_status vmps_sort_records(const void* records, void* out, int64_t n, int32_t record_bytes, int32_t key_offset,
                              vmps_dtype kt, uint32_t flags, void* ws, size_t ws_bytes, void* stream)
{
    if (n < 0 || (uint64_t)n >= (1ull << 32) || (kt != VMPS_U32 && kt != VMPS_U64)) return VMPS_ERR_INVALID_ARG;
    if (flags & ~VMPS_DESCENDING_RUNS) return VMPS_ERR_INVALID_ARG;
    const int32_t kbytes = (int32_t)key_bytes(kt);
    if (record_bytes < kbytes || record_bytes % 4 || key_offset < 0 || key_offset % kbytes ||
        key_offset + kbytes > record_bytes)
        return VMPS_ERR_INVALID_ARG;
    if (n == 0) return VMPS_OK;
    if (!records || !out || ((uintptr_t)records & 3) || ((uintptr_t)out & 3)) return VMPS_ERR_INVALID_ARG;
    if (kbytes == 8 && (record_bytes % 8 || ((uintptr_t)records & 7))) return VMPS_ERR_INVALID_ARG;
    const size_t total = (size_t)n * (size_t)record_bytes;
    if (ranges_overlap(records, total, out, total)) return VMPS_ERR_INVALID_ARG;
    size_t need = 0;
    vmps_sort_records_workspace_size(n, kt, &need);
    if (!ws || ws_bytes < need) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    const int kb = key_bits_of(kt);
    vmps_status st = VMPS_OK;
    const vmps_status g = guarded([&] {
        return records_enqueue(records, out, (uint64_t)n, (uint32_t)record_bytes, (uint32_t)key_offset, kb, flags, ws,
                               need - records_workspace_bytes((uint64_t)n, kb), (hipStream_t)stream, &st);
    });
    return g != VMPS_OK ? g : st;
}

vmps_status vmps_sort_vm_layout(int64_t n, vmps_dtype kt, int has_values, int64_t window_pages,
                                vmps_vm_layout* out)
{
    if (!out || n < 0 || (uint64_t)n >= (1ull << 32) || window_pages < 0) return VMPS_ERR_INVALID_ARG;
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    const int kb = key_bits_of(kt), hv = has_values ? 1 : 0;
    const uint64_t P = vm_page_elems(kb, hv);
    out->page_elems = (int64_t)P;
    out->pages = (int64_t)ceil_div(n > 0 ? (uint64_t)n : 1, P);
    out->window_pages = (int64_t)vm_window_pages((uint64_t)n, kb, hv, (uint64_t)window_pages);
    out->pool_pages = out->window_pages + 9;
    out->copy_pages = (int64_t)ceil_div((uint64_t)out->pages, 64);
    out->buffer_bytes = vm_buffer_bytes((uint64_t)n, kb, hv, (uint64_t)window_pages);
    out->workspace_bytes = vm_workspace_bytes((uint64_t)n, kb, hv, (uint64_t)window_pages);
    return VMPS_OK;
}

vmps_status vmps_sort_vm(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                         int64_t window_pages, void* ws, size_t ws_bytes, uint64_t* stats, void* stream)
{
    const vmps_status st = check_sort_args(keys, values, n, kt, flags);
    if (st != VMPS_OK) return st;
    if (window_pages < 0 || (stats && ((uintptr_t)stats & 7))) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n <= 1) {
        if (n == 1 && (flags & VMPS_VALUES_IOTA))
            return guarded([&] { k_write_zero_u32<<<1, 1, 0, s>>>(values); return hipGetLastError(); });
        return VMPS_OK;
    }
    const int kb = key_bits_of(kt), hv = values ? 1 : 0;
    if (!ws || ws_bytes < vm_workspace_bytes((uint64_t)n, kb, hv, (uint64_t)window_pages))
        return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    const int vmode = values ? ((flags & VMPS_VALUES_IOTA) ? 2 : 1) : 0;
    return guarded([&] {
        return vm_sort_enqueue(keys, values, (uint64_t)n, kb, vmode, (flags & VMPS_DESCENDING_RUNS) ? 1u : 0u,
                               (uint64_t)window_pages, ws, (unsigned long long*)stats, s);
    });
}

}  // extern "C"

namespace vmps {

vmps_status check_sort_args(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (flags & ~(VMPS_VALUES_IOTA | VMPS_DESCENDING_RUNS)) return VMPS_ERR_INVALID_ARG;
    if ((flags & VMPS_VALUES_IOTA) && !values && n > 0) return VMPS_ERR_INVALID_ARG;
    if (values && ((uintptr_t)values & 3)) return VMPS_ERR_INVALID_ARG;
    if (values && n > 0 && ranges_overlap(keys, key_bytes(kt) * n, values, 4 * (size_t)n)) return VMPS_ERR_INVALID_ARG;
    return VMPS_OK;
}

vmps_status sort_in_workspace(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags, void* ws,
                              size_t ws_bytes, hipStream_t s, bool allow_host_wait, bool fused_levels)
{
    if (n <= 1) {
        if (n == 1 && (flags & VMPS_VALUES_IOTA))
            return guarded([&] { k_write_zero_u32<<<1, 1, 0, s>>>(values); return hipGetLastError(); });
        return VMPS_OK;
    }
    const int has_values = values ? 1 : 0;
    const SortLayout L = sort_layout((uint64_t)n, 1, kt, has_values, rule_min_len((uint64_t)n));
    if (!ws || ws_bytes < L.total) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    const int kb = key_bits_of(kt);
    const int vmode = values ? ((flags & VMPS_VALUES_IOTA) ? 2 : 1) : 0;
    uint8_t* w = (uint8_t*)ws;
    void* keysB = w + L.keys_b;
    uint32_t* valsB = has_values ? (uint32_t*)(w + L.vals_b) : nullptr;
    Plan P;
    const uint32_t T = tilesort_capacity(kb, has_values);
    plan_carve(P, w + L.plan, (uint64_t)n, 1, T, merge_tile_out(kb, has_values), rule_min_len((uint64_t)n));
    P.big_min = T;
    P.desc = (flags & VMPS_DESCENDING_RUNS) ? 1u : 0u;
    return guarded([&]() -> hipError_t {
        if ((uint64_t)n <= T) {
            k_single_segment<<<1, 1, 0, s>>>(P.inst_start, (uint32_t)n, P.segs, P.counters);
            return tilesort_enqueue(P, keys, keysB, values, valsB, kb, vmode, 0, s);
        }
        VMPS_HIP(plan_enqueue(P, keys, kb, 0, s));
        VMPS_HIP(level_probe_enqueue(P, kb, has_values, s, allow_host_wait));
        VMPS_HIP(tilesort_enqueue(P, keys, keysB, values, valsB, kb, vmode, 0, s));
        // up to 2^20 elements a level holds at most a few hundred tiles,
        // about one per workgroup: the fused levels save the partition
        // launches at no cost
        const bool fused = fused_levels || (uint64_t)n <= (1ull << 20);
        return merge_levels_enqueue(P, keys, keysB, values, valsB, kb, has_values, s, fused);
    });
}

}  // namespace vmps

extern "C" {

vmps_status vmps_merge_workspace_size(int64_t na, int64_t nb, vmps_dtype kt, size_t* bytes)
{
    if (!bytes || na < 0 || nb < 0 || (uint64_t)(na + nb) >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    *bytes = align256(4 * (ceil_div((uint64_t)(na + nb), 4096) + 2));
    return VMPS_OK;
}

vmps_status vmps_merge(const void* a, const uint32_t* va, int64_t na, const void* b, const uint32_t* vb, int64_t nb,
                       void* out, uint32_t* vout, vmps_dtype kt, void* ws, size_t ws_bytes, void* stream)
{
    if (na < 0 || nb < 0 || (uint64_t)(na + nb) >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    vmps_status st = check_keys(a, na, kt);
    if (st == VMPS_OK) st = check_keys(b, nb, kt);
    if (st == VMPS_OK) st = check_keys(out, na + nb, kt);
    if (st != VMPS_OK) return st;
    const bool vals = va || vb || vout;
    if (vals && ((na > 0 && !va) || (nb > 0 && !vb) || (na + nb > 0 && !vout))) return VMPS_ERR_INVALID_ARG;
    const size_t kbytes = key_bytes(kt);
    if (na + nb > 0) {
        if (na > 0 && ranges_overlap(out, kbytes * (na + nb), a, kbytes * na)) return VMPS_ERR_INVALID_ARG;
        if (nb > 0 && ranges_overlap(out, kbytes * (na + nb), b, kbytes * nb)) return VMPS_ERR_INVALID_ARG;
    }
    size_t need = 0;
    vmps_merge_workspace_size(na, nb, kt, &need);
    if (na + nb == 0) return VMPS_OK;
    if (!ws || ws_bytes < need) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        return merge_two_enqueue(a, vals ? va : nullptr, (uint32_t)na, b, vals ? vb : nullptr, (uint32_t)nb, out,
                                 vals ? vout : nullptr, key_bits_of(kt), (uint32_t*)ws, s);
    });
}

static vmps_status extract_runs_impl(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun,
                                     uint32_t* run_bounds, int64_t* num_runs, void* ws, size_t ws_bytes,
                                     void* stream, bool desc);

vmps_status vmps_extract_runs(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun, uint32_t* run_bounds,
                              int64_t* num_runs, void* ws, size_t ws_bytes, void* stream)
{
    return extract_runs_impl(keys, n, kt, minrun, run_bounds, num_runs, ws, ws_bytes, stream, false);
}

vmps_status vmps_extract_runs_desc(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun, uint32_t* run_bounds,
                                   int64_t* num_runs, void* ws, size_t ws_bytes, void* stream)
{
    return extract_runs_impl(keys, n, kt, minrun, run_bounds, num_runs, ws, ws_bytes, stream, true);
}

static vmps_status extract_runs_impl(const void* keys, int64_t n, vmps_dtype kt, int32_t minrun,
                                     uint32_t* run_bounds, int64_t* num_runs, void* ws, size_t ws_bytes,
                                     void* stream, bool desc)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (!run_bounds || !num_runs) return VMPS_ERR_INVALID_ARG;
    const uint32_t ell = minrun > 0 ? (uint32_t)minrun : (n > 0 ? minrun_of((uint64_t)n) : 1u);
    if (minrun > 0 && (int64_t)ell < (n < 16 ? n : 16)) return VMPS_ERR_INVALID_ARG;
    // the documented workspace is vmps_sort's; the run chain needs no second
    // array, so its plan (sized for runs of ell) starts at the front
    const SortLayout L = sort_layout((uint64_t)n, 1, kt, 0, rule_min_len((uint64_t)n));
    if (!ws || ws_bytes < L.total) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        return guarded([&] {
            k_write_zero_u32<<<1, 1, 0, s>>>(run_bounds);
            k_write_zero_i64<<<1, 1, 0, s>>>(num_runs);
            return hipGetLastError();
        });
    }
    const int kb = key_bits_of(kt);
    Plan P;
    if (plan_workspace_bytes((uint64_t)n, 1, tilesort_capacity(kb, 0), merge_tile_out(kb, 0), ell) > ws_bytes)
        return VMPS_ERR_WORKSPACE_TOO_SMALL;
    plan_carve(P, ws, (uint64_t)n, 1, tilesort_capacity(kb, 0), merge_tile_out(kb, 0), ell);
    P.big_min = 0;
    P.desc = desc ? 1u : 0u;
    return guarded([&]() -> hipError_t {
        VMPS_HIP(plan_enqueue(P, keys, kb, minrun > 0 ? (uint32_t)minrun : 0u, s));
        const uint64_t cap = (uint64_t)vmps_max_runs(n, minrun);
        k_export_runs<<<(unsigned)ceil_div(cap + 1, 256), 256, 0, s>>>(P.run_start, P.counters, run_bounds,
                                                                       num_runs, cap);
        return hipGetLastError();
    });
}

vmps_status vmps_run_powers(const uint32_t* run_bounds, const int64_t* num_runs, int64_t n, int64_t max_runs,
                            uint8_t* powers, void* stream)
{
    if (!run_bounds || !num_runs || !powers || n < 1 || (uint64_t)n >= (1ull << 32) || max_runs < 0)
        return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (max_runs < 2) return VMPS_OK;
    return guarded([&] {
        k_powers<<<(unsigned)ceil_div((uint64_t)max_runs, 256), 256, 0, s>>>(run_bounds, num_runs, (uint64_t)n,
                                                                            powers, (uint64_t)max_runs);
        return hipGetLastError();
    });
}

vmps_status vmps_sort_schedule(const void* keys, int64_t n, vmps_dtype kt, int has_values, uint32_t* node_l,
                               uint32_t* node_m, uint32_t* node_r, uint8_t* node_level, uint8_t* node_buf,
                               uint32_t* seg_start, uint32_t* seg_end, uint8_t* seg_buf, int64_t* counts,
                               int32_t* tile, void* ws, size_t ws_bytes, void* stream)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (n < 1 || !node_l || !node_m || !node_r || !node_level || !node_buf || !seg_start || !seg_end || !seg_buf ||
        !counts || !tile)
        return VMPS_ERR_INVALID_ARG;
    const SortLayout L = sort_layout((uint64_t)n, 1, kt, has_values ? 1 : 0, rule_min_len((uint64_t)n));
    if (!ws || ws_bytes < L.total) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    const int kb = key_bits_of(kt);
    const uint32_t T = tilesort_capacity(kb, has_values ? 1 : 0);
    *tile = (int32_t)T;
    Plan P;
    plan_carve(P, (uint8_t*)ws + L.plan, (uint64_t)n, 1, T, merge_tile_out(kb, has_values ? 1 : 0),
               rule_min_len((uint64_t)n));
    P.big_min = 0;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&]() -> hipError_t {
        VMPS_HIP(plan_enqueue(P, keys, kb, 0, s));
        const uint64_t cap = (uint64_t)vmps_max_runs(n, 0) + 1;
        k_export_schedule<<<(unsigned)ceil_div(cap, 256), 256, 0, s>>>(P, node_l, node_m, node_r, node_level,
                                                                       node_buf, seg_start, seg_end, seg_buf,
                                                                       counts);
        return hipGetLastError();
    });
}

vmps_status vmps_segmented_sort_workspace_size(int64_t total, int64_t nseg, vmps_dtype kt, int has_values,
                                               size_t* bytes)
{
    if (!bytes || total < 0 || (uint64_t)total >= (1ull << 32) || nseg < 0 || (uint64_t)nseg >= (1ull << 31))
        return VMPS_ERR_INVALID_ARG;
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    const uint64_t k = (uint64_t)(nseg > 0 ? nseg : 1);
    size_t b = sort_layout((uint64_t)total, k, kt, has_values ? 1 : 0, 16).total;
    // 32-bit keys without values may run on the tuned 8192-element tile
    if (kt == VMPS_U32 && !has_values) {
        const size_t b2 = sort_layout((uint64_t)total, k, kt, 0, 16, 8192).total;
        if (b2 > b) b = b2;
    }
    *bytes = b;
    return VMPS_OK;
}

vmps_status vmps_segmented_sort(void* keys, uint32_t* values, const int64_t* seg_offsets, int64_t nseg,
                                int64_t total, vmps_dtype kt, void* ws, size_t ws_bytes, void* stream)
{
    vmps_status st = check_keys(keys, total, kt);
    if (st != VMPS_OK) return st;
    if (nseg < 0 || (uint64_t)nseg >= (1ull << 31) || !seg_offsets) return VMPS_ERR_INVALID_ARG;
    if ((uintptr_t)seg_offsets & 7) return VMPS_ERR_INVALID_ARG;
    if (values && ((uintptr_t)values & 3)) return VMPS_ERR_INVALID_ARG;
    if (values && total > 0 && ranges_overlap(keys, key_bytes(kt) * total, values, 4 * (size_t)total))
        return VMPS_ERR_INVALID_ARG;
    if (nseg == 0 || total <= 1) return VMPS_OK;
    const int has_values = values ? 1 : 0;
    const int kb = key_bits_of(kt);
    // the tile length (and workgroup size) tuned for this configuration
    const Tuning& tu = tuning_for(kb, has_values != 0);
    const uint32_t T = tu.tile_elems ? (uint32_t)tu.tile_elems : tilesort_capacity(kb, has_values);
    const SortLayout L = sort_layout((uint64_t)total, (uint64_t)nseg, kt, has_values, 16, T);
    if (!ws || ws_bytes < L.total) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    uint8_t* w = (uint8_t*)ws;
    void* keysB = w + L.keys_b;
    uint32_t* valsB = has_values ? (uint32_t*)(w + L.vals_b) : nullptr;
    Plan P;
    plan_carve(P, w + L.plan, (uint64_t)total, (uint64_t)nseg, T, merge_tile_out(kb, has_values));
    P.inst_off64 = seg_offsets;
    P.big_min = T;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&]() -> hipError_t {
        VMPS_HIP(plan_enqueue(P, keys, kb, 0, s));
        VMPS_HIP(level_probe_enqueue(P, kb, has_values, s));
        VMPS_HIP(tilesort_enqueue(P, keys, keysB, values, valsB, kb, values ? 1 : 0, 0, s, tu.tile_threads));
        // levels above the longest array's powers are empty: one launch each
        return merge_levels_enqueue(P, keys, keysB, values, valsB, kb, has_values, s, true);
    });
}

}  // extern "C"

// ------------------------------------------------------------ learned --
namespace {
bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

vmps_status check_config(const vmps_learned_config& c, int64_t n)
{
    if (c.num_buckets != 0 && (!pow2((uint64_t)c.num_buckets) || c.num_buckets < 2 || c.num_buckets > VMPS_MAX_BUCKETS))
        return VMPS_ERR_INVALID_ARG;
    if (c.hidden != 16 && c.hidden != 32 && c.hidden != 64) return VMPS_ERR_INVALID_ARG;
    if (c.steps < 0 || c.batch < 64 || (c.batch % 64) || c.batch > VMPS_CDF_MAX_BATCH) return VMPS_ERR_INVALID_ARG;
    if (!(c.lr >= 0.f) || c.knots < 1 || c.knots > VMPS_CDF_MAX_KNOTS) return VMPS_ERR_INVALID_ARG;
    if (c.feature_bits < 4 || c.feature_bits > 24) return VMPS_ERR_INVALID_ARG;
    if (c.sample_size < 2 || c.sample_size > n || c.sample_size > VMPS_CDF_MAX_SAMPLE) return VMPS_ERR_INVALID_ARG;
    if (c.flags & ~VMPS_CDF_KEEP_TRAINED) return VMPS_ERR_INVALID_ARG;
    return VMPS_OK;
}

uint32_t auto_buckets(uint64_t n, uint32_t T, int key_bits, bool has_values)
{
    // about an eighth of an LDS tile per bucket (tunable): small buckets,
    // which the grouping packs into segments that fill the tile pass
    const int div = tuning_for(key_bits, has_values).bucket_div;
    uint64_t target = T / (uint64_t)(div > 0 ? div : 8);
    if (target < 1) target = 1;
    uint64_t b = 2;
    while (b < VMPS_MAX_BUCKETS && b * target < n) b <<= 1;
    return (uint32_t)b;
}

struct LearnedLayout {
    size_t keys_b, vals_b, sample, sample_ws, u, tb, model, boff, goff, gscr, judge, arena, plan, total;
    uint32_t B, T;
    uint64_t m;
};

LearnedLayout learned_layout(uint64_t n, vmps_dtype kt, int has_values, const vmps_learned_config& c)
{
    const int kb = key_bits_of(kt);
    LearnedLayout L;
    L.T = tilesort_capacity(kb, has_values);
    L.B = c.num_buckets ? (uint32_t)c.num_buckets : auto_buckets(n, L.T, kb, has_values != 0);
    L.m = (uint64_t)c.sample_size;
    size_t off = 0;
    L.keys_b = off; off += align256(key_bytes(kt) * n);
    L.vals_b = off; off += has_values ? align256(4 * n) : 0;
    L.sample = off; off += align256(key_bytes(kt) * L.m);
    L.sample_ws = off; off += align256(sort_layout(L.m, 1, kt, 0, rule_min_len(L.m)).total);
    L.u = off; off += align256(4 * L.m);
    L.tb = off; off += align256(4 * train_buf_floats());
    L.model = off; off += align256(sizeof(vmps_cdf_model));
    L.boff = off; off += align256(8 * ((uint64_t)L.B + 1));
    L.goff = off; off += align256(8 * ((uint64_t)L.B + 1));
    L.gscr = off; off += align256(4 * group_scratch_words(L.B));
    L.judge = off; off += align256(8 * 6 * (size_t)JUDGE_GRID);
    L.arena = off; off += align256(4 * partition_arena_words(n, L.B));
    L.plan = off;
    off += plan_workspace_bytes(n, L.B, L.T, merge_tile_out(kb, has_values));
    L.total = off;
    return L;
}
}  // namespace

extern "C" {

vmps_status vmps_learned_default_config(int64_t n, vmps_dtype kt, vmps_learned_config* cfg)
{
    if (!cfg || n < 0 || (kt != VMPS_U32 && kt != VMPS_U64)) return VMPS_ERR_INVALID_ARG;
    memset(cfg, 0, sizeof *cfg);
    cfg->num_buckets = 0;
    cfg->hidden = 64;
    cfg->steps = 32;
    cfg->batch = 8192;
    cfg->lr = 5e-5f;
    cfg->knots = VMPS_CDF_MAX_KNOTS;
    cfg->feature_bits = 20;
    // n/256 sample keys, at least 8192 and at most 2^20 (2^20 from n = 2^28 on)
    int64_t m = n / 256;
    m = m < 8192 ? 8192 : (m > (1 << 20) ? (1 << 20) : m);
    cfg->sample_size = m < n ? m : n;
    cfg->seed = 55;
    return VMPS_OK;
}

vmps_status vmps_learned_workspace_size(int64_t n, vmps_dtype kt, int has_values, const vmps_learned_config* cfg,
                                        size_t* bytes)
{
    if (!bytes || n < 0 || (uint64_t)n >= (1ull << 32) || (kt != VMPS_U32 && kt != VMPS_U64))
        return VMPS_ERR_INVALID_ARG;
    vmps_learned_config c;
    if (cfg) c = *cfg; else vmps_learned_default_config(n, kt, &c);
    if (n < 2) { *bytes = 256; return VMPS_OK; }
    if (check_config(c, n) != VMPS_OK) return VMPS_ERR_INVALID_ARG;
    const size_t plain = sort_layout((uint64_t)n, 1, kt, has_values ? 1 : 0, rule_min_len((uint64_t)n)).total;
    const size_t lrn = learned_layout((uint64_t)n, kt, has_values ? 1 : 0, c).total;
    *bytes = plain > lrn ? plain : lrn;
    return VMPS_OK;
}

vmps_status vmps_sort_learned(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                              const vmps_learned_config* cfg, vmps_cdf_model* model, vmps_learned_stats* stats,
                              void* ws, size_t ws_bytes, void* stream)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (flags & ~VMPS_VALUES_IOTA) return VMPS_ERR_INVALID_ARG;
    if ((flags & VMPS_VALUES_IOTA) && !values && n > 0) return VMPS_ERR_INVALID_ARG;
    if (values && ((uintptr_t)values & 3)) return VMPS_ERR_INVALID_ARG;
    if (values && n > 0 && ranges_overlap(keys, key_bytes(kt) * n, values, 4 * (size_t)n)) return VMPS_ERR_INVALID_ARG;
    vmps_learned_config c;
    if (cfg) c = *cfg; else vmps_learned_default_config(n, kt, &c);
    const int has_values = values ? 1 : 0;
    const int kb = key_bits_of(kt);
    const uint32_t T = tilesort_capacity(kb, has_values);
    if (n < 2) return vmps_sort(keys, values, n, kt, flags, ws, ws_bytes, stream);
    if (check_config(c, n) != VMPS_OK) return VMPS_ERR_INVALID_ARG;
    size_t need = 0;
    vmps_learned_workspace_size(n, kt, has_values, &c, &need);
    if (!ws || ws_bytes < need) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    if ((uint64_t)n < 4ull * T || c.sample_size < 1024) return vmps_sort(keys, values, n, kt, flags, ws, ws_bytes, stream);
    const LearnedLayout L = learned_layout((uint64_t)n, kt, has_values, c);
    uint8_t* w = (uint8_t*)ws;
    void* keysB = w + L.keys_b;
    uint32_t* valsB = has_values ? (uint32_t*)(w + L.vals_b) : nullptr;
    vmps_cdf_model* M = (vmps_cdf_model*)(w + L.model);
    int64_t* boff = (int64_t*)(w + L.boff);
    hipStream_t s = (hipStream_t)stream;
    const int vmode = values ? ((flags & VMPS_VALUES_IOTA) ? 2 : 1) : 0;
    return guarded([&]() -> hipError_t {
        {
            TraceScope tr(VMPS_TRACE_SAMPLE, s);
            VMPS_HIP(sample_enqueue(keys, (uint64_t)n, kb, L.m, c.seed, w + L.sample, s));
            // the sample's levels as one launch each (a tile or two per
            // workgroup: searching the cuts in the merge costs no more)
            if (sort_in_workspace(w + L.sample, nullptr, (int64_t)L.m, kt, 0, w + L.sample_ws,
                                  sort_layout(L.m, 1, kt, 0, rule_min_len(L.m)).total, s, false, true) != VMPS_OK)
                return hipErrorLaunchFailure;
        }
        {
            TraceScope tr(VMPS_TRACE_TRAIN, s);
            VMPS_HIP(train_enqueue(w + L.sample, L.m, kb, c, (float*)(w + L.u), (float*)(w + L.tb), M, s));
        }
        VMPS_HIP(partition_enqueue(keys, values, keysB, valsB, keys, values, (uint32_t)n, kb, vmode, M, L.B, boff,
                                   (uint32_t*)(w + L.arena), s));
        // consecutive buckets grouped into instances that fill the tile
        // pass's segments (the shorter class of 64-bit keys without values)
        const uint32_t C = (kb == 64 && !has_values) ? T / 2 : T;
        int64_t* goff = (int64_t*)(w + L.goff);
        VMPS_HIP(group_enqueue(boff, L.B, (uint32_t)n, C, goff, (uint32_t*)(w + L.gscr), s));
        Plan P;
        plan_carve(P, w + L.plan, (uint64_t)n, L.B, T, merge_tile_out(kb, has_values));
        P.inst_off64 = goff;
        P.off_trusted = true;
        P.k_dev = group_count((const uint32_t*)(w + L.gscr), L.B);
        P.big_min = T;
        VMPS_HIP(plan_enqueue(P, keys, kb, 0, s));
        VMPS_HIP(level_probe_enqueue(P, kb, has_values, s));
        VMPS_HIP(tilesort_enqueue(P, keys, keysB, values, valsB, kb, values ? 1 : 0, 1, s));
        // only buckets longer than the tile reach the levels: mostly empty
        VMPS_HIP(merge_levels_enqueue(P, keys, keysB, values, valsB, kb, has_values, s, true));
        if (stats)
            VMPS_HIP(learned_stats_enqueue(boff, L.B, T, M, w + L.sample, L.m, kb, (uint64_t*)(w + L.judge), stats,
                                           s));
        if (model) VMPS_HIP(hipMemcpyAsync(model, M, sizeof(vmps_cdf_model), hipMemcpyDeviceToDevice, s));
        return hipGetLastError();
    });
}

vmps_status vmps_sample(const void* keys, int64_t n, vmps_dtype kt, int64_t m, uint64_t seed, void* out,
                        void* stream)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (n < 1 || m < 0 || !out || ((uintptr_t)out % key_bytes(kt))) return VMPS_ERR_INVALID_ARG;
    if (m == 0) return VMPS_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] { return sample_enqueue(keys, (uint64_t)n, key_bits_of(kt), (uint64_t)m, seed, out, s); });
}

vmps_status vmps_cdf_grad(const float* params, int32_t hidden, const float* u, const float* y, int32_t nb,
                          float* grad, float* loss, void* stream)
{
    if (!params || !u || !y || !grad || !loss || nb < 1) return VMPS_ERR_INVALID_ARG;
    if (hidden != 16 && hidden != 32 && hidden != 64) return VMPS_ERR_INVALID_ARG;
    if (nb % 64) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] { return grad_enqueue(params, hidden, u, y, nb, grad, loss, s); });
}

vmps_status vmps_cdf_train(const void* sorted_sample, int64_t m, vmps_dtype kt, const vmps_learned_config* cfg,
                           vmps_cdf_model* model, void* ws, size_t ws_bytes, void* stream)
{
    vmps_status st = check_keys(sorted_sample, m, kt);
    if (st != VMPS_OK) return st;
    if (!cfg || !model || m < 2) return VMPS_ERR_INVALID_ARG;
    vmps_learned_config c = *cfg;
    c.sample_size = m;
    if (check_config(c, m) != VMPS_OK) return VMPS_ERR_INVALID_ARG;
    size_t need = 0;
    vmps_cdf_train_workspace_size(m, &need);
    if (!ws || ws_bytes < need) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    float* tb = (float*)((uint8_t*)ws + align256(4 * (size_t)m));
    return guarded([&] {
        return train_enqueue(sorted_sample, (uint64_t)m, key_bits_of(kt), c, (float*)ws, tb, model, s);
    });
}

vmps_status vmps_cdf_train_workspace_size(int64_t m, size_t* bytes)
{
    if (!bytes || m < 0 || (uint64_t)m >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    *bytes = align256(4 * (size_t)m) + align256(4 * train_buf_floats());
    return VMPS_OK;
}

vmps_status vmps_cdf_compile(const float* params, int32_t hidden, uint64_t z_lo, uint64_t z_hi, int32_t key_bits,
                             int32_t feature_bits, int32_t knots, vmps_cdf_model* model, void* stream)
{
    if (!params || !model || (hidden != 16 && hidden != 32 && hidden != 64)) return VMPS_ERR_INVALID_ARG;
    if (z_hi < z_lo || (key_bits != 32 && key_bits != 64) || feature_bits < 4 || feature_bits > 24) return VMPS_ERR_INVALID_ARG;
    if (knots < 1 || knots > VMPS_CDF_MAX_KNOTS || z_hi - z_lo >= (1ull << 32)) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] { return compile_enqueue(params, hidden, z_lo, z_hi, key_bits, feature_bits, knots, model, s); });
}

vmps_status vmps_bucket_ids(const void* keys, int64_t n, vmps_dtype kt, const vmps_cdf_model* model,
                            int32_t num_buckets, uint32_t* ids, void* stream)
{
    vmps_status st = check_keys(keys, n, kt);
    if (st != VMPS_OK) return st;
    if (!model || !ids || num_buckets < 1) return VMPS_ERR_INVALID_ARG;
    if (n == 0) return VMPS_OK;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&] {
        return bucket_ids_enqueue(keys, (uint64_t)n, key_bits_of(kt), model, (uint32_t)num_buckets, ids, s);
    });
}

vmps_status vmps_partition_workspace_size(int64_t n, vmps_dtype kt, int has_values, int32_t num_buckets,
                                          size_t* bytes)
{
    if (!bytes || n < 0 || (uint64_t)n >= (1ull << 32) || (kt != VMPS_U32 && kt != VMPS_U64)) return VMPS_ERR_INVALID_ARG;
    if (!pow2((uint64_t)num_buckets) || num_buckets < 2 || num_buckets > VMPS_MAX_BUCKETS) return VMPS_ERR_INVALID_ARG;
    *bytes = align256(key_bytes(kt) * (size_t)n) + (has_values ? align256(4 * (size_t)n) : 0) +
             align256(4 * partition_arena_words((uint64_t)n, (uint32_t)num_buckets));
    return VMPS_OK;
}

vmps_status vmps_partition(const void* keys_in, const uint32_t* vals_in, int64_t n, vmps_dtype kt,
                           const vmps_cdf_model* model, int32_t num_buckets, void* keys_out, uint32_t* vals_out,
                           int64_t* bucket_offsets, void* ws, size_t ws_bytes, void* stream)
{
    vmps_status st = check_keys(keys_in, n, kt);
    if (st == VMPS_OK) st = check_keys(keys_out, n, kt);
    if (st != VMPS_OK) return st;
    if (!model || !bucket_offsets || !pow2((uint64_t)num_buckets) || num_buckets < 2 || num_buckets > VMPS_MAX_BUCKETS)
        return VMPS_ERR_INVALID_ARG;
    if ((vals_in == nullptr) != (vals_out == nullptr)) return VMPS_ERR_INVALID_ARG;
    if (n > 0 && ranges_overlap(keys_in, key_bytes(kt) * n, keys_out, key_bytes(kt) * n)) return VMPS_ERR_INVALID_ARG;
    size_t need = 0;
    vmps_partition_workspace_size(n, kt, vals_in != nullptr, num_buckets, &need);
    if (!ws || ws_bytes < need) return VMPS_ERR_WORKSPACE_TOO_SMALL;
    if ((uintptr_t)ws & 255) return VMPS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* w = (uint8_t*)ws;
    void* ktmp = w;
    size_t off = align256(key_bytes(kt) * (size_t)n);
    uint32_t* vtmp = vals_in ? (uint32_t*)(w + off) : nullptr;
    off += vals_in ? align256(4 * (size_t)n) : 0;
    uint32_t* arena = (uint32_t*)(w + off);
    return guarded([&] {
        return partition_enqueue(keys_in, vals_in, ktmp, vtmp, keys_out, vals_out, (uint32_t)n, key_bits_of(kt),
                                 vals_in ? 1 : 0, model, (uint32_t)num_buckets, bucket_offsets, arena, s);
    });
}

// ---------------------------------------------------------------- tuning --
vmps_status vmps_set_tuning(vmps_dtype kt, int has_values, const vmps_tuning* t)
{
    if (kt != VMPS_U32 && kt != VMPS_U64) return VMPS_ERR_INVALID_ARG;
    Tuning v{0, 0, 0, 0, 0, 0, 0};
    if (t) {
        if (t->tile_wg_per_cu < 0 || t->merge_grid < 0 || t->bucket_div < 0 || t->bucket_div > 64 ||
            (t->host_wait != 0 && t->host_wait != 1) || (t->merge_ki != 0 && t->merge_ki != 8 && t->merge_ki != 16))
            return VMPS_ERR_INVALID_ARG;
        // tile variants compiled for the segmented sort: 32-bit keys without
        // values, 512 x 16384 (default), 512 x 8192, 256 x 8192
        const bool seg32 = kt == VMPS_U32 && !has_values;
        const bool big = t->tile_elems == 0 || t->tile_elems == 16384;
        if (big ? (t->tile_threads != 0 && t->tile_threads != 512)
                : (!seg32 || t->tile_elems != 8192 ||
                   (t->tile_threads != 0 && t->tile_threads != 256 && t->tile_threads != 512)))
            return VMPS_ERR_INVALID_ARG;
        if (!seg32 && t->tile_elems != 0) return VMPS_ERR_INVALID_ARG;
        v = Tuning{t->tile_wg_per_cu, t->merge_grid, t->bucket_div, t->host_wait, t->merge_ki,
                   big ? 0 : 8192, big ? 0 : (t->tile_threads == 256 ? 256 : 0)};
    }
    tuning_table()[kt == VMPS_U64][has_values ? 1 : 0] = v;
    return VMPS_OK;
}

vmps_status vmps_get_tuning(vmps_dtype kt, int has_values, vmps_tuning* t)
{
    if ((kt != VMPS_U32 && kt != VMPS_U64) || !t) return VMPS_ERR_INVALID_ARG;
    const Tuning& v = tuning_table()[kt == VMPS_U64][has_values ? 1 : 0];
    t->tile_wg_per_cu = v.tile_wg_per_cu;
    t->merge_grid = v.merge_grid;
    t->bucket_div = v.bucket_div;
    t->host_wait = v.host_wait;
    t->merge_ki = v.merge_ki;
    t->tile_elems = v.tile_elems;
    t->tile_threads = v.tile_threads;
    return VMPS_OK;
}

// ---------------------------------------------------------------- graphs --
vmps_status vmps_segmented_sort_graph(void* keys, uint32_t* values, const int64_t* seg_offsets, int64_t nseg,
                                      int64_t total, vmps_dtype kt, void* ws, size_t ws_bytes, vmps_graph* graph)
{
    if (!graph) return VMPS_ERR_INVALID_ARG;
    return capture_graph(graph, [&](hipStream_t cs) {
        return vmps_segmented_sort(keys, values, seg_offsets, nseg, total, kt, ws, ws_bytes, cs);
    });
}

vmps_status vmps_sort_learned_graph(void* keys, uint32_t* values, int64_t n, vmps_dtype kt, uint32_t flags,
                                    const vmps_learned_config* cfg, vmps_learned_stats* stats, void* ws,
                                    size_t ws_bytes, vmps_graph* graph)
{
    if (!graph) return VMPS_ERR_INVALID_ARG;
    return capture_graph(graph, [&](hipStream_t cs) {
        return vmps_sort_learned(keys, values, n, kt, flags, cfg, nullptr, stats, ws, ws_bytes, cs);
    });
}

vmps_status vmps_graph_launch(vmps_graph graph, void* stream)
{
    if (!graph) return VMPS_ERR_INVALID_ARG;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? VMPS_OK : VMPS_ERR_DEVICE;
}

vmps_status vmps_graph_destroy(vmps_graph graph)
{
    if (!graph) return VMPS_ERR_INVALID_ARG;
    hipError_t e1 = hipGraphExecDestroy(graph->exec);
    hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    return (e1 == hipSuccess && e2 == hipSuccess) ? VMPS_OK : VMPS_ERR_DEVICE;
}

}  // extern "C"

namespace vmps {
const Tuning& tuning_for(int key_bits, bool has_values)
{
    return tuning_table()[key_bits == 64][has_values ? 1 : 0];
}
}  // namespace vmps
