"""Python binding of libvmps.so: stable run-adaptive sorting on MI355X.

Argument marshalling only.  Every step of the sort runs in the HIP kernels
of ``libvmps.so``; PyTorch provides device memory and the current stream.
Importing works without a GPU, but calling any entry point requires the
built library and a HIP device: there is no CPU fallback.

Tensors may be torch.int32/uint32 (keys compared as unsigned 32-bit) or
torch.int64/uint64 (unsigned 64-bit), contiguous, on the current device.
"""
from __future__ import annotations

import ctypes
import json
import os

__all__ = [
    "VmpsError", "load_library", "library_path", "minrun", "max_runs", "sort_", "argsort_", "merge",
    "extract_runs", "run_powers", "sort_schedule", "segmented_sort_", "sort_workspace_size",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libvmps.so")
_lib = None

OK, INVALID_ARG, WORKSPACE_TOO_SMALL, UNSUPPORTED, DEVICE = range(5)
U32, U64 = 0, 1
VALUES_IOTA = 1
DESCENDING_RUNS = 2
VM_STATS = 8  # vmps_sort_vm statistics: faults, carried, copied, merged, levels, page writes, kept in place
CDF_KEEP_TRAINED = 1


class LearnedConfig(ctypes.Structure):
    _fields_ = [("num_buckets", ctypes.c_int32), ("hidden", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("knots", ctypes.c_int32),
                ("feature_bits", ctypes.c_int32), ("flags", ctypes.c_int32), ("sample_size", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


CDF_MAX_HIDDEN, CDF_MAX_KNOTS = 64, 4096


class CdfModel(ctypes.Structure):
    _fields_ = [("z_lo", ctypes.c_uint64), ("z_hi", ctypes.c_uint64), ("key_bits", ctypes.c_int32),
                ("feature_bits", ctypes.c_int32), ("hidden", ctypes.c_int32), ("knots", ctypes.c_int32),
                ("shift", ctypes.c_int32), ("trained", ctypes.c_int32), ("loss_init", ctypes.c_float),
                ("loss_final", ctypes.c_float), ("w1", ctypes.c_float * CDF_MAX_HIDDEN),
                ("b1", ctypes.c_float * CDF_MAX_HIDDEN), ("w2", ctypes.c_float * CDF_MAX_HIDDEN),
                ("b2", ctypes.c_float), ("reserved", ctypes.c_float),
                ("table", ctypes.c_uint64 * (CDF_MAX_KNOTS + 1))]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_wg_per_cu", ctypes.c_int32), ("merge_grid", ctypes.c_int32),
                ("bucket_div", ctypes.c_int32), ("host_wait", ctypes.c_int32), ("merge_ki", ctypes.c_int32),
                ("tile_elems", ctypes.c_int32), ("tile_threads", ctypes.c_int32)]


class VmLayout(ctypes.Structure):
    _fields_ = [("page_elems", ctypes.c_int64), ("pages", ctypes.c_int64), ("window_pages", ctypes.c_int64),
                ("pool_pages", ctypes.c_int64), ("copy_pages", ctypes.c_int64), ("buffer_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t)]


class LearnedStats(ctypes.Structure):
    _fields_ = [("buckets", ctypes.c_int64), ("nonempty_buckets", ctypes.c_int64),
                ("fallback_buckets", ctypes.c_int64), ("fallback_keys", ctypes.c_int64),
                ("max_bucket", ctypes.c_int64), ("loss_init", ctypes.c_float), ("loss_final", ctypes.c_float),
                ("judge_samples", ctypes.c_int64), ("judge_max_bucket_err", ctypes.c_int64),
                ("judge_mean_bucket_err", ctypes.c_double), ("judge_max_err", ctypes.c_double),
                ("judge_mean_err", ctypes.c_double), ("overflow_fraction", ctypes.c_double)]


class VmpsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libvmps.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2605_27147_amd/build.py")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "vmps_status_string": (ctypes.c_char_p, [st]),
        "vmps_minrun": (i32, [i64]),
        "vmps_max_runs": (i64, [i64, i32]),
        "vmps_sort_workspace_size": (st, [i64, st, st, ctypes.POINTER(sz)]),
        "vmps_sort": (st, [vp, vp, i64, st, u32, vp, sz, vp]),
        "vmps_sort_noalloc": (st, [vp, vp, i64, st, u32, vp]),
        "vmps_noalloc_scratch_bytes": (sz, []),
        "vmps_merge_workspace_size": (st, [i64, i64, st, ctypes.POINTER(sz)]),
        "vmps_merge": (st, [vp, vp, i64, vp, vp, i64, vp, vp, st, vp, sz, vp]),
        "vmps_extract_runs": (st, [vp, i64, st, i32, vp, vp, vp, sz, vp]),
        "vmps_extract_runs_desc": (st, [vp, i64, st, i32, vp, vp, vp, sz, vp]),
        "vmps_run_powers": (st, [vp, vp, i64, i64, vp, vp]),
        "vmps_sort_schedule": (st, [vp, i64, st, st, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                    ctypes.POINTER(i32), vp, sz, vp]),
        "vmps_segmented_sort_workspace_size": (st, [i64, i64, st, st, ctypes.POINTER(sz)]),
        "vmps_segmented_sort": (st, [vp, vp, vp, i64, i64, st, vp, sz, vp]),
        "vmps_learned_default_config": (st, [i64, st, ctypes.POINTER(LearnedConfig)]),
        "vmps_learned_workspace_size": (st, [i64, st, st, ctypes.POINTER(LearnedConfig), ctypes.POINTER(sz)]),
        "vmps_sort_learned": (st, [vp, vp, i64, st, u32, ctypes.POINTER(LearnedConfig), vp, vp, vp, sz, vp]),
        "vmps_sample": (st, [vp, i64, st, i64, ctypes.c_uint64, vp, vp]),
        "vmps_cdf_grad": (st, [vp, i32, vp, vp, i32, vp, vp, vp]),
        "vmps_cdf_train": (st, [vp, i64, st, ctypes.POINTER(LearnedConfig), vp, vp, sz, vp]),
        "vmps_cdf_train_workspace_size": (st, [i64, ctypes.POINTER(sz)]),
        "vmps_cdf_compile": (st, [vp, i32, ctypes.c_uint64, ctypes.c_uint64, i32, i32, i32, vp, vp]),
        "vmps_bucket_ids": (st, [vp, i64, st, vp, i32, vp, vp]),
        "vmps_partition_workspace_size": (st, [i64, st, st, i32, ctypes.POINTER(sz)]),
        "vmps_partition": (st, [vp, vp, i64, st, vp, i32, vp, vp, vp, vp, sz, vp]),
        "vmps_set_tuning": (st, [st, st, ctypes.POINTER(Tuning)]),
        "vmps_get_tuning": (st, [st, st, ctypes.POINTER(Tuning)]),
        "vmps_segmented_sort_graph": (st, [vp, vp, vp, i64, i64, st, vp, sz, ctypes.POINTER(vp)]),
        "vmps_sort_learned_graph": (st, [vp, vp, i64, st, u32, ctypes.POINTER(LearnedConfig), vp, vp, sz,
                                         ctypes.POINTER(vp)]),
        "vmps_graph_launch": (st, [vp, vp]),
        "vmps_graph_destroy": (st, [vp]),
        "vmps_sort_vm_layout": (st, [i64, st, st, i64, ctypes.POINTER(VmLayout)]),
        "vmps_sort_records_workspace_size": (st, [i64, st, ctypes.POINTER(sz)]),
        "vmps_sort_records": (st, [vp, vp, i64, i32, i32, st, u32, vp, sz, vp]),
        "vmps_sort_vm": (st, [vp, vp, i64, st, u32, i64, vp, sz, vp, vp]),
        "vmps_trace_enable": (st, [st]),
        "vmps_trace_collect": (st, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    _apply_autotune(lib)
    return lib


AUTOTUNE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune.json")


def _apply_autotune(lib, path: str = AUTOTUNE_PATH):
    """Loads the tuning table measured for this GPU (if there is one) into the
    library.  Tuning changes speed, never results."""
    try:
        with open(path) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return
    arch = _gpu_arch()
    if arch is None or table.get("arch") != arch:
        return
    for e in table.get("entries", []):
        if e.get("merge_ki", 0) not in (0, 8, 16):
            continue
        t = Tuning(int(e.get("tile_wg_per_cu", 0)), int(e.get("merge_grid", 0)), int(e.get("bucket_div", 0)), 0,
                   int(e.get("merge_ki", 0)), int(e.get("tile_elems", 0)), int(e.get("tile_threads", 0)))
        kt = U64 if e["dtype"] == "u64" else U32
        # an entry the library rejects (INVALID_ARG) leaves the defaults
        lib.vmps_set_tuning(kt, int(bool(e["values"])), ctypes.byref(t))


def _gpu_arch():
    try:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return None


def set_tuning(dtype_code: int, has_values: bool, tile_wg_per_cu: int = 0, merge_grid: int = 0,
               bucket_div: int = 0, host_wait: int = 0, merge_ki: int = 0, tile_elems: int = 0,
               tile_threads: int = 0):
    t = Tuning(tile_wg_per_cu, merge_grid, bucket_div, host_wait, merge_ki, tile_elems, tile_threads)
    _check(load_library().vmps_set_tuning(dtype_code, int(bool(has_values)), ctypes.byref(t)), "vmps_set_tuning")


def reset_tuning(dtype_code: int, has_values: bool):
    _check(load_library().vmps_set_tuning(dtype_code, int(bool(has_values)), None), "vmps_set_tuning")


def get_tuning(dtype_code: int, has_values: bool) -> dict:
    t = Tuning()
    _check(load_library().vmps_get_tuning(dtype_code, int(bool(has_values)), ctypes.byref(t)), "vmps_get_tuning")
    return {"tile_wg_per_cu": t.tile_wg_per_cu, "merge_grid": t.merge_grid, "bucket_div": t.bucket_div,
            "host_wait": t.host_wait, "merge_ki": t.merge_ki, "tile_elems": t.tile_elems,
            "tile_threads": t.tile_threads}


def status_string(s: int) -> str:
    try:
        return load_library().vmps_status_string(s).decode()
    except ImportError:
        return {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "unsupported",
                4: "device error"}.get(s, "unknown status")


def _check(status: int, where: str):
    if status != OK:
        raise VmpsError(status, where)


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype in (torch.int32, getattr(torch, "uint32", torch.int32)):
        return U32
    if t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)):
        return U64
    raise TypeError(f"keys must be 32- or 64-bit integers, got {t.dtype}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_cuda(*ts):
    for t in ts:
        if t is not None:
            if not t.is_cuda:
                raise ValueError("tensors must live on the GPU")
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous")


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def minrun(n: int) -> int:
    return int(load_library().vmps_minrun(n))


def max_runs(n: int, minrun_: int = 0) -> int:
    return int(load_library().vmps_max_runs(n, minrun_))


def sort_workspace_size(n: int, dtype_code: int, has_values: bool) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().vmps_sort_workspace_size(n, dtype_code, int(bool(has_values)), ctypes.byref(out)),
           "vmps_sort_workspace_size")
    return out.value


def sort_(keys, values=None, *, iota: bool = False, workspace=None, desc: bool = False):
    """Stable in-place sort of keys (and values).  iota=True fills `values`
    with the stable permutation instead of reading it; desc=True reverses
    strictly decreasing runs (VMPS_DESCENDING_RUNS)."""
    lib = load_library()
    _require_cuda(keys, values)
    kt = _dtype_code(keys)
    n = keys.numel()
    ws_bytes = sort_workspace_size(n, kt, values is not None)
    ws = workspace if workspace is not None else _workspace(ws_bytes, keys.device)
    flags = (VALUES_IOTA if iota else 0) | (DESCENDING_RUNS if desc else 0)
    _check(lib.vmps_sort(_ptr(keys), _ptr(values), n, kt, flags, _ptr(ws), ws.numel(), _stream(keys.device)),
           "vmps_sort")
    return keys


def sort_noalloc_(keys, values=None, *, iota: bool = False):
    """sort_ with the library's own device scratch array as the workspace
    (no allocation; calls on one GPU must not overlap in time)."""
    lib = load_library()
    _require_cuda(keys, values)
    kt = _dtype_code(keys)
    flags = VALUES_IOTA if iota else 0
    _check(lib.vmps_sort_noalloc(_ptr(keys), _ptr(values), keys.numel(), kt, flags, _stream(keys.device)),
           "vmps_sort_noalloc")
    return keys


def vm_layout(n: int, dtype_code: int, has_values: bool, window_pages: int = 0) -> dict:
    """Page length, page counts and bytes of the paged sort (vmps_sort_vm)."""
    out = VmLayout()
    _check(load_library().vmps_sort_vm_layout(n, dtype_code, int(bool(has_values)), window_pages,
                                              ctypes.byref(out)), "vmps_sort_vm_layout")
    return {name: getattr(out, name) for name, _ in VmLayout._fields_}


def sort_vm_(keys, values=None, *, iota: bool = False, desc: bool = False, window_pages: int = 0, workspace=None,
             stats=None):
    """Stable in-place sort with paged merge levels (Virtual-Memory
    Powersort): no second array, a pool of window_pages + 9 pages.  stats:
    None or an int64 GPU tensor of VM_STATS entries (see vmps_sort_vm)."""
    lib = load_library()
    _require_cuda(keys, values, stats)
    kt = _dtype_code(keys)
    n = keys.numel()
    lay = vm_layout(n, kt, values is not None, window_pages)
    ws = workspace if workspace is not None else _workspace(lay["workspace_bytes"], keys.device)
    if stats is not None and stats.numel() < VM_STATS:
        raise ValueError(f"stats needs {VM_STATS} entries")
    flags = (VALUES_IOTA if iota else 0) | (DESCENDING_RUNS if desc else 0)
    _check(lib.vmps_sort_vm(_ptr(keys), _ptr(values), n, kt, flags, window_pages, _ptr(ws), ws.numel(), _ptr(stats),
                            _stream(keys.device)), "vmps_sort_vm")
    return keys


def records_workspace_size(n: int, key_dtype_code: int) -> int:
    sz = ctypes.c_size_t(0)
    _check(load_library().vmps_sort_records_workspace_size(n, key_dtype_code, ctypes.byref(sz)),
           "vmps_sort_records_workspace_size")
    return sz.value


def sort_records(records, key_offset: int, key_dtype_code: int, *, out=None, desc: bool = False, workspace=None):
    """Stable sort of records (a contiguous GPU tensor whose last dimension
    holds one record's bytes or words) by the u32/u64 key field at byte
    key_offset; returns `out` (a new tensor of the same shape unless given)."""
    lib = load_library()
    _require_cuda(records, out)
    n = records.shape[0] if records.dim() > 0 else 0
    rb = records.numel() * records.element_size() // max(n, 1)
    if out is None:
        out = _torch().empty_like(records)
    ws = workspace if workspace is not None else _workspace(records_workspace_size(n, key_dtype_code),
                                                            records.device)
    _check(lib.vmps_sort_records(_ptr(records), _ptr(out), n, rb, key_offset, key_dtype_code,
                                 DESCENDING_RUNS if desc else 0, _ptr(ws), ws.numel(), _stream(records.device)),
           "vmps_sort_records")
    return out


def noalloc_scratch_bytes() -> int:
    return int(load_library().vmps_noalloc_scratch_bytes())


def argsort_(keys, indices):
    """Sort keys in place and write the stable permutation into indices (int32)."""
    return sort_(keys, indices, iota=True)


def merge(a, b, va=None, vb=None, out=None, vout=None):
    torch = _torch()
    lib = load_library()
    _require_cuda(a, b, va, vb)
    kt = _dtype_code(a)
    if _dtype_code(b) != kt:
        raise TypeError("a and b must have the same key type")
    na, nb = a.numel(), b.numel()
    if out is None:
        out = torch.empty(na + nb, dtype=a.dtype, device=a.device)
    if va is not None and vout is None:
        vout = torch.empty(na + nb, dtype=va.dtype, device=a.device)
    need = ctypes.c_size_t(0)
    _check(lib.vmps_merge_workspace_size(na, nb, kt, ctypes.byref(need)), "vmps_merge_workspace_size")
    ws = _workspace(need.value, a.device)
    _check(lib.vmps_merge(_ptr(a), _ptr(va), na, _ptr(b), _ptr(vb), nb, _ptr(out), _ptr(vout), kt, _ptr(ws),
                          ws.numel(), _stream(a.device)), "vmps_merge")
    return out, vout


def extract_runs(keys, minrun_: int = 0, desc: bool = False):
    """(run_bounds int32 tensor of r+1 bounds, r) — synchronises to read r.
    desc: the chain with descending runs (vmps_extract_runs_desc)."""
    torch = _torch()
    lib = load_library()
    _require_cuda(keys)
    kt = _dtype_code(keys)
    n = keys.numel()
    cap = max_runs(n, minrun_)
    bounds = torch.empty(cap + 1, dtype=torch.int32, device=keys.device)
    nr = torch.zeros(1, dtype=torch.int64, device=keys.device)
    ws = _workspace(sort_workspace_size(n, kt, False), keys.device)
    fn = lib.vmps_extract_runs_desc if desc else lib.vmps_extract_runs
    _check(fn(_ptr(keys), n, kt, minrun_, _ptr(bounds), _ptr(nr), _ptr(ws), ws.numel(), _stream(keys.device)),
           "vmps_extract_runs")
    r = int(nr.item())
    return bounds[: r + 1], r


def run_powers(bounds, r: int, n: int):
    torch = _torch()
    lib = load_library()
    _require_cuda(bounds)
    nr = torch.tensor([r], dtype=torch.int64, device=bounds.device)
    powers = torch.zeros(max(r - 1, 1), dtype=torch.uint8, device=bounds.device)
    _check(lib.vmps_run_powers(_ptr(bounds), _ptr(nr), n, max(r, 0), _ptr(powers), _stream(bounds.device)),
           "vmps_run_powers")
    return powers[: max(r - 1, 0)]


def sort_schedule(keys, has_values: bool = False):
    """The merge schedule vmps_sort would run: dict of host numpy arrays."""
    torch = _torch()
    lib = load_library()
    _require_cuda(keys)
    kt = _dtype_code(keys)
    n = keys.numel()
    cap = max_runs(n, 0) + 1
    dev = keys.device
    u32 = lambda: torch.zeros(cap, dtype=torch.int32, device=dev)
    u8 = lambda: torch.zeros(cap, dtype=torch.uint8, device=dev)
    nl, nm, nr_, nlev, nbuf, ss, se, sb = u32(), u32(), u32(), u8(), u8(), u32(), u32(), u8()
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    tile = ctypes.c_int32(0)
    ws = _workspace(sort_workspace_size(n, kt, has_values), dev)
    _check(lib.vmps_sort_schedule(_ptr(keys), n, kt, int(bool(has_values)), _ptr(nl), _ptr(nm), _ptr(nr_),
                                  _ptr(nlev), _ptr(nbuf), _ptr(ss), _ptr(se), _ptr(sb), _ptr(counts),
                                  ctypes.byref(tile), _ptr(ws), ws.numel(), _stream(dev)), "vmps_sort_schedule")
    c = counts.cpu().tolist()
    h, ns = int(c[1]), int(c[2])
    return {
        "runs": int(c[0]), "merge_cost": int(c[3]), "tile": tile.value,
        "node_l": nl[:h].cpu().numpy(), "node_m": nm[:h].cpu().numpy(), "node_r": nr_[:h].cpu().numpy(),
        "node_level": nlev[:h].cpu().numpy(), "node_buf": nbuf[:h].cpu().numpy(),
        "seg_start": ss[:ns].cpu().numpy(), "seg_end": se[:ns].cpu().numpy(), "seg_buf": sb[:ns].cpu().numpy(),
    }


TRACE_KINDS = ["plan", "tilesort", "level_partition", "level_merge", "histogram", "scatter", "train", "sample"]


def trace_enable(on: bool = True):
    _check(load_library().vmps_trace_enable(int(bool(on))), "vmps_trace_enable")


def trace_collect() -> dict:
    """{kind: (milliseconds, launches)} since the previous collect (waits for the events)."""
    k = len(TRACE_KINDS)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    _check(load_library().vmps_trace_collect(ms, cnt, k), "vmps_trace_collect")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(TRACE_KINDS)}


def segmented_sort_(keys, offsets, values=None, workspace=None):
    """Independent stable sorts of keys[offsets[s]:offsets[s+1]] (offsets: int64 on the GPU)."""
    lib = load_library()
    _require_cuda(keys, values, offsets)
    kt = _dtype_code(keys)
    total = keys.numel()
    nseg = offsets.numel() - 1
    need = ctypes.c_size_t(0)
    _check(lib.vmps_segmented_sort_workspace_size(total, max(nseg, 0), kt, int(values is not None),
                                                  ctypes.byref(need)), "vmps_segmented_sort_workspace_size")
    if workspace is not None and workspace.numel() < need.value:
        raise ValueError("workspace too small")
    ws = workspace if workspace is not None else _workspace(need.value, keys.device)
    _check(lib.vmps_segmented_sort(_ptr(keys), _ptr(values), _ptr(offsets), nseg, total, kt, _ptr(ws),
                                   ws.numel(), _stream(keys.device)), "vmps_segmented_sort")
    return keys


class Graph:
    """A captured sort (vmps_*_graph): replay() enqueues it on the current
    stream.  It keeps the tensors it was captured with alive."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def replay(self):
        _check(load_library().vmps_graph_launch(self._h, _stream()), "vmps_graph_launch")

    def close(self):
        if self._h:
            load_library().vmps_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def segmented_sort_graph(keys, offsets, values=None) -> Graph:
    """Captures segmented_sort_(keys, offsets, values) into a graph."""
    lib = load_library()
    _require_cuda(keys, values, offsets)
    kt = _dtype_code(keys)
    total = keys.numel()
    nseg = offsets.numel() - 1
    need = ctypes.c_size_t(0)
    _check(lib.vmps_segmented_sort_workspace_size(total, max(nseg, 0), kt, int(values is not None),
                                                  ctypes.byref(need)), "vmps_segmented_sort_workspace_size")
    ws = _workspace(need.value, keys.device)
    h = ctypes.c_void_p()
    _check(lib.vmps_segmented_sort_graph(_ptr(keys), _ptr(values), _ptr(offsets), nseg, total, kt, _ptr(ws),
                                         ws.numel(), ctypes.byref(h)), "vmps_segmented_sort_graph")
    return Graph(h, (keys, values, offsets, ws))


def sort_learned_graph(keys, values=None, *, iota: bool = False, cfg=None) -> Graph:
    """Captures sort_learned_(keys, values) into a graph (no statistics)."""
    lib = load_library()
    _require_cuda(keys, values)
    kt = _dtype_code(keys)
    n = keys.numel()
    if cfg is None:
        cfg = learned_default_config(n, kt)
    need = ctypes.c_size_t(0)
    _check(lib.vmps_learned_workspace_size(n, kt, int(values is not None), ctypes.byref(cfg), ctypes.byref(need)),
           "vmps_learned_workspace_size")
    ws = _workspace(need.value, keys.device)
    h = ctypes.c_void_p()
    _check(lib.vmps_sort_learned_graph(_ptr(keys), _ptr(values), n, kt, VALUES_IOTA if iota else 0, ctypes.byref(cfg),
                                       None, _ptr(ws), ws.numel(), ctypes.byref(h)), "vmps_sort_learned_graph")
    return Graph(h, (keys, values, ws, cfg))


# ------------------------------------------------------------- learned --
def learned_default_config(n: int, dtype_code: int) -> LearnedConfig:
    cfg = LearnedConfig()
    _check(load_library().vmps_learned_default_config(n, dtype_code, ctypes.byref(cfg)), "vmps_learned_default_config")
    return cfg


def _struct_from_tensor(t, cls):
    raw = t.cpu().numpy().tobytes()
    return cls.from_buffer_copy(raw[: ctypes.sizeof(cls)])


def model_to_tensor(model: CdfModel, device="cuda"):
    """Copy a host model struct into a device byte tensor."""
    torch = _torch()
    raw = bytes(model)
    import numpy as np
    return torch.from_numpy(np.frombuffer(raw, dtype=np.uint8).copy()).to(device)


def model_from_tensor(t) -> CdfModel:
    return _struct_from_tensor(t, CdfModel)


def sort_learned_(keys, values=None, *, iota: bool = False, cfg: LearnedConfig | None = None, workspace=None,
                  want_model: bool = False, read_stats: bool = True):
    """Stable in-place sort through the learned partition.  Returns
    (stats dict, model struct or None), synchronising to read them; with
    read_stats=False it only enqueues the sort and returns (None, None)."""
    torch = _torch()
    lib = load_library()
    _require_cuda(keys, values)
    kt = _dtype_code(keys)
    n = keys.numel()
    if cfg is None:
        cfg = learned_default_config(n, kt)
    need = ctypes.c_size_t(0)
    _check(lib.vmps_learned_workspace_size(n, kt, int(values is not None), ctypes.byref(cfg), ctypes.byref(need)),
           "vmps_learned_workspace_size")
    ws = workspace if workspace is not None else _workspace(need.value, keys.device)
    want_model = want_model and read_stats
    model_t = torch.zeros(ctypes.sizeof(CdfModel), dtype=torch.uint8, device=keys.device) if want_model else None
    stats_t = torch.zeros(ctypes.sizeof(LearnedStats), dtype=torch.uint8, device=keys.device) if read_stats else None
    _check(lib.vmps_sort_learned(_ptr(keys), _ptr(values), n, kt, VALUES_IOTA if iota else 0, ctypes.byref(cfg),
                                 _ptr(model_t), _ptr(stats_t), _ptr(ws), ws.numel(), _stream(keys.device)),
           "vmps_sort_learned")
    if not read_stats:
        return None, None
    st = _struct_from_tensor(stats_t, LearnedStats)
    stats = {name: getattr(st, name) for name, _ in LearnedStats._fields_}
    return stats, (model_from_tensor(model_t) if want_model else None)


def learned_workspace_size(n: int, dtype_code: int, has_values: bool, cfg: LearnedConfig) -> int:
    need = ctypes.c_size_t(0)
    _check(load_library().vmps_learned_workspace_size(n, dtype_code, int(bool(has_values)), ctypes.byref(cfg),
                                                      ctypes.byref(need)), "vmps_learned_workspace_size")
    return need.value


def sample(keys, m: int, seed: int):
    torch = _torch()
    _require_cuda(keys)
    out = torch.empty(m, dtype=keys.dtype, device=keys.device)
    _check(load_library().vmps_sample(_ptr(keys), keys.numel(), _dtype_code(keys), m, seed, _ptr(out),
                                      _stream(keys.device)), "vmps_sample")
    return out


def cdf_grad(params, hidden: int, u, y):
    """params, u, y: float32 device tensors. Returns (grad[3H+1], loss)."""
    torch = _torch()
    grad = torch.empty(3 * hidden + 1, dtype=torch.float32, device=params.device)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(load_library().vmps_cdf_grad(_ptr(params), hidden, _ptr(u), _ptr(y), u.numel(), _ptr(grad), _ptr(loss),
                                        _stream(params.device)), "vmps_cdf_grad")
    return grad, loss


def cdf_train(sorted_sample, cfg: LearnedConfig, want_features: bool = False):
    """Trains and compiles the model on a sorted sample; returns the model
    (and with want_features the fp32 features u it was trained on)."""
    torch = _torch()
    _require_cuda(sorted_sample)
    m = sorted_sample.numel()
    model_t = torch.zeros(ctypes.sizeof(CdfModel), dtype=torch.uint8, device=sorted_sample.device)
    need = ctypes.c_size_t(0)
    _check(load_library().vmps_cdf_train_workspace_size(m, ctypes.byref(need)), "vmps_cdf_train_workspace_size")
    ws = _workspace(need.value, sorted_sample.device)
    _check(load_library().vmps_cdf_train(_ptr(sorted_sample), m, _dtype_code(sorted_sample), ctypes.byref(cfg),
                                         _ptr(model_t), _ptr(ws), ws.numel(), _stream(sorted_sample.device)),
           "vmps_cdf_train")
    model = model_from_tensor(model_t)
    if want_features:
        return model, ws[: 4 * m].view(torch.float32).clone()
    return model


def cdf_compile(params, hidden: int, z_lo: int, z_hi: int, key_bits: int, feature_bits: int, knots: int):
    """Returns the compiled model as a device byte tensor."""
    torch = _torch()
    model_t = torch.zeros(ctypes.sizeof(CdfModel), dtype=torch.uint8, device=params.device)
    _check(load_library().vmps_cdf_compile(_ptr(params), hidden, z_lo, z_hi, key_bits, feature_bits, knots,
                                           _ptr(model_t), _stream(params.device)), "vmps_cdf_compile")
    return model_t


def bucket_ids(keys, model_t, num_buckets: int):
    torch = _torch()
    ids = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    _check(load_library().vmps_bucket_ids(_ptr(keys), keys.numel(), _dtype_code(keys), _ptr(model_t), num_buckets,
                                          _ptr(ids), _stream(keys.device)), "vmps_bucket_ids")
    return ids


def partition(keys, model_t, num_buckets: int, values=None):
    """Stable partition by bucket: (keys_out, vals_out, offsets int64[B+1])."""
    torch = _torch()
    lib = load_library()
    kt = _dtype_code(keys)
    n = keys.numel()
    need = ctypes.c_size_t(0)
    _check(lib.vmps_partition_workspace_size(n, kt, int(values is not None), num_buckets, ctypes.byref(need)),
           "vmps_partition_workspace_size")
    ws = _workspace(need.value, keys.device)
    ko = torch.empty_like(keys)
    vo = None if values is None else torch.empty_like(values)
    off = torch.empty(num_buckets + 1, dtype=torch.int64, device=keys.device)
    _check(lib.vmps_partition(_ptr(keys), _ptr(values), n, kt, _ptr(model_t), num_buckets, _ptr(ko), _ptr(vo),
                              _ptr(off), _ptr(ws), ws.numel(), _stream(keys.device)), "vmps_partition")
    return ko, vo, off
