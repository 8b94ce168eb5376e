"""Powersort CPU oracle: TEST INFRASTRUCTURE ONLY.

Thin ctypes/numpy wrapper over ``liboracle.so`` (plain C, ``oracle.c``).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.

Every function follows the paper "Virtual-Memory Powersort":
Algorithm 1 (Abstract Powersort), the Power theorem of Section 2, Pingpong
Powersort (Section 3), StandardMerge (Algorithm 2), and the minrun rule of
Section 5.  The learned-partition helpers are the fp64 reference of the
project's CDF model (a monotone integer feature, one hidden ReLU layer, an
integer knot table, and a stable counting sort by bucket id).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PINGPONG, PINGPONG_LASTPOP, CPYTHON = 0, 1, 2
DESC_RUNS = 4  # flag or-ed into a variant: strictly decreasing runs are reversed


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "n", "runs", "merges", "merge_cost", "max_stack", "cmp_run", "cmp_ins",
        "cmp_merge", "mov_ins", "mov_push", "mov_merge")] + [("entropy", ctypes.c_double), ("mov_rev", ctypes.c_int64),
                                                               ("mov_copy", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class VmStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "page", "input_pages", "extra_pages", "meta_words", "max_buffers")]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, u64, vp, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double
        lib.orc_adam_update.restype = None
        lib.orc_adam_update.argtypes = [vp, vp, vp, vp, i32, i64, dbl]
        lib.orc_minrun.restype = i32
        lib.orc_minrun.argtypes = [i64]
        lib.orc_power_def.restype = i32
        lib.orc_power_def.argtypes = [i64, i64, i64, i64]
        lib.orc_power_closed.restype = i32
        lib.orc_power_closed.argtypes = [i64, i64, i64, i64]
        lib.orc_extract_runs.restype = i64
        lib.orc_extract_runs.argtypes = [vp, i64, i32, vp]
        lib.orc_extract_runs_dir.restype = i64
        lib.orc_extract_runs_dir.argtypes = [vp, i64, i32, ctypes.c_int, vp, vp]
        lib.orc_run_powers.restype = None
        lib.orc_run_powers.argtypes = [vp, i64, i64, vp]
        lib.orc_powersort.restype = ctypes.c_int
        lib.orc_powersort.argtypes = [vp, vp, i64, i32, ctypes.c_int, ctypes.POINTER(Stats), vp, i64]
        lib.orc_vm_powersort.restype = ctypes.c_int
        lib.orc_vm_powersort.argtypes = [vp, vp, i64, i32, i64, ctypes.c_int, ctypes.POINTER(Stats),
                                         ctypes.POINTER(VmStats), vp, i64]
        lib.orc_vm_page.restype = i64
        lib.orc_vm_page.argtypes = [i64, i32]
        lib.orc_segmented_powersort.restype = ctypes.c_int
        lib.orc_segmented_powersort.argtypes = [vp, vp, vp, i64, i32, ctypes.c_int]
        lib.orc_standard_merge.restype = None
        lib.orc_standard_merge.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp]
        lib.orc_tree_nodes.restype = None
        lib.orc_tree_nodes.argtypes = [vp, i64, i64, vp, vp]
        lib.orc_plan.restype = i64
        lib.orc_plan.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp, vp, vp]
        lib.orc_mix64.restype = u64
        lib.orc_mix64.argtypes = [u64, u64]
        lib.orc_sample_positions.restype = None
        lib.orc_sample_positions.argtypes = [i64, i64, u64, vp]
        lib.orc_feature.restype = u64
        lib.orc_feature.argtypes = [u64, i32, i32]
        lib.orc_mlp_forward.restype = dbl
        lib.orc_mlp_forward.argtypes = [vp, vp, vp, dbl, i32, dbl]
        lib.orc_mlp_grad.restype = dbl
        lib.orc_mlp_grad.argtypes = [vp, vp, vp, dbl, i32, vp, vp, i64, vp, vp, vp, vp]
        lib.orc_cdf_grid.restype = None
        lib.orc_cdf_grid.argtypes = [u64, u64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.orc_cdf_table.restype = None
        lib.orc_cdf_table.argtypes = [vp, vp, vp, dbl, i32, u64, u64, i32, vp, ctypes.POINTER(i32),
                                      ctypes.POINTER(i32)]
        lib.orc_bucket_of.restype = ctypes.c_uint32
        lib.orc_bucket_of.argtypes = [u64, i32, i32, u64, u64, vp, i32, i32, ctypes.c_uint32]
        lib.orc_cdf_pos.restype = u64
        lib.orc_cdf_pos.argtypes = [u64, i32, i32, u64, u64, vp, i32, i32]
        lib.orc_judge.restype = None
        lib.orc_judge.argtypes = [vp, i64, i32, i32, u64, u64, vp, i32, i32, ctypes.c_uint32, vp, vp, vp, vp]
        lib.orc_cdf_init.restype = None
        lib.orc_cdf_init.argtypes = [vp, i64, i32, vp, vp, vp, vp]
        lib.orc_cdf_loss.restype = dbl
        lib.orc_cdf_loss.argtypes = [vp, vp, vp, dbl, i32, vp, i64, i64]
        lib.orc_cdf_adam_steps.restype = None
        lib.orc_cdf_adam_steps.argtypes = [vp, i64, i32, i32, i32, dbl, vp, vp]
        lib.orc_cdf_train2.restype = dbl
        lib.orc_cdf_train2.argtypes = [vp, i64, i32, i32, i32, dbl, vp, ctypes.POINTER(i32)]
        lib.orc_cdf_train.restype = dbl
        lib.orc_cdf_train.argtypes = [vp, i64, i32, i32, i32, dbl, vp]
        lib.orc_partition.restype = None
        lib.orc_partition.argtypes = [vp, vp, i64, i32, i32, u64, u64, vp, i32, i32, ctypes.c_uint32,
                                      vp, vp, vp]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _keys64(keys) -> np.ndarray:
    keys = np.asarray(keys)
    if keys.dtype in (np.uint32, np.int32):
        return keys.view(np.uint32).astype(np.uint64)
    return np.ascontiguousarray(keys.view(np.uint64) if keys.dtype == np.int64 else keys.astype(np.uint64))


def minrun(n: int) -> int:
    return int(_L().orc_minrun(n))


def power_def(n, i, j, k) -> int:
    return int(_L().orc_power_def(n, i, j, k))


def power_closed(n, i, j, k) -> int:
    return int(_L().orc_power_closed(n, i, j, k))


def extract_runs(keys, ell: int | None = None, desc: bool = False, want_desc: bool = False):
    """Run bounds (r+1 int64) of the sequential ExtractRun chain; with desc,
    maximal strictly decreasing runs count too (want_desc: also the flags of
    the runs that are reversed)."""
    x = _keys64(keys)
    n = x.size
    if ell is None:
        ell = minrun(n)
    bounds = np.zeros(n + 2, dtype=np.int64)
    flags = np.zeros(n + 2, dtype=np.uint8)
    r = _L().orc_extract_runs_dir(_p(x), n, ell, int(desc), _p(bounds), _p(flags))
    if want_desc:
        return bounds[: r + 1].copy(), flags[:r].copy()
    return bounds[: r + 1].copy()


def run_powers(bounds: np.ndarray, n: int) -> np.ndarray:
    bounds = np.ascontiguousarray(bounds, dtype=np.int64)
    r = bounds.size - 1
    out = np.zeros(max(r - 1, 1), dtype=np.uint8)
    _L().orc_run_powers(_p(bounds), r, n, _p(out))
    return out[: max(r - 1, 0)].copy()


def powersort(keys, vals=None, variant: int = PINGPONG, ell: int = 0, log_merges: bool = False):
    """Algorithm 1 on a copy of keys (and vals). Returns (keys, vals, stats, merge_log)."""
    orig = np.asarray(keys)
    x = _keys64(orig).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    n = x.size
    st = Stats()
    cap = n if log_merges else 0
    log = np.zeros(3 * max(cap, 1), dtype=np.int64)
    rc = _L().orc_powersort(_p(x), _p(v), n, ell, variant, ctypes.byref(st),
                            _p(log) if log_merges else None, cap)
    if rc != 0:
        raise RuntimeError("oracle powersort failed")
    out = x.astype(orig.dtype) if orig.dtype in (np.uint32, np.int32) else x.view(orig.dtype) if orig.dtype == np.int64 else x
    merges = log[: 3 * st.merges].reshape(-1, 3).copy() if log_merges else None
    return out, v, st.as_dict(), merges


def vm_page(n: int, rec_words: int) -> int:
    return int(_L().orc_vm_page(n, rec_words))


def vm_powersort(keys, vals=None, page: int = 0, ell: int = 0, desc: bool = False, log_merges: bool = False):
    """Virtual-Memory Powersort (Section 4) on a copy: (keys, vals, stats,
    vm_stats, merge_log)."""
    orig = np.asarray(keys)
    x = _keys64(orig).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    n = x.size
    st, vst = Stats(), VmStats()
    cap = n if log_merges else 0
    log = np.zeros(3 * max(cap, 1), dtype=np.int64)
    rc = _L().orc_vm_powersort(_p(x), _p(v), n, ell, page, DESC_RUNS if desc else 0, ctypes.byref(st),
                               ctypes.byref(vst), _p(log) if log_merges else None, cap)
    if rc != 0:
        raise RuntimeError("oracle vm powersort failed")
    out = x.astype(orig.dtype) if orig.dtype in (np.uint32, np.int32) else x
    merges = log[: 3 * st.merges].reshape(-1, 3).copy() if log_merges else None
    return out, v, st.as_dict(), vst.as_dict(), merges


def records_sort(records, key_offset: int, key_bytes: int, desc: bool = False):
    """Stable sort of records (an (n, record_bytes) uint8 array) by the
    little-endian unsigned key field of key_bytes bytes at key_offset: the
    record types of Sec. 5 sorted as whole elements.  The order is Algorithm
    1's on the keys (indices as values, so equal keys keep input order);
    the records are then taken in that order."""
    rec = np.ascontiguousarray(records, dtype=np.uint8)
    n = rec.shape[0]
    field = rec[:, key_offset:key_offset + key_bytes].copy()
    keys = field.view(np.uint32 if key_bytes == 4 else np.uint64).reshape(n)
    _, perm, _, _ = powersort(keys, np.arange(n, dtype=np.uint32), variant=PINGPONG | (DESC_RUNS if desc else 0))
    return rec[perm.astype(np.int64)]


def segmented_powersort(keys, offsets, vals=None, variant: int = PINGPONG, ell: int = 0):
    """Every segment [offsets[s], offsets[s+1]) sorted as its own instance
    (ell <= 0: the minrun rule for the segment's length)."""
    orig = np.asarray(keys)
    x = _keys64(orig).copy()
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    rc = _L().orc_segmented_powersort(_p(x), _p(v), _p(off), off.size - 1, ell, variant)
    if rc != 0:
        raise RuntimeError("oracle segmented powersort failed")
    out = x.astype(orig.dtype) if orig.dtype in (np.uint32, np.int32) else x
    return out, v


def standard_merge(a, b, va=None, vb=None):
    A, B = _keys64(a), _keys64(b)
    out = np.zeros(A.size + B.size, dtype=np.uint64)
    vout = None
    if va is not None:
        va = np.ascontiguousarray(va, dtype=np.uint32)
        vb = np.ascontiguousarray(vb, dtype=np.uint32)
        vout = np.zeros(out.size, dtype=np.uint32)
    _L().orc_standard_merge(_p(A), _p(va), A.size, _p(B), _p(vb), B.size, _p(out), _p(vout))
    return out, vout


def tree_nodes(bounds, n, powers) -> np.ndarray:
    bounds = np.ascontiguousarray(bounds, dtype=np.int64)
    powers = np.ascontiguousarray(powers, dtype=np.uint8)
    r = bounds.size - 1
    nodes = np.zeros(4 * max(r - 1, 1), dtype=np.int64)
    _L().orc_tree_nodes(_p(bounds), r, n, _p(powers), _p(nodes))
    return nodes[: 4 * max(r - 1, 0)].reshape(-1, 4).copy()


def plan(bounds, n, powers, T):
    """Pingpong placement: (node_buf, node_depth, segs[(start,end,buf)], M, M_hbm)."""
    bounds = np.ascontiguousarray(bounds, dtype=np.int64)
    powers = np.ascontiguousarray(powers, dtype=np.uint8)
    r = bounds.size - 1
    nb = max(r - 1, 0)
    node_buf = np.zeros(max(nb, 1), dtype=np.int8)
    node_depth = np.zeros(max(nb, 1), dtype=np.int32)
    segs = np.zeros(3 * (nb + 1), dtype=np.int64)
    mt = ctypes.c_int64(0)
    mh = ctypes.c_int64(0)
    ns = _L().orc_plan(_p(bounds), r, n, _p(powers), T, _p(node_buf), _p(node_depth), _p(segs),
                       ctypes.byref(mt), ctypes.byref(mh))
    return node_buf[:nb].copy(), node_depth[:nb].copy(), segs[: 3 * ns].reshape(-1, 3).copy(), mt.value, mh.value


# ---- learned CDF partitioner reference (fp64) ----

def mix64(seed: int, counter: int) -> int:
    return int(_L().orc_mix64(seed & (2**64 - 1), counter))


def sample_positions(n: int, m: int, seed: int) -> np.ndarray:
    out = np.zeros(m, dtype=np.int64)
    _L().orc_sample_positions(n, m, seed & (2**64 - 1), _p(out))
    return out


def feature(key: int, key_bits: int, fbits: int) -> int:
    return int(_L().orc_feature(key, key_bits, fbits))


def features(keys, key_bits: int, fbits: int) -> np.ndarray:
    return np.array([feature(int(k), key_bits, fbits) for k in np.asarray(keys).ravel()], dtype=np.uint64)


def mlp_forward(params: dict, u: float) -> float:
    w1, b1, w2 = (np.ascontiguousarray(params[k], dtype=np.float64) for k in ("w1", "b1", "w2"))
    return float(_L().orc_mlp_forward(_p(w1), _p(b1), _p(w2), float(params["b2"]), w1.size, u))


def mlp_grad(params: dict, u, y):
    """(loss, grads dict) of the minibatch MSE, fp64."""
    w1, b1, w2 = (np.ascontiguousarray(params[k], dtype=np.float64) for k in ("w1", "b1", "w2"))
    H = w1.size
    u = np.ascontiguousarray(u, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = {k: np.zeros(H, dtype=np.float64) for k in ("w1", "b1", "w2")}
    gb2 = ctypes.c_double(0.0)
    loss = _L().orc_mlp_grad(_p(w1), _p(b1), _p(w2), float(params["b2"]), H, _p(u), _p(y), u.size,
                             _p(g["w1"]), _p(g["b1"]), _p(g["w2"]), ctypes.byref(gb2))
    g["b2"] = gb2.value
    return float(loss), g


class Table:
    """Compiled CDF model: knot positions (Q32) every 2^shift feature units."""

    def __init__(self, table, shift, knots, z_lo, z_hi):
        self.table, self.shift, self.knots, self.z_lo, self.z_hi = table, shift, knots, z_lo, z_hi


def cdf_grid(z_lo: int, z_hi: int, K: int):
    sh, kn = ctypes.c_int32(0), ctypes.c_int32(0)
    _L().orc_cdf_grid(z_lo, z_hi, K, ctypes.byref(sh), ctypes.byref(kn))
    return sh.value, kn.value


def cdf_table(params: dict, z_lo: int, z_hi: int, K: int) -> Table:
    w1, b1, w2 = (np.ascontiguousarray(params[k], dtype=np.float64) for k in ("w1", "b1", "w2"))
    table = np.zeros(K + 2, dtype=np.uint64)
    sh, kn = ctypes.c_int32(0), ctypes.c_int32(0)
    _L().orc_cdf_table(_p(w1), _p(b1), _p(w2), float(params["b2"]), w1.size, z_lo, z_hi, K, _p(table),
                       ctypes.byref(sh), ctypes.byref(kn))
    return Table(table[: kn.value + 1].copy(), sh.value, kn.value, z_lo, z_hi)


def bucket_of(key: int, key_bits: int, fbits: int, tab: Table, B: int) -> int:
    t = np.ascontiguousarray(tab.table, dtype=np.uint64)
    return int(_L().orc_bucket_of(key, key_bits, fbits, tab.z_lo, tab.z_hi, _p(t), tab.shift, tab.knots, B))


def cdf_pos(key: int, key_bits: int, fbits: int, tab: Table) -> int:
    """F(key) of the compiled table in Q32."""
    t = np.ascontiguousarray(tab.table, dtype=np.uint64)
    return int(_L().orc_cdf_pos(key, key_bits, fbits, tab.z_lo, tab.z_hi, _p(t), tab.shift, tab.knots))


def judge(sorted_keys, key_bits: int, fbits: int, tab: Table, B: int) -> dict:
    """Error judge on a sorted sample (targets y_i = (i + 1/2)/m): maximum and
    mean of |bucket(x_i) - floor(B y_i)| and of |B F(x_i) - B y_i|, the last
    two as exact rationals rounded once to float."""
    from fractions import Fraction
    x = _keys64(sorted_keys)
    m = x.size
    t = np.ascontiguousarray(tab.table, dtype=np.uint64)
    mb = np.zeros(1, dtype=np.uint64)
    sb = np.zeros(1, dtype=np.uint64)
    dm = np.zeros(2, dtype=np.uint64)
    ds = np.zeros(2, dtype=np.uint64)
    _L().orc_judge(_p(x), m, key_bits, fbits, tab.z_lo, tab.z_hi, _p(t), tab.shift, tab.knots, B,
                   _p(mb), _p(sb), _p(dm), _p(ds))
    d_max = int(dm[0]) + (int(dm[1]) << 64)
    d_sum = int(ds[0]) + (int(ds[1]) << 64)
    return {"samples": m, "max_bucket_err": int(mb[0]), "sum_bucket_err": int(sb[0]),
            "mean_bucket_err": float(Fraction(int(sb[0]), m)) if m else 0.0,
            "d_max": d_max, "d_sum": d_sum,
            "max_err": float(Fraction(B * d_max, (1 << 33) * m)) if m else 0.0,
            "mean_err": float(Fraction(B * d_sum, (1 << 33) * m * m)) if m else 0.0}


def partition(keys, key_bits: int, fbits: int, tab: Table, B: int, vals=None):
    """Stable counting sort by bucket id: (keys_out, vals_out, offsets[B+1])."""
    orig = np.asarray(keys)
    x = _keys64(orig)
    t = np.ascontiguousarray(tab.table, dtype=np.uint64)
    n = x.size
    ko = np.zeros(n, dtype=np.uint64)
    v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32)
    vo = None if v is None else np.zeros(n, dtype=np.uint32)
    off = np.zeros(B + 1, dtype=np.int64)
    _L().orc_partition(_p(x), _p(v), n, key_bits, fbits, tab.z_lo, tab.z_hi, _p(t), tab.shift, tab.knots, B,
                       _p(ko), _p(vo), _p(off))
    if orig.dtype in (np.uint32, np.int32):
        ko = ko.astype(np.uint32)
    return ko, vo, off


def _unpack(p, H):
    return {"w1": p[:H].copy(), "b1": p[H:2 * H].copy(), "w2": p[2 * H:3 * H].copy(), "b2": float(p[3 * H])}


def normalised_features(sorted_keys, key_bits: int, fbits: int):
    """(u in [0,1], z_lo, z_hi) of a sorted sample, fp64."""
    z = features(sorted_keys, key_bits, fbits).astype(np.float64)
    z_lo, z_hi = int(features(sorted_keys[:1], key_bits, fbits)[0]), int(features(sorted_keys[-1:], key_bits, fbits)[0])
    rng_ = z_hi - z_lo
    u = (z - z_lo) / rng_ if rng_ > 0 else np.zeros_like(z)
    return u, z_lo, z_hi


def cdf_init(u, H: int) -> dict:
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.zeros(3 * H + 1, dtype=np.float64)
    b2 = ctypes.c_double(0.0)
    _L().orc_cdf_init(_p(u), u.size, H, _p(p), p[H:].ctypes.data, p[2 * H:].ctypes.data, ctypes.byref(b2))
    p[3 * H] = b2.value
    return _unpack(p, H)


def adam_update(p, g, m1, m2, step: int, lr: float):
    """One Adam step on fp64 arrays, in place (p, m1, m2 are updated)."""
    for a in (p, g, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _L().orc_adam_update(_p(p), _p(g), _p(m1), _p(m2), p.size, step, lr)


def cdf_loss(params: dict, u, stride: int = 64) -> float:
    w1, b1, w2 = (np.ascontiguousarray(params[k], dtype=np.float64) for k in ("w1", "b1", "w2"))
    u = np.ascontiguousarray(u, dtype=np.float64)
    return float(_L().orc_cdf_loss(_p(w1), _p(b1), _p(w2), float(params["b2"]), w1.size, _p(u), u.size, stride))


def cdf_train(u, H: int, steps: int, nb: int, lr: float, want_trained: bool = False):
    """fp64 reference training: quantile init + Adam, then the better of the
    two models; returns (params, loss) or (params, loss, trained)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.zeros(3 * H + 1, dtype=np.float64)
    tr = ctypes.c_int32(0)
    loss = _L().orc_cdf_train2(_p(u), u.size, H, steps, nb, lr, _p(p), ctypes.byref(tr))
    if want_trained:
        return _unpack(p, H), float(loss), bool(tr.value)
    return _unpack(p, H), float(loss)


def flat_params(params: dict) -> np.ndarray:
    return np.concatenate([params["w1"], params["b1"], params["w2"], [params["b2"]]]).astype(np.float64)


def cdf_adam_steps(u, params: dict, steps: int, nb: int, lr: float):
    """Adam from the given parameters (no initialisation, no model choice);
    returns the trajectory, steps x (3H+1) fp64 (row s: after step s+1)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    H = len(params["w1"])
    p = np.ascontiguousarray(flat_params(params))
    traj = np.zeros((max(steps, 1), 3 * H + 1), dtype=np.float64)
    _L().orc_cdf_adam_steps(_p(u), u.size, H, steps, nb, lr, _p(p), _p(traj))
    return traj[:steps].copy()
