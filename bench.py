"""Throughput of stable Powersort on one MI355X: learned partition vs plain.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--path learned|plain] [--log2n 28]

A step is one full stable sort of n = 2^28 uint64 keys drawn from the
lognormal workload (floor(exp(2 N(0,1)) 2^40), seeded, synthetic) resident
in HBM.  The default path is the learned one: sample, sort the sample with
the plain path, train the CDF model, compile, stable two-level scatter,
Powersort of every bucket (the segmented path).  The plain path (run
detection, powers, merge tree, LDS subtrees, merge levels) is timed in the
same run for comparison.  The input is restored from a pristine device copy
before every step, outside the timed events.

The JSON line carries the throughput (Gkeys/s), the roofline of the
dominant kernel (its average launch time measured with HIP events on the
sort's stream, bytes = what the method must move in that kernel), and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s + % HBM roofline at n=2^28 u64, learned/batched vs plain GPU path"
HBM_PEAK_GBS = 8000.0
# LDS: 128 bytes per clock per CU, 256 CUs at 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
# VALU issue: one wave64 vector instruction per clock per CU (four SIMDs of
# 16 lanes, 64 lane-operations per clock), 256 CUs at 2.4 GHz
VALU_PEAK_GIPS = 256 * 2.4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def is_sorted_u64(t):
    import torch
    s = t ^ torch.iinfo(torch.int64).min  # unsigned order as signed order
    return bool((s[1:] >= s[:-1]).all().item())


def kernel_bytes(path: str, kind: str, n: int, kb: int, vb: int, m_hbm: int, sample: int) -> float:
    """Algorithmic bytes per sort of one kernel kind: every pass reads and
    writes each element once; cache re-reads are not counted."""
    kv = kb + vb
    if kind == "level_merge":
        return 2.0 * kv * m_hbm                 # merges longer than the LDS tile
    if kind == "tilesort":
        return float(kb * n + kv * n)           # read keys, write keys (+ values)
    if kind == "histogram":
        return (kb + 2 + 2) * float(n)          # level 1: keys in, 16-bit ids out; level 2: ids in
    if kind == "scatter":
        return (2 * (kv + 2) + (kv + 2) + kv) * float(n)  # level 1 moves keys+ids, level 2 reads both, writes keys
    if kind == "plan":
        return float(kb * n) if path == "plain" else 0.0
    if kind == "sample":
        return float(kb * sample)
    return 0.0


def run_path(vm, path, keys, pristine, steps, warmup, traced_steps=None):
    """Times `steps` sorts (HIP events around each, input restored from the
    pristine copy before each, outside the events), then runs `traced_steps`
    more with the library's per-kernel launch tracing for the breakdown (the
    tracing events are kept out of the timed steps)."""
    import numpy as np
    import torch

    stream = torch.cuda.current_stream()

    def step():
        if path == "learned":
            vm.sort_learned_(keys, workspace=WS[0], read_stats=False)
        else:
            vm.sort_(keys, workspace=WS[0])

    for _ in range(warmup):
        keys.copy_(pristine)
        step()
    torch.cuda.synchronize()
    ev = []
    for _ in range(steps):
        keys.copy_(pristine)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step()
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    assert is_sorted_u64(keys), f"{path}: output not sorted"
    MEDIAN[path] = float(np.median(ms))
    trace = None
    if traced_steps:
        vm.trace_collect()
        vm.trace_enable(True)
        for _ in range(traced_steps):
            keys.copy_(pristine)
            step()
        torch.cuda.synchronize()
        vm.trace_enable(False)
        trace = vm.trace_collect()
    return float(np.mean(ms)), trace


def _timed(fn, restore, steps):
    """Mean ms of `steps` calls after one warm-up call, HIP events around
    each call, input restored before each (outside the events)."""
    import numpy as np
    import torch
    ts = []
    for i in range(steps + 1):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        if i:
            ts.append(e0.elapsed_time(e1))
    return float(np.mean(ts))


def _m_hbm(vm, keys, has_values=False):
    import numpy as np
    sch = vm.sort_schedule(keys, has_values=has_values)
    return int((sch["node_r"].astype(np.int64) - sch["node_l"].astype(np.int64)).sum()), int(sch["tile"])


def bench_configs(vm, dev, steps):
    """The other workload configurations, each timed on its own input:
    algorithmic bytes of the plain path = bitmap read (kb per key), tile pass
    (kb in, kb + vb out; index values are generated, not read), merges
    beyond the LDS tile (2 (kb + vb) per element of M_HBM)."""
    import numpy as np
    import torch

    import workloads
    out = {}

    def entry(name, n, ms, b_alg=None, **kw):
        e = {"workload": name, "n": n, "ms_per_step": round(ms, 4), "value": round(n / (ms / 1e3) / 1e9, 4),
             "unit": "Gkeys/s"}
        if b_alg is not None:
            e.update({"bytes_alg": b_alg, "achieved_GBs": round(b_alg / (ms / 1e3) / 1e9, 1),
                      "frac": round(b_alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)})
        e.update(kw)
        return e

    # 2^16 uint32 keys, uniform, plain path (launch-bound at this size)
    n1 = 1 << 16
    x1 = workloads.uniform(n1, 32, 1)
    src1 = torch.from_numpy(x1.view(np.int32)).to(dev)
    k1 = torch.empty_like(src1)
    ws1 = torch.empty(vm.sort_workspace_size(n1, vm.U32, False), dtype=torch.uint8, device=dev)
    log(f"config uniform32 2^16: timed {steps * 10}")
    ms1 = _timed(lambda: vm.sort_(k1, workspace=ws1), lambda: k1.copy_(src1), steps * 10)
    assert np.array_equal(k1.cpu().numpy().view(np.uint32), np.sort(x1)), "uniform32: wrong output"
    m1, _ = _m_hbm(vm, src1)
    out["uniform32_2p16"] = entry("n=2^16 uint32 uniform keys, plain path", n1, ms1, 4 * n1 + 8 * n1 + 8 * m1,
                                  merge_cost_hbm=m1)

    # 2^24 uint64 keys with presortedness (geometric runs of mean 2^10, 10%
    # reversed, 1% random swaps), plain path, with and without the reversal
    # of strictly decreasing runs
    n2 = 1 << 24
    x2 = workloads.presorted(n2, 33, mean_run=1024, bits=64)
    src2 = torch.from_numpy(x2.view(np.int64)).to(dev)
    k2 = torch.empty_like(src2)
    ws2 = torch.empty(vm.sort_workspace_size(n2, vm.U64, False), dtype=torch.uint8, device=dev)
    log(f"config presorted64 2^24: timed {steps * 3}")
    ms2 = _timed(lambda: vm.sort_(k2, workspace=ws2), lambda: k2.copy_(src2), steps * 3)
    ref2 = np.sort(x2)
    assert np.array_equal(k2.cpu().numpy().view(np.uint64), ref2), "presorted64: wrong output"
    ms2d = _timed(lambda: vm.sort_(k2, workspace=ws2, desc=True), lambda: k2.copy_(src2), steps * 3)
    assert np.array_equal(k2.cpu().numpy().view(np.uint64), ref2), "presorted64 (descending runs): wrong output"
    m2, _ = _m_hbm(vm, src2)
    out["presorted64_2p24"] = entry("n=2^24 uint64 keys, geometric runs (mean 2^10), 10% reversed, 1% swaps, "
                                    "plain path", n2, ms2, 8 * n2 + 16 * n2 + 16 * m2, merge_cost_hbm=m2,
                                    descending_runs_ms=round(ms2d, 4),
                                    descending_runs_value=round(n2 / (ms2d / 1e3) / 1e9, 4))
    del src2, k2, ws2

    # 2^28 uint64 keys, mixture (50% uniform, 30% Zipf 1.1 over 2^20
    # values, 20% normal around 64 centres), stable sort of (key, u32 index)
    # pairs: plain and learned paths
    n3 = 1 << 28
    log("config mixture64 pairs 2^28: generating")
    x3 = workloads.mixture(n3, 36)
    src3 = torch.from_numpy(x3.view(np.int64)).to(dev)
    del x3
    k3 = torch.empty_like(src3)
    v3 = torch.empty(n3, dtype=torch.int32, device=dev)
    ws3 = torch.empty(vm.sort_workspace_size(n3, vm.U64, True), dtype=torch.uint8, device=dev)

    def check3(what):
        s = k3 ^ torch.iinfo(torch.int64).min
        assert bool((s[1:] >= s[:-1]).all().item()), f"{what}: keys out of order"
        idx = v3.to(torch.int64)
        assert bool((src3[idx] == k3).all().item()), f"{what}: a value does not index its key"
        hit = torch.zeros(n3, dtype=torch.bool, device=dev)
        hit[idx] = True
        assert bool(hit.all().item()), f"{what}: values are not a permutation"
        del idx, hit
        eq = s[1:] == s[:-1]
        assert bool(((v3[1:] > v3[:-1]) | ~eq).all().item()), f"{what}: equal keys out of input order"

    log(f"config mixture64 pairs 2^28, plain: timed {steps}")
    ms3 = _timed(lambda: vm.sort_(k3, v3, iota=True, workspace=ws3), lambda: k3.copy_(src3), steps)
    check3("mixture64 pairs, plain")
    del ws3
    torch.cuda.empty_cache()
    lcfg = vm.learned_default_config(n3, vm.U64)
    lws = torch.empty(vm.learned_workspace_size(n3, vm.U64, True, lcfg), dtype=torch.uint8, device=dev)
    log(f"config mixture64 pairs 2^28, learned: timed {steps}")
    ms3l = _timed(lambda: vm.sort_learned_(k3, v3, iota=True, workspace=lws, read_stats=False),
                  lambda: k3.copy_(src3), steps)
    check3("mixture64 pairs, learned")
    m3, _ = _m_hbm(vm, src3, has_values=True)
    out["mixture64_pairs_2p28"] = entry("n=2^28 uint64 mixture keys, stable sort of (key, u32 index) pairs, "
                                        "plain path", n3, ms3, 8 * n3 + 20 * n3 + 24 * m3, merge_cost_hbm=m3,
                                        learned_ms=round(ms3l, 4),
                                        learned_value=round(n3 / (ms3l / 1e3) / 1e9, 4))
    del src3, k3, v3, lws
    torch.cuda.empty_cache()
    return out


WS = [None]
MEDIAN = {}
TRACED = 3  # extra sorts run with per-kernel tracing for the breakdown


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", default="learned", choices=["learned", "plain"])
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--compare-steps", type=int, default=3, help="steps of the other path (0: skip)")
    ap.add_argument("--vm-steps", type=int, default=3,
                    help="steps of the paged (virtual-memory) sort at two window sizes (0: skip)")
    ap.add_argument("--records-log2", type=int, default=24,
                    help="records of 120 bytes sorted by a u64 key field (0: skip)")
    ap.add_argument("--batch-nseg", type=int, default=4096,
                    help="arrays of the batched u32 workload sorted in one segmented call (0: skip)")
    ap.add_argument("--configs-steps", type=int, default=3,
                    help="steps of the other workload configurations: 2^16 u32 uniform, 2^24 u64 presorted, "
                         "2^28 u64 mixture (key, index) pairs (0: skip)")
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the sort runs on one GPU only (asked for --gpus {args.gpus}); "
              "a sharded multi-GPU sort is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_27147_amd as vm
    import workloads

    vm.load_library()
    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    log(f"generating lognormal keys n=2^{args.log2n}")
    keys_np = workloads.lognormal(n, 5)
    pristine = torch.from_numpy(keys_np.view(np.int64)).to(dev)
    keys = torch.empty_like(pristine)
    checksum = int(pristine.sum().item())
    cfg = vm.learned_default_config(n, vm.U64)
    ws_bytes = max(vm.sort_workspace_size(n, vm.U64, False), vm.learned_workspace_size(n, vm.U64, False, cfg))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    WS[0] = ws

    sch = vm.sort_schedule(pristine)
    m_hbm_plain = int((sch["node_r"].astype(np.int64) - sch["node_l"].astype(np.int64)).sum())

    log(f"{args.path}: warmup {args.warmup}, timed {args.steps}")
    ms, trace = run_path(vm, args.path, keys, pristine, args.steps, args.warmup, traced_steps=TRACED)
    assert int(keys.sum().item()) == checksum, "output is not a permutation of the input"
    stats = stats0 = None
    if args.path == "learned":
        keys.copy_(pristine)
        stats, _ = vm.sort_learned_(keys, workspace=ws)
        # the same sort with the quantile initialisation alone (no Adam
        # step), outside the timed steps: what training adds
        cfg0 = vm.learned_default_config(n, vm.U64)
        cfg0.steps = 0
        keys.copy_(pristine)
        stats0, _ = vm.sort_learned_(keys, workspace=ws, cfg=cfg0)
    other = "plain" if args.path == "learned" else "learned"
    other_ms = None
    if args.compare_steps > 0:
        log(f"{other}: timed {args.compare_steps}")
        other_ms, _ = run_path(vm, other, keys, pristine, args.compare_steps, 1)

    vm_out = None
    if args.vm_steps > 0:
        # Virtual-Memory Powersort (Section 4): the same input through the
        # paged merge levels, no second array; extra memory against the
        # Pingpong buffer and time against the plain path
        plain_ms = ms if args.path == "plain" else other_ms
        nvm = vm.vm_layout(n, vm.U64, False)["pages"]
        vm_out = {"pingpong_buffer_bytes": 8 * n, "plain_workspace_bytes": vm.sort_workspace_size(n, vm.U64, False),
                  "plain_ms_per_step": round(plain_ms, 4) if plain_ms else None, "windows": []}
        for wreq in (0, nvm // 4):
            lay = vm.vm_layout(n, vm.U64, False, wreq)
            vws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device=dev)
            vst = torch.zeros(vm.VM_STATS, dtype=torch.int64, device=dev)
            log(f"paged sort, window {lay['window_pages']} pages: timed {args.vm_steps}")
            tms = []
            for i in range(args.vm_steps + 1):
                keys.copy_(pristine)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                vm.sort_vm_(keys, window_pages=wreq, workspace=vws, stats=vst)
                e1.record()
                torch.cuda.synchronize()
                if i:
                    tms.append(e0.elapsed_time(e1))
            assert is_sorted_u64(keys) and int(keys.sum().item()) == checksum, "paged sort: wrong output"
            s = vst.cpu().tolist()
            assert s[0] == 0, "paged sort: schedule fault"
            vms = float(np.mean(tms))
            vm_out["windows"].append({
                "window_pages": lay["window_pages"], "page_elems": lay["page_elems"], "pages": lay["pages"],
                "ms_per_step": round(vms, 4), "value": round(n / (vms / 1e3) / 1e9, 4), "unit": "Gkeys/s",
                "page_buffer_bytes": lay["buffer_bytes"], "workspace_bytes": lay["workspace_bytes"],
                "page_buffer_vs_pingpong": round(lay["buffer_bytes"] / (8 * n), 4),
                "workspace_vs_plain": round(lay["workspace_bytes"] / vm_out["plain_workspace_bytes"], 4),
                "slowdown_vs_plain": round(vms / plain_ms, 3) if plain_ms else None,
                "carried": s[1], "copy_moves": s[2], "merged": s[3], "levels": s[4], "page_writes": s[5]})
            del vws
        # a nearly sorted input (key i is i * 2^20 plus a jitter below
        # 3 * 2^20, so every key is out of place by at most a few
        # positions): merges that mostly concatenate, where the
        # page-skipping merge leaves pages in place
        ns = 1 << 26
        rng = np.random.default_rng(11)
        xs = np.arange(ns, dtype=np.uint64) * np.uint64(1 << 20) + rng.integers(0, 3 << 20, ns, dtype=np.uint64)
        src_ns = torch.from_numpy(xs.view(np.int64)).to(dev)
        k_ns = torch.empty_like(src_ns)
        pws = torch.empty(vm.sort_workspace_size(ns, vm.U64, False), dtype=torch.uint8, device=dev)
        lay = vm.vm_layout(ns, vm.U64, False)
        vws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device=dev)
        vst = torch.zeros(vm.VM_STATS, dtype=torch.int64, device=dev)
        t_p, t_v = [], []
        for i in range(args.vm_steps + 1):
            for fn, acc in ((lambda: vm.sort_(k_ns, workspace=pws), t_p),
                            (lambda: vm.sort_vm_(k_ns, workspace=vws, stats=vst), t_v)):
                k_ns.copy_(src_ns)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                if i:
                    acc.append(e0.elapsed_time(e1))
        assert is_sorted_u64(k_ns), "paged sort: nearly sorted input not sorted"
        s = vst.cpu().tolist()
        vm_out["jittered_sorted_2p26"] = {
            "plain_ms": round(float(np.mean(t_p)), 4), "paged_ms": round(float(np.mean(t_v)), 4),
            "merged": s[3], "kept_in_place": s[6], "kept_share": round(s[6] / max(1, s[3] + s[6]), 4),
            "copy_moves": s[2], "page_writes": s[5]}
        del src_ns, k_ns, pws, vws
        torch.cuda.empty_cache()

    rec_out = None
    if args.records_log2 > 0:
        # large records (the 30-word element types of Sec. 5, hypothesis H4):
        # 120-byte records of random 32-bit words sorted by the u64 in words
        # 2-3, as (key, index) pairs and one gather, against the bytes a
        # record-moving Pingpong sort would need
        nr = 1 << args.records_log2
        g = torch.Generator(device=dev)
        g.manual_seed(7)
        rec = torch.randint(100, 10**9, (nr, 30), dtype=torch.int32, device=dev, generator=g)
        rec[:, 0] = torch.arange(nr, dtype=torch.int32, device=dev)
        out_rec = torch.empty_like(rec)
        rws = torch.empty(vm.records_workspace_size(nr, vm.U64), dtype=torch.uint8, device=dev)
        log(f"records: 2^{args.records_log2} x 120 bytes")
        tms = []
        for i in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vm.sort_records(rec, 8, vm.U64, out=out_rec, workspace=rws)
            e1.record()
            torch.cuda.synchronize()
            if i:
                tms.append(e0.elapsed_time(e1))
        keys_r = out_rec[:, 2:4].contiguous().view(torch.int64).reshape(-1)
        assert is_sorted_u64(keys_r), "records: keys out of order"
        idx = out_rec[:, 0].to(torch.int64)
        assert bool((rec[idx] == out_rec).all().item()), "records: a record changed"
        sch_r = vm.sort_schedule(rec[:, 2:4].contiguous().view(torch.int64).reshape(-1), has_values=True)
        m_r = int((sch_r["node_r"].astype(np.int64) - sch_r["node_l"].astype(np.int64)).sum())
        rms = float(np.mean(tms))
        # algorithmic bytes: key extraction (8 B read per record), the (key,
        # index) sort (bitmap 8, tile pass 8 + 12, levels 2 * 12 per element
        # per merge beyond the tile), the gather (120 read + 120 written)
        pairs_then_gather = nr * (8 + 8 + 8 + 12 + 240) + 2 * 12 * m_r
        # the same sort moving whole records: bitmap on the keys, tile pass
        # reading and writing records, every merge beyond the tile moving them
        record_merging = nr * (8 + 240) + 2 * 120 * m_r
        rec_out = {"records": nr, "record_bytes": 120, "key": "u64 in words 2-3", "ms_per_step": round(rms, 4),
                   "Mrecords_per_s": round(nr / (rms / 1e3) / 1e6, 1),
                   "record_GB_per_s": round(nr * 240 / (rms / 1e3) / 1e9, 1), "merge_cost_hbm": m_r,
                   "bytes_pairs_then_gather": pairs_then_gather, "bytes_record_merging": record_merging,
                   "byte_ratio": round(record_merging / pairs_then_gather, 2)}
        del rec, out_rec, rws
        torch.cuda.empty_cache()

    cfg_out = None
    if args.configs_steps > 0:
        cfg_out = bench_configs(vm, dev, args.configs_steps)

    batch_out = None
    if args.batch_nseg > 0:
        # the batched workload: arrays of 2^6..2^20 u32 keys (log-uniform
        # lengths; even arrays uniform, odd ones Zipf), one segmented call
        log(f"batch: generating {args.batch_nseg} arrays")
        bk, boff = workloads.batch32(args.batch_nseg, 1)
        nb = int(bk.size)
        src_b = torch.from_numpy(bk.view(np.int32)).to(dev)
        off_b = torch.from_numpy(boff).to(dev)
        kb_ = torch.empty_like(src_b)
        need = ctypes.c_size_t(0)
        vm.load_library().vmps_segmented_sort_workspace_size(nb, args.batch_nseg, vm.U32, 0, ctypes.byref(need))
        bws = torch.empty(need.value, dtype=torch.uint8, device=dev)
        tms = []
        for i in range(4):
            kb_.copy_(src_b)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vm.segmented_sort_(kb_, off_b, workspace=bws)
            e1.record()
            torch.cuda.synchronize()
            if i:
                tms.append(e0.elapsed_time(e1))
        bms = float(np.mean(tms))
        # algorithmic bytes: the tile pass reads and writes every key; arrays
        # longer than the LDS tile also have the descent bitmap read and
        # their merges beyond the tile (M_HBM) read and write.  Counted with
        # the 16384-key tile's schedule, the fewest bytes of the compiled
        # tiles (the tuned 8192-key tile sends more merges to HBM)
        T32 = 16384
        m_b, big = 0, 0
        for s in range(args.batch_nseg):
            a, b = int(boff[s]), int(boff[s + 1])
            if b - a > T32:
                big += b - a
                sch_b = vm.sort_schedule(src_b[a:b].contiguous())
                m_b += int((sch_b["node_r"].astype(np.int64) - sch_b["node_l"].astype(np.int64)).sum())
        b_alg = 4 * big + 8 * nb + 8 * m_b
        out_b = kb_.cpu().numpy().view(np.uint32)
        for s in range(0, args.batch_nseg, 97):
            a, b = int(boff[s]), int(boff[s + 1])
            assert np.array_equal(out_b[a:b], np.sort(bk[a:b])), "batch: segment not sorted"
        tu = vm.get_tuning(vm.U32, False)
        batch_out = {"arrays": args.batch_nseg, "keys": nb, "key_bits": 32, "ms_per_step": round(bms, 4),
                     "lds_tile": tu["tile_elems"] or T32, "tile_threads": tu["tile_threads"] or 512,
                     "value": round(nb / (bms / 1e3) / 1e9, 4), "unit": "Gkeys/s", "merge_cost_hbm": m_b,
                     "bytes_alg": b_alg, "achieved_GBs": round(b_alg / (bms / 1e3) / 1e9, 1),
                     "frac": round(b_alg / (bms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del src_b, off_b, kb_, bws
        torch.cuda.empty_cache()

    value = n / (ms / 1e3) / 1e9
    kinds = {k: v for k, v in trace.items() if v[1] > 0}
    dom = max(kinds, key=lambda k: kinds[k][0])
    dom_ms, dom_launches = kinds[dom]
    m_hbm = m_hbm_plain if args.path == "plain" else 0
    bytes_per_sort = kernel_bytes(args.path, dom, n, 8, 0, m_hbm, cfg.sample_size)
    achieved = bytes_per_sort * TRACED / (dom_ms / 1e3) / 1e9
    # HBM bytes per launch measured by rocprofv3 counters for this kernel, while
    # its source is unchanged since they were taken
    from paper_2605_27147_amd import profiling
    tfile = os.path.join(ROOT, "profiles", f"traffic_{args.path}_lognormal64_2p{args.log2n}_{dom}.json")
    tr = profiling.load_traffic(tfile)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(tr["traffic_bytes_per_launch"]) if tr else None,
                "traffic_source": os.path.relpath(tfile, ROOT) if tr else None, "kernel": dom,
                "avg_launch_ms": round(dom_ms / dom_launches, 4),
                "launches_per_step": dom_launches / TRACED,
                "bytes_per_launch": bytes_per_sort * TRACED / dom_launches}
    # the same kernel against the LDS and the VALU-issue roofs: LDS bytes and
    # wave-level VALU instructions per launch from rocprofv3 SQ counters
    # (while its source is unchanged since they were taken), over the live
    # average launch time
    cfile = os.path.join(ROOT, "profiles", f"counters_{args.path}_lognormal64_2p{args.log2n}_{dom}.json")
    cn = profiling.load_counters(cfile)
    if cn:
        pl = cn["per_launch"]
        launch_s = dom_ms / dom_launches / 1e3
        lds_b = 64.0 * (pl["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + pl["SQ_INSTS_LDS_STORE_BANDWIDTH"])
        roofline["lds"] = {"achieved": round(lds_b / launch_s / 1e9, 1), "peak": LDS_PEAK_GBS, "unit": "GB/s",
                           "frac": round(lds_b / launch_s / 1e9 / LDS_PEAK_GBS, 4), "bytes_per_launch": lds_b,
                           "bank_conflict_share": round(pl["SQ_LDS_BANK_CONFLICT"] / pl["SQ_LDS_IDX_ACTIVE"], 4)}
        roofline["valu"] = {"achieved": round(pl["SQ_INSTS_VALU"] / launch_s / 1e9, 1), "peak": VALU_PEAK_GIPS,
                            "unit": "G wave-instructions/s",
                            "frac": round(pl["SQ_INSTS_VALU"] / launch_s / 1e9 / VALU_PEAK_GIPS, 4),
                            "instructions_per_launch": pl["SQ_INSTS_VALU"]}
        roofline["counters_source"] = os.path.relpath(cfile, ROOT)
        roofline["binding_roof"] = max(("hbm", roofline["frac"]), ("lds", roofline["lds"]["frac"]),
                                       ("valu", roofline["valu"]["frac"]), key=lambda t: t[1])[0]
    breakdown = {k: {"ms_per_step": round(v[0] / TRACED, 4), "launches_per_step": v[1] / TRACED}
                 for k, v in kinds.items()}
    path_bytes = sum(kernel_bytes(args.path, k, n, 8, 0, m_hbm, cfg.sample_size) for k in kinds)

    cfgd = {"workload": f"lognormal64: n=2^{args.log2n} uint64 keys floor(exp(2 N(0,1)) 2^40), stable sort, "
                        f"{args.path} Powersort path", "n": n, "key_bits": 64, "values": False, "path": args.path,
            "lds_tile": sch["tile"]}
    if args.path == "learned":
        cfgd.update({"buckets": stats["buckets"], "sample": int(cfg.sample_size), "hidden": cfg.hidden,
                     "adam_steps": cfg.steps, "fallback_keys": stats["fallback_keys"],
                     "fallback_buckets": stats["fallback_buckets"], "max_bucket": stats["max_bucket"],
                     "model_loss_init": stats["loss_init"], "model_loss_final": stats["loss_final"],
                     "init_model_fallback_keys": stats0["fallback_keys"],
                     "init_model_max_bucket": stats0["max_bucket"]})
    else:
        cfgd.update({"merge_cost": sch["merge_cost"], "merge_cost_hbm": m_hbm_plain, "runs": sch["runs"]})
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "ms_per_step_median": round(MEDIAN[args.path], 4),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic", "config": cfgd, "roofline": roofline,
        "path_roofline": {"bytes_per_step": path_bytes, "achieved_GBs": round(path_bytes / (ms / 1e3) / 1e9, 1),
                          "frac": round(path_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "breakdown": breakdown,
    }
    # the goal set for this path: the whole path at 60% of HBM peak
    out["target"] = {"hbm_frac_goal": 0.6, "path_frac": out["path_roofline"]["frac"],
                     "dominant_kernel_frac": roofline["frac"], "met": out["path_roofline"]["frac"] >= 0.6}
    if vm_out is not None:
        out["vm"] = vm_out
    if rec_out is not None:
        out["records"] = rec_out
    if batch_out is not None:
        out["batch"] = batch_out
    if cfg_out is not None:
        out["configs"] = cfg_out
    if other_ms is not None:
        out["compare"] = {"path": other, "ms_per_step": round(other_ms, 4),
                          "value": round(n / (other_ms / 1e3) / 1e9, 4), "unit": "Gkeys/s"}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        import oracle
        oracle.build()
        msz = min(n, 1 << args.cpu_sample_log2)
        sample = np.ascontiguousarray(keys_np[:msz])
        # one host core: the oracle is single-threaded; pin it so the time
        # is one core's
        prev = os.sched_getaffinity(0)
        core = min(prev)
        os.sched_setaffinity(0, {core})
        try:
            t0 = time.perf_counter()
            oracle.powersort(sample)
            dt = time.perf_counter() - t0
        finally:
            os.sched_setaffinity(0, prev)
        cpu_model = "unknown"
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        cpu_model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        out["cpu_baseline"] = {"value": round(msz / dt / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
                               "sample": f"first 2^{args.cpu_sample_log2} keys of the same lognormal input, "
                                         f"single-threaded oracle Powersort (Pingpong) in {dt:.2f} s, "
                                         f"pinned to host core {core}",
                               "host_cpu": cpu_model, "host_nproc": os.cpu_count(),
                               "host_cores_allowed": len(prev)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
