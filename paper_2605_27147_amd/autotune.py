"""Autotuner for the launch parameters (vmps_set_tuning).

    python -m paper_2605_27147_amd.autotune [--out PATH] [--log2n 28] [--batch 4096]

For each tuned configuration it times every candidate on its workload
(median of a few steps after a warm-up, input restored before each step),
checks that every candidate produces byte-identical output, and writes the
fastest into the JSON table the binding loads with the library
(paper_2605_27147_amd/autotune.json), keyed by the GPU architecture.

  u64 keys (learned path): lognormal keys, n = 2^log2n
  u32 keys (segmented path): `batch` arrays of log-uniform length in [2^6, 2^20]
  u64 keys with values, u32 keys with values (plain path): (key, index)
      pairs of n = 2^(log2n - 2) lognormal / uniform keys

The candidates cover the persistent tile pass's workgroups per CU, the
merge-level grid, the merge tile's outputs per thread (merge_ki 8 or 16:
tiles of 2048 or 4096 elements), for the learned path the bucket size, and
for the segmented sort of u32 keys the LDS tile and its workgroup size
(512 threads x 16384 keys, 512 x 8192 or 256 x 8192).
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _median_ms(run, restore, steps):
    import torch
    ts = []
    for i in range(steps + 1):
        restore()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        torch.cuda.synchronize()
        if i:
            ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def tune(space, apply, reset, run, restore, output, steps):
    import torch
    results, ref = [], None
    for cand in space:
        apply(cand)
        try:
            ms = _median_ms(run, restore, steps)
            out = output()
            if ref is None:
                ref = out.clone()
            same = bool(torch.equal(out, ref))
        finally:
            reset()
        results.append({**cand, "ms": round(ms, 4), "identical": same})
        print(json.dumps(results[-1]), flush=True)
        if not same:
            raise SystemExit(f"candidate {cand} changed the output")
    best = min(results, key=lambda r: r["ms"])
    return best, results


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "autotune.json"))
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=3)
    a = ap.parse_args(argv)

    import torch
    import paper_2605_27147_amd as vm
    import workloads

    vm.load_library()
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    entries = []

    # u64 keys, learned path
    n = 1 << a.log2n
    x = workloads.lognormal(n, 5)
    pristine = torch.from_numpy(x.view(np.int64)).to(dev)
    keys = torch.empty_like(pristine)
    cfg = vm.learned_default_config(n, vm.U64)
    ws = torch.empty(vm.learned_workspace_size(n, vm.U64, False, cfg) + (1 << 20), dtype=torch.uint8, device=dev)
    fields = ("tile_wg_per_cu", "merge_grid", "bucket_div", "merge_ki", "tile_elems", "tile_threads")
    # merge_ki stays at its default here: this entry (u64 keys, no values)
    # also serves the plain sort of u64 keys, whose merge levels need the
    # 4096-element tiles (2048 measured 7% slower there), while the learned
    # sort's few merges cannot tell the two apart
    space = [{"tile_wg_per_cu": t, "merge_grid": m, "bucket_div": b, "merge_ki": 0, "tile_elems": 0,
              "tile_threads": 0}
             for t, m, b in itertools.product([0, 1], [1024, 2048], [0, 4])]
    best, res = tune(space,
                     lambda c: vm.set_tuning(vm.U64, False, **c), lambda: vm.reset_tuning(vm.U64, False),
                     lambda: vm.sort_learned_(keys, workspace=ws, read_stats=False),
                     lambda: keys.copy_(pristine), lambda: keys, a.steps)
    entries.append({"dtype": "u64", "values": False, **{k: best[k] for k in fields},
                    "workload": f"learned sort, lognormal n=2^{a.log2n}", "ms": best["ms"], "candidates": res})
    del pristine, keys, ws
    torch.cuda.empty_cache()

    # u32 keys, segmented path
    kb, off = workloads.batch32(a.batch, 4)
    pristine = torch.from_numpy(kb.view(np.int32)).to(dev)
    offs = torch.from_numpy(off).to(dev)
    keys = torch.empty_like(pristine)
    # the LDS tile and the workgroup size of its pass: 512 x 16384 (32 keys
    # per thread), 512 x 8192 (16) and 256 x 8192 (32)
    space = [{"tile_wg_per_cu": t, "merge_grid": m, "bucket_div": 0, "merge_ki": k, "tile_elems": te,
              "tile_threads": tt}
             for t, m, k, (te, tt) in itertools.product([0, 1], [1024, 2048, 4096], [0, 8],
                                                        [(0, 0), (8192, 512), (8192, 256)])]
    best, res = tune(space,
                     lambda c: vm.set_tuning(vm.U32, False, **c), lambda: vm.reset_tuning(vm.U32, False),
                     lambda: vm.segmented_sort_(keys, offs), lambda: keys.copy_(pristine), lambda: keys, a.steps)
    entries.append({"dtype": "u32", "values": False, **{k: best[k] for k in fields},
                    "workload": f"segmented sort, {a.batch} arrays, {kb.size} keys", "ms": best["ms"],
                    "candidates": res})
    del pristine, offs, keys
    torch.cuda.empty_cache()

    # (key, index) pairs, plain path: u64 and u32 keys
    npairs = 1 << (a.log2n - 2)
    for dtype, code, gen, ki_alt in (("u64", vm.U64, lambda: workloads.lognormal(npairs, 8), 16),
                                     ("u32", vm.U32, lambda: workloads.uniform(npairs, 32, 9), 8)):
        xk = gen()
        pristine = torch.from_numpy(xk.view(np.int64 if dtype == "u64" else np.int32)).to(dev)
        keys = torch.empty_like(pristine)
        vals = torch.empty(npairs, dtype=torch.int32, device=dev)
        pws = torch.empty(vm.sort_workspace_size(npairs, code, True), dtype=torch.uint8, device=dev)
        space = [{"tile_wg_per_cu": t, "merge_grid": m, "bucket_div": 0, "merge_ki": k, "tile_elems": 0,
                  "tile_threads": 0}
                 for t, m, k in itertools.product([0, 1], [1024, 2048, 4096], [0, ki_alt])]
        best, res = tune(space,
                         lambda c, code=code: vm.set_tuning(code, True, **c),
                         lambda code=code: vm.reset_tuning(code, True),
                         lambda: vm.sort_(keys, vals, iota=True, workspace=pws),
                         lambda: keys.copy_(pristine), lambda: vals, a.steps)
        entries.append({"dtype": dtype, "values": True, **{k: best[k] for k in fields},
                        "workload": f"plain sort of (key, index) pairs, n=2^{a.log2n - 2}", "ms": best["ms"],
                        "candidates": res})
        del pristine, keys, vals, pws
        torch.cuda.empty_cache()

    table = {"arch": arch, "cus": props.multi_processor_count,
             "generated": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}
    with open(a.out, "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
