"""The segmented (batched) launcher: graph capture and replay, and launch
tuning, both checked against eager runs and the oracle bit for bit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_27147_amd as vm
    vm.load_library()
    return vm


def _t(x):
    import torch
    return torch.from_numpy(x.view(np.int64 if x.dtype == np.uint64 else np.int32).copy()).cuda()


def _np(t, dtype):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype)


def _say(*a):
    print(*a, flush=True)


def test_segmented_graph_replays_match_eager_and_oracle(vm, orc):
    import torch
    keys_np, off = workloads.batch32(384, 41, lengths=workloads.batch_lengths(384, 41, hi_log2=17))
    _say("graph batch", keys_np.size, off.size - 1)
    want, _ = orc.segmented_powersort(keys_np, off)
    pristine = _t(keys_np)
    offs = torch.from_numpy(off).cuda()
    keys = pristine.clone()
    vm.segmented_sort_(keys, offs)
    eager = _np(keys, np.uint32).copy()
    assert np.array_equal(eager, want.astype(np.uint32))
    keys.copy_(pristine)
    g = vm.segmented_sort_graph(keys, offs)
    for rep in range(3):
        keys.copy_(pristine)
        torch.cuda.synchronize()
        g.replay()
        got = _np(keys, np.uint32)
        assert np.array_equal(got, eager), rep
        # unrelated eager work between replays
        torch.cuda.synchronize()
        (pristine.float() * 2).sum().item()
    g.close()


def test_segmented_graph_with_values(vm, orc):
    import torch
    keys_np, off = workloads.batch32(96, 43, lengths=workloads.batch_lengths(96, 43, hi_log2=16))
    n = keys_np.size
    v = np.random.default_rng(5).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    want, wantv = orc.segmented_powersort(keys_np, off, v)
    keys, vals = _t(keys_np), _t(v)
    offs = torch.from_numpy(off).cuda()
    g = vm.segmented_sort_graph(keys, offs, vals)
    for rep in range(2):
        keys.copy_(_t(keys_np))
        vals.copy_(_t(v))
        g.replay()
        assert np.array_equal(_np(keys, np.uint32), want.astype(np.uint32)), rep
        assert np.array_equal(_np(vals, np.uint32), wantv), rep
    g.close()


def test_learned_graph_replays_match_oracle(vm, orc):
    import torch
    x = workloads.lognormal(1 << 20, 44)
    want, _, _, _ = orc.powersort(x)
    pristine = _t(x)
    keys = pristine.clone()
    g = vm.sort_learned_graph(keys)
    for rep in range(3):
        keys.copy_(pristine)
        g.replay()
        assert np.array_equal(_np(keys, np.uint64), want), rep
        torch.cuda.synchronize()
    g.close()


@pytest.mark.parametrize("tile_wg, merge_grid, bucket_div, host_wait, merge_ki",
                         [(1, 256, 2, 1, 8), (2, 4096, 4, 0, 16), (0, 0, 3, 0, 0), (0, 0, 0, 0, 8)])
def test_tuning_never_changes_results(vm, orc, tile_wg, merge_grid, bucket_div, host_wait, merge_ki):
    import torch
    keys_np, off = workloads.batch32(128, 45, lengths=workloads.batch_lengths(128, 45, hi_log2=17))
    want, _ = orc.segmented_powersort(keys_np, off)
    x = workloads.lognormal(1 << 19, 46)
    wantx, _, _, _ = orc.powersort(x)
    try:
        for hv in (False, True):
            vm.set_tuning(vm.U32, hv, tile_wg, merge_grid, bucket_div, host_wait, merge_ki)
            vm.set_tuning(vm.U64, hv, tile_wg, merge_grid, bucket_div, host_wait, merge_ki)
        keys = _t(keys_np)
        vm.segmented_sort_(keys, torch.from_numpy(off).cuda())
        assert np.array_equal(_np(keys, np.uint32), want.astype(np.uint32))
        k2 = _t(x)
        vm.sort_learned_(k2)
        assert np.array_equal(_np(k2, np.uint64), wantx)
        # plain sorts of (key, index) pairs at both merge tile sizes
        for bits in (32, 64):
            xp = workloads.uniform(300007, bits, 47)
            kp = _t(xp)
            vp = torch.empty(xp.size, dtype=torch.int32, device="cuda")
            vm.sort_(kp, vp, iota=True)
            _, wantv, _, _ = orc.powersort(xp, np.arange(xp.size, dtype=np.uint32))
            assert np.array_equal(_np(vp, np.uint32), wantv), bits
    finally:
        for hv in (False, True):
            vm.reset_tuning(vm.U32, hv)
            vm.reset_tuning(vm.U64, hv)



@pytest.mark.parametrize("tile_threads, extra", [(512, {}), (256, {}),
                                                 (256, {"tile_wg_per_cu": 1, "merge_ki": 8, "merge_grid": 1024})])
def test_segmented_tuned_tile_8192(vm, orc, tile_threads, extra):
    """The segmented sort on the 8192-element LDS tile (u32 keys without
    values, 512 or 256 threads a workgroup): eager and graph replays against
    the oracle, with segment lengths around both tile sizes, single natural
    runs longer than the tile, duplicates, and empty segments."""
    import torch
    g0 = np.random.default_rng(48)
    keys_np, off = workloads.batch32(96, 48, lengths=workloads.batch_lengths(96, 48, hi_log2=17))
    parts, lens = [keys_np], list(np.diff(off))
    for ln in (0, 1, 2, 31, 32, 33, 4095, 4096, 4097, 8191, 8192, 8193, 12000, 16383, 16384, 16385, 40000, 0):
        parts.append(g0.integers(0, 2**32, ln, dtype=np.uint64).astype(np.uint32))
        lens.append(ln)
    for ln in (8193, 20000):
        parts.append(np.sort(g0.integers(0, 2**32, ln, dtype=np.uint64).astype(np.uint32)))        # one run
        parts.append(np.sort(g0.integers(0, 2**32, ln, dtype=np.uint64).astype(np.uint32))[::-1].copy())
        parts.append(g0.integers(0, 16, ln, dtype=np.uint64).astype(np.uint32))                   # duplicates
        lens += [ln, ln, ln]
    kn = np.concatenate(parts).astype(np.uint32)
    offs_np = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    _say("tuned tile 8192 x", tile_threads, "keys", kn.size, "segments", offs_np.size - 1)
    want, _ = orc.segmented_powersort(kn, offs_np)
    want = want.astype(np.uint32)
    pristine = _t(kn)
    offs = torch.from_numpy(offs_np).cuda()
    try:
        vm.set_tuning(vm.U32, False, tile_elems=8192, tile_threads=tile_threads, **extra)
        keys = pristine.clone()
        vm.segmented_sort_(keys, offs)
        assert np.array_equal(_np(keys, np.uint32), want)
        g = vm.segmented_sort_graph(keys, offs)
        for rep in range(3):
            keys.copy_(pristine)
            torch.cuda.synchronize()
            g.replay()
            assert np.array_equal(_np(keys, np.uint32), want), rep
            (pristine.float() * 2).sum().item()
        g.close()
    finally:
        vm.reset_tuning(vm.U32, False)
    # back on the default tile, the same workspace size query still fits
    keys = pristine.clone()
    vm.segmented_sort_(keys, offs)
    assert np.array_equal(_np(keys, np.uint32), want)


def test_segmented_long_runs_across_instances(vm, orc):
    """Segments longer than the tile made of natural runs of 33 to 70 keys
    (thousands of long runs, so the planner's run-start chain spans several
    blocks and sub-blocks, with instances opening inside them), next to
    short random segments; each segment against the oracle."""
    import torch
    rng = np.random.default_rng(49)
    parts, lens = [], []
    for sidx in range(40):
        if sidx % 3 == 2:
            ln = int(rng.integers(0, 3000))
            parts.append(rng.integers(0, 2**32, ln, dtype=np.uint64).astype(np.uint32))
        else:
            ln = int(rng.integers(17000, 90000))
            x = rng.integers(0, 2**32, ln, dtype=np.uint64).astype(np.uint32)
            pos = 0
            while pos < ln:
                L = int(rng.integers(33, 71))
                x[pos:pos + L] = np.sort(x[pos:pos + L])
                pos += L + int(rng.integers(0, 2))
            parts.append(x)
        lens.append(ln)
    kn = np.concatenate(parts).astype(np.uint32)
    offs_np = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    _say("long-run segments", kn.size, len(lens))
    want, _ = orc.segmented_powersort(kn, offs_np)
    keys = _t(kn)
    vals = torch.arange(kn.size, dtype=torch.int32, device="cuda")
    vm.segmented_sort_(keys, torch.from_numpy(offs_np).cuda(), vals)
    got = _np(keys, np.uint32)
    assert np.array_equal(got, want.astype(np.uint32))
    # the index payload is the stable permutation of every segment
    gv = _np(vals, np.uint32).astype(np.int64)
    for a, b in zip(offs_np[:-1], offs_np[1:]):
        assert np.array_equal(gv[a:b], a + np.argsort(kn[a:b], kind="stable"))

def _brute_force_segments():
    """Every permutation of 0..n-1 for n <= 9 and every word over {0,1,2} of
    length n <= 12, each as one segment (u32 keys), in one array."""
    import itertools
    parts, lengths = [], []
    for n in range(1, 10):
        p = np.array(list(itertools.permutations(range(n))), dtype=np.uint32)
        parts.append(p.ravel())
        lengths += [n] * p.shape[0]
    for n in range(1, 13):
        w = np.indices((3,) * n, dtype=np.uint32).reshape(n, -1).T
        parts.append(np.ascontiguousarray(w).ravel())
        lengths += [n] * w.shape[0]
    x = np.concatenate(parts)
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return x, off


def test_segmented_brute_force_tiny_inputs(vm, orc):
    """Tiny inputs exhaustively, through the batched path in one call: every
    permutation of n <= 9 and every {0,1,2}^n word of n <= 12 (1.21 M
    segments, 12.8 M keys) with their positions as values, against the
    definition (the unique order by segment, key, then position) and the
    oracle's per-segment Powersort."""
    import torch
    x, off = _brute_force_segments()
    total, nseg = x.size, off.size - 1
    _say("brute force segments", nseg, "keys", total)
    seg = np.repeat(np.arange(nseg, dtype=np.int64), np.diff(off))
    order = np.lexsort((np.arange(total), x, seg))
    want_k, want_v = x[order], order.astype(np.uint32)
    ok, ov = orc.segmented_powersort(x, off, vals=np.arange(total, dtype=np.uint32))
    assert np.array_equal(ok.astype(np.uint32), want_k) and np.array_equal(ov, want_v)
    keys = _t(x)
    vals = _t(np.arange(total, dtype=np.uint32))
    vm.segmented_sort_(keys, torch.from_numpy(off).cuda(), vals)
    assert np.array_equal(_np(keys, np.uint32), want_k)
    assert np.array_equal(_np(vals, np.uint32), want_v)
