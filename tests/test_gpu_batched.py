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


@pytest.mark.parametrize("tile_wg, merge_grid, bucket_div, host_wait", [(1, 256, 2, 1), (2, 4096, 4, 0), (0, 0, 3, 0)])
def test_tuning_never_changes_results(vm, orc, tile_wg, merge_grid, bucket_div, host_wait):
    import torch
    keys_np, off = workloads.batch32(128, 45, lengths=workloads.batch_lengths(128, 45, hi_log2=17))
    want, _ = orc.segmented_powersort(keys_np, off)
    x = workloads.lognormal(1 << 19, 46)
    wantx, _, _, _ = orc.powersort(x)
    try:
        vm.set_tuning(vm.U32, False, tile_wg, merge_grid, bucket_div, host_wait)
        vm.set_tuning(vm.U64, False, tile_wg, merge_grid, bucket_div, host_wait)
        keys = _t(keys_np)
        vm.segmented_sort_(keys, torch.from_numpy(off).cuda())
        assert np.array_equal(_np(keys, np.uint32), want.astype(np.uint32))
        k2 = _t(x)
        vm.sort_learned_(k2)
        assert np.array_equal(_np(k2, np.uint64), wantx)
    finally:
        vm.reset_tuning(vm.U32, False)
        vm.reset_tuning(vm.U64, False)
