"""vmps_sort_noalloc (workspace in the library's fixed device array) against
vmps_sort (caller workspace) through the C ABI: element by element, on two
calls in a row with the second one smaller, so that the second call runs on
what the first one left in the array.  Also the host-side rejection of a
sort larger than the array."""
import ctypes

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
    if x.dtype == np.uint64:
        return torch.from_numpy(x.view(np.int64).copy()).cuda()
    return torch.from_numpy(x.view(np.int32).copy()).cuda()


def _np(t, dtype):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype)


def _pair(vm, x, values):
    """(keys, values) after vmps_sort and after vmps_sort_noalloc."""
    import torch
    dt = x.dtype
    out = []
    for noalloc in (False, True):
        keys = _t(x)
        vals = None
        if values:
            vals = torch.full((x.size,), -1, dtype=torch.int32, device="cuda")
        if noalloc:
            vm.sort_noalloc_(keys, vals, iota=values)
        else:
            vm.sort_(keys, vals, iota=values)
        out.append((_np(keys, dt), None if vals is None else _np(vals, np.uint32)))
    return out


@pytest.mark.parametrize("bits,values", [(64, True), (32, False), (64, False)])
def test_noalloc_matches_sort_twice(vm, bits, values):
    sizes = [(1 << 22) - 12345, (1 << 17) + 77]   # second call smaller
    for i, n in enumerate(sizes):
        print("noalloc", bits, values, "call", i, "n", n, flush=True)
        if bits == 64:
            x = workloads.mixture(n, 60 + i) if i == 0 else workloads.presorted(n, 61, mean_run=500)
        else:
            x = workloads.uniform(n, 32, 62 + i)
        (k0, v0), (k1, v1) = _pair(vm, x, values)
        assert np.array_equal(k0, k1)
        if values:
            assert np.array_equal(v0, v1)
        # and the result is the sort itself
        order = np.argsort(x, kind="stable")
        assert np.array_equal(k1, x[order])
        if values:
            assert np.array_equal(v1, order.astype(np.uint32))


def test_noalloc_rejects_oversize(vm):
    import torch
    lib = vm.load_library()
    cap = vm.noalloc_scratch_bytes()
    assert cap == 96 << 20
    n = 1 << 23   # u64 keys with values need about 164 MiB of workspace
    keys = torch.zeros(n, dtype=torch.int64, device="cuda")
    vals = torch.zeros(n, dtype=torch.int32, device="cuda")
    st = lib.vmps_sort_noalloc(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()), n, vm.U64, 0,
                               None)
    assert st == vm.WORKSPACE_TOO_SMALL
    torch.cuda.synchronize()
    assert int(keys.abs().sum().item()) == 0   # nothing enqueued
