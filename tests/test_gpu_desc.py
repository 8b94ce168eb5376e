"""Descending-run reversal (VMPS_DESCENDING_RUNS; the remark on decreasing
runs in Section 5) on the GPU against the oracle's ExtractRun with the same
rule: run bounds element by element, and the sorts (keys, values, stable
permutation) element by element."""
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


def _desc_inputs(bits=64):
    dt = np.uint32 if bits == 32 else np.uint64
    rng = np.random.default_rng(91)
    yield "presorted_c2", workloads.presorted(1 << 18, 5, mean_run=1000, bits=bits).astype(dt)
    yield "half_reversed", workloads.presorted(100003, 6, mean_run=300, desc_frac=0.5, swap_frac=0.0,
                                               bits=bits).astype(dt)
    # strictly decreasing blocks of minrun .. 2 minrun: phase-dependent jumps
    for L in (32, 33, 40, 63, 64, 65, 200):
        n = 60013
        x = rng.integers(0, 2**31, n).astype(dt)
        pos = 0
        while pos < n:
            x[pos:pos + L] = np.sort(x[pos:pos + L])[::-1]
            pos += L + int(rng.integers(0, 3))
        yield f"desc_blocks{L}", x
    # increasing and decreasing runs sharing their end elements
    x = np.concatenate([np.arange(0, 50), np.arange(49, -1, -1), np.arange(1, 60), np.arange(58, 0, -1)] * 700)
    yield "zigzag", x.astype(dt)
    # ties inside decreasing stretches: only strict decreases are reversed
    yield "steps", np.repeat(np.arange(40000, 0, -1), 3).astype(dt)
    yield "reverse", np.arange(1 << 18, dtype=dt)[::-1].copy()
    yield "sorted", np.arange(1 << 17, dtype=dt)
    yield "uniform", workloads.uniform(70001, bits, 7)
    yield "tiny", np.array([5, 3, 1, 2, 4, 6, 0], dtype=dt)


@pytest.mark.parametrize("minrun", [0, 16, 40])
def test_extract_runs_desc_matches_oracle(vm, orc, minrun):
    for name, x in _desc_inputs():
        ell = minrun if minrun else orc.minrun(x.size)
        if minrun and x.size < minrun:
            continue
        _say("desc runs", name, x.size, ell)
        want = orc.extract_runs(x, ell, desc=True)
        got, r = vm.extract_runs(_t(x), minrun, desc=True)
        assert r == want.size - 1, name
        assert np.array_equal(_np(got, np.uint32).astype(np.int64), want), name


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("values", ["none", "input", "iota"])
def test_sort_desc_matches_oracle(vm, orc, bits, values):
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    extra = [("long_desc_runs", np.concatenate([np.arange(30000, 0, -1) + 100000 * i for i in range(9)]).astype(dt)),
             ("reverse_2p20", np.arange(1 << 20, dtype=dt)[::-1].copy())]
    for name, x in list(_desc_inputs(bits)) + extra:
        n = x.size
        _say("desc sort", bits, values, name, n)
        v = np.random.default_rng(n).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        want, wantv, st, _ = orc.powersort(x, v if values == "input" else np.arange(n, dtype=np.uint32),
                                           variant=orc.DESC_RUNS)
        keys = _t(x)
        if values == "none":
            vm.sort_(keys, desc=True)
        elif values == "input":
            vals = _t(v)
            vm.sort_(keys, vals, desc=True)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        else:
            vals = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            vm.sort_(keys, vals, iota=True, desc=True)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        assert np.array_equal(_np(keys, dt), want.astype(dt)), name


def test_presorted_2p24_desc_matches_oracle(vm, orc):
    """The presorted workload at its full size (n = 2^24 u64, geometric runs
    of mean 2^10, a tenth decreasing, 1% swaps) with the reversal, element
    by element, and the merge cost it saves (oracle counters)."""
    import torch
    x = workloads.presorted(1 << 24, 2)
    want, wantv, st1, _ = orc.powersort(x, np.arange(x.size, dtype=np.uint32), variant=orc.DESC_RUNS)
    _, _, st0, _ = orc.powersort(x)
    _say("M increasing-only", st0["merge_cost"], "M with reversal", st1["merge_cost"], "runs", st0["runs"],
         st1["runs"])
    keys = _t(x)
    vals = torch.empty(x.size, dtype=torch.int32, device="cuda")
    vm.sort_(keys, vals, iota=True, desc=True)
    assert np.array_equal(_np(keys, np.uint64), want)
    assert np.array_equal(_np(vals, np.uint32), wantv)
    assert st1["merge_cost"] < st0["merge_cost"]
