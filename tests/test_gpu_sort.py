"""GPU parity: the HIP path against the CPU oracle, element by element.

Every test calls libvmps.so through the C ABI (via the thin binding) on
seeded inputs from `workloads` and compares with the oracle on the same
bytes.  Integer results must be bit-exact.
"""
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
    if x.dtype == np.uint32:
        return torch.from_numpy(x.view(np.int32).copy()).cuda()
    return torch.from_numpy(x.copy()).cuda()


def _np(t, dtype):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(dtype)


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ merge --
@pytest.mark.parametrize("bits", [32, 64])
def test_merge_matches_standard_merge(vm, orc, bits):
    rng = np.random.default_rng(10 + bits)
    dt = np.uint32 if bits == 32 else np.uint64
    cases = [(0, 0), (0, 5), (7, 0), (1, 1), (4096, 4096), (4095, 4097), (10000, 3), (3, 10000),
             (123457, 54321), (1 << 18, 1 << 18)]
    for na, nb in cases:
        for kind in ("random", "ties", "disjoint"):
            if kind == "random":
                a = np.sort(rng.integers(0, 2**bits, na, dtype=np.uint64)).astype(dt)
                b = np.sort(rng.integers(0, 2**bits, nb, dtype=np.uint64)).astype(dt)
            elif kind == "ties":
                a = np.sort(rng.integers(0, 5, na)).astype(dt)
                b = np.sort(rng.integers(0, 5, nb)).astype(dt)
            else:
                a = np.arange(na, dtype=dt)
                b = np.arange(na, na + nb, dtype=dt)
            _say("merge", bits, na, nb, kind)
            va = np.arange(na, dtype=np.uint32)
            vb = np.arange(na, na + nb, dtype=np.uint32)
            want, wantv = orc.standard_merge(a, b, va, vb)
            if na + nb == 0:
                continue
            out, vout = vm.merge(_t(a), _t(b), _t(va), _t(vb))
            assert np.array_equal(_np(out, dt), want.astype(dt))
            assert np.array_equal(_np(vout, np.uint32), wantv)


# ------------------------------------------------------------- run chain --
def _run_inputs():
    rng = np.random.default_rng(77)
    yield "uniform", workloads.uniform(70001, 64, 1)
    yield "presorted1000", workloads.presorted(1 << 18, 2, mean_run=1000)
    yield "presorted40", workloads.presorted(100003, 3, mean_run=40, swap_frac=0.0)
    yield "presorted5000", workloads.presorted(1 << 20, 4, mean_run=5000)
    # natural runs of exactly minrun .. 2 minrun: the chain's phase-dependent jumps
    for L in (32, 33, 40, 47, 63, 64, 65):
        n = 90011
        x = rng.integers(0, 2**40, n).astype(np.uint64)
        pos = 0
        while pos < n:
            x[pos:pos + L] = np.sort(x[pos:pos + L])
            pos += L + int(rng.integers(0, 3))
        yield f"blocks{L}", x
    yield "sorted", np.arange(300000, dtype=np.uint64)
    yield "reverse", np.arange(300000, dtype=np.uint64)[::-1].copy()
    yield "equal", np.full(200000, 9, dtype=np.uint64)
    yield "tiny", workloads.uniform(50, 64, 5)


@pytest.mark.parametrize("minrun", [0, 16, 40])
def test_extract_runs(vm, orc, minrun):
    for name, x in _run_inputs():
        ell = minrun if minrun else orc.minrun(x.size)
        if minrun and x.size < minrun:
            continue
        _say("runs", name, x.size, ell)
        want = orc.extract_runs(x, ell)
        got, r = vm.extract_runs(_t(x), minrun)
        assert r == want.size - 1, name
        assert np.array_equal(_np(got, np.uint32).astype(np.int64), want), name


def test_run_powers(vm, orc):
    for name, x in _run_inputs():
        b = orc.extract_runs(x)
        want = orc.run_powers(b, x.size)
        got = vm.run_powers(_t(b.astype(np.uint32)), b.size - 1, x.size)
        _say("powers", name)
        assert np.array_equal(_np(got, np.uint8), want), name


def test_schedule_matches_oracle_plan(vm, orc):
    for name, x in _run_inputs():
        for has_values in (False, True):
            sch = vm.sort_schedule(_t(x), has_values)
            T = sch["tile"]
            b = orc.extract_runs(x)
            P = orc.run_powers(b, x.size)
            node_buf, depth, segs, M, Mh = orc.plan(b, x.size, P, T)
            nodes = orc.tree_nodes(b, x.size, P)
            hbm = nodes[(nodes[:, 2] - nodes[:, 0]) > T]
            _say("schedule", name, has_values, T, sch["runs"], hbm.shape[0], segs.shape[0])
            assert sch["runs"] == b.size - 1
            assert sch["merge_cost"] == M
            assert np.array_equal(sch["node_l"], hbm[:, 0]) and np.array_equal(sch["node_m"], hbm[:, 1])
            assert np.array_equal(sch["node_r"], hbm[:, 2]) and np.array_equal(sch["node_level"], hbm[:, 3])
            hbm_buf = node_buf[(nodes[:, 2] - nodes[:, 0]) > T]
            assert np.array_equal(sch["node_buf"], hbm_buf)
            got_segs = sorted(zip(sch["seg_start"].tolist(), sch["seg_end"].tolist(), sch["seg_buf"].tolist()))
            assert got_segs == sorted(map(tuple, segs.tolist()))


# ------------------------------------------------------------------ sort --
def _sort_inputs(bits):
    dt = np.uint32 if bits == 32 else np.uint64
    T = 16384 if bits == 32 else 8192
    for n in (2, 3, 63, 64, 65, 1000, T - 1, T, T + 1, 3 * T + 17, (1 << 20) + 12345):
        yield f"uniform{n}", workloads.uniform(n, bits, n)
    yield "presorted", workloads.presorted(1 << 20, 6, mean_run=1024, bits=bits).astype(dt)
    yield "presorted64", workloads.presorted(300007, 7, mean_run=64, bits=bits).astype(dt)
    if bits == 64:
        yield "mixture", workloads.mixture(1 << 20, 8)
        yield "lognormal", workloads.lognormal(1 << 20, 9)
        yield "dup16", workloads.dup16(1 << 19, 10)
    else:
        yield "paperS100", workloads.paper_workload(11, 100, n=1 << 20)
        yield "few", (workloads.uniform(1 << 20, 32, 12) % 7).astype(np.uint32)
    yield "sorted", np.arange(1 << 19, dtype=dt)
    yield "reverse", np.arange(1 << 19, dtype=dt)[::-1].copy()
    yield "equal", np.full(1 << 19, 3, dtype=dt)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("values", ["none", "input", "iota"])
def test_sort_matches_oracle(vm, orc, bits, values):
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    for name, x in _sort_inputs(bits):
        n = x.size
        _say("sort", bits, values, name, n)
        v = np.random.default_rng(n).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        want, wantv, _, _ = orc.powersort(x, v if values == "input" else np.arange(n, dtype=np.uint32))
        keys = _t(x)
        if values == "none":
            vm.sort_(keys)
        elif values == "input":
            vals = _t(v)
            vm.sort_(keys, vals)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        else:
            vals = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            vm.argsort_(keys, vals)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        assert np.array_equal(_np(keys, dt), want.astype(dt)), name


def test_sort_trivial_sizes(vm):
    import torch
    for n in (0, 1):
        k = torch.arange(n, dtype=torch.int64, device="cuda")
        v = torch.full((n,), 7, dtype=torch.int32, device="cuda")
        vm.argsort_(k, v)
        torch.cuda.synchronize()
        assert v.cpu().tolist() == list(range(n))


def test_sort_repeatable_with_poisoned_workspace(vm, orc):
    import torch
    x = workloads.presorted(1 << 20, 13, mean_run=500)
    want, _, _, _ = orc.powersort(x)
    n = x.size
    ws_bytes = vm.sort_workspace_size(n, vm.U64, False)
    for trial in range(3):
        ws = torch.full((ws_bytes,), 0xA5 if trial % 2 else 0x00, dtype=torch.uint8, device="cuda")
        keys = _t(x)
        vm.sort_(keys, workspace=ws)
        assert np.array_equal(_np(keys, np.uint64), want)


def _long_next_to_tiny(n, seed, bits):
    """Sorted runs of one to three keys next to sorted runs of up to half the
    input: the run structure whose long merges reach the highest power a
    merge longer than the tile can have, where the launched merge levels
    stop (2^p < 9 n / T)."""
    rng = np.random.default_rng(seed)
    parts, tot = [], 0
    while tot < n:
        L = min(int(rng.choice([1, 2, 3, int(rng.integers(1, n // 2 + 2))])), n - tot)
        parts.append(np.sort(rng.integers(0, 1 << (bits - 8), L)))
        tot += L
    return np.concatenate(parts).astype(np.uint32 if bits == 32 else np.uint64)


@pytest.mark.parametrize("bits", [32, 64])
def test_sort_long_runs_next_to_tiny_runs(vm, orc, bits):
    """Plain sort (keys, and the stable argsort) and paged sort on long runs
    next to tiny ones, against the oracle: no merge level the sorts skip
    holds a merge."""
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    for seed in range(3):
        for n in ((1 << 20) + 77, 3 << 19):
            x = _long_next_to_tiny(n, seed, bits)
            _say("long next to tiny", bits, seed, n)
            want, wantv, _, _ = orc.powersort(x, np.arange(n, dtype=np.uint32))
            keys = _t(x)
            vm.sort_(keys)
            assert np.array_equal(_np(keys, dt), want.astype(dt)), (seed, n)
            keys = _t(x)
            vals = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            vm.argsort_(keys, vals)
            assert np.array_equal(_np(keys, dt), want.astype(dt)), (seed, n)
            assert np.array_equal(_np(vals, np.uint32), wantv), (seed, n)
            keys = _t(x)
            vm.sort_vm_(keys, window_pages=3)
            assert np.array_equal(_np(keys, dt), want.astype(dt)), (seed, n)


# ------------------------------------------------------------- segmented --
@pytest.mark.parametrize("bits", [32, 64])
def test_segmented_sort_matches_oracle(vm, orc, bits):
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    T = 16384 if bits == 32 else 8192
    lengths = [0, 1, 2, 63, 64, 65, 0, T - 1, T, T + 1, 1000, 3 * T + 5, 1 << 17, 5, 0]
    rng = np.random.default_rng(bits)
    lengths += rng.integers(1, 5000, 40).tolist()
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    x = workloads.uniform(int(off[-1]), bits, 3)
    x[: off[6]] = np.sort(x[: off[6]])  # some presorted segments
    v = np.arange(x.size, dtype=np.uint32)
    want, wantv = orc.segmented_powersort(x, off, vals=v)
    keys, vals = _t(x), _t(v)
    vm.segmented_sort_(keys, torch.from_numpy(off).cuda(), vals)
    assert np.array_equal(_np(keys, dt), want.astype(dt))
    assert np.array_equal(_np(vals, np.uint32), wantv)


def test_segmented_batch_workload(vm, orc):
    import torch
    keys_np, off = workloads.batch32(256, 4)
    want, _ = orc.segmented_powersort(keys_np, off)
    keys = _t(keys_np)
    vm.segmented_sort_(keys, torch.from_numpy(off).cuda())
    assert np.array_equal(_np(keys, np.uint32), want.astype(np.uint32))


def test_segmented_bad_offsets_leave_keys(vm):
    import torch
    x = workloads.uniform(100000, 32, 1)
    off = np.array([0, 500, 400, 100000], dtype=np.int64)  # decreasing
    keys = _t(x)
    vm.segmented_sort_(keys, torch.from_numpy(off).cuda())
    assert np.array_equal(_np(keys, np.uint32), x)
