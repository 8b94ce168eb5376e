"""Virtual-Memory Powersort on the GPU (vmps_sort_vm, Section 4): paged
merge levels with a free sequence of pages, a page table and the final
page-permuting Copy.  Output against the oracle element by element (keys,
values, stable permutation); the page merges write exactly the merge cost of
the nodes longer than a tile (the oracle's M_hbm); no page is handed out
before it is free (the device's schedule check); extra memory against the
second Pingpong buffer."""
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


def _tile(bits, has_values):
    if bits == 32:
        return 8192 if has_values else 16384
    return 4096 if has_values else 8192


def _inputs(bits):
    dt = np.uint32 if bits == 32 else np.uint64
    rng = np.random.default_rng(17)
    yield "uniform_ragged", workloads.uniform((1 << 20) + 12345, bits, 3)
    yield "presorted", workloads.presorted(1 << 19, 4, mean_run=3000, bits=bits).astype(dt)
    yield "dup16", workloads.dup16(1 << 18, 5).astype(dt) if bits == 64 else (workloads.dup16(1 << 18, 5) & 0xFFFFFFFF).astype(dt)
    yield "sorted", np.arange(300000, dtype=dt)
    yield "reverse", np.arange(300001, dtype=dt)[::-1].copy()
    yield "pages_exact", rng.integers(0, 1000, 4096 * 37).astype(dt)  # n a multiple of every page length
    yield "one_tile", rng.integers(0, 2**31, 5000).astype(dt)
    yield "tile_plus_one", rng.integers(0, 50, 16385).astype(dt)
    yield "two", np.array([2, 1], dtype=dt)


def _check(vm, orc, x, values, window, desc, bits):
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    n = x.size
    v = np.random.default_rng(n).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    variant = orc.DESC_RUNS if desc else orc.PINGPONG
    want, wantv, st, _ = orc.powersort(x, v if values == "input" else np.arange(n, dtype=np.uint32), variant=variant)
    stats = torch.full((vm.VM_STATS,), -1, dtype=torch.int64, device="cuda")
    keys = _t(x)
    vals = None
    if values == "input":
        vals = _t(v)
        vm.sort_vm_(keys, vals, desc=desc, window_pages=window, stats=stats)
    elif values == "iota":
        vals = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        vm.sort_vm_(keys, vals, iota=True, desc=desc, window_pages=window, stats=stats)
    else:
        vm.sort_vm_(keys, desc=desc, window_pages=window, stats=stats)
    got = _np(keys, dt)
    s = _np(stats, np.int64)
    if not np.array_equal(got, want.astype(dt)):
        bad = np.nonzero(got != want.astype(dt))[0]
        P = vm.vm_layout(n, vm.U32 if bits == 32 else vm.U64, values != "none", window)["page_elems"]
        _say("  wrong", bad.size, "first", bad[:8].tolist(), "pages", sorted(set((bad // P).tolist()))[:16],
             "stats", s.tolist())
    assert np.array_equal(got, want.astype(dt))
    if vals is not None:
        assert np.array_equal(_np(vals, np.uint32), wantv)
    assert s[0] == 0, "a page was handed out before it was free"
    # the page merges write each node longer than a tile once, but for the
    # pages a merge leaves in place
    T = _tile(bits, values != "none")
    b = orc.extract_runs(x, desc=desc)
    _, _, _, _, m_hbm = orc.plan(b, n, orc.run_powers(b, n), T)
    assert s[3] + s[6] == m_hbm
    assert 0 <= s[2] <= n and s[1] >= 0
    return s


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("values", ["none", "input", "iota"])
def test_vm_sort_matches_oracle(vm, orc, bits, values):
    for name, x in _inputs(bits):
        _say("vm sort", bits, values, name, x.size)
        _check(vm, orc, x, values, 0, False, bits)


@pytest.mark.parametrize("window", [1, 2, 7, 64])
def test_vm_small_windows(vm, orc, window):
    """Rounds of 1, 2, 7 and 64 pages: many rounds per level, the pool at its
    smallest (window + 9 pages), pages recycled across rounds."""
    for bits in (32, 64):
        for name, x in (("uniform", workloads.uniform(300007, bits, 11)),
                        ("presorted", workloads.presorted(400000, 12, mean_run=500, bits=bits))):
            for values in ("none", "input"):
                _say("vm window", window, bits, name, values)
                _check(vm, orc, x.astype(np.uint32 if bits == 32 else np.uint64), values, window, False, bits)


def test_vm_descending_runs(vm, orc):
    """With the reversal of strictly decreasing runs (Section 5 remark):
    long decreasing runs are reversed in place by the tile pass."""
    for bits in (32, 64):
        dt = np.uint32 if bits == 32 else np.uint64
        for name, x in (("presorted_c2", workloads.presorted(1 << 18, 5, mean_run=1000, bits=bits).astype(dt)),
                        ("long_desc", np.concatenate([np.arange(30000, 0, -1) + 100000 * i
                                                      for i in range(9)]).astype(dt)),
                        ("reverse", np.arange(1 << 18, dtype=dt)[::-1].copy())):
            for values in ("none", "iota"):
                _say("vm desc", bits, name, values)
                _check(vm, orc, x, values, 3, True, bits)


def test_vm_memory_2p24(vm, orc):
    """n = 2^24 u64 keys with values: the same sort as vmps_sort, with pool
    and Copy pages under a tenth of the second Pingpong buffer (n * 12
    bytes)."""
    import torch
    n = 1 << 24
    x = workloads.uniform(n, 64, 21)
    lay = vm.vm_layout(n, vm.U64, True)
    _say("vm layout", lay)
    assert lay["buffer_bytes"] < 0.1 * n * 12
    want, wantv, _, _ = orc.powersort(x, np.arange(n, dtype=np.uint32))
    keys = _t(x)
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(vm.VM_STATS, dtype=torch.int64, device="cuda")
    vm.sort_vm_(keys, vals, iota=True, stats=stats)
    assert np.array_equal(_np(keys, np.uint64), want)
    assert np.array_equal(_np(vals, np.uint32), wantv)
    s = _np(stats, np.int64)
    _say("vm stats", s.tolist())
    assert s[0] == 0


def test_vm_workspace_reuse(vm, orc):
    """Two sorts in a row through one workspace, the second smaller: nothing
    stale from the first call (carry marks, pool, page table) leaks."""
    import torch
    lay = vm.vm_layout(1 << 20, vm.U32, False, 5)
    ws = torch.empty(lay["workspace_bytes"], dtype=torch.uint8, device="cuda")
    for n, seed in ((1 << 20, 1), (700001, 2), (1 << 20, 3)):
        x = workloads.uniform(n, 32, seed)
        keys = _t(x)
        vm.sort_vm_(keys, window_pages=5, workspace=ws)
        assert np.array_equal(_np(keys, np.uint32), np.sort(x)), n


def test_vm_pages_kept_in_place(vm, orc):
    """The page-skipping merge: when runs of a sorted sequence overlap only
    where they meet, almost every merge output stays where it is (kept
    pages, no fresh page, no Copy for them); the output and the merge cost
    are unchanged."""
    for bits in (32, 64):
        dt = np.uint32 if bits == 32 else np.uint64
        # a sorted sequence with a small step back every 5000 keys: runs of
        # 5000 whose merges interleave two keys each
        x = np.arange(1 << 19, dtype=np.int64) + 10
        x[::5000] -= 2
        s = _check(vm, orc, x.astype(dt), "iota", 0, False, bits)
        _say("steps", bits, s.tolist())
        assert s[6] > 0.75 * (s[3] + s[6])
        # blocks of a sorted sequence in shuffled order: a merge of a lower
        # block with a higher one keeps its pages, the reverse moves them all
        x = np.arange(1 << 19, dtype=np.int64).reshape(64, -1)
        x = x[np.random.default_rng(bits).permutation(64)].reshape(-1).astype(dt)
        s = _check(vm, orc, x, "input", 0, False, bits)
        _say("blocks", bits, s.tolist())
        assert s[6] > 0 and s[3] > 0
