"""Parity at the benchmark sizes, in the launch configurations bench.py and
the batched workload use.

The oracle cannot sort 2^28 keys in a test's time, so the full-size results
are checked through properties that determine a stable sort exactly:

  * keys non-decreasing (unsigned order);
  * the values (the input index of each output key, from the iota mode or
    from index payloads) hit every index once, and gathering the input at
    them gives the output keys, so the output is a permutation of the input
    that carries each key with its index;
  * among equal keys the indices increase (stability).

A key-only sort of the same input must then equal those keys.  The oracle
itself checks the 2^24 presorted input element by element and a sample of
whole segments of the batch.
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


def _say(*a):
    print(*a, flush=True)


def _unsigned(t):
    """Order-preserving signed view of unsigned keys held in a signed tensor."""
    import torch
    if t.dtype == torch.int64:
        return t ^ torch.iinfo(torch.int64).min
    return t.to(torch.int64) & 0xFFFFFFFF


def _check_stable_sort(x_dev, keys, vals, seg_of=None):
    """The properties above; seg_of (optional): segment of every position."""
    import torch
    n = x_dev.numel()
    u = _unsigned(keys)
    ordered = u[1:] >= u[:-1]
    same = keys[1:] == keys[:-1]
    if seg_of is not None:
        head = seg_of[1:] != seg_of[:-1]
        ordered = ordered | head
        same = same & ~head
    assert bool(ordered.all().item()), "keys out of order"
    idx = vals.to(torch.int64)
    assert int(idx.min().item()) >= 0 and int(idx.max().item()) < n
    hits = torch.zeros(n, dtype=torch.int32, device=keys.device)
    hits.scatter_add_(0, idx, torch.ones_like(vals, dtype=torch.int32))
    assert bool((hits == 1).all().item()), "values are not a permutation"
    del hits
    assert bool((x_dev[idx] == keys).all().item()), "keys do not travel with their indices"
    if seg_of is not None:
        assert bool((seg_of[idx] == seg_of).all().item()), "a key left its segment"
    assert bool(((vals[1:] > vals[:-1]) | ~same).all().item()), "equal keys out of input order"


def test_full_learned_lognormal_2p28(vm):
    """The learned path on the benchmark's input (n = 2^28 lognormal u64,
    seed 5, default configuration): the iota run is checked by the
    properties, the key-only run (the benchmark's launch) must equal it."""
    import torch
    n = 1 << 28
    _say("full learned: generating", n)
    x = workloads.lognormal(n, 5)
    x_dev = torch.from_numpy(x.view(np.int64)).cuda()
    del x
    keys = x_dev.clone()
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    _say("full learned: sort with iota values")
    stats, _ = vm.sort_learned_(keys, vals, iota=True)
    _say("  stats", {k: stats[k] for k in ("buckets", "fallback_buckets", "fallback_keys", "max_bucket")})
    _check_stable_sort(x_dev, keys, vals)
    _say("full learned: key-only sort")
    k2 = x_dev.clone()
    vm.sort_learned_(k2, read_stats=False)
    assert bool((k2 == keys).all().item())


def test_full_learned_dup16_2p28(vm):
    """The learned path's adversary at the benchmark size: n = 2^28 u64 keys
    drawn from 16 distinct lognormal values (every bucket that is not empty
    holds one value, far longer than the LDS tile, so all keys take the
    fallback), with index values, checked by the properties."""
    import torch
    n = 1 << 28
    _say("full dup16: generating", n)
    x = workloads.dup16(n, 6)
    x_dev = torch.from_numpy(x.view(np.int64)).cuda()
    del x
    keys = x_dev.clone()
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    _say("full dup16: sort with iota values")
    stats, _ = vm.sort_learned_(keys, vals, iota=True)
    _say("  stats", {k: stats[k] for k in ("buckets", "nonempty_buckets", "fallback_buckets", "fallback_keys",
                                           "max_bucket")})
    assert stats["nonempty_buckets"] <= 16 and stats["fallback_keys"] == n
    _check_stable_sort(x_dev, keys, vals)


def test_full_plain_pairs_mixture_2p28(vm):
    """(key, u32 index) pairs, n = 2^28 of the mixture input, plain path."""
    import torch
    n = 1 << 28
    _say("full pairs: generating", n)
    x = workloads.mixture(n, 36)
    x_dev = torch.from_numpy(x.view(np.int64)).cuda()
    del x
    keys = x_dev.clone()
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    _say("full pairs: sort with iota values")
    vm.sort_(keys, vals, iota=True)
    _check_stable_sort(x_dev, keys, vals)


def test_full_plain_presorted_2p24_matches_oracle(vm, orc):
    """n = 2^24 presorted u64 (geometric runs of mean 2^10, a tenth
    reversed, 1% swaps), plain path, element by element against the oracle
    with index payloads."""
    import torch
    n = 1 << 24
    x = workloads.presorted(n, 33, mean_run=1024, bits=64)
    v = np.arange(n, dtype=np.uint32)
    _say("full presorted: oracle", n)
    want, wantv, _, _ = orc.powersort(x, v)
    keys = torch.from_numpy(x.view(np.int64).copy()).cuda()
    vals = torch.from_numpy(v.view(np.int32).copy()).cuda()
    vm.sort_(keys, vals)
    torch.cuda.synchronize()
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), want)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), wantv)


def test_full_batch_4096_arrays(vm, orc):
    """4096 u32 arrays of log-uniform length in [2^6, 2^20], uniform and
    Zipf alternating: the segmented launcher eagerly and replayed from its
    graph; the properties per segment, and the oracle on a sample of whole
    segments."""
    import torch
    _say("full batch: generating")
    kb, off = workloads.batch32(4096, 4)
    total = kb.size
    _say("full batch: keys", total)
    x_dev = torch.from_numpy(kb.view(np.int32)).cuda()
    offs = torch.from_numpy(off).cuda()
    lengths = torch.from_numpy(np.diff(off)).cuda()
    seg_of = torch.repeat_interleave(torch.arange(off.size - 1, device="cuda"), lengths)
    keys = x_dev.clone()
    vals = torch.arange(total, dtype=torch.int32, device="cuda")
    vm.segmented_sort_(keys, offs, vals)
    _check_stable_sort(x_dev, keys, vals, seg_of)
    # the captured graph replays the same sort
    k2 = x_dev.clone()
    g = vm.segmented_sort_graph(k2, offs)
    for rep in range(2):
        k2.copy_(x_dev)
        g.replay()
        torch.cuda.synchronize()
        assert bool((k2 == keys).all().item()), rep
    g.close()
    got = keys.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(4)
    for s in sorted(rng.choice(off.size - 1, 8, replace=False).tolist()):
        a, b = int(off[s]), int(off[s + 1])
        want, _ = orc.segmented_powersort(kb[a:b], np.array([0, b - a], dtype=np.int64))
        assert np.array_equal(got[a:b], want.astype(np.uint32)), s


def test_full_uniform_2p16_u32_matches_oracle(vm, orc):
    """n = 2^16 uniform u32, plain path, against the oracle."""
    import torch
    x = workloads.uniform(1 << 16, 32, 1)
    want, wantv, _, _ = orc.powersort(x, np.arange(x.size, dtype=np.uint32))
    keys = torch.from_numpy(x.view(np.int32).copy()).cuda()
    vals = torch.empty(x.size, dtype=torch.int32, device="cuda")
    vm.sort_(keys, vals, iota=True)
    torch.cuda.synchronize()
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), want.astype(np.uint32))
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), wantv)


def test_full_vm_lognormal_2p28(vm):
    """The paged sort (Virtual-Memory Powersort, Section 4) on the
    benchmark's input (n = 2^28 lognormal u64, seed 5) at the default window
    with index values, checked by the properties; its key-only run (the
    benchmark's launch) must equal it, with no schedule fault."""
    import torch
    n = 1 << 28
    _say("full vm: generating", n)
    x = workloads.lognormal(n, 5)
    x_dev = torch.from_numpy(x.view(np.int64)).cuda()
    del x
    keys = x_dev.clone()
    vals = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.zeros(vm.VM_STATS, dtype=torch.int64, device="cuda")
    _say("full vm: sort with iota values")
    vm.sort_vm_(keys, vals, iota=True, stats=st)
    assert int(st[0].item()) == 0
    _check_stable_sort(x_dev, keys, vals)
    del vals
    _say("full vm: key-only sort")
    k2 = x_dev.clone()
    vm.sort_vm_(k2, stats=st)
    assert int(st[0].item()) == 0
    assert bool((k2 == keys).all().item())
