"""Large records on the GPU (vmps_sort_records; the 30-word record types of
Sec. 5 and hypothesis H4): records sorted by a key field through a (key,
index) sort and one gather, compared with the oracle's record sort byte for
byte."""
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


def _records(n, words, seed):
    """n records of `words` 32-bit words: uniform payload in [100, 10^9]
    (the paper's random words), record index in word 0."""
    rng = np.random.default_rng(seed)
    rec = rng.integers(100, 10**9, (n, words), dtype=np.uint64).astype(np.uint32)
    rec[:, 0] = np.arange(n, dtype=np.uint32)
    return rec


@pytest.mark.parametrize("key", ["u32_last", "u32_mid", "u64_front", "u64_presorted"])
def test_records_match_oracle(vm, orc, key):
    import torch
    for n in (1, 2, 1000, 70001, (1 << 18) + 3):
        rec = _records(n, 30, n)
        if key == "u32_last":      # zeroBlob30-like: only the last word decides
            rec[:, 1:29] = 0
            off, kb, kt = 116, 4, vm.U32
        elif key == "u32_mid":     # few distinct keys: long runs of ties
            rec[:, 7] %= 16
            off, kb, kt = 28, 4, vm.U32
        elif key == "u64_front":   # randomBlob30-like: words 2-3 as one u64 key
            off, kb, kt = 8, 8, vm.U64
        else:                      # the presorted generator's keys in words 2-3
            k = workloads.presorted(n, 3, mean_run=500)
            rec[:, 2:4] = k.view(np.uint32).reshape(n, 2)
            off, kb, kt = 8, 8, vm.U64
        _say("records", key, n)
        want = orc.records_sort(rec.view(np.uint8), off, kb).view(np.uint32).reshape(n, 30)
        src = torch.from_numpy(rec.view(np.int32).copy()).cuda()
        out = vm.sort_records(src, off, kt, desc=(key == "u64_presorted"))
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (key, n)
        assert torch.equal(src.cpu(), torch.from_numpy(rec.view(np.int32))), "input modified"


def test_records_odd_sizes_and_errors(vm, orc):
    """Records of 12 bytes (u32 words, 4-byte gather) and 40 bytes (8-byte
    gather); bad arguments are rejected before anything runs."""
    import torch
    for words in (3, 10):
        n = 50003
        rec = _records(n, words, words)
        rec[:, 1] %= 1000
        want = orc.records_sort(rec.view(np.uint8), 4, 4).view(np.uint32).reshape(n, words)
        src = torch.from_numpy(rec.view(np.int32).copy()).cuda()
        out = vm.sort_records(src, 4, vm.U32)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want), words
    src = torch.zeros((10, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(vm.VmpsError):
        vm.sort_records(src, 8, vm.U64)  # 12-byte records cannot hold an aligned u64 key
    with pytest.raises(vm.VmpsError):
        vm.sort_records(src, 10, vm.U32)  # key off its alignment
    with pytest.raises(vm.VmpsError):
        vm.sort_records(src, 0, vm.U32, out=src)  # output overlaps the input
