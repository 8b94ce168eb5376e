"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here compares the oracle with itself: every check is a hand-derived
value (tests/golden, derived from the paper's definitions), a closed form, an
invariant stated by the paper's theorem or analysis, a library special case
(Python's stable sort), or brute force on tiny inputs.
"""
import itertools
import math
import random

import numpy as np
import pytest

from conftest import read_golden

import workloads


# ---------------------------------------------------------------- minrun --
def test_minrun_golden(orc):
    for ((n, l),) in read_golden("minrun.txt"):
        assert orc.minrun(n) == l, n


def test_minrun_closed_form(orc):
    # Nested ceilings collapse: ceil(ceil(n/2)/2) = ceil(n/4), so the rule
    # returns ceil(n / 2^k) for the least k with ceil(n / 2^k) < 64.
    rng = random.Random(5)
    for n in list(range(1, 3000)) + [rng.randrange(1, 2**40) for _ in range(3000)]:
        k = 0
        while -(-n // (1 << k)) >= 64:
            k += 1
        assert orc.minrun(n) == -(-n // (1 << k))


# ----------------------------------------------------------------- power --
def test_power_golden(orc):
    for (n,), bounds, powers, (M,) in read_golden("powers.txt"):
        b = np.array(bounds, dtype=np.int64)
        got = orc.run_powers(b, n)
        assert got.tolist() == powers
        nodes = orc.tree_nodes(b, n, got)
        assert int((nodes[:, 2] - nodes[:, 0]).sum()) == M


def test_power_ruler_sequence(orc):
    # Equal runs of length l with n = l * 2^K form a perfect binary tree:
    # the boundary after run t has power K - (trailing zeros of t+1).
    for K in range(1, 9):
        for l in (1, 3, 32):
            n = l << K
            bounds = np.arange(0, n + 1, l, dtype=np.int64)
            got = orc.run_powers(bounds, n)
            want = [K - ((t + 1) & -(t + 1)).bit_length() + 1 for t in range(bounds.size - 2)]
            assert got.tolist() == want


def test_power_closed_form_matches_definition(orc):
    for n in range(2, 41):
        for i in range(0, n):
            for j in range(i + 1, n):
                for k in range(j + 1, n + 1):
                    assert orc.power_def(n, i, j, k) == orc.power_closed(n, i, j, k)
    rng = random.Random(11)
    for _ in range(20000):
        n = rng.randrange(3, 2**32 + 1)
        i, j, k = sorted(rng.sample(range(0, min(n, 2**62) + 1), 3)) if n < 1000 else sorted(
            [rng.randrange(0, n - 1), rng.randrange(0, n - 1), rng.randrange(0, n + 1)])
        if not (i < j < k <= n):
            continue
        assert orc.power_def(n, i, j, k) == orc.power_closed(n, i, j, k)


def test_power_tree_invariants(orc):
    # Derived from the theorem: adjacent boundaries never share a power, two
    # equal powers are separated by a smaller one, max power <= ceil(log2 n).
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(2, 5000))
        cuts = np.unique(np.concatenate([[0, n], rng.integers(1, n, size=int(rng.integers(1, n)))]))
        P = orc.run_powers(cuts.astype(np.int64), n)
        if P.size == 0:
            continue
        assert int(P.max()) <= math.ceil(math.log2(n))
        assert np.all(P[1:] != P[:-1])
        last = {}
        for t, p in enumerate(P.tolist()):
            if p in last:
                assert P[last[p] + 1:t].min() < p
            last[p] = t


# ------------------------------------------------------------ ExtractRun --
def test_extract_runs_golden(orc):
    for (ell,), keys, bounds in read_golden("extract_runs.txt"):
        assert orc.extract_runs(np.array(keys, dtype=np.uint64), ell).tolist() == bounds


def _check_runs_characterisation(x, bounds, ell):
    n = x.size
    assert bounds[0] == 0 and bounds[-1] == n
    for s, e in zip(bounds[:-1], bounds[1:]):
        nat = s + 1
        while nat < n and x[nat - 1] <= x[nat]:
            nat += 1
        if nat - s >= ell:
            assert e == nat
        else:
            assert e == min(n, s + ell)


def test_extract_runs_characterisation(orc):
    rng = np.random.default_rng(9)
    for trial in range(40):
        n = int(rng.integers(1, 3000))
        x = workloads.presorted(n, int(rng.integers(1 << 30)), mean_run=int(rng.choice([2, 20, 80, 400])),
                                swap_frac=0.0)
        for ell in (1, 4, 32, orc.minrun(n)):
            _check_runs_characterisation(x, orc.extract_runs(x, ell), ell)


# ------------------------------------------------------------ full sorts --
def _stable_positions(keys):
    return sorted(range(len(keys)), key=lambda i: (keys[i], i))


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_bruteforce_permutations(orc, variant):
    for n in range(0, 8):
        for perm in itertools.permutations(range(n)):
            keys = np.array(perm, dtype=np.uint64)
            out, v, st, _ = orc.powersort(keys, np.arange(n, dtype=np.uint32), variant=variant, ell=2)
            assert out.tolist() == sorted(perm)
            assert v.tolist() == _stable_positions(list(perm))


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_bruteforce_words_stability(orc, variant):
    # every word over {0,1,2} of length <= 9, minrun forced to 2 so merges happen
    for n in range(1, 10):
        for w in itertools.product(range(3), repeat=n):
            keys = np.array(w, dtype=np.uint64)
            out, v, _, _ = orc.powersort(keys, np.arange(n, dtype=np.uint32), variant=variant, ell=2)
            assert v.tolist() == _stable_positions(list(w))


def test_stability_golden(orc):
    for keys, pos in read_golden("stability.txt"):
        _, v, _, _ = orc.powersort(np.array(keys, dtype=np.uint64), np.arange(len(keys), dtype=np.uint32), ell=2)
        assert v.tolist() == pos


@pytest.mark.parametrize("maker", ["uniform32", "presorted", "mixture", "lognormal", "dup16", "paper"])
def test_matches_library_stable_sort(orc, maker):
    rng = np.random.default_rng(21)
    for trial in range(4):
        n = int(rng.integers(1, 40000))
        seed = int(rng.integers(1 << 30))
        x = {"uniform32": lambda: workloads.uniform(n, 32, seed),
             "presorted": lambda: workloads.presorted(n, seed, mean_run=256),
             "mixture": lambda: workloads.mixture(n, seed),
             "lognormal": lambda: workloads.lognormal(n, seed),
             "dup16": lambda: workloads.dup16(n, seed),
             "paper": lambda: workloads.paper_workload(seed, 100, n=n)}[maker]()
        want = np.argsort(x, kind="stable").astype(np.uint32)
        for variant in (0, 1, 2):
            out, v, _, _ = orc.powersort(x, np.arange(n, dtype=np.uint32), variant=variant)
            assert np.array_equal(v, want)
            assert np.array_equal(out, x[want])


# ------------------------------------------------------------ invariants --
def test_theorem_bounds_and_counters(orc):
    rng = np.random.default_rng(4)
    for trial in range(30):
        n = int(rng.integers(2, 60000))
        x = workloads.presorted(n, int(rng.integers(1 << 30)), mean_run=int(rng.choice([4, 64, 1000, 20000])))
        _, _, pp, log_pp = orc.powersort(x, variant=0, log_merges=True)
        _, _, lp, log_lp = orc.powersort(x, variant=1, log_merges=True)
        _, _, cp, log_cp = orc.powersort(x, variant=2, log_merges=True)
        for st in (pp, lp, cp):
            # Theorem (Section 2): stack height and merge cost bounds
            assert st["max_stack"] <= math.ceil(math.log2(n)) + 1
            assert st["merge_cost"] <= n * (st["entropy"] + 2) + 1e-6
            # run detection compares each adjacent pair at most once
            assert st["cmp_run"] <= n - 1
            assert st["cmp_merge"] <= st["merge_cost"] - st["merges"]
        # same merges, same merge cost in every buffer scheme
        assert np.array_equal(log_pp, log_lp) and np.array_equal(log_pp, log_cp)
        # Pingpong (Section 3): with the right-to-left last pop, pushes copy
        # only freshly extracted runs, so at most n copies and M + n moves
        # outside insertion sort.  Without it a merged run is copied again on
        # push; merges alone still write at most M elements.
        assert lp["mov_push"] <= n
        assert lp["mov_push"] + lp["mov_merge"] <= lp["merge_cost"] + n
        assert pp["mov_merge"] <= pp["merge_cost"]
        assert lp["mov_push"] + lp["mov_merge"] <= pp["mov_push"] + pp["mov_merge"]
        # CPython style: copy the smaller run, merge back: <= 1.5 M moves
        assert cp["mov_merge"] <= 1.5 * cp["merge_cost"]


def test_merge_cost_closed_form_perfect_tree(orc):
    # n = 2^16 uniform keys: every run is forced to l = 32 (a natural run of
    # 32 has probability ~1/32!), 2^11 runs in a perfect tree, M = 11 n.
    x = workloads.uniform(1 << 16, 32, 1)
    _, _, st, _ = orc.powersort(x)
    assert st["runs"] == 2048
    assert st["merge_cost"] == 11 * (1 << 16) == 720896


def test_sorted_and_constant_inputs(orc):
    for x in (np.arange(5000, dtype=np.uint64), np.full(5000, 7, dtype=np.uint64)):
        out, _, st, _ = orc.powersort(x)
        assert st["runs"] == 1 and st["merge_cost"] == 0 and st["cmp_run"] == x.size - 1
        assert st["mov_push"] + st["mov_merge"] + st["mov_ins"] == 0
        assert np.array_equal(out, x)


def test_merge_log_equals_tree_form(orc):
    rng = np.random.default_rng(12)
    for trial in range(40):
        n = int(rng.integers(2, 30000))
        x = workloads.presorted(n, int(rng.integers(1 << 30)), mean_run=int(rng.choice([8, 100, 3000])))
        _, _, st, log = orc.powersort(x, log_merges=True)
        b = orc.extract_runs(x)
        P = orc.run_powers(b, n)
        nodes = orc.tree_nodes(b, n, P)
        assert sorted(map(tuple, log.tolist())) == sorted(map(tuple, nodes[:, :3].tolist()))
        assert st["runs"] == b.size - 1


def test_standard_merge(orc):
    rng = np.random.default_rng(2)
    for trial in range(100):
        na, nb = int(rng.integers(0, 300)), int(rng.integers(0, 300))
        a = np.sort(rng.integers(0, 20, size=na).astype(np.uint64))
        b = np.sort(rng.integers(0, 20, size=nb).astype(np.uint64))
        va = np.arange(na, dtype=np.uint32)
        vb = np.arange(na, na + nb, dtype=np.uint32)
        out, vout = orc.standard_merge(a, b, va, vb)
        cat = np.concatenate([a, b])
        want = np.argsort(cat, kind="stable")
        assert np.array_equal(out, cat[want]) and np.array_equal(vout, want.astype(np.uint32))


# ------------------------------------------------------------------ plan --
def _execute_plan(x, bounds, powers, T, node_buf, segs, nodes):
    """Run the planned schedule with two numpy buffers, tracking which buffer
    holds valid data for every position; merges are stable sorts of the
    concatenation of two sorted runs (a library special case)."""
    n = x.size
    A, B = x.copy(), np.zeros_like(x)
    bufs = [A, B]
    where = np.zeros(n, dtype=np.int8)          # everything starts in A
    for s, e, b in segs:
        seg = np.sort(A[s:e], kind="stable")
        bufs[b][s:e] = seg
        where[s:e] = b
    order = np.argsort(-nodes[:, 3], kind="stable")
    for t in order:
        L, mid, R, p = nodes[t]
        if R - L <= T:
            continue
        src = 1 - node_buf[t]
        assert np.all(where[L:R] == src), "children not in the opposite buffer"
        cat = bufs[src][L:R]
        assert np.all(np.diff(cat[: mid - L].astype(np.float64)) >= 0)
        bufs[node_buf[t]][L:R] = np.sort(cat, kind="stable")
        where[L:R] = node_buf[t]
    assert np.all(where == 0), "result not in the input buffer"
    return A


def test_plan_executes_to_sorted_result(orc):
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(1, 50000))
        x = workloads.presorted(n, int(rng.integers(1 << 30)), mean_run=int(rng.choice([2, 50, 2000])))
        b = orc.extract_runs(x)
        P = orc.run_powers(b, n)
        nodes = orc.tree_nodes(b, n, P)
        for T in (64, 512, 4096):
            node_buf, depth, segs, M, Mh = orc.plan(b, n, P, T)
            assert segs[0, 0] == 0 and segs[-1, 1] == n and np.all(segs[1:, 0] == segs[:-1, 1])
            for s, e, _ in segs:
                assert e - s <= T or np.count_nonzero((b > s) & (b < e)) == 0
            got = _execute_plan(x, b, P, T, node_buf, segs, nodes)
            assert np.array_equal(got, np.sort(x))
            assert M == int((nodes[:, 2] - nodes[:, 0]).sum())
            assert Mh == int(sum(R - L for L, _, R, _ in nodes if R - L > T))


def _hbm_top_level(n, T):
    """Largest power p with 2^p < 9 n / T, at most ceil(log2 n): the highest
    merge level the GPU launches for nodes longer than T."""
    top = 1
    while top < 32 and (1 << top) < n:
        top += 1
    p = 1
    while p < top and ((2 * T) << p) < 9 * n:
        p += 1
    return p


def test_long_merges_power_bound(orc):
    """A node of power p has its run midpoints in a window of width n 2^(1-p)
    and each of its runs borders a boundary of power >= p, so it is shorter
    than about 3 n 2^(1-p): every merge of Algorithm 1 longer than T has
    2^p < 9 n / T, and the merge levels above that power are empty.  Checked
    on the merges Algorithm 1 performs, for random, presorted, block-shuffled
    and long-next-to-tiny run structures; the bound comes within one level
    of the largest power seen (it is not vacuous)."""
    closest = -99
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        for n in (1000, 4097, 30000, 1 << 17):
            inputs = [workloads.uniform(n, 64, seed),
                      workloads.presorted(n, seed, mean_run=int(rng.integers(2, 5000))).astype(np.uint64)]
            parts, tot = [], 0
            while tot < n:  # long runs next to runs of one to three keys
                L = min(int(rng.choice([1, 2, 3, int(rng.integers(1, n // 2 + 2))])), n - tot)
                parts.append(np.sort(rng.integers(0, 1 << 40, L)))
                tot += L
            inputs.append(np.concatenate(parts).astype(np.uint64))
            cut = np.sort(rng.choice(np.arange(1, n), size=int(rng.integers(2, 64)), replace=False))
            inputs.append(np.concatenate(np.split(np.arange(n, dtype=np.uint64), cut)[::-1]))
            for x in inputs:
                for ell in (0, 16):
                    b = orc.extract_runs(x, ell or None)
                    pw = orc.run_powers(b, n)
                    _, _, _, log = orc.powersort(x, ell=ell, log_merges=True)
                    where = {int(v): i for i, v in enumerate(b)}
                    for T in (32, 100, 1024, 8192):
                        top = _hbm_top_level(n, T)
                        for L, M, R in log:
                            if R - L > T:
                                p = int(pw[where[int(M)] - 1])
                                assert p <= top, (n, T, int(L), int(M), int(R), p, top)
                                closest = max(closest, p - top)
    assert closest >= -1, closest


def test_plan_depth_perfect_tree(orc):
    # perfect tree: depth = power - 1, so the buffer is (power - 1) mod 2
    n = 32 << 8
    b = np.arange(0, n + 1, 32, dtype=np.int64)
    P = orc.run_powers(b, n)
    node_buf, depth, segs, M, Mh = orc.plan(b, n, P, 1024)
    assert np.array_equal(depth, P.astype(np.int32) - 1)
    assert M == 8 * n and Mh == 3 * n
    assert segs.shape[0] == n // 1024 and np.all(segs[:, 2] == 1)


def test_segmented_equals_per_segment_library_sort(orc):
    # each segment is an independent stable sort (library special case),
    # values record the original positions
    rng = np.random.default_rng(11)
    for trial in range(20):
        nseg = int(rng.integers(1, 40))
        lens = rng.integers(0, 400, size=nseg)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        n = int(off[-1])
        keys = rng.integers(0, 7 if trial % 2 else 2**63, size=n, dtype=np.uint64)
        out, v = orc.segmented_powersort(keys, off, np.arange(n, dtype=np.uint32))[:2]
        for s in range(nseg):
            a, b = off[s], off[s + 1]
            order = np.argsort(keys[a:b], kind="stable") + a
            assert out[a:b].tolist() == keys[order].tolist()
            assert v[a:b].tolist() == order.tolist()


# ------------------------------------------- exhaustive small inputs --
def _all_permutations(n):
    return np.fromiter(itertools.chain.from_iterable(itertools.permutations(range(n))), dtype=np.uint8,
                       count=math.factorial(n) * n).reshape(-1, n)


def _all_words(n):
    # row r is r written in base 3 with n digits (most significant first)
    r = np.arange(3 ** n, dtype=np.int64)[:, None]
    return ((r // (3 ** np.arange(n - 1, -1, -1, dtype=np.int64))) % 3).astype(np.uint8)


def _sort_rows_with_oracle(orc, rows, ell, variant):
    cnt, n = rows.shape
    keys = rows.reshape(-1).astype(np.uint64)
    off = np.arange(cnt + 1, dtype=np.int64) * n
    vals = np.tile(np.arange(n, dtype=np.uint32), cnt)  # index inside the row
    out, v = orc.segmented_powersort(keys, off, vals, variant=variant, ell=ell)
    return out.reshape(cnt, n), v.reshape(cnt, n)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_exhaustive_permutations_up_to_10(orc, variant):
    # every permutation of n <= 10 (3.6 million at n = 10), each sorted as
    # its own instance with minrun 2 so that runs, powers and merges are
    # exercised; with distinct keys the stable sort is the inverse
    # permutation (numpy's argsort of the row)
    for n in range(1, 11):
        rows = _all_permutations(n)
        out, v = _sort_rows_with_oracle(orc, rows, 2, variant)
        assert np.array_equal(out, np.broadcast_to(np.arange(n, dtype=np.uint64), out.shape)), n
        assert np.array_equal(v, np.argsort(rows, axis=1).astype(np.uint32)), n


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_exhaustive_words_up_to_12(orc, variant):
    # every word over {0,1,2} of length <= 12: equal keys keep their order
    # (numpy's stable argsort of the row is the definition)
    for n in range(1, 13):
        rows = _all_words(n)
        out, v = _sort_rows_with_oracle(orc, rows, 2, variant)
        want = np.argsort(rows, axis=1, kind="stable")
        assert np.array_equal(v, want.astype(np.uint32)), n
        assert np.array_equal(out, np.take_along_axis(rows, want, axis=1).astype(np.uint64)), n


# ---------------------------------------------------- descending runs --
DESC_VARIANTS = [0, 1, 2]


def test_desc_runs_golden(orc):
    for (ell,), keys, bounds, flags, (M,) in read_golden("desc_runs.txt"):
        x = np.array(keys, dtype=np.uint64)
        b, f = orc.extract_runs(x, ell, desc=True, want_desc=True)
        assert b.tolist() == bounds and f.tolist() == flags, keys
        for variant in DESC_VARIANTS:
            k, v, st, _ = orc.powersort(x, np.arange(x.size, dtype=np.uint32), variant=variant | orc.DESC_RUNS, ell=ell)
            assert st["merge_cost"] == M and st["runs"] == len(bounds) - 1
            assert np.array_equal(k, np.sort(x)) and np.array_equal(v, np.argsort(x, kind="stable"))


@pytest.mark.parametrize("variant", DESC_VARIANTS)
def test_desc_runs_bruteforce(orc, variant):
    """Every permutation of n <= 8 and every {0,1,2}^n word of n <= 10 (ties:
    a reversed run must be strictly decreasing) sorts stably with the
    reversal on, at minrun 2 and at the rule's minrun."""
    cases = []
    for n in range(1, 9):
        cases += [np.array(p, dtype=np.uint64) for p in itertools.permutations(range(n))]
    for n in range(1, 11):
        cases += [np.array(w, dtype=np.uint64) for w in itertools.product(range(3), repeat=n)]
    for x in cases:
        order = np.argsort(x, kind="stable")
        for ell in (2, 0):
            k, v, _, _ = orc.powersort(x, np.arange(x.size, dtype=np.uint32), variant=variant | orc.DESC_RUNS, ell=ell)
            assert np.array_equal(v, order), (x, ell)


def test_desc_runs_special_cases(orc):
    rng = np.random.default_rng(9)
    for n in (2, 3, 64, 65, 1000, 4097):
        # strictly decreasing: one reversed run, no merge, every element
        # written once by the reversal except the middle one of an odd n
        x = np.arange(n, 0, -1, dtype=np.uint64) * 3
        k, v, st, _ = orc.powersort(x, np.arange(n, dtype=np.uint32), variant=orc.DESC_RUNS)
        assert st["runs"] == 1 and st["merge_cost"] == 0 and st["mov_rev"] == 2 * (n // 2)
        assert np.array_equal(k, np.sort(x)) and v[0] == n - 1
        # no strict descent anywhere: the same runs and merges as without
        y = np.sort(rng.integers(0, 50, n).astype(np.uint64))
        y[: n // 3] = y[0]
        b0 = orc.extract_runs(y)
        b1, f1 = orc.extract_runs(y, desc=True, want_desc=True)
        assert np.array_equal(b0, b1) and not f1.any()
        # non-increasing with ties: only the strictly decreasing stretches
        # are reversed, ties keep their input order
        z = np.repeat(np.arange(n, 0, -1, dtype=np.uint64), 2)
        kz, vz, _, _ = orc.powersort(z, np.arange(z.size, dtype=np.uint32), variant=orc.DESC_RUNS)
        assert np.array_equal(vz, np.argsort(z, kind="stable"))


def test_desc_runs_theorem_bound_and_counters(orc):
    """M <= n (H + 2) (merge-cost theorem of Section 2) and the Pingpong
    moves M + n (Section 3, with the last pop) hold for the reversed runs
    too; on these inputs (runs of mean length 300, a tenth of them
    decreasing) the reversal leaves fewer runs than the increasing-only
    chain, which cuts each decreasing run into forced runs."""
    for seed in range(6):
        x = workloads.presorted(1 << 14, seed, mean_run=300)
        _, _, s0, _ = orc.powersort(x)
        _, _, s1, _ = orc.powersort(x, variant=orc.PINGPONG_LASTPOP | orc.DESC_RUNS)
        n = x.size
        assert s1["merge_cost"] <= n * (s1["entropy"] + 2)
        assert s1["mov_push"] + s1["mov_merge"] <= s1["merge_cost"] + n
        assert s1["runs"] <= s0["runs"]
        assert s1["mov_rev"] > 0


# --- Virtual-Memory Powersort (Section 4) ---------------------------------

def test_vm_golden_pages(orc):
    """Hand-derived page traces (fixture header): output, copy moves, extra
    pages, live buffers and metadata entries."""
    for (page,), (ell,), keys, (extra,), (copies,), (bufs,), (meta,) in read_golden("vm_pages.txt"):
        x = np.array(keys, dtype=np.uint64)
        k, v, st, vs, log = orc.vm_powersort(x, np.arange(x.size, dtype=np.uint32), page=page, ell=ell,
                                             log_merges=True)
        n = x.size
        assert np.array_equal(v, np.argsort(x, kind="stable")) and np.array_equal(k, np.sort(x))
        assert log.tolist() == [[0, 2, n]]
        assert (vs["extra_pages"], st["mov_copy"], vs["max_buffers"], vs["meta_words"]) == (extra, copies, bufs, meta)
        assert st["mov_push"] == n and st["mov_merge"] == n and vs["input_pages"] == (n + page - 1) // page


@pytest.mark.parametrize("desc", [False, True])
def test_vm_bruteforce_small_pages(orc, desc):
    """Every permutation of n <= 7 and every {0,1,2}^n word of n <= 8 sorts
    stably with pages of 1, 2 and 3 elements (a partial last page whenever
    the page does not divide n)."""
    cases = []
    for n in range(0, 8):
        cases += [np.array(p, dtype=np.uint64) for p in itertools.permutations(range(n))]
    for n in range(1, 9):
        cases += [np.array(w, dtype=np.uint64) for w in itertools.product(range(3), repeat=n)]
    for x in cases:
        order = np.argsort(x, kind="stable")
        for page in (1, 2, 3):
            k, v, _, _, _ = orc.vm_powersort(x, np.arange(x.size, dtype=np.uint32), page=page, ell=2, desc=desc)
            assert np.array_equal(v, order), (x, page)


def test_vm_page_rule(orc):
    """P: the largest power of two <= sqrt(n / (T log2 n)) (Section 4 and its
    footnote on powers of two), worked by hand: 2^20 keys give
    sqrt(2^20/20) = 228.9 -> 128; key-value records (T = 2) sqrt(2^20/40) =
    161.9 -> 128; 2^28 keys sqrt(2^28/28) = 3096.3 -> 2048; 2^28 records
    2189.4 -> 2048; 10 keys sqrt(10/4) = 1.58 -> 1; 4096 keys sqrt(4096/12)
    = 18.5 -> 16."""
    for n, t, p in ((1 << 20, 1, 128), (1 << 20, 2, 128), (1 << 28, 1, 2048), (1 << 28, 2, 2048),
                    (10, 1, 1), (4096, 1, 16), (1, 1, 1)):
        assert orc.vm_page(n, t) == p, (n, t)


@pytest.mark.parametrize("kind", ["uniform", "presorted", "dup16", "desc"])
def test_vm_same_merges_and_move_bound(orc, kind):
    """The paged buffers change where elements live, not what Algorithm 1
    does: the merge log and merge comparisons equal Pingpong's.  Moves:
    n into pages, M by the merges, at most 2n by the final Copy, so at most
    M + 3n (the bound stated at the start of Section 4)."""
    for n in (2, 3, 100, 1000, 4097, 1 << 15):
        x = {"uniform": lambda: workloads.uniform(n, 64, n),
             "presorted": lambda: workloads.presorted(n, n, mean_run=300),
             "dup16": lambda: workloads.dup16(n, n),
             "desc": lambda: np.arange(n, 0, -1, dtype=np.uint64)}[kind]()
        for page in (0, 1, 5, 64):
            for desc in (False, True):
                k, v, st, vs, log = orc.vm_powersort(x, np.arange(n, dtype=np.uint32), page=page, desc=desc,
                                                     log_merges=True)
                k2, v2, st2, log2 = orc.powersort(x, np.arange(n, dtype=np.uint32),
                                                  variant=orc.PINGPONG | (orc.DESC_RUNS if desc else 0),
                                                  log_merges=True)
                assert np.array_equal(v, v2) and np.array_equal(k, k2)
                assert np.array_equal(log, log2)
                assert st["cmp_merge"] == st2["cmp_merge"] and st["merge_cost"] == st2["merge_cost"]
                assert st["mov_push"] == n and st["mov_merge"] == st["merge_cost"]
                assert st["mov_copy"] <= 2 * n
                assert st["mov_push"] + st["mov_merge"] + st["mov_copy"] <= st["merge_cost"] + 3 * n


def test_vm_pages_and_memory(orc):
    """Pages in use: each live buffer holds all its elements in full pages
    but for a partial page at each end, so pages in use stay below n/P +
    buffers + 3; a fresh page is made only when none is free, so the extra
    pages stay at most buffers + 4.  Buffers: the run stack (at most
    ceil(log2 n) + 1 runs, the powers on it strictly increase) plus work,
    curr, next and a merge result.  Metadata: one entry per page in a list,
    at most every page.  With the page rule the extra words grow like
    sqrt(n T log n) (Section 4's memory bound)."""
    for n in (1000, 1 << 14, 1 << 17, 1 << 20):
        for kind in ("uniform", "presorted", "dup16"):
            x = {"uniform": workloads.uniform, "dup16": workloads.dup16}.get(kind)
            x = workloads.presorted(n, 5, mean_run=300) if x is None else (
                x(n, 64, 5) if kind == "uniform" else x(n, 5))
            for vals in (None, np.arange(n, dtype=np.uint32)):
                t = 1 if vals is None else 2
                _, _, st, vs, _ = orc.vm_powersort(x, vals)
                P = vs["page"]
                assert P == orc.vm_page(n, t)
                assert vs["max_buffers"] <= math.ceil(math.log2(n)) + 1 + 4
                assert vs["extra_pages"] <= vs["max_buffers"] + 4
                assert vs["meta_words"] <= vs["input_pages"] + vs["extra_pages"]
                extra_words = vs["extra_pages"] * P * t + vs["meta_words"]
                assert extra_words <= 4 * math.sqrt(n * t * math.log2(n)), (n, kind, t, extra_words)


# --- large records (Sec. 5 record types) ------------------------------------

def test_records_golden(orc):
    for (off,), words, want in read_golden("records.txt"):
        rec = np.array(words, dtype=np.uint32).reshape(-1, 2).view(np.uint8)
        got = orc.records_sort(rec, off, 4).view(np.uint32).reshape(-1)
        assert got.tolist() == want


def test_records_bruteforce_and_stability(orc):
    """Every permutation of n <= 6 keys with repeats (keys in {0,1,2}),
    30-word records whose payload words record the input position: the
    output keys are non-decreasing, each record is intact, and equal keys
    keep input order (the definition of a stable sort, checked directly);
    with u64 keys at a word offset inside the record as well."""
    for n in range(0, 7):
        for w in itertools.product(range(3), repeat=n):
            rec = np.zeros((n, 30), dtype=np.uint32)
            rec[:, 5] = np.array(w, dtype=np.uint32)
            rec[:, 0] = np.arange(n)
            rec[:, 29] = np.arange(n) * 7 + 1
            out = orc.records_sort(rec.view(np.uint8), 20, 4).view(np.uint32).reshape(n, 30)
            k, pos = out[:, 5].astype(np.int64), out[:, 0].astype(np.int64)
            assert np.all(np.diff(k) >= 0)
            assert np.array_equal(out, rec[pos])
            assert np.all((np.diff(k) > 0) | (np.diff(pos) > 0))
            rec64 = np.zeros((n, 16), dtype=np.uint64)
            rec64[:, 3] = np.array(w, dtype=np.uint64) << np.uint64(40)
            rec64[:, 0] = np.arange(n)
            out64 = orc.records_sort(rec64.view(np.uint8), 24, 8).view(np.uint64).reshape(n, 16)
            assert np.array_equal(out64, rec64[np.argsort(rec64[:, 3], kind="stable")])
