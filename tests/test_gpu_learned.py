"""GPU parity of the learned CDF partitioner against the oracle.

Inputs to both sides come from `workloads` or from seeded parameters; the
model tables given to the GPU partition are built by the oracle.  Integer
results (sample, bucket ids, partition, final sort) are compared exactly;
fp32 gradients and tables against the oracle's fp64 within tolerances
derived from fp32 rounding.
"""
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
    if x.dtype == np.uint32:
        return torch.from_numpy(x.view(np.int32).copy()).cuda()
    return torch.from_numpy(x.copy()).cuda()


def _np(t, dtype):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype)


def _say(*a):
    print(*a, flush=True)


def _params(rng, H):
    return {"w1": rng.normal(1, 0.5, H), "b1": rng.normal(-0.5, 0.3, H), "w2": rng.normal(0, 1, H),
            "b2": float(rng.normal())}


def _flat32(p):
    return np.concatenate([p["w1"], p["b1"], p["w2"], [p["b2"]]]).astype(np.float32)


def _as64(p32, H):
    p = p32.astype(np.float64)
    return {"w1": p[:H], "b1": p[H:2 * H], "w2": p[2 * H:3 * H], "b2": float(p[3 * H])}


def _host_model(vm, orc, params64, tab, key_bits, fbits):
    m = vm.CdfModel()
    m.z_lo, m.z_hi = tab.z_lo, tab.z_hi
    m.key_bits, m.feature_bits, m.hidden = key_bits, fbits, len(params64["w1"])
    m.knots, m.shift = tab.knots, tab.shift
    for i, v in enumerate(tab.table.tolist()):
        m.table[i] = v
    return m


def test_sample_positions(vm, orc):
    for n, m, seed in ((1000, 5000, 1234567), (1 << 20, 1 << 16, 55), (17, 100, 0)):
        x = workloads.uniform(n, 64, seed % 1000)
        pos = orc.sample_positions(n, m, seed)
        got = _np(vm.sample(_t(x), m, seed), np.uint64)
        assert np.array_equal(got, x[pos])


def _abs_sums(p, u, y):
    """Sum over the points of the absolute value of every term of each
    gradient component (the scale that bounds the rounding error of an fp32
    sum of those terms), fp64."""
    a = np.outer(u, p["w1"]) + p["b1"]
    r = np.maximum(a, 0.0)
    f = r @ p["w2"] + p["b2"]
    d = np.abs(2.0 * (f - y) / u.size)[:, None]
    act = (a > 0).astype(np.float64)
    return np.concatenate([(d * act * np.abs(p["w2"]) * np.abs(u)[:, None]).sum(0),
                           (d * act * np.abs(p["w2"])).sum(0), (d * r).sum(0), [d.sum()]])


@pytest.mark.parametrize("H", [16, 32, 64])
def test_gradient_matches_fp64(vm, orc, H):
    """fp32 forward/backward kernels against the fp64 oracle on the same
    fp32 parameters and points: relative 1e-4, plus an absolute allowance of
    1e-5 times the sum of the absolute terms of each component.  Each GPU
    thread sums at most nb/(1024/H) points in order and 1024/H partial sums
    follow, so an fp32 sum carries at most about (nb*H/1024 + 1024/H) * 2^-24
    of that absolute sum (below 2^-24 * 272 = 1.6e-5 for nb = 4096, H = 64,
    and far smaller in practice); the forward pass adds a relative error of
    about H * 2^-24 to each point's residual."""
    import torch
    rng = np.random.default_rng(H)
    for trial in range(4):
        p32 = _flat32(_params(rng, H))
        nb = [64, 1024, 4096, 192][trial]
        u = rng.random(nb).astype(np.float32)
        y = rng.random(nb).astype(np.float32)
        grad, loss = vm.cdf_grad(torch.from_numpy(p32).cuda(), H, torch.from_numpy(u).cuda(),
                                 torch.from_numpy(y).cuda())
        g = grad.cpu().numpy().astype(np.float64)
        p64 = _as64(p32, H)
        ref_loss, ref = orc.mlp_grad(p64, u.astype(np.float64), y.astype(np.float64))
        want = np.concatenate([ref["w1"], ref["b1"], ref["w2"], [ref["b2"]]])
        absum = _abs_sums(p64, u.astype(np.float64), y.astype(np.float64))
        excess = np.abs(g - want) / (1e-4 * np.abs(want) + 1e-5 * absum + 1e-30)
        _say("grad", H, nb, "max |diff|", float(np.abs(g - want).max()), "worst fraction of the bound",
             float(excess.max()))
        assert np.all(np.abs(g - want) <= 1e-4 * np.abs(want) + 1e-5 * absum)
        assert float(loss.item()) == pytest.approx(ref_loss, rel=1e-4)


def _model_params(model, H):
    return {"w1": np.array(model.w1[:H], dtype=np.float64), "b1": np.array(model.b1[:H], dtype=np.float64),
            "w2": np.array(model.w2[:H], dtype=np.float64), "b2": float(model.b2)}


@pytest.mark.parametrize("H,lr,nb", [(16, 1e-3, 512), (64, 6e-4, 512), (64, 5e-5, 8192)])
def test_training_trajectory_matches_oracle(vm, orc, H, lr, nb):
    """The GPU's Adam against the oracle's from the same start: the GPU's
    fp32 features and fp32 quantile initialisation are handed to the
    oracle's fp64 Adam (minibatch rule, gradient, bias-corrected update) and
    the parameters are compared after 1, 2 and 8 steps, kept even when they
    are worse than the start (VMPS_CDF_KEEP_TRAINED).  Every Adam step moves a
    parameter by at most about lr, and by lr * g/(|g| + eps) on the first one,
    so a wrong minibatch, step counter or update shows up as a difference of
    the order of lr; fp32 rounding of the gradient changes a step by a
    relative 1e-4 or less, except where a gradient component is itself at the
    level of its rounding error (checked separately below).  With nb = 8192
    the minibatch is spread over 32 workgroups whose parts are summed in a
    fixed order."""
    m = 1 << 16
    keys = np.sort(workloads.lognormal(m, 21))
    cfg = vm.learned_default_config(m, vm.U64)
    cfg.hidden, cfg.batch, cfg.lr, cfg.flags = H, nb, lr, vm.CDF_KEEP_TRAINED
    cfg.steps = 0
    m0, u32 = vm.cdf_train(_t(keys), cfg, want_features=True)
    u = u32.cpu().numpy().astype(np.float64)
    u_ref, z_lo, z_hi = orc.normalised_features(keys, 64, 20)
    assert (m0.z_lo, m0.z_hi) == (z_lo, z_hi)
    assert np.abs(u - u_ref).max() <= 2.0 ** -23          # one fp32 rounding of a value in [0, 1]
    p0 = _model_params(m0, H)
    # the fp32 quantile initialisation is the oracle's one up to fp32 rounding
    init_ref = orc.cdf_init(u, H)
    f_gpu = np.array([orc.mlp_forward(p0, x) for x in u[::257]])
    f_ref = np.array([orc.mlp_forward(init_ref, x) for x in u[::257]])
    assert np.abs(f_gpu - f_ref).max() <= 1e-5
    traj = orc.cdf_adam_steps(u, p0, 8, nb, lr)
    # conditioning: components whose oracle gradient at some step is within
    # 1e-4 of the largest component's magnitude take steps that fp32 may
    # round differently; they get the coarse bound of 2 lr per step
    weak = np.zeros(3 * H + 1, dtype=bool)
    prev = p0
    for s in range(8):
        idx = np.array([((s * nb + j) * 0x9E3779B1) % m for j in range(nb)])
        _, g = orc.mlp_grad(prev, u[idx], (idx + 0.5) / m)
        gf = np.concatenate([g["w1"], g["b1"], g["w2"], [g["b2"]]])
        weak |= np.abs(gf) <= 1e-4 * np.abs(gf).max()
        row = traj[s]
        prev = {"w1": row[:H], "b1": row[H:2 * H], "w2": row[2 * H:3 * H], "b2": float(row[3 * H])}
    for k in (1, 2, 8):
        cfg.steps = k
        mk = vm.cdf_train(_t(keys), cfg)
        assert mk.trained == 1
        got = np.concatenate([np.array(mk.w1[:H]), np.array(mk.b1[:H]), np.array(mk.w2[:H]), [mk.b2]])
        want = traj[k - 1]
        diff = np.abs(got - want)
        start = orc.flat_params(p0)
        moved = np.abs(want - start)
        bound = np.where(weak, 2.0 * lr * k, 0.01 * lr * k) + 2.0 ** -22 * np.abs(want)
        _say("trajectory", H, k, "max diff", float(diff.max()), "max diff on well-conditioned",
             float(diff[~weak].max()), "weak", int(weak.sum()), "max move", float(moved.max()))
        assert np.all(diff <= bound), np.nonzero(diff > bound)
    # keep/discard: with the default choice the GPU keeps the trained model
    # exactly when its loss is not above the initial one (losses compared in
    # fp64 here; cases within fp32 rounding of each other are not decided)
    cfg.flags = 0
    for k, lr_k in ((8, lr), (8, 0.5)):
        cfg.steps, cfg.lr = k, lr_k
        mk = vm.cdf_train(_t(keys), cfg)
        last = orc.cdf_adam_steps(u, p0, k, nb, lr_k)[-1]
        l0 = orc.cdf_loss(p0, u)
        l1 = orc.cdf_loss({"w1": last[:H], "b1": last[H:2 * H], "w2": last[2 * H:3 * H], "b2": float(last[3 * H])}, u)
        _say("choice", H, lr_k, "oracle losses", l0, l1, "gpu", mk.loss_init, mk.loss_final, mk.trained)
        if abs(l1 - l0) > 1e-3 * l0:
            assert mk.trained == (1 if l1 <= l0 else 0)


@pytest.mark.parametrize("H", [16, 32])
def test_compile_matches_oracle(vm, orc, H):
    import torch
    rng = np.random.default_rng(100 + H)
    for trial in range(4):
        p32 = _flat32(_params(rng, H))
        z_lo = int(rng.integers(0, 2**30))
        rng_ = int(rng.choice([0, 1, 1000, 2**20 + 3, 2**27]))
        K = int(rng.choice([1, 64, 4096]))
        t = vm.cdf_compile(torch.from_numpy(p32).cuda(), H, z_lo, z_lo + rng_, 64, 20, K)
        got = vm.model_from_tensor(t)
        tab = orc.cdf_table(_as64(p32, H), z_lo, z_lo + rng_, K)
        assert (got.shift, got.knots) == (tab.shift, tab.knots)
        gt = np.array(got.table[: tab.knots + 1], dtype=np.float64)
        assert np.all(np.diff(gt) >= 0)
        # fp32 evaluation (and fp32 knot positions) against fp64: within 1e-5
        # of the full Q32 scale
        assert np.abs(gt - tab.table.astype(np.float64)).max() <= 2**32 * 1e-5


def _models(vm, orc, keys_sorted, key_bits, fbits, rng):
    """Oracle-built tables: trained fp64, random, identity, constant."""
    u, z_lo, z_hi = orc.normalised_features(keys_sorted, key_bits, fbits)
    out = []
    p, _ = orc.cdf_train(u, 16, 16, 256, 1e-4)
    out.append(("trained", p))
    out.append(("random", _params(rng, 8)))
    out.append(("identity", {"w1": np.array([1.0]), "b1": np.array([0.0]), "w2": np.array([1.0]), "b2": 0.0}))
    out.append(("constant", {"w1": np.array([0.0]), "b1": np.array([0.0]), "w2": np.array([0.0]), "b2": 0.37}))
    return [(name, orc.cdf_table(prm, z_lo, z_hi, 512), prm) for name, prm in out]


@pytest.mark.parametrize("bits", [32, 64])
def test_bucket_ids_and_partition_exact(vm, orc, bits):
    rng = np.random.default_rng(bits)
    fbits = 20
    dt = np.uint32 if bits == 32 else np.uint64
    for maker in ("lognormal", "uniform", "dup16"):
        n = 50001 if maker != "dup16" else 30000
        if maker == "lognormal":
            x = (workloads.lognormal(n, 3) >> np.uint64(0 if bits == 64 else 32)).astype(dt)
        elif maker == "uniform":
            x = workloads.uniform(n, bits, 4)
        else:
            x = workloads.dup16(n, 5).astype(dt)
        xs = np.sort(x[:: max(1, n // 4000)])
        for name, tab, prm in _models(vm, orc, xs, bits, fbits, rng):
            model_t = vm.model_to_tensor(_host_model(vm, orc, prm, tab, bits, fbits))
            for B in (2, 16, 256, 1024, 8192, 65536, 131072):
                _say("partition", bits, maker, name, B)
                ids = _np(vm.bucket_ids(_t(x), model_t, B), np.uint32)
                want_ids = np.array([orc.bucket_of(int(k), bits, fbits, tab, B) for k in x[:2000]])
                assert np.array_equal(ids[:2000], want_ids)
                v = np.arange(n, dtype=np.uint32)
                ko, vo, off = vm.partition(_t(x), model_t, B, _t(v))
                wk, wv, woff = orc.partition(x, bits, fbits, tab, B, vals=v)
                assert np.array_equal(_np(off, np.int64), woff)
                assert np.array_equal(_np(vo, np.uint32), wv)
                assert np.array_equal(_np(ko, dt), wk.astype(dt))


def test_partition_tiny_and_ragged(vm, orc):
    rng = np.random.default_rng(9)
    for n in (1, 2, 4095, 4096, 4097, 3 * 4096 + 11):
        x = workloads.lognormal(n, n)
        tab = orc.cdf_table(_params(rng, 4), 0, int(orc.feature(int(x.max()), 64, 20)) + 1, 64)
        model_t = vm.model_to_tensor(_host_model(vm, orc, _params(rng, 4), tab, 64, 20))
        ko, _, off = vm.partition(_t(x), model_t, 4096)
        wk, _, woff = orc.partition(x, 64, 20, tab, 4096)
        assert np.array_equal(_np(off, np.int64), woff) and np.array_equal(_np(ko, np.uint64), wk)


def test_partition_caller_tables(vm, orc):
    """Tables a caller may build: not monotone, values of 2^32 and above, a
    segment width of 2^40, a z_lo above every feature.  The histogram
    evaluates monotone 32-bit tables in 32-bit arithmetic and every other
    table in 64-bit arithmetic; the partition equals the oracle's in each
    case."""
    rng = np.random.default_rng(17)
    x = workloads.lognormal(3 * 8192 + 77, 3)
    zmax = int(orc.feature(int(x.max()), 64, 20)) + 1
    sh, kn = orc.cdf_grid(0, zmax, 64)

    def table(k, hi, sort=True):
        t = rng.integers(0, hi, k + 1, dtype=np.uint64)
        return np.sort(t) if sort else t

    cases = [("not monotone", orc.Table(table(kn, 1 << 32, sort=False), sh, kn, 0, zmax)),
             ("above 2^32", orc.Table(table(kn, 1 << 40), sh, kn, 0, zmax)),
             ("monotone 32-bit", orc.Table(table(kn, 1 << 32), sh, kn, 0, zmax)),
             ("shift 40", orc.Table(table(4, 1 << 32), 40, 4, 0, zmax)),
             ("z_lo above the features", orc.Table(table(kn, 1 << 32), sh, kn, 1 << 33, (1 << 33) + zmax))]
    for name, tab in cases:
        _say("caller table", name)
        model_t = vm.model_to_tensor(_host_model(vm, orc, _params(rng, 4), tab, 64, 20))
        ko, _, off = vm.partition(_t(x), model_t, 4096)
        wk, _, woff = orc.partition(x, 64, 20, tab, 4096)
        assert np.array_equal(_np(off, np.int64), woff), name
        assert np.array_equal(_np(ko, np.uint64), wk), name


@pytest.mark.parametrize("H,steps,batch,lr", [(32, 64, 1024, 1e-4), (32, 32, 512, 4e-4), (64, 8, 512, 2e-4),
                                               (64, 24, 512, 6e-4), (64, 32, 8192, 5e-5)])
def test_training_reaches_oracle_quality(vm, orc, H, steps, batch, lr):
    import torch
    keys = np.sort(workloads.lognormal(1 << 16, 21))
    cfg = vm.learned_default_config(1 << 16, vm.U64)
    cfg.hidden, cfg.steps, cfg.batch, cfg.lr = H, steps, batch, lr
    model = vm.cdf_train(_t(keys), cfg)
    u, z_lo, z_hi = orc.normalised_features(keys, 64, 20)
    assert (model.z_lo, model.z_hi) == (z_lo, z_hi)
    p_ref, loss_ref = orc.cdf_train(u, H, steps, batch, lr)
    init_ref = orc.cdf_loss(orc.cdf_init(u, H), u)
    _say("train", model.loss_init, model.loss_final, init_ref, loss_ref)
    assert model.loss_final <= model.loss_init
    assert model.loss_init == pytest.approx(init_ref, rel=0.05, abs=1e-8)
    assert model.loss_final <= 1.5 * loss_ref + 1e-8
    assert np.all(np.diff(np.array(model.table[: model.knots + 1], dtype=np.float64)) >= 0)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("values", ["none", "input", "iota"])
def test_sort_learned_matches_oracle(vm, orc, bits, values):
    import torch
    dt = np.uint32 if bits == 32 else np.uint64
    inputs = [
        ("lognormal", (workloads.lognormal(1 << 20, 31) >> np.uint64(32 if bits == 32 else 0)).astype(dt)),
        ("uniform", workloads.uniform((1 << 19) + 777, bits, 32)),
        ("presorted", workloads.presorted(1 << 19, 33, mean_run=800, bits=bits).astype(dt)),
        ("dup16", workloads.dup16(1 << 19, 34).astype(dt)),
        ("dup16x16", workloads.dup16(1 << 18, 35, every_16=True).astype(dt)),
        ("equal", np.full(1 << 18, 5, dtype=dt)),
    ]
    if bits == 64:
        inputs.append(("mixture", workloads.mixture(1 << 20, 36)))
    for name, x in inputs:
        n = x.size
        _say("learned sort", bits, values, name, n)
        v = np.random.default_rng(n).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        want, wantv, _, _ = orc.powersort(x, v if values == "input" else np.arange(n, dtype=np.uint32))
        keys = _t(x)
        if values == "none":
            stats, _ = vm.sort_learned_(keys)
        elif values == "input":
            vals = _t(v)
            stats, _ = vm.sort_learned_(keys, vals)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        else:
            vals = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            stats, _ = vm.sort_learned_(keys, vals, iota=True)
            assert np.array_equal(_np(vals, np.uint32), wantv), name
        _say("  stats", stats)
        assert np.array_equal(_np(keys, dt), want.astype(dt)), name


def test_trained_model_beats_untrained(vm, orc):
    """What Adam adds to the quantile initialisation, at the benchmark's
    model configuration (a 2^20-key sample, H = 64, 32 steps of 8192 points
    at 5e-5) on n = 2^24 lognormal keys (B = 4096 buckets of 4096 keys on
    average): the trained model is kept, its loss is below the initial
    model's, and fewer keys land in buckets longer than the LDS tile than
    with the initial model (steps = 0).  The oracle's fp64 training on the
    same sample measures loss 1.64e-6 -> 1.06e-6 and 412k -> 377k fallback
    keys.  Beside it, the untrained identity model f(u) = u sends most keys
    to the merge levels."""
    import torch
    n = 1 << 24
    x = workloads.lognormal(n, 41)
    cfg = vm.learned_default_config(n, vm.U64)
    cfg.sample_size, cfg.num_buckets = 1 << 20, 4096
    assert (cfg.hidden, cfg.steps, cfg.batch) == (64, 32, 8192) and abs(cfg.lr - 5e-5) < 1e-9
    keys = _t(x)
    stats, model = vm.sort_learned_(keys, cfg=cfg, want_model=True)
    assert np.array_equal(_np(keys, np.uint64), np.sort(x))
    cfg0 = vm.learned_default_config(n, vm.U64)
    cfg0.sample_size, cfg0.num_buckets, cfg0.steps = 1 << 20, 4096, 0
    k0 = _t(x)
    stats0, model0 = vm.sort_learned_(k0, cfg=cfg0, want_model=True)
    assert np.array_equal(_np(k0, np.uint64), np.sort(x))
    _say("trained", stats, "\ninitial", stats0)
    assert model.trained == 1
    assert stats["loss_final"] < 0.8 * stats["loss_init"]
    assert stats0["loss_init"] == pytest.approx(stats["loss_init"], rel=1e-6)
    assert stats["fallback_keys"] < stats0["fallback_keys"]
    # f(u) = u with H = 16: w1 = 1, b1 = 0, w2 = (1, 0, ..., 0), b2 = 0
    ident = [1.0] * 16 + [0.0] * 16 + [1.0] + [0.0] * 15 + [0.0]
    id_t = vm.cdf_compile(torch.tensor(ident, dtype=torch.float32, device="cuda"), 16, model.z_lo, model.z_hi,
                          64, 20, 4096)
    B = stats["buckets"]
    _, _, off_id = vm.partition(_t(x), id_t, B)
    sizes = np.diff(_np(off_id, np.int64))
    id_fallback = int(sizes[sizes > 8192].sum())
    _say("identity fallback keys", id_fallback, "identity max", int(sizes.max()))
    assert stats["fallback_keys"] * 4 < id_fallback


def test_sort_learned_sample_2p20_matches_oracle(vm, orc):
    """The learned sort with the benchmark's 2^20-key sample (n = 2^21
    lognormal keys, and 2^21 mixture keys with index values) against the
    oracle's Powersort, element by element."""
    import torch
    for name, x, values in (("lognormal", workloads.lognormal(1 << 21, 51), False),
                            ("mixture", workloads.mixture((1 << 21) + 999, 52), True)):
        n = x.size
        cfg = vm.learned_default_config(n, vm.U64)
        cfg.sample_size = 1 << 20
        _say("learned sample 2^20", name, n)
        want, wantv, _, _ = orc.powersort(x, np.arange(n, dtype=np.uint32))
        keys = _t(x)
        vals = torch.full((n,), -1, dtype=torch.int32, device="cuda") if values else None
        stats, model = vm.sort_learned_(keys, vals, iota=values, cfg=cfg, want_model=True)
        _say("  stats", stats, "trained", model.trained)
        assert np.array_equal(_np(keys, np.uint64), want), name
        if values:
            assert np.array_equal(_np(vals, np.uint32), wantv), name


@pytest.mark.parametrize("bits", [32, 64])
def test_error_judge_matches_oracle(vm, orc, bits):
    """The judge in the statistics equals the oracle's judge of the returned
    compiled model on the same sorted sample: integer fields exactly, the
    doubles (exact 128-bit numerators, rounded once or twice at the end) to a
    relative 1e-12."""
    dt = np.uint32 if bits == 32 else np.uint64
    inputs = [("lognormal", (workloads.lognormal(1 << 20, 51) >> np.uint64(32 if bits == 32 else 0)).astype(dt)),
              ("uniform", workloads.uniform((1 << 19) + 99, bits, 52)),
              ("dup16", workloads.dup16(1 << 19, 53).astype(dt))]
    for name, x in inputs:
        n = x.size
        cfg = vm.learned_default_config(n, vm.U32 if bits == 32 else vm.U64)
        if name == "uniform":
            cfg.sample_size = 5000   # not a power of two
        _say("judge", bits, name, n, cfg.sample_size)
        stats, model = vm.sort_learned_(_t(x), cfg=cfg, want_model=True)
        sample = np.sort(x[orc.sample_positions(n, cfg.sample_size, cfg.seed)])
        tab = orc.Table(np.array(model.table[: model.knots + 1], dtype=np.uint64), model.shift, model.knots,
                        model.z_lo, model.z_hi)
        B = stats["buckets"]
        want = orc.judge(sample, bits, model.feature_bits, tab, B)
        _say("  gpu", {k: v for k, v in stats.items() if k.startswith(("judge", "overflow"))})
        _say("  oracle", {k: v for k, v in want.items() if k not in ("d_max", "d_sum")})
        assert stats["judge_samples"] == cfg.sample_size
        assert stats["judge_max_bucket_err"] == want["max_bucket_err"]
        assert stats["judge_mean_bucket_err"] == want["mean_bucket_err"]
        assert stats["judge_max_err"] == pytest.approx(want["max_err"], rel=1e-12, abs=0)
        assert stats["judge_mean_err"] == pytest.approx(want["mean_err"], rel=1e-12, abs=0)
        assert stats["overflow_fraction"] == stats["fallback_buckets"] / B


def test_error_judge_zero_on_plain_path(vm):
    x = workloads.lognormal(5000, 54)
    stats, _ = vm.sort_learned_(_t(x))
    assert stats["judge_samples"] == 0 and stats["buckets"] == 0
