"""Pins of the oracle's learned-partition reference (fp64).

Hand-derived feature values, finite differences for the backward pass, a
closed form for the identity model's buckets, the published SplitMix64
outputs, and numpy's stable argsort as the partition's library special case.
"""
import numpy as np
import pytest

import workloads


def test_splitmix64_published_vectors(orc):
    # first outputs of splitmix64.c (Vigna, public domain) for seed 1234567
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [orc.mix64(1234567, i) for i in range(5)] == want
    pos = orc.sample_positions(1000, 5, 1234567)
    assert pos.tolist() == [w % 1000 for w in want]


def test_feature_hand_values(orc):
    F = 4
    cases = {0: 0, 1: 16, 2: 32, 3: 40, 22: 86, 91: 118, 2**63: 64 << 4, 2**64 - 1: (64 << 4) | 15}
    for k, z in cases.items():
        assert orc.feature(k, 64, F) == z, k
    assert orc.feature(2**32 - 1, 32, F) == (32 << 4) | 15
    assert orc.feature(2**32 + 5, 32, F) == orc.feature(5, 32, F)  # high bits ignored


def test_feature_monotone(orc):
    keys = np.sort(workloads.mixture(3000, 4))
    z = orc.features(keys, 64, 20)
    assert np.all(np.diff(z.astype(np.float64)) >= 0)


def _rand_params(rng, H):
    return {"w1": rng.normal(1, 0.5, H), "b1": rng.normal(-0.5, 0.3, H), "w2": rng.normal(0, 1, H),
            "b2": float(rng.normal())}


def test_forward_hand_value(orc):
    p = {"w1": np.array([1.0, 2.0]), "b1": np.array([0.0, -1.0]), "w2": np.array([0.5, -0.25]), "b2": 0.1}
    # u = 0.75: 0.1 + 0.5*relu(0.75) - 0.25*relu(0.5) = 0.1 + 0.375 - 0.125
    assert orc.mlp_forward(p, 0.75) == pytest.approx(0.35, abs=1e-15)
    # u = 0.25: second unit inactive
    assert orc.mlp_forward(p, 0.25) == pytest.approx(0.225, abs=1e-15)


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(1)
    for H in (1, 4, 32):
        p = _rand_params(rng, H)
        u = rng.random(257)
        y = rng.random(257)
        loss, g = orc.mlp_grad(p, u, y)
        eps = 1e-6
        for name in ("w1", "b1", "w2", "b2"):
            for idx in (range(H) if name != "b2" else [None]):
                hi = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
                lo = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
                if idx is None:
                    hi[name] += eps; lo[name] -= eps
                    gi = g[name]
                else:
                    hi[name][idx] += eps; lo[name][idx] -= eps
                    gi = g[name][idx]
                fd = (orc.mlp_grad(hi, u, y)[0] - orc.mlp_grad(lo, u, y)[0]) / (2 * eps)
                assert gi == pytest.approx(fd, rel=1e-4, abs=1e-7), (H, name, idx)


def test_grid_is_least_power_of_two_cover(orc):
    rng = np.random.default_rng(4)
    for _ in range(500):
        z_lo = int(rng.integers(0, 2**40))
        rng_ = int(rng.integers(0, 2**31))
        K = int(rng.choice([1, 7, 64, 4096]))
        sh, kn = orc.cdf_grid(z_lo, z_lo + rng_, K)
        assert 1 <= kn <= K
        assert -(-rng_ // (1 << sh)) == (kn if rng_ else 0)
        if sh > 0:
            assert -(-rng_ // (1 << (sh - 1))) > K


def test_identity_table_and_buckets_closed_form(orc):
    # f(u) = u over a range 2^20 with K = 64 knots: segments of 2^14, knots
    # floor(s/64 * 2^32) (the last saturates at 2^32-1), and for B a power of
    # two the bucket is floor(d B / 2^20) by nested floors.
    K, B = 64, 256
    ident = {"w1": np.array([1.0]), "b1": np.array([0.0]), "w2": np.array([1.0]), "b2": 0.0}
    z_lo = orc.feature(1 << 40, 64, 40)
    tab = orc.cdf_table(ident, z_lo, z_lo + (1 << 20), K)
    assert (tab.shift, tab.knots) == (14, 64)
    assert tab.table[:K].tolist() == [(s << 32) // K for s in range(K)]
    assert tab.table[K] == 2**32 - 1
    rng = np.random.default_rng(0)
    for d in list(range(0, 200)) + rng.integers(0, 1 << 20, 500).tolist():
        if (d >> 14) >= K - 1:
            continue
        key = (1 << 40) + d   # bit length 41, feature = (41 << 40) | (key - 2^40)
        assert orc.bucket_of(key, 64, 40, tab, B) == d * B >> 20


def test_table_monotone_and_buckets_monotone(orc):
    rng = np.random.default_rng(7)
    for trial in range(10):
        p = _rand_params(rng, 8)
        keys = np.sort(workloads.lognormal(2000, trial))
        z = orc.features(keys, 64, 20)
        tab = orc.cdf_table(p, int(z[10]), int(z[-10]), 128)
        assert np.all(np.diff(tab.table.astype(np.float64)) >= 0)
        b = [orc.bucket_of(int(k), 64, 20, tab, 1000) for k in keys]
        assert all(x <= y for x, y in zip(b, b[1:]))
        assert max(b) < 1000


def test_partition_is_stable_counting_sort(orc):
    rng = np.random.default_rng(3)
    for trial in range(5):
        n = int(rng.integers(1, 5000))
        keys = workloads.lognormal(n, trial)
        vals = np.arange(n, dtype=np.uint32)
        p = _rand_params(rng, 4)
        zs = orc.features(np.sort(keys), 64, 20)
        tab = orc.cdf_table(p, int(zs[0]), int(zs[-1]), 64)
        B = 97
        ko, vo, off = orc.partition(keys, 64, 20, tab, B, vals=vals)
        ids = np.array([orc.bucket_of(int(k), 64, 20, tab, B) for k in keys])
        order = np.argsort(ids, kind="stable")
        assert np.array_equal(vo, order.astype(np.uint32)) and np.array_equal(ko, keys[order])
        assert np.array_equal(off, np.concatenate([[0], np.cumsum(np.bincount(ids, minlength=B))]))


def test_quantile_init_interpolates_ecdf(orc):
    keys = np.sort(workloads.lognormal(1 << 14, 5))
    u, z_lo, z_hi = orc.normalised_features(keys, 64, 20)
    H = 16
    p = orc.cdf_init(u, H)
    m = u.size
    for h in range(H):
        qi = h * (m - 1) // (H - 1)
        if h == 0 or u[qi] > u[(h - 1) * (m - 1) // (H - 1)]:
            assert orc.mlp_forward(p, float(u[qi])) == pytest.approx((qi + 0.5) / m, abs=1e-9)
    assert orc.mlp_forward(p, -1.0) == pytest.approx(0.5 / m)


BATCH_STRIDE = 0x9E3779B1  # minibatch rule of the training (odd multiplier mod m)


def _minibatch(u, m, s, nb):
    """Points of minibatch s: index (s*nb + j) * stride mod m, target (index + 1/2)/m."""
    idx = np.array([((s * nb + j) * BATCH_STRIDE) % m for j in range(nb)], dtype=np.int64)
    return u[idx], (idx + 0.5) / m


def _flat(g):
    return np.concatenate([g["w1"], g["b1"], g["w2"], [g["b2"]]])


def test_adam_steps_zero_learning_rate_keeps_start(orc):
    # lr = 0 leaves every parameter bit for bit where it started; a step
    # counter starting at 0 (bias correction 1 - beta^0 = 0) would turn them
    # into NaN here
    rng = np.random.default_rng(8)
    u = np.sort(rng.random(37))
    p = _rand_params(rng, 3)
    traj = orc.cdf_adam_steps(u, p, 5, 64, 0.0)
    for row in traj:
        assert np.array_equal(row, orc.flat_params(p))
    keys = np.sort(workloads.lognormal(1 << 12, 3))
    uu, _, _ = orc.normalised_features(keys, 64, 20)
    p0 = orc.cdf_init(uu, 16)
    p1, l1, trained = orc.cdf_train(uu, 16, 4, 256, 0.0, want_trained=True)
    assert trained and np.array_equal(orc.flat_params(p1), orc.flat_params(p0))
    assert l1 == orc.cdf_loss(p0, uu)


@pytest.mark.parametrize("m,H,nb", [(4, 1, 8), (4, 2, 64), (37, 2, 64), (1000, 5, 128)])
def test_adam_first_two_steps_on_their_minibatches(orc, m, H, nb):
    # Step 1 of Adam moves every parameter by lr g / (|g| + eps) (both moment
    # estimates are exact after bias correction), with g the gradient of the
    # MSE on minibatch 0 (pinned by finite differences); step 2 uses the
    # gradient at the new parameters on minibatch 1 and the moments
    # m = (0.9*0.1 g1 + 0.1 g2) / (1 - 0.9^2), v = (0.999*0.001 g1^2 + 0.001 g2^2) / (1 - 0.999^2).
    # A wrong minibatch index, target, step counter or gradient fails here.
    rng = np.random.default_rng(m + H)
    u = np.sort(rng.random(m))
    p0 = _rand_params(rng, H)
    lr = 1e-2
    traj = orc.cdf_adam_steps(u, p0, 2, nb, lr)
    ub, yb = _minibatch(u, m, 0, nb)
    _, g1 = orc.mlp_grad(p0, ub, yb)
    g1 = _flat(g1)
    want1 = orc.flat_params(p0) - lr * g1 / (np.abs(g1) + 1e-8)
    assert np.allclose(traj[0], want1, rtol=1e-12, atol=1e-15)
    p1 = {"w1": traj[0][:H], "b1": traj[0][H:2 * H], "w2": traj[0][2 * H:3 * H], "b2": float(traj[0][3 * H])}
    ub, yb = _minibatch(u, m, 1, nb)
    _, g2 = orc.mlp_grad(p1, ub, yb)
    g2 = _flat(g2)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.9 ** 2)
    vh = (0.999 * 0.001 * g1 * g1 + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    want2 = traj[0] - lr * mh / (np.sqrt(vh) + 1e-8)
    assert np.allclose(traj[1], want2, rtol=1e-10, atol=1e-14)


def test_loss_identity_model_is_zero(orc):
    # f(u) = u on u_i = (i + 1/2)/m puts every point on its target
    ident = {"w1": np.array([1.0]), "b1": np.array([0.0]), "w2": np.array([1.0]), "b2": 0.0}
    for m in (1, 7, 64, 1000, 4096):
        u = (np.arange(m) + 0.5) / m
        for stride in (1, 3, 64):
            assert orc.cdf_loss(ident, u, stride) == 0.0


def test_loss_constant_model_closed_form(orc):
    # f = c: the mean over the k = ceil(m/s) points i = s*j of (c - (s*j + 1/2)/m)^2,
    # from sum_j (s j + 1/2) = s k(k-1)/2 + k/2 and
    # sum_j (s j + 1/2)^2 = s^2 (k-1)k(2k-1)/6 + s k(k-1)/2 + k/4
    from fractions import Fraction
    rng = np.random.default_rng(2)
    for m, s in ((1, 1), (10, 1), (10, 3), (4096, 64), (5000, 64), (777, 5)):
        c = float(rng.random())
        const = {"w1": np.array([0.0]), "b1": np.array([0.0]), "w2": np.array([0.0]), "b2": c}
        u = np.sort(rng.random(m))
        k = -(-m // s)
        C = Fraction(c)
        s1 = Fraction(s * k * (k - 1), 2) + Fraction(k, 2)
        s2 = Fraction(s * s * (k - 1) * k * (2 * k - 1), 6) + Fraction(s * k * (k - 1), 2) + Fraction(k, 4)
        want = (k * C * C - 2 * C * s1 / m + s2 / (m * m)) / k
        assert orc.cdf_loss(const, u, s) == pytest.approx(float(want), rel=1e-12, abs=1e-300)


def test_training_keeps_the_better_model(orc):
    # the trained parameters are the raw Adam trajectory's last row when
    # their strided loss is at most the initial one, else the initial model
    keys = np.sort(workloads.lognormal(1 << 14, 6))
    u, _, _ = orc.normalised_features(keys, 64, 20)
    H, steps, nb = 16, 24, 512
    init = orc.cdf_init(u, H)
    l0 = orc.cdf_loss(init, u)
    for lr, improves in ((3e-4, True), (5.0, False)):
        traj = orc.cdf_adam_steps(u, init, steps, nb, lr)
        last = {"w1": traj[-1][:H], "b1": traj[-1][H:2 * H], "w2": traj[-1][2 * H:3 * H], "b2": float(traj[-1][3 * H])}
        l_raw = orc.cdf_loss(last, u)
        assert (l_raw <= l0) == improves, (lr, l_raw, l0)
        p, l, trained = orc.cdf_train(u, H, steps, nb, lr, want_trained=True)
        assert trained == improves
        assert np.array_equal(orc.flat_params(p), traj[-1] if improves else orc.flat_params(init))
        assert l == (l_raw if improves else l0)


def test_adam_first_steps_closed_form(orc):
    # Adam (Kingma and Ba): the bias-corrected first step moves every
    # parameter by lr * g / (|g| + eps), i.e. almost exactly lr against the
    # sign of its gradient; a second step with the same gradient does the
    # same again (both moment estimates stay g and g^2 after correction).
    rng = np.random.default_rng(3)
    g = rng.normal(size=9) * 10.0 ** rng.integers(-3, 3, size=9)
    g[0] = 0.0
    p = rng.normal(size=9)
    p0 = p.copy()
    m1 = np.zeros(9)
    m2 = np.zeros(9)
    lr = 1e-3
    orc.adam_update(p, g, m1, m2, 1, lr)
    step = lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(p0 - p, step, rtol=1e-12, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)
    orc.adam_update(p, g, m1, m2, 2, lr)
    assert np.allclose(p0 - p, 2 * step, rtol=1e-9, atol=1e-15)


def _ident_table(orc, K=64):
    ident = {"w1": np.array([1.0]), "b1": np.array([0.0]), "w2": np.array([1.0]), "b2": 0.0}
    z_lo = orc.feature(1 << 40, 64, 40)
    return orc.cdf_table(ident, z_lo, z_lo + (1 << 20), K)


def test_judge_zero_for_a_perfect_model(orc):
    # identity table, keys 2^40 + d with F = d / 2^20 exactly below the last
    # knot (pinned above; 4096 knots put it at d = 4095 * 2^8); sample points
    # at d_i = (2i+1) 2^9 for m = 2^10 sit exactly on their targets
    # (2i+1)/(2m): every error is zero
    tab = _ident_table(orc, 4096)
    assert tab.shift == 8
    m, B = 1 << 10, 256
    keys = np.array([(1 << 40) + (2 * i + 1) * (1 << 9) for i in range(m)], dtype=np.uint64)
    j = orc.judge(keys, 64, 40, tab, B)
    assert j["d_max"] == 0 and j["max_err"] == 0.0 and j["max_bucket_err"] == 0


def test_judge_identity_model_brute_force(orc):
    # the same identity model on random sorted offsets: the judge is the
    # definition |B d_i / 2^20 - B (i + 1/2) / m| in exact rationals
    from fractions import Fraction
    tab = _ident_table(orc)
    rng = np.random.default_rng(17)
    for m, B in ((1000, 256), (4096, 65536), (3, 2)):
        d = np.sort(rng.integers(0, 63 << 14, m))
        keys = ((1 << 40) + d).astype(np.uint64)
        errs = [abs(Fraction(B * int(di), 1 << 20) - Fraction(B * (2 * i + 1), 2 * m)) for i, di in enumerate(d)]
        berrs = [abs((int(di) * B >> 20) - (B * (2 * i + 1)) // (2 * m)) for i, di in enumerate(d)]
        j = orc.judge(keys, 64, 40, tab, B)
        assert j["samples"] == m
        assert j["max_err"] == float(max(errs))
        assert j["mean_err"] == float(sum(errs) / m)
        assert j["max_bucket_err"] == max(berrs) and j["sum_bucket_err"] == sum(berrs)


def test_judge_constant_model_closed_form(orc):
    # F = 0 everywhere: bucket(x_i) = 0, so the bucket error is floor(B y_i);
    # with m = kB that is k copies of 0..B-1: mean (B-1)/2, maximum B-1.  The
    # CDF error B y_i has maximum B (2m-1)/(2m) and mean B/2.
    K = 16
    tab = orc.Table(np.zeros(K + 1, dtype=np.uint64), 4, K, 0, K << 4)
    for k, B in ((1, 8), (3, 1024), (7, 2)):
        m = k * B
        keys = np.sort(workloads.lognormal(m, B))
        j = orc.judge(keys, 64, 20, tab, B)
        assert j["max_bucket_err"] == B - 1 and j["mean_bucket_err"] == (B - 1) / 2
        assert j["d_max"] == (2 * m - 1) << 32
        assert j["max_err"] == B * (2 * m - 1) / (2 * m) and j["mean_err"] == B / 2
