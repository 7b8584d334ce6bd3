"""Pins of the surrogate oracle (oracle/mlp.py) against what mathematics and
library routines fix: bfloat16 rounding, GELU identities, finite-difference
gradients, Adam's closed-form first steps, zero rates of known curves, PCA of
curves built from known factors, hand-computed features and the exact
reserves the targets come from."""
import numpy as np
import pytest
import torch
from scipy.special import erf

import oracle
import synth
from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, 20000).astype(np.float32) * np.float32(10.0) ** rng.integers(-20, 20, 20000)
    # exact halfway cases, both parities of the kept last bit, and carries
    bits = rng.integers(0, 1 << 31, 4000).astype(np.uint32)
    bits = (bits & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    half = bits.view(np.float32)
    special = np.array([0.0, -0.0, 1.0, -1.0, 3.3895314e38, 1.17549435e-38,
                        np.float32(1.0) + np.float32(2 ** -8), 65504.0], np.float32)
    for arr in (x, half[np.isfinite(half)], special):
        ref = torch.from_numpy(arr.copy()).to(torch.bfloat16).to(torch.float32).numpy()
        got = mlp.bf16(arr)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_gelu_identities_and_erf_form():
    x = np.linspace(-12, 12, 4801)
    g = mlp.gelu(x)
    assert mlp.gelu(0.0) == 0.0
    # tanh is odd, so gelu(x) - gelu(-x) = x exactly in real arithmetic
    assert np.max(np.abs(g - mlp.gelu(-x) - x)) <= 1e-14 * np.max(np.abs(x))
    exact = 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))
    assert np.max(np.abs(g - exact)) < 1e-3           # tanh form vs the erf definition
    assert np.max(np.abs(g - exact)) > 1e-5           # ... and it is the tanh form
    assert abs(mlp.gelu(40.0) - 40.0) < 1e-12 and abs(mlp.gelu(-40.0)) < 1e-12


def test_gelu_grad_finite_differences():
    x = np.linspace(-6, 6, 601)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def _net(seed, n=7):
    rng = np.random.default_rng(seed)
    p = {k: np.asarray(v, np.float64) for k, v in synth.random_mlp_params(rng).items()}
    z = np.zeros((n, mlp.K_IN))
    z[:, :mlp.N_FEAT] = rng.normal(0, 1, (n, mlp.N_FEAT))
    t = rng.normal(0, 1, n)
    return p, z, t


def test_backward_fp64_matches_finite_differences():
    p, z, t = _net(2)
    g, _ = mlp.backward(p, z, t, quant=False)
    rng = np.random.default_rng(3)
    for name, shape in mlp.PARAM_SHAPES:
        arr = p[name]
        if shape == ():
            idxs = [()]
        else:
            flat = rng.choice(arr.size, min(25, arr.size), replace=False)
            if name == "W1":   # real input rows only: padded rows have zero inputs
                flat = rng.choice(mlp.N_FEAT * mlp.HIDDEN, 25, replace=False)
            idxs = [np.unravel_index(f, shape) for f in flat]
        gmax = np.max(np.abs(g[name]))
        for ix in idxs:
            q = {k: np.array(v, dtype=np.float64, copy=True) for k, v in p.items()}
            h = 1e-5 * max(1.0, abs(float(arr[ix])))
            q[name][ix] += h
            lp = mlp.loss(q, z, t, quant=False)
            q[name][ix] -= 2 * h
            lm = mlp.loss(q, z, t, quant=False)
            fd = (lp - lm) / (2 * h)
            got = float(np.asarray(g[name])[ix])
            assert abs(fd - got) <= 1e-6 * (abs(got) + 1e-3 * gmax), (name, ix, fd, got)
    # padded input rows get exactly zero gradient
    assert np.all(g["W1"][mlp.N_FEAT:] == 0.0)


def test_bf16_mode_is_close_to_fp64():
    p, z, t = _net(4, n=64)
    y64, _ = mlp.forward(p, z, quant=False)
    y16, s = mlp.forward(p, z, quant=True)
    assert np.linalg.norm(y16 - y64) <= 2e-2 * np.linalg.norm(y64)
    # quantisation points hold bfloat16 values
    for k in ("xq", "a1", "a2", "W1", "W2", "W3"):
        assert np.array_equal(mlp.bf16(s[k]), np.asarray(s[k], np.float32))
    g64, _ = mlp.backward(p, z, t, quant=False)
    g16, _ = mlp.backward(p, z, t, quant=True)
    for k, _ in mlp.PARAM_SHAPES:
        a, b = np.ravel(g16[k]).astype(np.float64), np.ravel(g64[k])
        assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b) + 1e-12, k


def test_adam_first_two_steps_closed_form():
    rng = np.random.default_rng(5)
    p = {k: np.asarray(v, np.float32) for k, v in synth.random_mlp_params(rng).items()}
    g1 = {k: rng.normal(0, 1e-2, np.shape(v)).astype(np.float32) for k, v in p.items()}
    g2 = {k: rng.normal(0, 1e-2, np.shape(v)).astype(np.float32) for k, v in p.items()}
    zeros = {k: np.zeros(np.shape(v), np.float32) for k, v in p.items()}
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = mlp.adam(p, g1, zeros, zeros, 1, lr)
    p2, _, _ = mlp.adam(p1, g2, m1, v1, 2, lr)
    for k in p:
        a = np.asarray(g1[k], np.float64)
        b = np.asarray(g2[k], np.float64)
        w0 = np.asarray(p[k], np.float64)
        w1 = w0 - lr * a / (np.abs(a) + eps)
        mh = (0.9 * 0.1 * a + 0.1 * b) / (1 - 0.9 ** 2)
        vh = (0.999 * 0.001 * a * a + 0.001 * b * b) / (1 - 0.999 ** 2)
        w2 = w1 - lr * mh / (np.sqrt(vh) + eps)
        assert np.max(np.abs(np.asarray(p1[k], np.float64) - w1)) <= 4e-7 * max(1.0, np.max(np.abs(w0)))
        assert np.max(np.abs(np.asarray(p2[k], np.float64) - w2)) <= 8e-7 * max(1.0, np.max(np.abs(w0)))


def test_zero_rates_of_flat_and_random_curves():
    v = synth.flat_v(600)
    z = mlp.zero_rates(v)
    assert np.allclose(z, np.log(1.03), rtol=0, atol=1e-15)
    assert abs(mlp.short_rate(v) - np.log(1.03)) < 1e-15
    rng = np.random.default_rng(6)
    v = rng.uniform(0.995, 1.001, (3, 300))
    z = mlp.zero_rates(v)
    for T in range(1, 51):
        m = min(12 * T, 300)
        D = np.prod(v[:, :m], axis=1)          # discount factor to month m
        assert np.allclose(np.exp(-z[:, T - 1] * m / 12.0), D, rtol=1e-13)
    assert np.array_equal(z[:, 24], z[:, 49])  # tenors beyond the curve use its end


def test_pca_recovers_known_factors():
    rng = np.random.default_rng(7)
    E0, _ = np.linalg.qr(rng.normal(size=(mlp.N_TENORS, 3)))
    zbar0 = np.linspace(0.01, 0.04, mlp.N_TENORS)
    # scores with zero sample mean, uncorrelated sample columns and known variances
    n = 20000
    s = rng.normal(size=(n, 3))
    s -= s.mean(axis=0)
    Q, _ = np.linalg.qr(s)
    sig = np.array([3.0, 2.0, 1.0]) * 1e-3
    scores = Q * np.sqrt(n) * sig
    z = zbar0 + scores @ E0.T
    zbar, E, w = mlp.fit_pca(z)
    assert np.allclose(zbar, zbar0, atol=1e-15)
    for j in range(3):
        c = abs(float(E[:, j] @ E0[:, j]))
        assert c > 1 - 1e-10
        assert E[np.argmax(np.abs(E[:, j])), j] > 0
        assert abs(w[j] - sig[j] ** 2) < 1e-9 * sig[j] ** 2
    assert np.allclose(E.T @ E, np.eye(3), atol=1e-12)


def test_policy_features_by_hand():
    pf = synth.Portfolio(product=np.array([0, 1, 4, 5, 2], np.int32),
                         age1_m=np.array([720, 600, 300, 480, 700], np.int32),
                         age2_m=np.array([0, 612, 0, 0, 650], np.int32),
                         term_m=np.array([300, 120, 240, 60, 100], np.int32),
                         table1=np.array([0, 0, 1, 2, 0], np.int32),
                         table2=np.array([0, 0, 1, 2, 0], np.int32),
                         timing=np.array([1, 1, 1, 1, 1], np.int32),
                         amount=np.array([1e4, 2e4, 1e5, 5e4, 1e4]),
                         premium=np.array([0.0, 0.0, 20.0, 100.0, 0.0]))
    f, ok = mlp.policy_features(pf, node=2, node_step=12)
    assert f[0].tolist() == [62.0, 23.0, 1, 0, 0, 0, np.log(1e4), 0.0, 0.0]
    assert f[1].tolist() == [52.0, 8.0, 0, 1, 0, 0, np.log(2e4), 0.0, 53.0]
    assert f[2, 7] == 12 * 20.0 / 1e5 and f[3, 7] == 12 * 100.0 / 5e4
    assert ok.tolist() == [True, True, True, True, False]     # reversionary annuity: no one-hot
    sig = mlp.product_signature(pf.subset([0, 1, 2, 3]))
    assert sig == [(0, -1, 1), (0, 0, 1), (1, -1, -1), (2, -1, -1)]
    pf.table1[2] = 2      # a term assurance on the endowment table is outside the domain
    _, ok = mlp.policy_features(pf, 0, 12, sig)
    assert ok.tolist() == [True, True, False, True, False]


def test_samples_come_from_exact_reserves():
    rng = np.random.default_rng(8)
    w = synth.random_small(rng, n=40, n_steps=48, n_scen=3, n_nodes=2, shock=True,
                           products=(0, 1, 2, 4, 5))
    b, pf = w.basis, w.portfolio
    ref = oracle.reserves(b, pf, 0, 2, 0, 3, 0)
    zbar, E, _ = mlp.fit_pca(mlp.zero_rates(b.v.reshape(-1, b.n_steps)))
    X, T = mlp.samples(w, 0, 2, 0, 3, 0, ref["r_all"], zbar, E)
    per = np.where(pf.product == 1, 3, np.where(pf.product == 2, 0, 1))
    assert X.shape == (2 * 3 * per.sum(), mlp.N_FEAT)
    # the first rows are node 0, scenario 0, in policy order
    i0 = int(np.flatnonzero(per > 0)[0])
    assert T[0] == ref["r_all"][0, i0, 0, 0] / pf.amount[i0]
    assert X[0, mlp.F_SHOCK] == b.shock[0]
    assert X[0, mlp.F_RATE] == -12.0 * np.log(b.v[0, 0, 0])
    jl = X[:, mlp.F_PROD + 1] == 1
    st = X[:, mlp.F_STATE:mlp.F_STATE + 3]
    assert np.all(st.sum(axis=1) == 1)
    # a joint-life annuity pays only while both live: states 1 and 2 hold 0
    assert np.all(T[jl & (st[:, 0] == 0)] == 0.0)
    mu, sd, lo, hi, tmu, tsd = mlp.normalisation(X, T)
    zs = mlp.standardise(X, mu, sd)
    assert np.allclose(zs[:, :mlp.N_FEAT].mean(axis=0), 0, atol=1e-6)
    live = X.std(axis=0) > 0
    assert np.allclose(zs[:, :mlp.N_FEAT][:, live].std(axis=0), 1, atol=1e-6)
    assert np.all(zs[:, mlp.N_FEAT:] == 0)
    ts = mlp.standardise_target(X, T, tmu, tsd)
    for j in range(4):
        sel = X[:, mlp.F_PROD + j] == 1
        if sel.sum() > 1 and np.std(T[sel]) > 0:
            assert abs(ts[sel].mean()) < 1e-6 and abs(ts[sel].std() - 1) < 1e-6
    assert mlp.in_range(X, lo, hi).all()
    assert not mlp.in_range(X[:1] + (hi - lo + 1), lo, hi).any()


def test_bf16_boundary_distance_by_brute_force():
    """The distance to the rounding boundary: moving a value by 90 % of it
    either way keeps its bfloat16 rounding, moving by 101 % towards the
    boundary changes it; exact midpoints are at distance 0 and bfloat16
    values at half a unit."""
    rng = np.random.default_rng(5)
    x = (rng.normal(0, 1, 2000) * 10.0 ** rng.integers(-8, 8, 2000)).astype(np.float32)
    d = mlp.bf16_boundary_distance(x)
    # moves that FP32 represents without landing on a boundary
    f32_ulp = np.spacing(np.abs(x)).astype(np.float64)
    far = d > 16 * f32_ulp
    assert far.mean() > 0.95
    for sgn in (-1.0, 1.0):
        moved = (x.astype(np.float64) + sgn * 0.9 * d).astype(np.float32)
        assert np.array_equal(mlp.bf16(moved)[far], mlp.bf16(x)[far])
    up = (x.astype(np.float64) + 1.01 * d).astype(np.float32)
    dn = (x.astype(np.float64) - 1.01 * d).astype(np.float32)
    changed = (mlp.bf16(up) != mlp.bf16(x)) | (mlp.bf16(dn) != mlp.bf16(x))
    assert np.all(changed[far])
    b = mlp.bf16(x)
    ulp = (np.abs((b.view(np.uint32) + np.uint32(0x10000)).view(np.float32).astype(np.float64))
           - np.abs(b.astype(np.float64)))
    # a bfloat16 value is half a unit from the boundary above it, and half
    # a unit below it from the one below (a quarter at powers of two)
    db = mlp.bf16_boundary_distance(b)
    pow2 = (b.view(np.uint32) & np.uint32(0x007F0000)) == 0
    np.testing.assert_array_equal(db[~pow2], 0.5 * ulp[~pow2])
    np.testing.assert_array_equal(db[pow2], 0.25 * ulp[pow2])
    mid = (np.abs(b).astype(np.float64) + 0.5 * ulp).astype(np.float32)
    assert np.all(mlp.bf16_boundary_distance(mid) == 0.0)


def test_abs_sums_equal_the_sums_for_nonnegative_terms():
    """With non-negative inputs, weights and gradient factors every term is
    non-negative, so each sum of absolute terms is the sum itself."""
    rng = np.random.default_rng(6)
    p = {k: np.abs(v) for k, v in synth.random_mlp_params(rng).items()}
    p["b3"] = np.float32(abs(p["b3"]))
    z = np.zeros((40, mlp.K_IN), np.float32)
    z[:, :mlp.N_FEAT] = np.abs(rng.normal(0, 1, (40, mlp.N_FEAT)))
    t = np.full(40, -100.0, np.float32)          # y > t: dy > 0
    g, y, s = mlp.backward(p, z, t, quant=False, keep=True)
    S = mlp.abs_sums(p, s, 40)
    np.testing.assert_allclose(S["z1"], s["z1"], rtol=1e-12)
    np.testing.assert_allclose(S["z2"], s["z2"], rtol=1e-12)
    np.testing.assert_allclose(S["y"], y, rtol=1e-12)
    assert np.all(np.asarray(s["dy"]) > 0)
    for k in ("W3", "b3"):
        np.testing.assert_allclose(S["grad"][k], g[k], rtol=1e-12)
    # GELU' is positive for positive pre-activations, so dz2, dz1 and all
    # remaining gradients are sums of non-negative terms too
    assert np.all(np.asarray(s["z1"]) > 0) and np.all(np.asarray(s["z2"]) > 0)
    for k in ("W2", "b2", "W1", "b1"):
        np.testing.assert_allclose(S["grad"][k], g[k], rtol=1e-12)
    assert mlp.gamma(1) > mlp.U32 and abs(mlp.gamma(1000) / (1000 * mlp.U32) - 1.0) < 1e-4
