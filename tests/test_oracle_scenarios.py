"""Pins of the oracle's scenario generator (CPU): the counter-based RNG
against numpy's independent Philox4x64-10, the normals by their law, and the
exact Vasicek step by the Ornstein-Uhlenbeck moments, the zero-coupon bond
closed form, the one-step covariance of (r, integral of r) and the
deterministic case sigma = 0."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import synth

A, B, SIG, DT = 0.1, 0.03, 0.01, 1.0 / 12.0


def _plus_one(c):
    """The 256-bit counter plus one (numpy's generator advances before each block)."""
    out = [int(x) for x in c]
    for i in range(4):
        out[i] = (out[i] + 1) % (1 << 64)
        if out[i] != 0:
            break
    return out


@pytest.mark.parametrize("seed", range(6))
def test_philox_matches_numpy(seed):
    rng = np.random.default_rng(seed)
    c = [int(x) for x in rng.integers(0, 1 << 63, 4, dtype=np.uint64)]
    k = [int(x) for x in rng.integers(0, 1 << 63, 2, dtype=np.uint64)]
    if seed == 0:
        c = [(1 << 64) - 1, (1 << 64) - 1, 5, 0]          # carries into word 2
    if seed == 1:
        k = [(1 << 64) - 1, (1 << 64) - 1]
    want = np.random.Philox(counter=np.array(c, np.uint64), key=np.array(k, np.uint64)).random_raw(4)
    got = oracle.philox4x64_10(_plus_one(c), k)
    assert np.array_equal(got, want)


def test_normals_have_the_standard_normal_law():
    key = (2024, 7)
    z = np.array([oracle.normals(key, 0, s, t) for s in range(200) for t in range(250)])
    n = z.shape[0]
    for j in range(2):
        assert abs(z[:, j].mean()) < 5 / math.sqrt(n)
        assert abs(z[:, j].var() - 1.0) < 5 * math.sqrt(2.0 / n)
        assert stats.kstest(z[:, j], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 5 / math.sqrt(n)
    # counters and keys give different blocks; the same ones the same block
    assert not np.array_equal(oracle.normals(key, 0, 1, 2), oracle.normals(key, 0, 2, 1))
    assert not np.array_equal(oracle.normals(key, 0, 1, 2), oracle.normals(key, 1, 1, 2))
    assert not np.array_equal(oracle.normals(key, 0, 1, 2), oracle.normals((2024, 8), 0, 1, 2))
    assert np.array_equal(oracle.normals(key, 3, 4, 5), oracle.normals(key, 3, 4, 5))


def test_vasicek_ou_moments_and_bond_prices():
    n, T = 40_000, 120
    v, r = oracle.vasicek_curves(A, B, SIG, DT, [0.05], n, T, (99, 1))
    for t in (1, 12, 60, 120):
        tau = t * DT
        mean = B + (0.05 - B) * math.exp(-A * tau)
        var = SIG ** 2 * (1 - math.exp(-2 * A * tau)) / (2 * A)
        assert abs(r[0, :, t].mean() - mean) < 5 * math.sqrt(var / n)
        assert abs(r[0, :, t].var() / var - 1.0) < 5 * math.sqrt(2.0 / n)
    disc = np.cumprod(v[0], axis=1)
    for t in (12, 60, 120):
        p = disc[:, t - 1]
        want = synth.vasicek_zcb(t * DT, 0.05, A, B, SIG)
        assert abs(p.mean() - want) < 5 * p.std() / math.sqrt(n)


def test_vasicek_one_step_joint_law():
    """From a common r_0: Var Y, Var r_1 and Cov(r_1, Y) of the first step."""
    n = 200_000
    v, r = oracle.vasicek_curves(A, B, SIG, DT, [0.02], n, 1, (5, 5))
    Y = -np.log(v[0, :, 0])
    r1 = r[0, :, 1]
    e = math.exp(-A * DT)
    var_r = SIG ** 2 * (1 - e * e) / (2 * A)
    var_y = SIG ** 2 / A ** 2 * (DT - 2 * (1 - e) / A + (1 - e * e) / (2 * A))
    cov = SIG ** 2 / (2 * A ** 2) * (1 - e) ** 2
    assert abs(Y.mean() - (B * DT + (0.02 - B) * (1 - e) / A)) < 5 * math.sqrt(var_y / n)
    assert abs(Y.var() / var_y - 1) < 5 * math.sqrt(2.0 / n)
    assert abs(r1.var() / var_r - 1) < 5 * math.sqrt(2.0 / n)
    c = np.cov(r1, Y)[0, 1]
    assert abs(c / cov - 1) < 0.02
    assert c > 0     # the integral moves with the end rate


def test_vasicek_without_volatility_is_the_ode_solution():
    T = 600
    v, r = oracle.vasicek_curves(A, B, 0.0, DT, [0.07, 0.01], 2, T, (1, 1))
    t = np.arange(T + 1) * DT
    for k, r0 in enumerate((0.07, 0.01)):
        np.testing.assert_allclose(r[k, 0], B + (r0 - B) * np.exp(-A * t), rtol=1e-13)
        integral = B * t[1:] + (r0 - B) * (1 - np.exp(-A * t[1:])) / A
        np.testing.assert_allclose(np.cumprod(v[k, 1]), np.exp(-integral), rtol=1e-12)
