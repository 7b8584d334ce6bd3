"""Checks of the seeded input generators: the mortality table against
numerical quadrature of the force of mortality, the Vasicek scenarios against
the model's closed-form moments and bond prices, and seed reproducibility."""
import math

import numpy as np
import pytest
from scipy import integrate

import synth


def test_gm_monthly_q_matches_quadrature():
    q = synth.gm_monthly_q(1500)
    A, B, c = synth.GM_A, synth.GM_B, synth.GM_C
    mu = lambda s: A + B * c ** s
    for a in (0, 1, 240, 777, 1020, 1439):
        H, _ = integrate.quad(mu, a / 12.0, (a + 1) / 12.0, epsabs=0, epsrel=2e-14)
        assert q[a] == pytest.approx(-math.expm1(-H), rel=1e-13)
    assert np.all(q[1440:] == 1.0)
    assert np.all(np.diff(q[:1440]) > 0)
    ql = synth.gm_monthly_q(1500, 1.2)
    assert np.all(ql <= 1.0)
    np.testing.assert_allclose(ql[:1000], np.minimum(1.0, 1.2 * q[:1000]), rtol=1e-15)


def test_vasicek_moments_and_bond_price():
    rng = np.random.default_rng(123)
    n, steps = 20000, 120
    v, r = synth.vasicek_paths(rng, n, steps, 0.05)
    a, b, s = synth.VAS_A, synth.VAS_B, synth.VAS_SIGMA
    for t in (12, 60, 120):
        T = t / 12.0
        mean = b + (0.05 - b) * math.exp(-a * T)
        var = s * s * (1 - math.exp(-2 * a * T)) / (2 * a)
        se = math.sqrt(var / n)
        assert abs(r[:, t].mean() - mean) < 4 * se
        assert r[:, t].var() == pytest.approx(var, rel=4 * math.sqrt(2.0 / n))
        D = np.prod(v[:, :t], axis=1)
        P = synth.vasicek_zcb(T, 0.05)
        assert abs(D.mean() - P) < 4 * D.std() / math.sqrt(n)


def test_workloads_reproducible_and_in_range():
    a = synth.config_c2(n=5000)
    b = synth.config_c2(n=5000)
    np.testing.assert_array_equal(a.portfolio.amount, b.portfolio.amount)
    pf = a.portfolio
    assert pf.term_m.min() >= 60 and pf.term_m.max() <= 600
    assert pf.age1_m.min() >= 240 and pf.age1_m.max() <= 1020
    counts = np.bincount(pf.product, minlength=7)
    assert counts[synth.SL_ANN] == 2000 and counts[synth.JL_ANN] == 1000
    assert counts[synth.TERM] == 1000 and counts[synth.ENDOW] == 1000
    assert np.all(pf.age1_m + pf.term_m < a.basis.q.shape[1])
    c1 = synth.config_c1()
    assert c1.portfolio.n == 1000 and c1.basis.n_steps == 300
    assert c1.portfolio.amount.mean() == pytest.approx(1.0e4, rel=0.1)
