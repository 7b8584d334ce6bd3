"""Pins of the CPU oracle against facts fixed by the paper and by the
mathematics: closed forms, textbook identities between products, the
transition matrices the paper prints, the summation definition (Eq. 3.5) on
tiny inputs, structural invariants and the complexity shape (Sec. 5.1.2)."""
import math
import os
import time

import numpy as np
import pytest

import oracle
import synth
from synth import (ADVANCE, ARREARS, CF_TABLE, FRACTIONAL, ENDOW, ENDOW_ASSUR, JL_ASSUR1, JL_ASSUR2, JL_ENDOW, MARKOV, JL_ANN, LS_ANN,
                   REV_ANN, SL_ANN, TERM, Basis, Portfolio)

HERE = os.path.dirname(os.path.abspath(__file__))


def make_pf(product, age1, term, amount=12.0, premium=0.0, timing=ARREARS,
            age2=0, table1=0, table2=0):
    n = len(product)
    arr = lambda x, dt: np.asarray(np.broadcast_to(x, (n,)), dt).copy()
    return Portfolio(product=arr(product, np.int32), age1_m=arr(age1, np.int32),
                     age2_m=arr(age2, np.int32), term_m=arr(term, np.int32),
                     table1=arr(table1, np.int32), table2=arr(table2, np.int32),
                     timing=arr(timing, np.int32), amount=arr(amount, np.float64),
                     premium=arr(premium, np.float64))


def basis(q_tables, v, shock=None):
    q = np.atleast_2d(np.asarray(q_tables, np.float64))
    v = np.asarray(v, np.float64)
    if v.ndim == 1:
        v = v[None, None, :]
    elif v.ndim == 2:
        v = v[None]
    return Basis(q=q, v=v, shock=shock)


def r0(b, pf, **kw):
    return oracle.reserves(b, pf, **kw)["r_all"][0, :, 0, :]


N_AGES = 2000
V_FLAT = 1.03 ** (-1.0 / 12.0)


def gm(load=1.0):
    return synth.gm_monthly_q(N_AGES, load)


# --------------------------------------------------------------------------
# Closed forms with zero mortality (annuities certain) and v = 1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 7, 120, 300, 600])
def test_annuity_certain_arrears_and_advance(n):
    b = basis(np.zeros(N_AGES), np.full(600, V_FLAT))
    pf = make_pf([SL_ANN, SL_ANN], 700, n, amount=12.0, timing=[ARREARS, ADVANCE])
    r = r0(b, pf)
    v = V_FLAT
    i_m = 1.0 / v - 1.0
    d = 1.0 - v
    assert r[0, 0] == pytest.approx((1 - v ** n) / i_m, rel=1e-13)
    assert r[1, 0] == pytest.approx((1 - v ** n) / d, rel=1e-13)


@pytest.mark.parametrize("n", [1, 60, 600])
def test_annuity_undiscounted_is_expected_number_of_payments(n):
    q = gm(1.0)
    b = basis(q, np.ones(600))
    age = 800
    pf = make_pf([SL_ANN, SL_ANN], age, n, amount=12.0, timing=[ARREARS, ADVANCE])
    r = r0(b, pf)
    p = 1.0 - q[age:age + n]
    kp = np.cumprod(p)                         # P(alive at k), k = 1..n
    assert r[0, 0] == pytest.approx(kp.sum(), rel=1e-13)
    assert r[1, 0] == pytest.approx(1.0 + kp[:-1].sum(), rel=1e-13)


def test_term_assurance_closed_forms():
    q = gm(1.2)
    n, age, SA, P = 240, 600, 1.0e5, 37.5
    # v = 1, no premium: probability of death within the term
    b = basis(q, np.ones(600))
    r = r0(b, make_pf([TERM], age, n, amount=SA))
    npx = np.prod(1.0 - q[age:age + n])
    assert r[0, 0] == pytest.approx(SA * (1.0 - npx), rel=1e-12)
    # zero mortality: only premiums, an annuity-certain due
    b0 = basis(np.zeros(N_AGES), np.full(600, V_FLAT))
    r = r0(b0, make_pf([TERM], age, n, amount=SA, premium=P))
    d = 1.0 - V_FLAT
    assert r[0, 0] == pytest.approx(-P * (1 - V_FLAT ** n) / d, rel=1e-13)
    assert r[0, 1] == 0.0 and r[0, 2] == 0.0


def test_endowment_closed_forms():
    n, age, SA, P = 180, 500, 5.0e4, 200.0
    b0 = basis(np.zeros(N_AGES), np.full(600, V_FLAT))
    v = V_FLAT
    r = r0(b0, make_pf([ENDOW, ENDOW], age, n, amount=SA, premium=[0.0, P]))
    assert r[0, 0] == pytest.approx(SA * v ** n, rel=1e-13)
    assert r[1, 0] == pytest.approx(SA * v ** n - P * (1 - v ** n) / (1 - v), rel=1e-12)


# --------------------------------------------------------------------------
# Textbook identities between products, any mortality
# --------------------------------------------------------------------------
def test_arrears_equals_due_minus_one_plus_pure_endowment():
    rng = np.random.default_rng(7)
    q = gm(0.9)
    v = rng.uniform(0.995, 1.0, 600)             # time-varying interest
    b = basis(q, v)
    age, n = 777, 333
    pf = make_pf([SL_ANN, SL_ANN, ENDOW], age, n, amount=[12.0, 12.0, 1.0],
                 timing=[ARREARS, ADVANCE, ARREARS])
    r = r0(b, pf)
    assert r[0, 0] == pytest.approx(r[1, 0] - 1.0 + r[2, 0], rel=1e-13)


def test_endowment_assurance_is_one_minus_d_times_annuity_due():
    q = gm(1.1)
    b = basis(q, np.full(600, V_FLAT))
    age, n = 400, 420
    pf = make_pf([ENDOW_ASSUR, SL_ANN], age, n, amount=[1.0, 12.0], timing=ADVANCE)
    r = r0(b, pf)
    d = 1.0 - V_FLAT
    assert r[0, 0] == pytest.approx(1.0 - d * r[1, 0], rel=1e-13)


def test_term_plus_pure_endowment_is_endowment_assurance():
    rng = np.random.default_rng(11)
    q = gm(1.0)
    b = basis(q, rng.uniform(0.996, 1.0, 600))
    pf = make_pf([TERM, ENDOW, ENDOW_ASSUR], 300, 480, amount=2.0e5,
                 premium=[55.0, 0.0, 55.0])
    r = r0(b, pf)
    assert r[2, 0] == pytest.approx(r[0, 0] + r[1, 0], rel=1e-12)


def test_two_life_annuity_identities():
    """a_xy(LS) = a_x + a_y - a_xy; a_x|y = a_y - a_xy; the reserve vectors
    read as in Sec. 4.2.1: REV -> (a_x|y, 0, a_y, 0), LS -> (LS, a_x, a_y, 0)."""
    rng = np.random.default_rng(3)
    q = np.stack([gm(0.8), gm(1.3)])
    b = basis(q, rng.uniform(0.996, 1.0, 600))
    x, y, n = 820, 760, 500
    for timing in (ARREARS, ADVANCE):
        pf = make_pf([SL_ANN, SL_ANN, JL_ANN, REV_ANN, LS_ANN],
                     [x, y, x, x, x], n, amount=1200.0, timing=timing,
                     age2=[0, 0, y, y, y], table1=[0, 1, 0, 0, 0],
                     table2=[0, 0, 1, 1, 1])
        r = r0(b, pf)
        ax, ay, axy, rev, ls = r[0, 0], r[1, 0], r[2, 0], r[3], r[4]
        assert ls[0] == pytest.approx(ax + ay - axy, rel=1e-12)
        assert rev[0] == pytest.approx(ay - axy, rel=1e-12)
        assert rev[1] == 0.0 and rev[3] == 0.0
        assert rev[2] == pytest.approx(ay, rel=1e-13)
        assert ls[1] == pytest.approx(ax, rel=1e-13)
        assert ls[2] == pytest.approx(ay, rel=1e-13)
        assert ls[3] == 0.0
        assert np.all(r[2, 1:] == 0.0)          # joint life: zero-reserve states


def test_joint_life_with_immortal_second_life_is_single_life():
    q1 = gm(1.0)
    q = np.stack([q1, np.zeros(N_AGES)])
    b = basis(q, np.full(600, V_FLAT))
    pf = make_pf([SL_ANN, JL_ANN], 700, 400, amount=999.0, age2=[0, 100],
                 table1=0, table2=1)
    r = r0(b, pf)
    assert r[1, 0] == r[0, 0]


def test_joint_life_symmetric():
    q = gm(1.0)
    b = basis(q, np.full(600, V_FLAT))
    pf = make_pf([JL_ANN, JL_ANN], [700, 850], 400, amount=999.0, age2=[850, 700])
    r = r0(b, pf)
    assert r[0, 0] == pytest.approx(r[1, 0], rel=1e-15)


# --------------------------------------------------------------------------
# Boundaries (Sec. 4.1.1 - 4.1.3): reserve at expiry, limiting age
# --------------------------------------------------------------------------
def test_boundaries_at_expiry_and_limiting_age():
    q = gm(1.0)
    b = basis(q, np.full(600, V_FLAT))
    n = 200
    pf = make_pf([TERM, ENDOW, SL_ANN], 1300, n, amount=1000.0, premium=[3.0, 3.0, 0.0])
    path, off = oracle.reserve_paths(b, pf)
    assert path[off[0] + n] == 0.0              # term assurance: 0 at expiry
    assert path[off[1] + n] == 1000.0           # endowment: sum assured at maturity
    sl = path[off[2]:off[3]]
    # life reaches 120 years (1440 months) at t = 140: q = 1 from then on, so
    # an annuity in arrears has no value from t = 140 on.
    assert np.all(sl[1440 - 1300:] == 0.0)
    assert sl[1440 - 1300 - 1] > 0.0


# --------------------------------------------------------------------------
# Recurrence (Eq. 3.1) == summation (Eq. 3.5) on tiny random inputs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_recurrence_equals_summation(seed):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=24, n_steps=60, n_scen=2, n_nodes=3, shock=True)
    b, pf = w.basis, w.portfolio
    for node in range(3):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=12)
        full = oracle.reserves(b, pf, node0=node, nnode=1, scen0=1, nscen=1, node_step=12)
        for i in range(pf.n):
            S = int(pf.term_m[i]) - 12 * node
            if S <= 0:
                assert path[off[i]] == 0.0
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=12)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0],
                                       rtol=0, atol=1e-12 * scale)
            ns = summ.shape[1]
            np.testing.assert_allclose(full["r_all"][0, i, 0, :min(ns, 4)], summ[0, :4],
                                       rtol=0, atol=1e-12 * scale)


# --------------------------------------------------------------------------
# Transition matrices: the paper's printed matrices, invariants
# --------------------------------------------------------------------------
def _golden_matrices():
    blocks, cur = [], None
    with open(os.path.join(HERE, "golden", "transition_matrices.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("matrix"):
                parts = line.split()
                cur = {"name": parts[1], "lives": int(parts[2].split("=")[1]),
                       "model": int(parts[3].split("=")[1]), "rows": []}
                blocks.append(cur)
            else:
                cur["rows"].append(line.split())
    return blocks


@pytest.mark.parametrize("g", [1.0, 0.0])
def test_kronecker_matrices_match_the_paper(g):
    qx, qy = 0.013, 0.041
    px, py = 1 - g * qx, 1 - g * qy
    env = {"px": px, "qx": g * qx, "py": py, "qy": g * qy}
    blocks = _golden_matrices()
    assert len(blocks) == 4
    for blk in blocks:
        expect = np.array([[eval(e, {}, dict(env)) for e in row] for row in blk["rows"]], float)
        got = oracle.build_w(blk["lives"], blk["model"], [qx, qy][: blk["lives"]], g)
        np.testing.assert_allclose(got, expect, rtol=0, atol=1e-15, err_msg=blk["name"])


def test_last_survivor_payment_probability_is_top_row():
    qx, qy, f = 0.02, 0.05, 1.0
    W = oracle.build_w(2, 2, [qx, qy], f)
    assert W[0, :3].sum() == pytest.approx(1.0 - qx * qy, rel=1e-15)


@pytest.mark.parametrize("lives,model,n,nnz", [(1, 2, 2, 3), (2, 2, 4, 9), (3, 2, 8, 27),
                                               (1, 3, 3, 4), (2, 3, 9, 16)])
def test_state_and_nonzero_counts(lives, model, n, nnz):
    """2^m / 3^m states and 3^m / 4^m non-zeros (Sec. 4.3); rows sum to 1;
    binary labelling makes W upper triangular (Sec. 2.4.2)."""
    q = [0.01, 0.02, 0.03][:lives]
    W = oracle.build_w(lives, model, q, 1.0)
    assert W.shape == (n, n)
    assert np.count_nonzero(W) == nnz
    np.testing.assert_allclose(W.sum(axis=1), 1.0, atol=1e-15)
    if model == 2:
        assert np.all(np.tril(W, -1) == 0.0)


# --------------------------------------------------------------------------
# Linearity, node shift (Eq. 3.2), gross PV, totals, expiry
# --------------------------------------------------------------------------
def test_doubling_amounts_doubles_reserves_bitwise():
    rng = np.random.default_rng(5)
    w = synth.random_small(rng, n=40, n_steps=120, n_scen=2)
    a = oracle.reserves(w.basis, w.portfolio)["r_all"]
    b = oracle.reserves(w.basis, w.portfolio.scaled(2.0))["r_all"]
    assert np.array_equal(b, 2.0 * a)


def test_node_shift_equals_path_under_flat_rates():
    q = gm(1.0)
    v = np.full((5, 1, 600), V_FLAT)
    b = Basis(q=np.atleast_2d(q), v=v)
    pf = make_pf([SL_ANN, TERM, ENDOW, JL_ANN], [700, 400, 500, 650], [600, 500, 480, 550],
                 amount=[1200.0, 1e5, 5e4, 900.0], premium=[0, 30.0, 120.0, 0],
                 age2=[0, 0, 0, 720])
    path, off = oracle.reserve_paths(b, pf, node=0)
    full = oracle.reserves(b, pf, node_step=12)
    for k in range(5):
        for i in range(pf.n):
            assert full["r_all"][k, i, 0, 0] == path[off[i] + 12 * k]


def test_gross_bounds_reserve_and_equals_it_for_annuities():
    rng = np.random.default_rng(9)
    w = synth.random_small(rng, n=60, n_steps=100)
    out = oracle.reserves(w.basis, w.portfolio)
    r = out["r_all"][0, :, 0, 0]
    g = out["gross"][0, :, 0]
    assert np.all(g + 1e-9 >= np.abs(r))
    ann = np.isin(w.portfolio.product, (SL_ANN, JL_ANN, REV_ANN, LS_ANN)) & (w.portfolio.premium == 0)
    np.testing.assert_array_equal(g[ann], r[ann])


def test_totals_are_accurately_rounded_sums_and_skip_expired():
    rng = np.random.default_rng(13)
    w = synth.random_small(rng, n=200, n_steps=48, n_scen=3, n_nodes=4)
    out = oracle.reserves(w.basis, w.portfolio, node_step=12)
    for k in range(4):
        live = w.portfolio.term_m - 12 * k > 0
        assert np.all(out["r_all"][k, ~live] == 0.0)
        for s in range(3):
            exact = math.fsum(out["r_all"][k, :, s, 0])
            assert out["totals"][k, s] == pytest.approx(exact, rel=1e-15, abs=1e-300)


def test_node_stats_quantile():
    tot = np.arange(1000, dtype=float)[None, ::-1].copy()
    mean, qv = oracle.node_stats(tot)
    assert qv[0] == 995.0                          # 5th largest of 1,000
    tot = np.arange(500, dtype=float)[None]
    assert oracle.node_stats(tot)[1][0] == 497.0   # 3rd largest of 500
    assert oracle.node_stats(tot)[0][0] == 249.5


def test_oracle_rejects_invalid_input():
    b = basis(gm(1.0), np.full(600, V_FLAT))
    with pytest.raises(ValueError):
        oracle.reserves(b, make_pf([SL_ANN], 700, 601))
    with pytest.raises(ValueError):
        oracle.reserves(b, make_pf([11], 700, 10))
    with pytest.raises(ValueError):
        oracle.reserves(b, make_pf([SL_ANN], N_AGES - 5, 10))


# --------------------------------------------------------------------------
# Complexity shape (Sec. 3.8, Fig. 1): linear vs quadratic in S
# --------------------------------------------------------------------------
def _min_time(fn, reps=7):
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        best = min(best, time.perf_counter() - t)
    return best


def test_complexity_linear_vs_quadratic():
    q = gm(1.0)
    b = basis(q, np.full(1200, V_FLAT))
    S1, S2 = 120, 960
    pf1 = make_pf([SL_ANN] * 2000, 100, S1)
    pf2 = make_pf([SL_ANN] * 2000, 100, S2)
    t1 = _min_time(lambda: oracle.reserves(b, pf1, want_gross=False, n_threads=1))
    t2 = _min_time(lambda: oracle.reserves(b, pf2, want_gross=False, n_threads=1))
    lin = math.log(t2 / t1) / math.log(S2 / S1)
    one1 = make_pf([SL_ANN], 100, S1)
    one2 = make_pf([SL_ANN], 100, S2)
    s1 = _min_time(lambda: oracle.reserve_path_summation(b, one1, 0))
    s2 = _min_time(lambda: oracle.reserve_path_summation(b, one2, 0))
    quad = math.log(s2 / s1) / math.log(S2 / S1)
    assert 0.7 < lin < 1.35, lin
    assert 1.7 < quad < 2.3, quad


def test_node_shock_equals_scaled_table_and_nodes_use_their_own_curves():
    """Node k: ages + 12k, term - 12k, curve v[k], q scaled by m_k (capped)."""
    rng = np.random.default_rng(21)
    q = rng.uniform(0.0, 0.3, 1400)
    v = rng.uniform(0.99, 1.0, (3, 2, 300))
    shock = np.array([1.0, 1.7, 3.5])
    pf = make_pf([SL_ANN, TERM, ENDOW_ASSUR, REV_ANN, LS_ANN], [100, 200, 300, 400, 500],
                 [300, 250, 200, 280, 290], amount=[1200.0, 1e4, 1e4, 600.0, 600.0],
                 premium=[0, 2.0, 9.0, 0, 0], age2=[0, 0, 0, 350, 450])
    full = oracle.reserves(Basis(q=q[None], v=v, shock=shock), pf, node_step=12)
    for k in range(3):
        qk = np.minimum(1.0, shock[k] * q)
        pk = pf.subset(np.arange(pf.n))
        pk.age1_m = pf.age1_m + 12 * k
        pk.age2_m = pf.age2_m + 12 * k
        pk.term_m = pf.term_m - 12 * k
        for s in range(2):
            bk = Basis(q=qk[None], v=v[k:k + 1, s:s + 1, :])
            ref = oracle.reserves(bk, pk)["r_all"][0, :, 0, :]
            np.testing.assert_array_equal(full["r_all"][k, :, s, :], ref)


def test_scenario_window_matches_single_scenario_basis():
    rng = np.random.default_rng(23)
    w = synth.random_small(rng, n=30, n_steps=50, n_scen=5)
    part = oracle.reserves(w.basis, w.portfolio, scen0=2, nscen=2)["r_all"]
    for s in (2, 3):
        b1 = Basis(q=w.basis.q, v=w.basis.v[:, s:s + 1, :])
        one = oracle.reserves(b1, w.portfolio)["r_all"]
        np.testing.assert_array_equal(part[:, :, s - 2, :], one[:, :, 0, :])


# --------------------------------------------------------------------------
# Annuity payment patterns (escalation on anniversaries, annual payment)
# --------------------------------------------------------------------------
def _pattern_pf(product, age1, term, amount, timing, esc, anniv, annual, age2=0):
    pf = make_pf(product, age1, term, amount=amount, timing=timing, age2=age2)
    n = pf.n
    pf.escalation = np.asarray(np.broadcast_to(esc, (n,)), np.float64).copy()
    pf.anniv_m = np.asarray(np.broadcast_to(anniv, (n,)), np.int32).copy()
    pf.annual = np.asarray(np.broadcast_to(annual, (n,)), np.int32).copy()
    return pf


@pytest.mark.parametrize("a", [1, 5, 12])
@pytest.mark.parametrize("S", [1, 11, 12, 13, 300, 599])
def test_escalating_annuities_certain_closed_forms(a, S):
    """Zero mortality: geometric sums over the anniversary years."""
    v, e, theta = V_FLAT, 0.05, 1200.0
    b = basis(np.zeros(N_AGES), np.full(600, v))
    pf = _pattern_pf([SL_ANN] * 4, 700, S, theta, [ARREARS, ADVANCE, ARREARS, ADVANCE],
                     e, a, [0, 0, 1, 1])
    r = r0(b, pf)[:, 0]
    g = 1.0 + e

    def blocks(first, last):
        # sum over months tau in [first, last] of g^(years passed) v^tau, by blocks
        tot = 0.0
        lo = first
        while lo <= last:
            k = 0 if lo < a else 1 + (lo - a) // 12           # anniversaries in (0, lo]
            hi = min(last, a - 1 if lo < a else a + 12 * k - 1)
            m = hi - lo + 1                                    # months at level g^k
            tot += g ** k * v ** lo * (1 - v ** m) / (1 - v)
            lo = hi + 1
        return tot

    monthly_arr = theta / 12 * blocks(1, S)
    monthly_adv = theta / 12 * blocks(0, S - 1)
    x = g * v ** 12
    m_arr = 0 if S < a else (S - a) // 12 + 1                 # anniversaries in [1, S]
    m_adv = 0 if S - 1 < a else (S - 1 - a) // 12 + 1         # anniversaries in [1, S-1]
    annual_arr = theta * g * v ** a * (1 - x ** m_arr) / (1 - x)
    annual_adv = theta * g * v ** a * (1 - x ** m_adv) / (1 - x)
    np.testing.assert_allclose(r, [monthly_arr, monthly_adv, annual_arr, annual_adv],
                               rtol=1e-13, atol=1e-12)


def test_level_patterns_equal_the_plain_annuity_bitwise():
    rng = np.random.default_rng(31)
    w = synth.random_small(rng, n=60, n_steps=90, n_scen=2, n_nodes=2, shock=True)
    pf = w.portfolio
    lv = pf.subset(np.arange(pf.n))
    lv.escalation = np.zeros(pf.n)
    lv.anniv_m = rng.integers(1, 13, pf.n).astype(np.int32)
    lv.annual = np.zeros(pf.n, np.int32)
    a = oracle.reserves(w.basis, pf)["r_all"]
    b = oracle.reserves(w.basis, lv)["r_all"]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("seed", [3, 4])
def test_payment_patterns_recurrence_equals_summation(seed):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=20, n_steps=60, n_scen=2, n_nodes=3, shock=True,
                           products=(SL_ANN, JL_ANN, REV_ANN, LS_ANN))
    b = w.basis
    pf = synth.with_payment_patterns(rng, w.portfolio, 0.6, 0.5)
    for node in range(3):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=7)
        for i in range(pf.n):
            if int(pf.term_m[i]) - 7 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=7)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=0,
                                       atol=1e-12 * scale)


@pytest.mark.parametrize("step", [12, 7])
def test_payment_patterns_node_shift_equals_path(step):
    """The payment factor depends on the time since node 0 only."""
    q = gm(1.0)
    b = Basis(q=np.atleast_2d(q), v=np.full((4, 1, 600), V_FLAT))
    pf = _pattern_pf([SL_ANN, SL_ANN, JL_ANN, SL_ANN], [700, 650, 600, 720], [600, 500, 550, 400],
                     [1200.0, 900.0, 600.0, 300.0], [ARREARS, ADVANCE, ARREARS, ARREARS],
                     [0.05, 0.03, 0.0425, 0.0], [3, 12, 7, 1], [0, 1, 0, 1], age2=[0, 0, 700, 0])
    path, off = oracle.reserve_paths(b, pf, node=0)
    full = oracle.reserves(b, pf, node_step=step)
    for k in range(4):
        for i in range(pf.n):
            assert full["r_all"][k, i, 0, 0] == path[off[i] + step * k]


# --------------------------------------------------------------------------
# Cash-flow tables (one life, c_t = amount x cf[row][t], Sec. 4.6)
# --------------------------------------------------------------------------
def _cf_pf(rows, row_of, age1, term, amount, premium=0.0, table1=0):
    n = np.broadcast(np.asarray(row_of), np.asarray(age1), np.asarray(term), np.asarray(amount),
                     np.asarray(premium)).size
    pf = make_pf([CF_TABLE] * n, age1, term, amount=amount, premium=premium, table1=table1)
    pf.cf = np.atleast_2d(np.asarray(rows, np.float64))
    pf.cf_row = np.asarray(np.broadcast_to(row_of, (pf.n,)), np.int32).copy()
    return pf


@pytest.mark.parametrize("S", [1, 2, 37, 600])
def test_cash_flow_table_closed_form_at_zero_mortality(S):
    rng = np.random.default_rng(S)
    v = rng.uniform(0.995, 1.0, 600)
    b = basis(np.zeros(N_AGES), v)
    rows = rng.uniform(-1.0, 3.0, (2, 600))
    pf = _cf_pf(rows, [0, 1], 700, S, [250.0, 40.0], premium=[3.0, 0.0])
    r = r0(b, pf)[:, 0]
    D = np.concatenate([[1.0], np.cumprod(v[:S])])          # discount to t = 0..S
    want = [a * (rows[k, :S] * D[1:S + 1]).sum() - P * D[:S].sum()
            for k, a, P in ((0, 250.0, 3.0), (1, 40.0, 0.0))]
    np.testing.assert_allclose(r, want, rtol=1e-12, atol=1e-12 * 250)


def test_cash_flow_table_reproduces_level_annuity_and_pure_endowment():
    b = basis(gm(1.0), np.full(600, V_FLAT))
    S, theta = 360, 1200.0
    level = _cf_pf(np.full((1, S), 1.0 / 12.0), 0, 720, S, theta)
    sl = make_pf([SL_ANN], 720, S, amount=theta, timing=ARREARS)
    np.testing.assert_allclose(r0(b, level), r0(b, sl), rtol=1e-14)
    lump = np.zeros((1, S)); lump[0, S - 1] = 1.0
    pe = _cf_pf(lump, 0, 600, S, 5000.0, premium=7.0)
    endow = make_pf([ENDOW], 600, S, amount=5000.0, premium=7.0)
    np.testing.assert_allclose(r0(b, pe), r0(b, endow), rtol=1e-13)


def test_cash_flow_table_is_linear_in_the_table():
    rng = np.random.default_rng(12)
    w = synth.random_small(rng, n=1, n_steps=200, n_scen=2)
    rows = rng.uniform(-1.0, 2.0, (2, 200))
    rows = np.vstack([rows, rows[0] + rows[1]])
    pf = _cf_pf(rows, [0, 1, 2], [300, 300, 300], 200, 100.0)
    r = oracle.reserves(w.basis, pf)["r_all"][0, :, :, 0]
    np.testing.assert_allclose(r[0] + r[1], r[2], rtol=1e-12, atol=1e-12 * np.abs(r).max())


@pytest.mark.parametrize("seed", [5, 6])
def test_cash_flow_tables_recurrence_equals_summation(seed):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=16, n_steps=50, n_scen=2, n_nodes=3, shock=True)
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.6)
    b = w.basis
    assert (pf.product == CF_TABLE).sum() >= 5
    for node in range(3):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=7)
        for i in np.flatnonzero(pf.product == CF_TABLE):
            if int(pf.term_m[i]) - 7 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=7)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=0,
                                       atol=1e-12 * scale)


@pytest.mark.parametrize("step", [12, 5])
def test_cash_flow_table_node_shift_equals_path(step):
    """The table is indexed by time since node 0."""
    rng = np.random.default_rng(step)
    b = Basis(q=np.atleast_2d(gm(1.0)), v=np.full((4, 1, 600), V_FLAT))
    rows = rng.uniform(0.0, 2.0, (3, 600))
    pf = _cf_pf(rows, [0, 1, 2], [700, 650, 600], [600, 500, 550], [1200.0, 900.0, 600.0],
                premium=[0.0, 2.0, 1.0])
    path, off = oracle.reserve_paths(b, pf, node=0)
    full = oracle.reserves(b, pf, node_step=step)
    for k in range(4):
        for i in range(pf.n):
            assert full["r_all"][k, i, 0, 0] == path[off[i] + step * k]


# --------------------------------------------------------------------------
# Two-life endowment and assurances (Sec. 4.2.2, 4.2.3; 9-state Kronecker W)
# --------------------------------------------------------------------------
def _two(product, q2, premium=0.0, S=240, amount=1000.0, age1=700, age2=650, v=None):
    """Life 1 on GM, life 2 on table 1 = q2 (scalar or table)."""
    q = np.vstack([gm(1.0), np.broadcast_to(np.asarray(q2, float), (N_AGES,))])
    b = basis(q, np.full(600, V_FLAT) if v is None else v)
    pf = make_pf([product], age1, S, amount=amount, premium=premium, age2=age2, table1=0, table2=1)
    return b, pf


def test_two_life_reduce_to_single_life_when_life_two_never_dies():
    for two, one in ((JL_ENDOW, ENDOW), (JL_ASSUR1, TERM)):
        b, pf2 = _two(two, 0.0, premium=3.0)
        pf1 = make_pf([one], 700, 240, amount=1000.0, premium=3.0)
        np.testing.assert_allclose(r0(b, pf2)[:, 0], r0(b, pf1)[:, 0], rtol=1e-13)


def test_second_death_assurance_is_single_life_when_life_two_dies_at_once():
    b, pf2 = _two(JL_ASSUR2, 1.0)
    pf1 = make_pf([TERM], 700, 240, amount=1000.0)
    np.testing.assert_allclose(r0(b, pf2)[:, 0], r0(b, pf1)[:, 0], rtol=1e-13)


@pytest.mark.parametrize("seed", [1, 2])
def test_first_plus_second_death_equals_two_single_life_assurances(seed):
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.0, 0.05, (2, N_AGES))
    v = rng.uniform(0.99, 1.0, (3, 300))
    b = Basis(q=q, v=v[None])
    mk = lambda prod, a1, t1: make_pf([prod], a1, 300, amount=500.0, age2=620, table1=t1, table2=1)
    first = oracle.reserves(b, mk(JL_ASSUR1, 710, 0))["r_all"][0, 0, :, 0]
    second = oracle.reserves(b, mk(JL_ASSUR2, 710, 0))["r_all"][0, 0, :, 0]
    tx = oracle.reserves(b, make_pf([TERM], 710, 300, amount=500.0, table1=0))["r_all"][0, 0, :, 0]
    ty = oracle.reserves(b, make_pf([TERM], 620, 300, amount=500.0, table1=1))["r_all"][0, 0, :, 0]
    np.testing.assert_allclose(first + second, tx + ty, rtol=1e-12)


def test_second_death_states_are_the_single_life_assurances():
    """The reserve with one life already dead is the other life's assurance."""
    rng = np.random.default_rng(3)
    q = rng.uniform(0.0, 0.05, (2, N_AGES))
    b = basis(q, rng.uniform(0.99, 1.0, 300))
    pf = make_pf([JL_ASSUR2], 710, 300, amount=500.0, age2=620, table1=0, table2=1)
    r = oracle.reserves(b, pf)["r_all"][0, 0, 0]
    tx = r0(b, make_pf([TERM], 710, 300, amount=500.0, table1=0))[0, 0]
    ty = r0(b, make_pf([TERM], 620, 300, amount=500.0, table1=1))[0, 0]
    np.testing.assert_allclose([r[1], r[2], r[3]], [tx, ty, 0.0], rtol=1e-13, atol=1e-12)


def test_joint_endowment_brute_force():
    rng = np.random.default_rng(4)
    q = rng.uniform(0.0, 0.05, (2, N_AGES))
    v = rng.uniform(0.99, 1.0, 300)
    b = basis(q, v)
    S = 180
    pf = make_pf([JL_ENDOW], 700, S, amount=800.0, age2=640, table1=0, table2=1)
    want = 800.0 * np.prod(v[:S]) * np.prod(1 - q[0, 700:700 + S]) * np.prod(1 - q[1, 640:640 + S])
    np.testing.assert_allclose(r0(b, pf)[0, 0], want, rtol=1e-13)


@pytest.mark.parametrize("product", [JL_ENDOW, JL_ASSUR1, JL_ASSUR2])
def test_two_life_insurance_recurrence_equals_summation(product):
    rng = np.random.default_rng(product)
    w = synth.random_small(rng, n=6, n_steps=40, n_scen=2, n_nodes=2, shock=True,
                           products=(product,))
    b, pf = w.basis, w.portfolio
    for node in range(2):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=5)
        for i in range(pf.n):
            if int(pf.term_m[i]) - 5 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=5)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=0,
                                       atol=1e-12 * scale)


def test_scenario_average_is_the_reserve_on_the_mean_discount_curve():
    """Eq. (3.5) is linear in the discount products D_t = v_0 ... v_{t-1}
    (mortality does not depend on the interest path): the reserve averaged
    over scenarios equals the reserve on the curve whose products are the
    scenario means of D_t."""
    rng = np.random.default_rng(21)
    w = synth.random_small(rng, n=40, n_steps=120, n_scen=25, n_nodes=2, shock=True,
                           products=tuple(range(7)) + (JL_ENDOW, JL_ASSUR1, JL_ASSUR2))
    b, pf = w.basis, w.portfolio
    ref = oracle.reserves(b, pf, 0, 2, 0, 25, 12)
    D = np.cumprod(b.v, axis=2)                                   # D_{t+1}
    Dbar = D.mean(axis=1)                                         # [node][t]
    vbar = Dbar / np.concatenate([np.ones((2, 1)), Dbar[:, :-1]], axis=1)
    mb = synth.Basis(q=b.q, v=vbar[:, None, :], shock=b.shock)
    mean_ref = oracle.reserves(mb, pf, 0, 2, 0, 1, 12)
    avg = ref["r_all"][..., 0].mean(axis=2)
    scale = np.maximum(np.abs(avg), ref["gross"].mean(axis=2))
    assert np.all(np.abs(mean_ref["r_all"][:, :, 0, 0] - avg) <= 1e-12 * scale + 1e-300)


# --------------------------------------------------------------------------
# Uploaded Markov models (Sec. 4.5: reversible, not upper-triangular W)
# --------------------------------------------------------------------------
def _mk_pf(models, model, age1, term, amount, premium=0.0):
    n = np.broadcast(np.asarray(model), np.asarray(age1), np.asarray(term), np.asarray(amount),
                     np.asarray(premium)).size
    pf = make_pf([MARKOV] * n, age1, term, amount=amount, premium=premium, table1=model)
    pf.markov = models
    return pf


def test_two_state_model_reproduces_the_single_life_annuity():
    q = gm(1.0)
    w = np.zeros((1, N_AGES, 2, 2))
    w[0, :, 0, 0], w[0, :, 0, 1], w[0, :, 1, 1] = 1 - q, q, 1.0
    c = np.array([[1.0 / 12.0, 0.0]])
    b = basis(q, np.full(600, V_FLAT))
    mk = _mk_pf((w, c), 0, 700, 360, 1200.0)
    sl = make_pf([SL_ANN], 700, 360, amount=1200.0, timing=ARREARS)
    np.testing.assert_allclose(r0(b, mk)[:, 0], r0(b, sl)[:, 0], rtol=1e-14)


@pytest.mark.parametrize("S", [1, 12, 240])
def test_reversible_model_closed_form(S):
    """Constant non-triangular W: r = amount sum_t v^t e0' W^t c minus the
    premium annuity sum_t v^t P(state 0 at t), by matrix powers."""
    W = np.array([[0.95, 0.04, 0.01], [0.10, 0.85, 0.05], [0.0, 0.0, 1.0]])
    c = np.array([0.0, 1.0 / 12.0, 0.0])
    w = np.broadcast_to(W, (1, N_AGES, 3, 3)).copy()
    b = basis(gm(1.0), np.full(600, V_FLAT))
    pf = _mk_pf((w, c[None]), 0, 500, S, 6000.0, premium=20.0)
    r = oracle.reserves(b, pf)["r_all"][0, 0, 0]
    e0 = np.array([1.0, 0.0, 0.0])
    ben = sum(V_FLAT ** t * e0 @ np.linalg.matrix_power(W, t) @ c for t in range(1, S + 1))
    prem = sum(V_FLAT ** t * (e0 @ np.linalg.matrix_power(W, t))[0] for t in range(S))
    np.testing.assert_allclose(r[0], 6000.0 * ben - 20.0 * prem, rtol=1e-12)
    # the sick state's reserve: the same sums from state 1, without premiums
    e1 = np.array([0.0, 1.0, 0.0])
    prem1 = sum(V_FLAT ** t * (e1 @ np.linalg.matrix_power(W, t))[0] for t in range(S))
    ben1 = sum(V_FLAT ** t * e1 @ np.linalg.matrix_power(W, t) @ c for t in range(1, S + 1))
    np.testing.assert_allclose(r[1], 6000.0 * ben1 - 20.0 * prem1, rtol=1e-12)


@pytest.mark.parametrize("seed", [8, 9])
def test_markov_recurrence_equals_summation(seed):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=10, n_steps=40, n_scen=2, n_nodes=2, shock=True)
    n_ages = w.basis.q.shape[1]
    raw = rng.uniform(0.0, 1.0, (2, n_ages, 4, 4))
    raw[:, :, 3, :] = [0, 0, 0, 1]                   # an absorbing state
    W = raw / raw.sum(axis=3, keepdims=True)
    c = rng.uniform(-1.0, 2.0, (2, 4))
    pf = synth.with_markov_policies(rng, w.portfolio, (W, c), frac=1.0)
    b = w.basis
    for node in range(2):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=5)
        for i in range(pf.n):
            if int(pf.term_m[i]) - 5 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=5)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=0,
                                       atol=1e-12 * scale)


def test_markov_node_shift_equals_path():
    w, c = synth.phi_models(N_AGES)
    b = Basis(q=np.atleast_2d(gm(1.0)), v=np.full((4, 1, 600), V_FLAT))
    pf = _mk_pf((w, c), [0, 1, 0], [600, 650, 700], [500, 400, 300], [1200.0, 900.0, 600.0],
                premium=[3.0, 0.0, 1.0])
    path, off = oracle.reserve_paths(b, pf, node=0)
    full = oracle.reserves(b, pf, node_step=12)
    for k in range(4):
        for i in range(pf.n):
            assert full["r_all"][k, i, 0, 0] == path[off[i] + 12 * k]


# --------------------------------------------------------------------------
# Fractional payment timing (Sec. 3.1's f in (0, 1); uniform deaths)
# --------------------------------------------------------------------------
def _frac_basis(q, v, f):
    b = basis(q, v)
    b.frac = f
    return b


@pytest.mark.parametrize("f", [0.25, 0.5, 0.9])
def test_fractional_annuity_certain(f):
    b = _frac_basis(np.zeros(N_AGES), np.full(600, V_FLAT), f)
    S = 240
    pf = make_pf([SL_ANN], 700, S, amount=1200.0, timing=FRACTIONAL)
    want = 100.0 * V_FLAT ** f * (1 - V_FLAT ** S) / (1 - V_FLAT)
    np.testing.assert_allclose(r0(b, pf)[0, 0], want, rtol=1e-13)


@pytest.mark.parametrize("f", [0.3, 0.7])
def test_fractional_timing_interpolates_without_discounting(f):
    """v = 1: survival to t + f is (1 - f) + f p, so the single-life value is
    (1 - f) x (advance) + f x (arrears); the joint-life value is the sum of
    the joint survival to t times (1 - f qx)(1 - f qy)."""
    q = np.vstack([gm(1.0), gm(1.3)])
    b = _frac_basis(q, np.ones(600), f)
    S = 300
    sl = [make_pf([SL_ANN], 700, S, amount=1200.0, timing=t) for t in (FRACTIONAL, ADVANCE, ARREARS)]
    r = [r0(b, p)[0, 0] for p in sl]
    np.testing.assert_allclose(r[0], (1 - f) * r[1] + f * r[2], rtol=1e-13)
    jl = make_pf([JL_ANN], 700, S, amount=1200.0, timing=FRACTIONAL, age2=650, table1=0, table2=1)
    qx, qy = q[0, 700:700 + S], q[1, 650:650 + S]
    surv = np.concatenate([[1.0], np.cumprod((1 - qx) * (1 - qy))[:-1]])
    want = 100.0 * math.fsum(surv * (1 - f * qx) * (1 - f * qy))
    np.testing.assert_allclose(r0(b, jl)[0, 0], want, rtol=1e-13)


@pytest.mark.parametrize("seed", [11, 12])
def test_fractional_recurrence_equals_summation(seed):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=16, n_steps=50, n_scen=2, n_nodes=2, shock=True,
                           products=(SL_ANN, JL_ANN, REV_ANN, LS_ANN))
    b, pf = w.basis, w.portfolio
    b.frac = 0.4
    pf.timing[:] = FRACTIONAL
    for node in range(2):
        path, off = oracle.reserve_paths(b, pf, node=node, scen=1, node_step=5)
        for i in range(pf.n):
            if int(pf.term_m[i]) - 5 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1, node_step=5)
            scale = np.abs(summ).max() + 1e-300
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=0,
                                       atol=1e-12 * scale)


# --------------------------------------------------------------------------
# The gross value G (the scale of every parity tolerance)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("S", [1, 13, 240])
def test_gross_closed_forms_at_zero_mortality(S):
    """q = 0: a premium-paying pure endowment or endowment assurance has
    G = SA v^S + P a-due_S and a term assurance G = P a-due_S, with
    a-due_S = (1 - v^S) / (1 - v) the annuity-certain due."""
    v = 0.997
    SA, P = 1000.0, 3.0
    pf = make_pf([ENDOW, ENDOW_ASSUR, TERM, JL_ENDOW, JL_ASSUR1, JL_ASSUR2], 300, S,
                 amount=SA, premium=P, age2=400)
    b = basis(np.zeros(N_AGES), np.full(S, v))
    g = oracle.reserves(b, pf)["gross"][0, :, 0]
    due = (1.0 - v ** S) / (1.0 - v)
    expect = [SA * v ** S + P * due, SA * v ** S + P * due, P * due, SA * v ** S + P * due,
              P * due, P * due]
    np.testing.assert_allclose(g, expect, rtol=1e-13)


def test_gross_is_reserve_plus_twice_the_premium_value():
    """For every product G = PV(benefits) + PV(premiums) while the reserve is
    PV(benefits) - PV(premiums), and -PV(premiums) is the reserve of the same
    policy with amount 0: G = r - 2 r(amount 0), random mortality and
    curves, non-negative cash-flow tables and Markov benefits."""
    rng = np.random.default_rng(31)
    w = synth.random_small(rng, n=400, n_steps=60, n_scen=3, n_nodes=2, shock=True,
                           products=tuple(range(7)) + (JL_ENDOW, JL_ASSUR1, JL_ASSUR2))
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.1, n_rows=3)
    pf.cf = np.abs(pf.cf)
    W, c = synth.phi_models(w.basis.q.shape[1])
    pf = synth.with_markov_policies(rng, pf, (W, c), frac=0.1)
    assert set(np.unique(pf.product)) == set(range(12))
    full = oracle.reserves(w.basis, pf, node_step=7)
    zero = pf.subset(np.arange(pf.n))
    zero.amount = np.zeros(pf.n)
    prem = oracle.reserves(w.basis, zero, node_step=7, want_gross=False)["r_all"][..., 0]
    expect = full["r_all"][..., 0] - 2.0 * prem
    scale = np.maximum(full["gross"], 1e-300)
    assert np.max(np.abs(full["gross"] - expect) / scale) < 1e-12


# --------------------------------------------------------------------------
# The reduced mode (zero-reserve states removed) against the dense mode
# --------------------------------------------------------------------------
def reduced_vs_dense(w, node_step):
    b, pf = w.basis, w.portfolio
    dense = oracle.reserves(b, pf, node_step=node_step)
    red = oracle.reserves_reduced(b, pf, node_step=node_step)
    scale = np.maximum(np.abs(dense["r_all"]), dense["gross"][..., None])
    err = np.abs(red["r_all"] - dense["r_all"]) / np.maximum(scale, 1e-300)
    assert err.max() <= 1e-13, (err.max(), np.unravel_index(np.argmax(err), err.shape))
    terr = np.abs(red["totals"] - dense["totals"]) / np.maximum(dense["gross_totals"], 1e-300)
    assert terr.max() <= 1e-13


@pytest.mark.parametrize("product", list(range(11)))
def test_reduced_mode_equals_dense_each_product(product):
    rng = np.random.default_rng(800 + product)
    w = synth.random_small(rng, n=80, n_steps=150, n_scen=3, n_nodes=2, shock=True,
                           products=(product,))
    if product == CF_TABLE:
        pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=1.0, n_rows=5)
        w = synth.Workload("cf", w.basis, pf)
    reduced_vs_dense(w, 12)


def test_reduced_mode_equals_dense_everything_together():
    """Every product with payment patterns, cash-flow tables, Markov models
    (permanent health and random 4-state), advance, arrears and fractional
    timing, three nodes 7 months apart with shocks."""
    rng = np.random.default_rng(830)
    w = synth.random_small(rng, n=600, n_steps=90, n_scen=4, n_nodes=3, shock=True,
                           products=tuple(range(7)) + (JL_ENDOW, JL_ASSUR1, JL_ASSUR2))
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.1, n_rows=4)
    pf = synth.with_payment_patterns(rng, pf, 0.4, 0.3)
    ann = np.isin(pf.product, (SL_ANN, JL_ANN, REV_ANN, LS_ANN))
    pf.timing = np.where(ann & (rng.uniform(size=pf.n) < 0.3), FRACTIONAL, pf.timing).astype(np.int32)
    n_ages = w.basis.q.shape[1]
    raw = rng.uniform(0.0, 1.0, (2, n_ages, 4, 4))
    raw[:, :, 3, :] = [0.0, 0.0, 0.0, 1.0]
    W = raw / raw.sum(axis=3, keepdims=True)
    pf = synth.with_markov_policies(rng, pf, (W, rng.uniform(-1.0, 2.0, (2, 4))), frac=0.1)
    w.basis.frac = 0.4
    w = synth.Workload("all", w.basis, pf)
    assert set(np.unique(pf.product)) == set(range(12))
    reduced_vs_dense(w, 7)


def test_reduced_mode_on_the_nested_workload_sample():
    """The benchmark's CPU workload (mixed products, Vasicek curves): a
    sample of policies and scenarios, reduced = dense."""
    w = synth.config_c3(n=300, n_scen=6)
    reduced_vs_dense(w, 12)


# --------------------------------------------------------------------------
# Three lives (Sec. 4.3: Kronecker W of 2^3 states)
# --------------------------------------------------------------------------
from synth import JL3_ANN, LS3_ANN  # noqa: E402


def make_pf3(product, ages, term, amount=12.0, premium=0.0, timing=ARREARS, tables=(0, 0, 0)):
    pf = make_pf(product, ages[0], term, amount=amount, premium=premium, timing=timing,
                 age2=ages[1], table1=tables[0], table2=tables[1])
    n = pf.n
    pf.age3_m = np.full(n, ages[2], np.int32)
    pf.table3 = np.full(n, tables[2], np.int32)
    return pf


@pytest.mark.parametrize("timing", [ADVANCE, ARREARS])
def test_three_lives_reduce_to_two_when_life_three_never_dies(timing):
    """q3 = 0: the three-life joint-life annuity is the two-life one exactly,
    and the last-survivor annuity the annuity certain (1 - v^n)/i."""
    q = np.stack([gm(), gm(1.3), np.zeros(N_AGES)])
    S = 240
    b = basis(q, np.full(S, V_FLAT))
    j3 = make_pf3([JL3_ANN, LS3_ANN], (700, 760, 500), S, timing=timing, tables=(0, 1, 2))
    j2 = make_pf([JL_ANN], 700, S, timing=timing, age2=760, table1=0, table2=1)
    r3 = r0(b, j3)
    assert r3[0, 0] == pytest.approx(r0(b, j2)[0, 0], rel=1e-14)
    i = 1.0 / V_FLAT - 1.0
    cert = (1.0 - V_FLAT ** S) / i * (1.0 / V_FLAT if timing == ADVANCE else 1.0)
    assert r3[1, 0] == pytest.approx(cert, rel=1e-13)


def test_three_lives_with_life_three_dead_at_once():
    """q3 = 1: an arrears joint-life annuity on three lives pays nothing and
    the last-survivor annuity is the two-life last-survivor annuity."""
    q = np.stack([gm(), gm(0.8), np.ones(N_AGES)])
    S = 180
    b = basis(q, np.full(S, V_FLAT))
    r3 = r0(b, make_pf3([JL3_ANN, LS3_ANN], (650, 700, 400), S, tables=(0, 1, 2)))
    ls2 = r0(b, make_pf([LS_ANN], 650, S, age2=700, table1=0, table2=1))
    assert r3[0, 0] == 0.0
    assert r3[1, 0] == pytest.approx(ls2[0, 0], rel=1e-13)


def test_three_lives_inclusion_exclusion():
    """Last survivor of three = sum of single-life annuities - sum of the
    pairs' joint-life annuities + the three-life joint-life annuity (the
    indicator that some life is alive, expanded); random mortality, random
    curve, both timings."""
    rng = np.random.default_rng(41)
    q = rng.uniform(0.0, 0.05, (3, 1200))
    S = 150
    v = rng.uniform(0.99, 1.0, S)
    b = basis(q, v)
    ages = (300, 420, 555)
    for timing in (ADVANCE, ARREARS):
        ls3 = r0(b, make_pf3([LS3_ANN], ages, S, timing=timing, tables=(0, 1, 2)))[0, 0]
        jl3 = r0(b, make_pf3([JL3_ANN], ages, S, timing=timing, tables=(0, 1, 2)))[0, 0]
        single = sum(r0(b, make_pf([SL_ANN], ages[l], S, timing=timing, table1=l))[0, 0] for l in range(3))
        pairs = sum(r0(b, make_pf([JL_ANN], ages[a], S, timing=timing, age2=ages[c], table1=a,
                                   table2=c))[0, 0] for a, c in ((0, 1), (0, 2), (1, 2)))
        assert ls3 == pytest.approx(single - pairs + jl3, rel=1e-12)


def test_three_lives_symmetric_and_states():
    """The reserves in the all-alive state do not depend on how the lives are
    numbered; the last-survivor reserve with life 3 dead (slot 1) is the
    two-life last-survivor reserve of lives 1 and 2 and with only life 1
    alive (slot 3) the single-life annuity."""
    q = np.stack([gm(), gm(0.7), gm(1.2)])
    S = 200
    b = basis(q, np.full(S, V_FLAT))
    base = r0(b, make_pf3([JL3_ANN, LS3_ANN], (600, 680, 720), S, premium=1.5, tables=(0, 1, 2)))
    perm = r0(b, make_pf3([JL3_ANN, LS3_ANN], (720, 600, 680), S, premium=1.5, tables=(2, 0, 1)))
    np.testing.assert_allclose(perm[:, 0], base[:, 0], rtol=1e-13)
    ls2 = r0(b, make_pf([LS_ANN], 600, S, age2=680, table1=0, table2=1))[0, 0]
    sl1 = r0(b, make_pf([SL_ANN], 600, S, table1=0))[0, 0]
    assert base[1, 1] == pytest.approx(ls2, rel=1e-13)
    assert base[1, 3] == pytest.approx(sl1, rel=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_three_lives_recurrence_equals_summation(seed):
    rng = np.random.default_rng(60 + seed)
    w = synth.random_small(rng, n=12, n_steps=40, n_scen=2, n_nodes=2, shock=True,
                           products=(JL3_ANN, LS3_ANN))
    w.basis.frac = 0.3
    w.portfolio.timing = rng.integers(0, 3, w.portfolio.n).astype(np.int32)
    b, pf = w.basis, w.portfolio
    for i in range(pf.n):
        for node in (0, 1):
            if pf.term_m[i] - 12 * node <= 0:
                continue
            summ = oracle.reserve_path_summation(b, pf, i, node=node, scen=1)
            path, off = oracle.reserve_paths(b, pf, node=node, scen=1)
            np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=1e-12, atol=1e-12)


def test_reduced_mode_three_lives():
    rng = np.random.default_rng(870)
    w = synth.random_small(rng, n=200, n_steps=120, n_scen=3, n_nodes=2, shock=True,
                           products=(JL3_ANN, LS3_ANN, SL_ANN, LS_ANN))
    w.basis.frac = 0.45
    pf = w.portfolio
    pf.timing = rng.integers(0, 3, pf.n).astype(np.int32)
    pf.premium = np.where(rng.uniform(size=pf.n) < 0.5, pf.premium, 0.0)
    reduced_vs_dense(synth.Workload("three", w.basis, pf), 12)


# --------------------------------------------------------------------------
# Uploaded models of up to nine states
# --------------------------------------------------------------------------
def two_life_assurance_tables(q, gap, model):
    """The 9-state two-life assurance model of Sec. 4.2.3 as an uploaded
    table by the attained age x of life 1, life 2 being x + gap."""
    n_ages = q.shape[1] - gap
    W = np.zeros((1, n_ages, 9, 9))
    for x in range(n_ages):
        W[0, x] = oracle.build_w(2, 3, [q[0, x], q[1, x + gap]])
    c = {JL_ASSUR1: [0, 1, 0, 1, 1, 0, 0, 0, 0], JL_ASSUR2: [0, 0, 0, 0, 1, 1, 0, 1, 0]}[model]
    return W, np.asarray([c], np.float64)


@pytest.mark.parametrize("model", [JL_ASSUR1, JL_ASSUR2])
def test_nine_state_upload_reproduces_two_life_assurances(model):
    """The paper's 9-state matrix uploaded as a table (life 2 a fixed 60
    months older) gives the built-in first- and second-death assurances."""
    rng = np.random.default_rng(880 + model)
    q = np.stack([gm(), gm(1.4)])
    S, gap = 300, 60
    W, c = two_life_assurance_tables(q, gap, model)
    b = basis(q, rng.uniform(0.995, 1.0, S))
    ages = rng.integers(300, 1000, 20)
    prem = rng.uniform(0.0, 40.0, 20)
    built = make_pf([model] * 20, ages, S, amount=1e4, premium=prem, age2=ages + gap, table1=0, table2=1)
    up = make_pf([MARKOV] * 20, ages, S, amount=1e4, premium=prem, table1=0)
    up.markov = (W, c)
    rb = oracle.reserves(b, built)
    ru = oracle.reserves(b, up)
    np.testing.assert_allclose(ru["r_all"][..., 0], rb["r_all"][..., 0], rtol=1e-13,
                               atol=1e-13 * float(rb["gross"].max()))
    red = oracle.reserves_reduced(b, up)
    np.testing.assert_allclose(red["r_all"][..., 0], ru["r_all"][..., 0], rtol=1e-13,
                               atol=1e-13 * float(rb["gross"].max()))


@pytest.mark.parametrize("m", [5, 9])
def test_large_markov_recurrence_equals_summation(m):
    rng = np.random.default_rng(890 + m)
    n_ages = 400
    raw = rng.uniform(0.0, 1.0, (2, n_ages, m, m))
    raw[:, :, m - 1, :] = 0.0
    raw[:, :, m - 1, m - 1] = 1.0
    W = raw / raw.sum(axis=3, keepdims=True)
    c = rng.uniform(-1.0, 2.0, (2, m))
    pf = make_pf([MARKOV] * 6, rng.integers(0, 300, 6), rng.integers(20, 90, 6), amount=100.0,
                 premium=rng.uniform(0, 2, 6), table1=rng.integers(0, 2, 6))
    pf.markov = (W, c)
    b = basis(np.zeros((1, n_ages)), rng.uniform(0.99, 1.0, (1, 2, 90)))
    for i in range(pf.n):
        summ = oracle.reserve_path_summation(b, pf, i, scen=1)
        path, off = oracle.reserve_paths(b, pf, scen=1)
        np.testing.assert_allclose(path[off[i]:off[i + 1]], summ[:, 0], rtol=1e-12, atol=1e-12)
    dense = oracle.reserves(b, pf)
    red = oracle.reserves_reduced(b, pf)
    np.testing.assert_allclose(red["r_all"], dense["r_all"], rtol=1e-13, atol=1e-11)


def test_reduced_mode_absolute_totals():
    rng = np.random.default_rng(900)
    w = synth.random_small(rng, n=150, n_steps=60, n_scen=3, n_nodes=2, shock=True)
    red = oracle.reserves_reduced(w.basis, w.portfolio, node_step=12)
    r = red["r_all"][..., 0]
    np.testing.assert_allclose(red["abs_totals"], np.abs(r).sum(axis=1), rtol=1e-14)
    np.testing.assert_allclose(red["totals"], r.sum(axis=1), rtol=1e-12, atol=1e-9)
