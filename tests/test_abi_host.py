"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/rr.h declares, and its input checks reject bad data
with a message naming the first bad value."""
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rr():
    import paper_1401_1757_amd as rr
    if not os.path.exists(rr.LIB_PATH):
        from paper_1401_1757_amd import build
        build.build()
    rr.load_library()
    return rr


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rr_\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(rr):
    names = declared_functions()
    assert len(names) >= 18
    lib = rr.load_library()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(rr.EXPORTS) == names


def test_create_without_gpu_fails_cleanly(rr):
    import ctypes
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert rr.load_library().rr_create(ctypes.byref(h), 0, 0) == rr.RR_EDEVICE


def test_portfolio_checks(rr):
    w = synth.config_c2(n=2000)
    n_ages = w.basis.q.shape[1]
    assert rr.check_portfolio(w.portfolio, 600, n_ages, 3) == ""
    cases = {
        "term": ("term_m", 7, 601, "policy 7 term 601"),
        "term0": ("term_m", 3, 0, "policy 3 term 0"),
        "product": ("product", 11, 14, "policy 11 has unknown product 14"),
        "three": ("product", 12, synth.LS3_ANN, "three-life products need age3_m and table3"),
        "age": ("age1_m", 5, n_ages, "policy 5 age"),
        "table": ("table1", 2, 3, "policy 2 table1 3"),
        "timing": ("timing", 9, 3, "policy 9 timing 3"),
        "amount": ("amount", 4, -1.0, "policy 4 amount"),
        "nan": ("premium", 6, float("nan"), "policy 6 premium"),
    }
    for name, (field, i, val, msg) in cases.items():
        pf = w.portfolio.subset(np.arange(20))
        getattr(pf, field)[i] = val
        got = rr.check_portfolio(pf, 600, n_ages, 3)
        assert msg in got, (name, got)
    two = w.portfolio.subset(np.arange(20))
    two.product[1] = synth.LS_ANN
    two.age2_m[1] = n_ages - 5
    assert "second age" in rr.check_portfolio(two, 600, n_ages, 3)
    three = w.portfolio.subset(np.arange(20))
    three.product[2] = synth.JL3_ANN
    three.age3_m = np.zeros(20, np.int32)
    three.table3 = np.zeros(20, np.int32)
    assert rr.check_portfolio(three, 600, n_ages, 3) == ""
    three.age3_m[2] = n_ages - 5
    assert "policy 2 third age" in rr.check_portfolio(three, 600, n_ages, 3)
    three.age3_m[2] = 0
    three.table3[2] = 3
    assert "policy 2 table3 3" in rr.check_portfolio(three, 600, n_ages, 3)


def test_basis_checks(rr):
    q = synth.gm_monthly_q(200)[None]
    v = np.full((1, 2, 50), 0.99)
    assert rr.check_basis(q, v) == ""
    q2 = q.copy(); q2[0, 17] = 1.5
    assert "q[17]" in rr.check_basis(q2, v)
    v2 = v.copy(); v2[0, 1, 3] = 0.0
    assert "v[53]" in rr.check_basis(q, v2)
    v3 = v.copy(); v3[0, 0, 0] = np.inf
    assert "v[0]" in rr.check_basis(q, v3)
    assert "shock[0]" in rr.check_basis(q, v, shock=np.array([-1.0]))


def test_payment_pattern_checks(rr):
    """Patterns only on annuities in payment; rates, anniversaries and the
    annual flag in range."""
    w = synth.config_c2(n=2000)
    n_ages = w.basis.q.shape[1]
    base = w.portfolio.subset(np.arange(40))
    ann = np.flatnonzero(np.isin(base.product, (synth.SL_ANN, synth.JL_ANN)))
    ins = np.flatnonzero(np.isin(base.product, (synth.TERM, synth.ENDOW)))
    assert ann.size and ins.size

    def patterned(esc=0.0, anniv=3, annual=0):
        pf = base.subset(np.arange(base.n))
        pf.escalation = np.zeros(pf.n)
        pf.anniv_m = np.full(pf.n, 12, np.int32)
        pf.annual = np.zeros(pf.n, np.int32)
        return pf

    ok = patterned()
    ok.escalation[ann] = 0.05
    ok.annual[ann[::2]] = 1
    ok.anniv_m[:] = np.arange(ok.n) % 12 + 1
    assert rr.check_portfolio(ok, 600, n_ages, 3) == ""
    i, k = int(ann[0]), int(ins[0])
    cases = [
        ("escalation", i, -0.01, f"policy {i} escalation"),
        ("escalation", i, float("nan"), f"policy {i} escalation"),
        ("escalation", i, 1.5, f"policy {i} escalation"),
        ("anniv_m", i, 0, f"policy {i} anniv_m 0"),
        ("anniv_m", k, 13, f"policy {k} anniv_m 13"),
        ("annual", i, 2, f"policy {i} annual 2"),
        ("escalation", k, 0.03, f"policy {k} has a payment pattern but product"),
        ("annual", k, 1, f"policy {k} has a payment pattern but product"),
    ]
    for field, j, val, msg in cases:
        pf = patterned()
        getattr(pf, field)[j] = val
        got = rr.check_portfolio(pf, 600, n_ages, 3)
        assert msg in got, (field, j, val, got)
    pf = patterned()
    pf.escalation[i] = 0.03
    pf.premium[i] = 1.0
    assert f"policy {i} has a payment pattern and premium" in rr.check_portfolio(pf, 600, n_ages, 3)
    # a level annuity may keep a premium whatever its anniversary
    pf = patterned()
    pf.premium[i] = 1.0
    pf.anniv_m[i] = 1
    assert rr.check_portfolio(pf, 600, n_ages, 3) == ""


def test_representative_portfolio_law():
    """The Sec. 5.3 recipe: composition, ages, sexes, frequencies, amounts,
    escalation, anniversaries and terms to the limiting age."""
    rng = np.random.default_rng(7)
    pf = synth.portfolio_representative(rng, 500_000)
    assert np.bincount(pf.product, minlength=4).tolist() == [300_000, 50_000, 100_000, 50_000]
    assert pf.age1_m.min() >= 57 * 12 and pf.age1_m.max() <= 67 * 12
    two = np.isin(pf.product, synth.TWO_LIFE)
    assert pf.age2_m[two].min() >= 57 * 12 and pf.age2_m[two].max() <= 67 * 12
    assert abs((pf.table1 == synth.TABLE_MALE).mean() - 0.75) < 0.005
    assert np.all(pf.table2[two] != pf.table1[two])
    assert abs(pf.annual.mean() - 0.20) < 0.005
    pay = np.where(pf.annual == 1, pf.amount, pf.amount / 12.0)
    assert abs(pay.mean() - 5.0) < 0.02 and abs(pay.std() - 1.5) < 0.02
    assert abs((pf.escalation > 0).mean() - 0.05) < 0.002
    assert set(np.unique(pf.escalation)) == {0.0, 0.03, 0.0425, 0.05}
    assert set(np.unique(pf.anniv_m)) == set(range(1, 13))
    youngest = np.where(two, np.minimum(pf.age1_m, pf.age2_m), pf.age1_m)
    assert np.all(pf.term_m == synth.LIMIT_AGE_M - youngest)
    assert abs(pf.term_m.mean() / 12 - 58) < 1.5     # the paper's average outstanding term
    assert np.all(pf.premium == 0) and np.all(pf.timing == synth.ARREARS)


def test_cash_flow_table_checks(rr):
    rng = np.random.default_rng(3)
    w = synth.random_small(rng, n=30, n_steps=120, n_scen=1)
    n_ages = w.basis.q.shape[1]
    ok = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.5, n_rows=4)
    tab = np.flatnonzero(ok.product == synth.CF_TABLE)
    assert tab.size >= 5
    assert rr.check_portfolio(ok, 120, n_ages, 2) == ""
    i = int(tab[0])
    bad = ok.subset(np.arange(ok.n)); bad.cf_row[i] = 4
    assert f"policy {i} cf_row 4" in rr.check_portfolio(bad, 120, n_ages, 2)
    bad = ok.subset(np.arange(ok.n)); bad.cf_row[i] = -1
    assert f"policy {i} cf_row -1" in rr.check_portfolio(bad, 120, n_ages, 2)
    bad = ok.subset(np.arange(ok.n)); bad.cf = bad.cf[:, :10].copy(); bad.term_m[i] = 11
    assert f"policy {i} term 11 exceeds cf_len 10" in rr.check_portfolio(bad, 120, n_ages, 2)
    bad = ok.subset(np.arange(ok.n)); bad.cf[2, 7] = np.nan
    assert "is not finite" in rr.check_portfolio(bad, 120, n_ages, 2)
    bad = ok.subset(np.arange(ok.n)); bad.cf = None
    assert "need cf_row and cf" in rr.check_portfolio(bad, 120, n_ages, 2)
    bad = ok.subset(np.arange(ok.n)); bad.product[i] = 14
    assert f"policy {i} has unknown product 14" in rr.check_portfolio(bad, 120, n_ages, 2)


def test_markov_policy_checks(rr):
    """Without a context the model bounds are unknown: the host check takes
    the model index and age as non-negative; the context's upload checks
    them against the uploaded models (GPU tests)."""
    rng = np.random.default_rng(4)
    w = synth.random_small(rng, n=20, n_steps=60, n_scen=1)
    n_ages = w.basis.q.shape[1]
    pf = synth.with_markov_policies(rng, w.portfolio, synth.phi_models(n_ages), frac=0.5)
    i = int(np.flatnonzero(pf.product == synth.MARKOV)[0])
    pf.table1[i] = 7                                  # beyond the q tables: fine for a model
    assert rr.check_portfolio(pf, 60, n_ages, 2) == ""
    bad = pf.subset(np.arange(pf.n)); bad.table1[i] = -1
    assert f"policy {i} model -1" in rr.check_portfolio(bad, 60, n_ages, 2)
    bad = pf.subset(np.arange(pf.n)); bad.age1_m[i] = -3
    assert f"policy {i} age -3" in rr.check_portfolio(bad, 60, n_ages, 2)


def test_fractional_timing_checks(rr):
    w = synth.config_c2(n=2000)
    n_ages = w.basis.q.shape[1]
    pf = w.portfolio.subset(np.arange(40))
    sl = np.flatnonzero(pf.product == synth.SL_ANN)
    term = np.flatnonzero(pf.product == synth.TERM)
    pf.timing[sl] = synth.FRACTIONAL
    assert rr.check_portfolio(pf, 600, n_ages, 3) == ""     # the basis's fraction is checked on upload
    bad = pf.subset(np.arange(pf.n)); bad.timing[term[0]] = synth.FRACTIONAL
    assert f"policy {term[0]}: fractional timing needs RR_SL_ANN" in rr.check_portfolio(bad, 600, n_ages, 3)
    bad = pf.subset(np.arange(pf.n))
    bad.escalation = np.zeros(bad.n); bad.escalation[sl[0]] = 0.03
    assert f"policy {sl[0]}: fractional timing with a payment pattern" in rr.check_portfolio(bad, 600, n_ages, 3)
