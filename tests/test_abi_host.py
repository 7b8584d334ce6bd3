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
        "product": ("product", 11, 9, "policy 11 has unknown product 9"),
        "age": ("age1_m", 5, n_ages, "policy 5 age"),
        "table": ("table1", 2, 3, "policy 2 table1 3"),
        "timing": ("timing", 9, 2, "policy 9 timing 2"),
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
