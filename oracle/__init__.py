"""Reserve oracle: TEST INFRASTRUCTURE ONLY.

Plain, slow CPU evaluation of reserves for the tests, the smoke check and the
CPU-baseline leg of the benchmark (see ``oracle.c`` for the method and the
readings of the paper it follows).  The GPU library never imports this
package and this package never imports the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
OUT_STATES = 4

_lib = None


_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no fast-math, no contraction).
    sanitize: liboracle_san.so instead, with AddressSanitizer and
    UndefinedBehaviorSanitizer (CPU only; load it with libasan preloaded)."""
    lib = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra"]
        if sanitize:
            cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined"]
        cmd += ["-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return lib


MAX_STATES = 9          # largest state model of the oracle


class _Basis(ctypes.Structure):
    _fields_ = [("n_ages", ctypes.c_int), ("n_tables", ctypes.c_int),
                ("q", ctypes.c_void_p), ("n_nodes", ctypes.c_int),
                ("n_scen", ctypes.c_int), ("n_steps", ctypes.c_int),
                ("v", ctypes.c_void_p), ("shock", ctypes.c_void_p), ("frac", ctypes.c_double)]


class _Portfolio(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("product", ctypes.c_void_p),
                ("age1", ctypes.c_void_p), ("age2", ctypes.c_void_p),
                ("term", ctypes.c_void_p), ("table1", ctypes.c_void_p),
                ("table2", ctypes.c_void_p), ("timing", ctypes.c_void_p),
                ("amount", ctypes.c_void_p), ("premium", ctypes.c_void_p),
                ("escalation", ctypes.c_void_p), ("anniv", ctypes.c_void_p),
                ("annual", ctypes.c_void_p), ("cf_row", ctypes.c_void_p),
                ("cf", ctypes.c_void_p), ("n_cf_rows", ctypes.c_int), ("cf_len", ctypes.c_int),
                ("mk_models", ctypes.c_int), ("mk_states", ctypes.c_int), ("mk_ages", ctypes.c_int),
                ("mk_w", ctypes.c_void_p), ("mk_c", ctypes.c_void_p),
                ("age3", ctypes.c_void_p), ("table3", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", "")   # e.g. the sanitizer build
        if not path:
            path = build()
        lib = ctypes.CDLL(path)
        vp, ci = ctypes.c_void_p, ctypes.c_int
        lib.orc_reserves.argtypes = [vp, vp, ci, ci, ci, ci, ci, vp, vp, vp, vp, ci]
        lib.orc_reserves.restype = ci
        lib.orc_reserves_reduced.argtypes = [vp, vp, ci, ci, ci, ci, ci, vp, vp, vp, ci]
        lib.orc_reserves_reduced.restype = ci
        lib.orc_reserve_paths.argtypes = [vp, vp, ci, ci, ci, vp, ci]
        lib.orc_reserve_paths.restype = ci
        lib.orc_reserve_path_summation.argtypes = [vp, vp, ci, ci, ci, ci, vp]
        lib.orc_reserve_path_summation.restype = ci
        lib.orc_build_w.argtypes = [ci, ci, vp, ctypes.c_double, vp]
        lib.orc_build_w.restype = ci
        lib.orc_n_states.argtypes = [ci]
        lib.orc_n_states.restype = ci
        u64, cd = ctypes.c_uint64, ctypes.c_double
        lib.orc_philox4x64_10.argtypes = [vp, vp, vp]
        lib.orc_philox4x64_10.restype = None
        lib.orc_normals.argtypes = [u64, u64, ci, ci, ci, vp]
        lib.orc_normals.restype = None
        lib.orc_vasicek_curves.argtypes = [cd, cd, cd, cd, vp, ci, ci, ci, u64, u64, vp, vp]
        lib.orc_vasicek_curves.restype = ci
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Args:
    """Holds contiguous copies so the pointers stay valid during a call."""

    def __init__(self, basis, pf):
        self.q = np.ascontiguousarray(basis.q, np.float64)
        self.v = np.ascontiguousarray(basis.v, np.float64)
        self.shock = None if basis.shock is None else np.ascontiguousarray(basis.shock, np.float64)
        self.b = _Basis(self.q.shape[1], self.q.shape[0], _ptr(self.q), self.v.shape[0],
                        self.v.shape[1], self.v.shape[2], _ptr(self.v), _ptr(self.shock),
                        float(getattr(basis, "frac", 0.0) or 0.0))
        i32 = lambda x: np.ascontiguousarray(x, np.int32)
        f64 = lambda x: np.ascontiguousarray(x, np.float64)
        opt = lambda x, f: None if x is None else f(x)
        self.arrs = [i32(pf.product), i32(pf.age1_m), i32(pf.age2_m), i32(pf.term_m),
                     i32(pf.table1), i32(pf.table2), i32(pf.timing), f64(pf.amount),
                     f64(pf.premium), opt(getattr(pf, "escalation", None), f64),
                     opt(getattr(pf, "anniv_m", None), i32), opt(getattr(pf, "annual", None), i32),
                     opt(getattr(pf, "cf_row", None), i32)]
        cf = getattr(pf, "cf", None)
        self.cf = None if cf is None else np.ascontiguousarray(np.atleast_2d(cf), np.float64)
        n_rows, cf_len = (0, 0) if self.cf is None else self.cf.shape
        mk = getattr(pf, "markov", None)      # (w [models][ages][m][m], c [models][m]) or None
        if mk is None:
            self.mk_w = self.mk_c = None
            mk_dims = (0, 0, 0)
        else:
            self.mk_w = np.ascontiguousarray(mk[0], np.float64)
            self.mk_c = np.ascontiguousarray(mk[1], np.float64)
            mk_dims = (self.mk_w.shape[0], self.mk_w.shape[2], self.mk_w.shape[1])
        self.three = [opt(getattr(pf, "age3_m", None), i32), opt(getattr(pf, "table3", None), i32)]
        self.p = _Portfolio(int(pf.product.shape[0]), *[_ptr(a) for a in self.arrs], _ptr(self.cf),
                            n_rows, cf_len, mk_dims[0], mk_dims[1], mk_dims[2], _ptr(self.mk_w),
                            _ptr(self.mk_c), _ptr(self.three[0]), _ptr(self.three[1]))
        self.n = int(pf.product.shape[0])


def default_threads() -> int:
    """ORACLE_THREADS, else OMP_NUM_THREADS (a machine's CPU share), else every core."""
    for var in ("ORACLE_THREADS", "OMP_NUM_THREADS"):
        val = os.environ.get(var, "").strip()
        if val.isdigit() and int(val) > 0:
            return int(val)
    return os.cpu_count() or 1


def reserves(basis, pf, node0=0, nnode=None, scen0=0, nscen=None, node_step=12,
             want_gross=True, n_threads=None):
    """Dense backward recurrence (Eq. 3.1) for every policy/node/scenario.

    Returns dict with r_all [nnode, n, nscen, 4], gross [nnode, n, nscen],
    totals [nnode, nscen], gross_totals [nnode, nscen].
    """
    lib = _load()
    a = _Args(basis, pf)
    nnode = basis.v.shape[0] - node0 if nnode is None else nnode
    nscen = basis.v.shape[1] - scen0 if nscen is None else nscen
    r_all = np.zeros((nnode, a.n, nscen, OUT_STATES))
    gross = np.zeros((nnode, a.n, nscen)) if want_gross else None
    totals = np.zeros((nnode, nscen))
    gtot = np.zeros((nnode, nscen)) if want_gross else None
    rc = lib.orc_reserves(ctypes.byref(a.b), ctypes.byref(a.p), node0, nnode, scen0, nscen,
                          node_step, _ptr(r_all), _ptr(gross), _ptr(totals), _ptr(gtot),
                          n_threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle rejected the input (rc={rc})")
    return {"r_all": r_all, "gross": gross, "totals": totals, "gross_totals": gtot}


def reserves_reduced(basis, pf, node0=0, nnode=None, scen0=0, nscen=None, node_step=12,
                     n_threads=None, want_r=True):
    """The same reserves by the zero-reserve-state-reduced recurrence of each
    product (see oracle.c, orc_reserves_reduced): r_all [nnode, n, nscen, 4]
    (None unless want_r), totals [nnode, nscen] and abs_totals (the sums of
    |r_0|); no gross values."""
    lib = _load()
    a = _Args(basis, pf)
    nnode = basis.v.shape[0] - node0 if nnode is None else nnode
    nscen = basis.v.shape[1] - scen0 if nscen is None else nscen
    r_all = np.zeros((nnode, a.n, nscen, OUT_STATES)) if want_r else None
    totals = np.zeros((nnode, nscen))
    abs_totals = np.zeros((nnode, nscen))
    rc = lib.orc_reserves_reduced(ctypes.byref(a.b), ctypes.byref(a.p), node0, nnode, scen0, nscen,
                                  node_step, _ptr(r_all), _ptr(totals), _ptr(abs_totals),
                                  n_threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle rejected the input (rc={rc})")
    return {"r_all": r_all, "totals": totals, "abs_totals": abs_totals}


def path_offsets(term_m, node=0, node_step=12):
    S = np.maximum(np.asarray(term_m, np.int64) - node * node_step, 0)
    off = np.zeros(S.shape[0] + 1, np.int64)
    np.cumsum(S + 1, out=off[1:])
    return off


def reserve_paths(basis, pf, node=0, scen=0, node_step=12, n_threads=None):
    """State-0 reserve at every step of every policy (ragged, see oracle.c)."""
    lib = _load()
    a = _Args(basis, pf)
    off = path_offsets(pf.term_m, node, node_step)
    path = np.zeros(int(off[-1]))
    rc = lib.orc_reserve_paths(ctypes.byref(a.b), ctypes.byref(a.p), node, scen, node_step,
                               _ptr(path), n_threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle rejected the input (rc={rc})")
    return path, off


def reserve_path_summation(basis, pf, i, node=0, scen=0, node_step=12):
    """Eq. (3.5) evaluated directly at each t = 0..S for policy i: [S+1, n_states]."""
    lib = _load()
    a = _Args(basis, pf)
    S = int(pf.term_m[i]) - node * node_step
    out = np.zeros((S + 1) * MAX_STATES)     # room for any model's states
    rc = lib.orc_reserve_path_summation(ctypes.byref(a.b), ctypes.byref(a.p), i, node, scen,
                                        node_step, _ptr(out))
    if rc < 0:
        raise ValueError("oracle rejected the input")
    return out[: (S + 1) * rc].reshape(S + 1, rc)


def build_w(n_lives: int, model: int, q, g: float = 1.0) -> np.ndarray:
    """Transition matrix of n_lives independent lives (Kronecker form)."""
    lib = _load()
    qa = np.ascontiguousarray(q, np.float64)
    W = np.zeros(81)
    n = lib.orc_build_w(n_lives, model, _ptr(qa), float(g), _ptr(W))
    if n < 0:
        raise ValueError("too many states")
    return W[: n * n].reshape(n, n)


def n_states(product: int) -> int:
    return int(_load().orc_n_states(int(product)))


def node_stats(totals: np.ndarray, tail: float = 0.005):
    """Per-node mean and the ceil(tail*K)-th largest of K scenario totals
    (the paper's 5th largest of 1,000 scenarios, Sec. 2.1)."""
    K = totals.shape[1]
    j = max(1, int(np.ceil(tail * K - 1e-12)))
    srt = np.sort(totals, axis=1)[:, ::-1]
    return totals.mean(axis=1), srt[:, j - 1]


# ---------------------------------------------------------------------------
# Scenario generation
# ---------------------------------------------------------------------------
def philox4x64_10(counter, key):
    """Philox4x64-10 block of a 4-word counter under a 2-word key (uint64[4])."""
    lib = _load()
    c = np.ascontiguousarray(counter, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib.orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(key, node, scen, step):
    """The two standard normals of (node, scenario, step)."""
    lib = _load()
    z = np.zeros(2)
    lib.orc_normals(int(key[0]), int(key[1]), node, scen, step, _ptr(z))
    return z


def vasicek_curves(a, b, sigma, dt, r0, n_scen, n_steps, key):
    """Exact-step Vasicek scenarios: (v[n_nodes][n_scen][n_steps] one-step
    discount factors, r[n_nodes][n_scen][n_steps + 1] short rates)."""
    lib = _load()
    r0 = np.ascontiguousarray(np.atleast_1d(r0), np.float64)
    n_nodes = r0.shape[0]
    v = np.zeros((n_nodes, n_scen, n_steps))
    r = np.zeros((n_nodes, n_scen, n_steps + 1))
    rc = lib.orc_vasicek_curves(a, b, sigma, dt, _ptr(r0), n_nodes, n_scen, n_steps,
                                int(key[0]), int(key[1]), _ptr(v), _ptr(r))
    if rc != 0:
        raise ValueError("orc_vasicek_curves: invalid input")
    return v, r
