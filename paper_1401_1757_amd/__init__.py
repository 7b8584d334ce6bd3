"""MI355X reserve-recurrence library: thin Python binding of librr.so.

Argument marshalling only.  Every step of the valuation runs in the HIP
kernels behind the C ABI declared in include/rr.h; torch is used for device
memory and the stream.  Loading fails loudly when librr.so is missing or no
GPU is present.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RR_LIB names another build of the same library (e.g. the host-sanitizer
# build of the CPU checks); by default the in-tree librr.so.
LIB_PATH = os.environ.get("RR_LIB") or os.path.join(_HERE, "librr.so")

RR_OK, RR_EINVAL, RR_ENOMEM, RR_EDEVICE, RR_ERANGE, RR_ESTATE = 0, -1, -2, -3, -4, -5
SL_ANN, JL_ANN, REV_ANN, LS_ANN, TERM, ENDOW, ENDOW_ASSUR, CF_TABLE = range(8)
JL_ENDOW, JL_ASSUR1, JL_ASSUR2, MARKOV = 8, 9, 10, 11
JL3_ANN, LS3_ANN = 12, 13


class Markov(ctypes.Structure):
    _fields_ = [("n_models", ctypes.c_int32), ("n_states", ctypes.c_int32),
                ("n_ages", ctypes.c_int32), ("w", ctypes.c_void_p), ("benefit", ctypes.c_void_p),
                ("mem_kind", ctypes.c_int32)]


class Vasicek(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("sigma", ctypes.c_double),
                ("dt", ctypes.c_double), ("r0", ctypes.c_void_p), ("key", ctypes.c_uint64 * 2)]


def vasicek_struct(a, b, sigma, dt, r0, key, keep):
    r0 = _np(np.atleast_1d(r0), np.float64)
    keep.append(r0)
    k = (ctypes.c_uint64 * 2)(int(key[0]), int(key[1]))
    return Vasicek(a, b, sigma, dt, r0.ctypes.data, k)
ADVANCE, ARREARS, FRACTIONAL = 0, 1, 2
HOST, DEVICE = 0, 1
OUT_R0, OUT_TOTALS, OUT_PATH, OUT_ALL_STATES, OUT_STATS = 1, 2, 4, 8, 16
OPT_BLOCK_K, OPT_WG_PER_CU, OPT_USE_GRAPH, OPT_KERNEL_TIMING, OPT_XCD_QUEUES = 1, 2, 3, 4, 5
OPT_LAST_K, OPT_LAST_WG, OPT_BLOCK_J, OPT_LAST_J, OPT_TERM_BUCKET = 6, 7, 8, 9, 10
OPT_CURVE_RING, OPT_LAST_RING, OPT_LANE_SPREAD, OPT_CURVE_SHARE, OPT_LAST_WINDOWS = 11, 12, 13, 14, 15
OPT_LAST_TABLES_LDS = 16

# Every symbol include/rr.h declares.
EXPORTS = (
    "rr_create", "rr_destroy", "rr_last_error", "rr_set_stream", "rr_sync",
    "rr_check_basis", "rr_check_portfolio", "rr_basis_upload", "rr_portfolio_upload",
    "rr_path_size", "rr_reserve_recurrence", "rr_set_option", "rr_get_option",
    "rr_kernel_times", "rr_surrogate_train", "rr_surrogate_get_weights",
    "rr_surrogate_set_weights", "rr_surrogate_infer", "rr_surrogate_forward",
    "rr_surrogate_gradients", "rr_surrogate_adam_step", "rr_surrogate_features",
    "rr_basis_generate_vasicek", "rr_curves_generate_vasicek", "rr_vasicek_curves",
    "rr_node_surrogate_train", "rr_node_surrogate_infer", "rr_node_surrogate_get_weights",
    "rr_node_surrogate_set_weights", "rr_node_expected_reserves", "rr_markov_upload",
    "rr_reserve_recurrence_noalloc",
)

# Surrogate dimensions (include/rr.h).
SG_FEATURES, SG_INPUTS, SG_HIDDEN, SG_TENORS, SG_FACTORS, SG_PARAMS = 17, 32, 256, 50, 3, 74497


class RRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rr error {code}: {msg}")
        self.code = code


class Basis(ctypes.Structure):
    _fields_ = [("n_tables", ctypes.c_int32), ("n_ages", ctypes.c_int32),
                ("q", ctypes.c_void_p), ("n_nodes", ctypes.c_int32),
                ("n_scen", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("v", ctypes.c_void_p), ("shock", ctypes.c_void_p),
                ("mem_kind", ctypes.c_int32), ("frac", ctypes.c_double)]


class Portfolio(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("product", ctypes.c_void_p),
                ("age1_m", ctypes.c_void_p), ("age2_m", ctypes.c_void_p),
                ("term_m", ctypes.c_void_p), ("table1", ctypes.c_void_p),
                ("table2", ctypes.c_void_p), ("timing", ctypes.c_void_p),
                ("amount", ctypes.c_void_p), ("premium", ctypes.c_void_p),
                ("mem_kind", ctypes.c_int32), ("escalation", ctypes.c_void_p),
                ("anniv_m", ctypes.c_void_p), ("annual", ctypes.c_void_p),
                ("cf_row", ctypes.c_void_p), ("cf", ctypes.c_void_p),
                ("cf_n_rows", ctypes.c_int32), ("cf_len", ctypes.c_int32),
                ("age3_m", ctypes.c_void_p), ("table3", ctypes.c_void_p)]


class Run(ctypes.Structure):
    _fields_ = [("node_begin", ctypes.c_int32), ("node_count", ctypes.c_int32),
                ("scen_begin", ctypes.c_int32), ("scen_count", ctypes.c_int32),
                ("node_step_m", ctypes.c_int32), ("out_mask", ctypes.c_uint32),
                ("tail", ctypes.c_double)]


class Outputs(ctypes.Structure):
    _fields_ = [("r0", ctypes.c_void_p), ("totals", ctypes.c_void_p),
                ("path", ctypes.c_void_p), ("path_cap", ctypes.c_int64),
                ("stats", ctypes.c_void_p)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("run", Run), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("lr_final", ctypes.c_float),
                ("holdout", ctypes.c_float), ("init", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class TrainReport(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("n_train", ctypes.c_int64),
                ("n_holdout", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("first_loss", ctypes.c_float), ("final_loss", ctypes.c_float),
                ("holdout_loss", ctypes.c_float), ("calibration", ctypes.c_float * 4),
                ("data_ms", ctypes.c_double), ("train_ms", ctypes.c_double)]


class InferReport(ctypes.Structure):
    _fields_ = [("n_in_range", ctypes.c_int64), ("n_fallback", ctypes.c_int64)]


# Model blob layout (include/rr.h): header, FP64 statistics, FP32 arrays.
_BLOB_HEADER = np.dtype([("magic", "S8"), ("version", "<i4"), ("n_feat", "<i4"),
                         ("k_in", "<i4"), ("hidden", "<i4"), ("n_tenors", "<i4"),
                         ("n_factors", "<i4"), ("n_params", "<i4"), ("adam_step", "<i4"),
                         ("signature", "<i4", (4, 3)), ("reserved", "<i4", (2,))])
_BLOB_F64 = [("mu", SG_FEATURES), ("sd", SG_FEATURES), ("lo", SG_FEATURES), ("hi", SG_FEATURES),
             ("tmu", 4), ("tsd", 4), ("zbar", SG_TENORS), ("evec", SG_FACTORS * SG_TENORS)]


def pack_surrogate_blob(params, mu, sd, lo, hi, tmu, tsd, zbar, evec, signature,
                        adam_m=None, adam_v=None, adam_step=0, node=False) -> bytes:
    """Serialise a model into the blob rr_surrogate_set_weights (node: the
    node-level rr_node_surrogate_set_weights) reads.
    params: FP32 vector [SG_PARAMS]; evec: [3][50]; signature: [4][3]."""
    h = np.zeros((), _BLOB_HEADER)
    h["magic"] = b"RRSURN01" if node else b"RRSURR01"
    for k, v in (("version", 1), ("n_feat", SG_FEATURES), ("k_in", SG_INPUTS),
                 ("hidden", SG_HIDDEN), ("n_tenors", SG_TENORS), ("n_factors", SG_FACTORS),
                 ("n_params", SG_PARAMS), ("adam_step", adam_step)):
        h[k] = v
    h["signature"] = np.asarray(signature, np.int32).reshape(4, 3)
    vals = dict(mu=mu, sd=sd, lo=lo, hi=hi, tmu=tmu, tsd=tsd, zbar=zbar, evec=evec)
    f64 = np.concatenate([np.asarray(vals[k], np.float64).reshape(-1) for k, _ in _BLOB_F64])
    zeros = np.zeros(SG_PARAMS, np.float32)
    f32 = np.concatenate([np.asarray(params, np.float32).reshape(-1),
                          zeros if adam_m is None else np.asarray(adam_m, np.float32).reshape(-1),
                          zeros if adam_v is None else np.asarray(adam_v, np.float32).reshape(-1)])
    return h.tobytes() + f64.astype("<f8").tobytes() + f32.astype("<f4").tobytes()


def unpack_surrogate_blob(blob: bytes) -> dict:
    h = np.frombuffer(blob[:_BLOB_HEADER.itemsize], _BLOB_HEADER)[0]
    off = _BLOB_HEADER.itemsize
    out = {"adam_step": int(h["adam_step"]), "signature": np.array(h["signature"])}
    for k, size in _BLOB_F64:
        a = np.frombuffer(blob[off:off + 8 * size], "<f8").copy()
        out[k] = a[0] if size == 1 else a
        off += 8 * size
    out["evec"] = out["evec"].reshape(SG_FACTORS, SG_TENORS)
    for k in ("params", "adam_m", "adam_v"):
        out[k] = np.frombuffer(blob[off:off + 4 * SG_PARAMS], "<f4").copy()
        off += 4 * SG_PARAMS
    return out


_lib = None


def load_library(path: str = LIB_PATH):
    """dlopen librr.so and declare argument types (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1401_1757_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, u64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64
    sig = {
        "rr_create": ([ctypes.POINTER(vp), ctypes.c_int, u64], ctypes.c_int),
        "rr_destroy": ([vp], ctypes.c_int),
        "rr_last_error": ([vp], ctypes.c_char_p),
        "rr_set_stream": ([vp, u64], ctypes.c_int),
        "rr_sync": ([vp], ctypes.c_int),
        "rr_check_basis": ([ctypes.POINTER(Basis), ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
        "rr_check_portfolio": ([ctypes.POINTER(Portfolio), i32, i32, i32, ctypes.c_char_p,
                                ctypes.c_size_t], ctypes.c_int),
        "rr_basis_upload": ([vp, ctypes.POINTER(Basis)], ctypes.c_int),
        "rr_portfolio_upload": ([vp, ctypes.POINTER(Portfolio)], ctypes.c_int),
        "rr_path_size": ([vp, i32, i32, ctypes.POINTER(i64)], ctypes.c_int),
        "rr_reserve_recurrence": ([vp, ctypes.POINTER(Run), ctypes.POINTER(Outputs)], ctypes.c_int),
        "rr_set_option": ([vp, i32, i64], ctypes.c_int),
        "rr_get_option": ([vp, i32, ctypes.POINTER(i64)], ctypes.c_int),
        "rr_kernel_times": ([vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)], ctypes.c_int),
        "rr_surrogate_train": ([vp, ctypes.POINTER(TrainCfg), ctypes.POINTER(TrainReport)], ctypes.c_int),
        "rr_surrogate_get_weights": ([vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "rr_surrogate_set_weights": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "rr_surrogate_infer": ([vp, ctypes.POINTER(Run), ctypes.POINTER(Outputs),
                                ctypes.POINTER(InferReport)], ctypes.c_int),
        "rr_surrogate_forward": ([vp, vp, i64, vp], ctypes.c_int),
        "rr_surrogate_gradients": ([vp, vp, vp, i64, vp, vp], ctypes.c_int),
        "rr_surrogate_adam_step": ([vp, vp, ctypes.c_float], ctypes.c_int),
        "rr_surrogate_features": ([vp, ctypes.POINTER(Run), vp, vp, vp, vp], ctypes.c_int),
        "rr_basis_generate_vasicek": ([vp, ctypes.POINTER(Basis), ctypes.POINTER(Vasicek)], ctypes.c_int),
        "rr_curves_generate_vasicek": ([vp, ctypes.POINTER(Vasicek)], ctypes.c_int),
        "rr_vasicek_curves": ([vp, ctypes.POINTER(Vasicek), i32, i32, i32, vp, vp], ctypes.c_int),
        "rr_node_surrogate_train": ([vp, ctypes.POINTER(TrainCfg), ctypes.POINTER(TrainReport)], ctypes.c_int),
        "rr_node_surrogate_infer": ([vp, ctypes.POINTER(Run), vp, vp, ctypes.POINTER(InferReport)],
                                    ctypes.c_int),
        "rr_node_surrogate_get_weights": ([vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
                                          ctypes.c_int),
        "rr_node_surrogate_set_weights": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "rr_node_expected_reserves": ([vp, ctypes.POINTER(Run), vp, vp], ctypes.c_int),
        "rr_markov_upload": ([vp, ctypes.POINTER(Markov)], ctypes.c_int),
        "rr_reserve_recurrence_noalloc": ([vp, ctypes.POINTER(Run), ctypes.POINTER(Outputs)],
                                          ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _np(x, dt):
    return np.ascontiguousarray(x, dtype=dt)


def basis_struct(q, v, shock=None, keep=None, frac=0.0):
    """Host-memory rr_basis; `keep` collects the arrays that must outlive it."""
    q = _np(q, np.float64)
    v = _np(v, np.float64)
    sh = None if shock is None else _np(shock, np.float64)
    if keep is not None:
        keep.extend([q, v, sh])
    return Basis(q.shape[0], q.shape[1], q.ctypes.data, v.shape[0], v.shape[1], v.shape[2],
                 v.ctypes.data, None if sh is None else sh.ctypes.data, HOST, float(frac))


def portfolio_struct(pf, keep=None):
    arrs = [_np(pf.product, np.int32), _np(pf.age1_m, np.int32), _np(pf.age2_m, np.int32),
            _np(pf.term_m, np.int32), _np(pf.table1, np.int32), _np(pf.table2, np.int32),
            _np(pf.timing, np.int32), _np(pf.amount, np.float64), _np(pf.premium, np.float64)]
    # Optional annuity payment patterns (None: level payments) and cash-flow tables.
    opt = [None if getattr(pf, name, None) is None else _np(getattr(pf, name), dt)
           for name, dt in (("escalation", np.float64), ("anniv_m", np.int32), ("annual", np.int32),
                            ("cf_row", np.int32))]
    cf = getattr(pf, "cf", None)
    cf = None if cf is None else np.ascontiguousarray(np.atleast_2d(cf), np.float64)
    n_rows, cf_len = (0, 0) if cf is None else cf.shape
    three = [None if getattr(pf, name, None) is None else _np(getattr(pf, name), np.int32)
             for name in ("age3_m", "table3")]
    if keep is not None:
        keep.extend(arrs)
        keep.extend(opt)
        keep.append(cf)
        keep.extend(three)
    return Portfolio(arrs[0].shape[0], *[a.ctypes.data for a in arrs], HOST,
                     *[None if a is None else a.ctypes.data for a in opt],
                     None if cf is None else cf.ctypes.data, n_rows, cf_len,
                     *[None if a is None else a.ctypes.data for a in three])


def check_portfolio(pf, n_steps, n_ages, n_tables):
    """Host-only validation; returns '' or the reason."""
    lib = load_library()
    keep = []
    st = portfolio_struct(pf, keep)
    buf = ctypes.create_string_buffer(512)
    rc = lib.rr_check_portfolio(ctypes.byref(st), n_steps, n_ages, n_tables, buf, 512)
    return "" if rc == RR_OK else buf.value.decode()


def check_basis(q, v, shock=None):
    lib = load_library()
    keep = []
    st = basis_struct(q, v, shock, keep)
    buf = ctypes.create_string_buffer(512)
    rc = lib.rr_check_basis(ctypes.byref(st), buf, 512)
    return "" if rc == RR_OK else buf.value.decode()


def _ptr(t):
    return None if t is None else t.data_ptr()


class Context:
    """One rr_ctx on a CUDA (HIP) device, bound to torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the reserve library runs only on a HIP device")
        self._torch = torch
        self.lib = load_library()
        self.device = device
        with torch.cuda.device(device):
            s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = ctypes.c_void_p()
        rc = self.lib.rr_create(ctypes.byref(h), device, s.cuda_stream)
        if rc != RR_OK:
            raise RRError(rc, "rr_create failed")
        self.h = h
        self.n = 0
        self.n_nodes = self.n_scen = self.n_steps = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.rr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != RR_OK:
            raise RRError(rc, self.lib.rr_last_error(self.h).decode())

    def set_option(self, opt, value):
        self._check(self.lib.rr_set_option(self.h, opt, int(value)))

    def get_option(self, opt):
        v = ctypes.c_int64()
        self._check(self.lib.rr_get_option(self.h, opt, ctypes.byref(v)))
        return v.value

    def basis_upload(self, q, v, shock=None, frac=0.0):
        keep = []
        st = basis_struct(q, v, shock, keep, frac)
        self._check(self.lib.rr_basis_upload(self.h, ctypes.byref(st)))
        self.n_nodes, self.n_scen, self.n_steps = st.n_nodes, st.n_scen, st.n_steps

    def basis_generate_vasicek(self, q, n_scen, n_steps, r0, a, b, sigma, dt, key, shock=None,
                               frac=0.0):
        """Install a basis (q, shock) whose curves are generated on the device:
        len(r0) nodes x n_scen scenarios x n_steps steps."""
        keep = []
        q = _np(q, np.float64)
        r0 = _np(np.atleast_1d(r0), np.float64)
        sh = None if shock is None else _np(shock, np.float64)
        keep.extend([q, sh])
        bs = Basis(q.shape[0], q.shape[1], q.ctypes.data, r0.shape[0], n_scen, n_steps, None,
                   None if sh is None else sh.ctypes.data, HOST, float(frac))
        vs = vasicek_struct(a, b, sigma, dt, r0, key, keep)
        self._check(self.lib.rr_basis_generate_vasicek(self.h, ctypes.byref(bs), ctypes.byref(vs)))
        self.n_nodes, self.n_scen, self.n_steps = r0.shape[0], n_scen, n_steps

    def curves_generate_vasicek(self, r0, a, b, sigma, dt, key):
        """Regenerate the installed basis's curves in place (asynchronous)."""
        keep = []
        vs = vasicek_struct(a, b, sigma, dt, r0, key, keep)
        self._check(self.lib.rr_curves_generate_vasicek(self.h, ctypes.byref(vs)))

    def vasicek_curves(self, n_scen, n_steps, r0, a, b, sigma, dt, key, rates=True):
        """Device tensors v [n_nodes][n_scen][n_steps] (and r [..][n_steps + 1])."""
        torch = self._torch
        keep = []
        vs = vasicek_struct(a, b, sigma, dt, r0, key, keep)
        n_nodes = len(np.atleast_1d(r0))
        dev = torch.device("cuda", self.device)
        v = torch.empty((n_nodes, n_scen, n_steps), dtype=torch.float64, device=dev)
        r = torch.empty((n_nodes, n_scen, n_steps + 1), dtype=torch.float64, device=dev) if rates else None
        self._check(self.lib.rr_vasicek_curves(self.h, ctypes.byref(vs), n_nodes, n_scen, n_steps,
                                               v.data_ptr(), None if r is None else r.data_ptr()))
        return v, r

    def markov_upload(self, w, benefit):
        """Markov models for MARKOV policies: w [models][ages][m][m], benefit [models][m]."""
        w = _np(w, np.float64)
        c = _np(benefit, np.float64)
        st = Markov(w.shape[0], w.shape[2], w.shape[1], w.ctypes.data, c.ctypes.data, HOST)
        self._check(self.lib.rr_markov_upload(self.h, ctypes.byref(st)))

    def portfolio_upload(self, pf):
        keep = []
        st = portfolio_struct(pf, keep)
        self._check(self.lib.rr_portfolio_upload(self.h, ctypes.byref(st)))
        self.n = st.n

    def path_size(self, node=0, node_step=12):
        n = ctypes.c_int64()
        self._check(self.lib.rr_path_size(self.h, node, node_step, ctypes.byref(n)))
        return n.value

    def alloc_outputs(self, node_count, scen_count, r0=True, totals=True, all_states=False,
                      stats=False, path_node=None, node_step=12):
        torch = self._torch
        dev = torch.device("cuda", self.device)
        out = {}
        if r0:
            shape = (node_count, self.n, scen_count) + ((4,) if all_states else ())
            out["r0"] = torch.empty(shape, dtype=torch.float64, device=dev)
        if totals:
            out["totals"] = torch.empty((node_count, scen_count), dtype=torch.float64, device=dev)
        if stats:
            out["stats"] = torch.empty((node_count, 2), dtype=torch.float64, device=dev)
        if path_node is not None:
            out["path"] = torch.empty(self.path_size(path_node, node_step), dtype=torch.float64,
                                      device=dev)
        return out

    def reserve_recurrence(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                           node_step=12, outputs=None, all_states=False, tail=0.005):
        """Run the recurrence; outputs is a dict of preallocated device tensors
        (keys r0, totals, path, stats) or None to allocate r0 + totals."""
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        if outputs is None:
            outputs = self.alloc_outputs(node_count, scen_count, all_states=all_states)
        mask = 0
        if outputs.get("r0") is not None:
            mask |= OUT_R0
            if outputs["r0"].dim() == 4:
                mask |= OUT_ALL_STATES
        if outputs.get("totals") is not None:
            mask |= OUT_TOTALS
        if outputs.get("path") is not None:
            mask |= OUT_PATH
        if outputs.get("stats") is not None:
            mask |= OUT_STATS
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, mask, tail)
        path = outputs.get("path")
        o = Outputs(_ptr(outputs.get("r0")), _ptr(outputs.get("totals")), _ptr(path),
                    0 if path is None else path.numel(), _ptr(outputs.get("stats")))
        self._check(self.lib.rr_reserve_recurrence(self.h, ctypes.byref(run), ctypes.byref(o)))
        return outputs

    def reserve_recurrence_noalloc(self, node_begin=0, node_count=None, scen_begin=0,
                                   scen_count=None, node_step=12, outputs=None, tail=0.005):
        """rr_reserve_recurrence_noalloc: the same valuation with the library's
        static scratch (no device allocation); outputs as for reserve_recurrence
        (a path is RR_EINVAL)."""
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        if outputs is None:
            outputs = self.alloc_outputs(node_count, scen_count)
        mask = 0
        if outputs.get("r0") is not None:
            mask |= OUT_R0
            if outputs["r0"].dim() == 4:
                mask |= OUT_ALL_STATES
        if outputs.get("totals") is not None:
            mask |= OUT_TOTALS
        if outputs.get("stats") is not None:
            mask |= OUT_STATS
        if outputs.get("path") is not None:     # the library rejects it
            mask |= OUT_PATH
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, mask, tail)
        path = outputs.get("path")
        o = Outputs(_ptr(outputs.get("r0")), _ptr(outputs.get("totals")), _ptr(path),
                    0 if path is None else path.numel(), _ptr(outputs.get("stats")))
        self._check(self.lib.rr_reserve_recurrence_noalloc(self.h, ctypes.byref(run), ctypes.byref(o)))
        return outputs

    def sync(self):
        self._check(self.lib.rr_sync(self.h))

    def kernel_times(self, cap=4096):
        buf = (ctypes.c_double * cap)()
        n = ctypes.c_int32()
        self._check(self.lib.rr_kernel_times(self.h, buf, cap, ctypes.byref(n)))
        return [buf[i] for i in range(min(n.value, cap))]

    # -- surrogate ----------------------------------------------------------
    def surrogate_train(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                        node_step=0, epochs=20, batch=4096, lr=2e-3, lr_final=1e-5,
                        holdout=0.02, init=True, seed=7):
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, 0, 0.0)
        cfg = TrainCfg(run, epochs, batch, lr, lr_final, holdout, 1 if init else 0, seed)
        rep = TrainReport()
        self._check(self.lib.rr_surrogate_train(self.h, ctypes.byref(cfg), ctypes.byref(rep)))
        out = {k: getattr(rep, k) for k, _ in TrainReport._fields_}
        out["calibration"] = list(rep.calibration)
        return out

    def surrogate_get_weights(self) -> bytes:
        need = ctypes.c_size_t()
        self._check(self.lib.rr_surrogate_get_weights(self.h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        self._check(self.lib.rr_surrogate_get_weights(self.h, buf, need.value, ctypes.byref(need)))
        return buf.raw

    def surrogate_set_weights(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.rr_surrogate_set_weights(self.h, buf, len(blob)))

    def surrogate_infer(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                        node_step=12, outputs=None, tail=0.005, report=True):
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        if outputs is None:
            outputs = self.alloc_outputs(node_count, scen_count)
        mask = 0
        if outputs.get("r0") is not None:
            mask |= OUT_R0
        if outputs.get("totals") is not None:
            mask |= OUT_TOTALS
        if outputs.get("stats") is not None:
            mask |= OUT_STATS
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, mask, tail)
        o = Outputs(_ptr(outputs.get("r0")), _ptr(outputs.get("totals")), None, 0,
                    _ptr(outputs.get("stats")))
        rep = InferReport()
        self._check(self.lib.rr_surrogate_infer(self.h, ctypes.byref(run), ctypes.byref(o),
                                                ctypes.byref(rep) if report else None))
        if report:
            outputs["report"] = {"n_in_range": rep.n_in_range, "n_fallback": rep.n_fallback}
        return outputs

    def node_expected_reserves(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                               node_step=12, r0=True, totals=True):
        """Exact scenario-averaged reserves (mean discount curve): device
        tensors r0 [node_count][n] and totals [node_count]."""
        torch = self._torch
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        dev = torch.device("cuda", self.device)
        out = {"r0": torch.empty((node_count, self.n), dtype=torch.float64, device=dev) if r0 else None,
               "totals": torch.empty(node_count, dtype=torch.float64, device=dev) if totals else None}
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, 0, 0.0)
        self._check(self.lib.rr_node_expected_reserves(self.h, ctypes.byref(run), _ptr(out["r0"]),
                                                       _ptr(out["totals"])))
        return out

    # -- node-level surrogate ------------------------------------------------
    def node_surrogate_train(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                             node_step=12, epochs=20, batch=4096, lr=2e-3, lr_final=1e-5,
                             holdout=0.02, init=True, seed=7):
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, 0, 0.0)
        cfg = TrainCfg(run, epochs, batch, lr, lr_final, holdout, 1 if init else 0, seed)
        rep = TrainReport()
        self._check(self.lib.rr_node_surrogate_train(self.h, ctypes.byref(cfg), ctypes.byref(rep)))
        out = {k: getattr(rep, k) for k, _ in TrainReport._fields_}
        out["calibration"] = list(rep.calibration)
        return out

    def node_surrogate_get_weights(self) -> bytes:
        need = ctypes.c_size_t()
        self._check(self.lib.rr_node_surrogate_get_weights(self.h, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        self._check(self.lib.rr_node_surrogate_get_weights(self.h, buf, need.value, ctypes.byref(need)))
        return buf.raw

    def node_surrogate_set_weights(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.rr_node_surrogate_set_weights(self.h, buf, len(blob)))

    def node_surrogate_infer(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                             node_step=12, r0=True, totals=True, report=True):
        """Expected (scenario-averaged) reserves: dict with device tensors
        r0 [node_count][n] and totals [node_count] (None when not asked)."""
        torch = self._torch
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        dev = torch.device("cuda", self.device)
        out = {"r0": torch.empty((node_count, self.n), dtype=torch.float64, device=dev) if r0 else None,
               "totals": torch.empty(node_count, dtype=torch.float64, device=dev) if totals else None}
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, 0, 0.0)
        rep = InferReport()
        self._check(self.lib.rr_node_surrogate_infer(self.h, ctypes.byref(run), _ptr(out["r0"]),
                                                     _ptr(out["totals"]),
                                                     ctypes.byref(rep) if report else None))
        if report:
            out["report"] = {"n_in_range": rep.n_in_range, "n_fallback": rep.n_fallback}
        return out

    def surrogate_forward(self, z):
        """z: device float32 [n][32] standardised inputs -> device float32 [n]."""
        z = z.contiguous()
        y = self._torch.empty(z.shape[0], dtype=self._torch.float32, device=z.device)
        self._check(self.lib.rr_surrogate_forward(self.h, _ptr(z), z.shape[0], _ptr(y)))
        return y

    def surrogate_gradients(self, z, t):
        z, t = z.contiguous(), t.contiguous()
        torch = self._torch
        g = torch.empty(SG_PARAMS, dtype=torch.float32, device=z.device)
        loss = torch.empty(1, dtype=torch.float32, device=z.device)
        self._check(self.lib.rr_surrogate_gradients(self.h, _ptr(z), _ptr(t), z.shape[0],
                                                     _ptr(g), _ptr(loss)))
        return g, loss

    def surrogate_adam_step(self, grad, lr):
        self._check(self.lib.rr_surrogate_adam_step(self.h, _ptr(grad.contiguous()), float(lr)))

    def surrogate_features(self, node_begin=0, node_count=None, scen_begin=0, scen_count=None,
                           node_step=12):
        node_count = self.n_nodes - node_begin if node_count is None else node_count
        scen_count = self.n_scen - scen_begin if scen_count is None else scen_count
        torch = self._torch
        dev = torch.device("cuda", self.device)
        pol = torch.empty((node_count, self.n, 9), dtype=torch.float64, device=dev)
        scen = torch.empty((node_count, scen_count, 5), dtype=torch.float64, device=dev)
        pflag = torch.empty((node_count, self.n), dtype=torch.int32, device=dev)
        sflag = torch.empty((node_count, scen_count), dtype=torch.int32, device=dev)
        run = Run(node_begin, node_count, scen_begin, scen_count, node_step, 0, 0.0)
        self._check(self.lib.rr_surrogate_features(self.h, ctypes.byref(run), _ptr(pol),
                                                   _ptr(scen), _ptr(pflag), _ptr(sflag)))
        return {"pol": pol, "scen": scen, "pflag": pflag, "sflag": sflag}
