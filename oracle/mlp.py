"""Reserve-surrogate oracle: TEST INFRASTRUCTURE ONLY.

Plain numpy definitions of the learned reserve surrogate that sits beside the
exact recurrence: its input features, their normalisation and range box, the
yield-curve factors, the multilayer perceptron (forward and backward, in FP64
and in a mode that rounds to bfloat16 where the GPU kernels do), the Adam
update and the training samples.  The surrogate is not part of the paper's
method; the paper only supplies the exact reserves it is fitted to (the
recurrence of Eq. (3.1), evaluated here by ``oracle.reserves``).  Only the
tests, the smoke check and the benchmark's CPU leg use this module.

Definitions (the same ones the GPU library documents):

* Features of one (node k, scenario s, policy i, state j) row, raw, FP64:
    0 age of life 1 in years at the node, (age1_m + k*node_step)/12
    1 remaining term in years, (term_m - k*node_step)/12
    2..5 product one-hot over (single-life annuity, joint-life annuity,
         term assurance, pure endowment)
    6 log of the amount (annual annuity or sum assured)
    7 annual premium per unit amount, 12*premium/amount
    8 short rate, -12 log v_{k,s,0}
    9..11 the first three principal-component scores of the scenario's
         zero-rate curve at 50 annual tenors
   12 mortality shock of the node (1 without shocks)
   13..15 one-hot of the reserve-vector state j (0, 1, 2)
   16 age of life 2 in years at the node (joint-life annuities; 0 otherwise)
* Zero rates: with m_T = min(12 T, n_steps) months, z_T = -(12/m_T) * sum of
  log v_t over t < m_T, for T = 1..50.
* Curve factors: f = E^T (z - zbar), with zbar the mean training curve and E
  the eigenvectors of the population covariance of the training curves for
  the three largest eigenvalues, each signed so that its component of
  largest magnitude is positive.
* Target: reserve of state j divided by the amount.  Features are
  standardised with the training mean and population standard deviation
  (1 where that is 0), the target with the mean and population standard
  deviation of the training rows of the same product; a row is in range
  when every raw feature lies in the training [min, max] box.
* Network: z (17 features, zero-padded to 32) -> 256 -> GELU -> 256 -> GELU
  -> 1, GELU in the tanh form of Hendrycks and Gimpel (2016); loss = mean
  squared error of the standardised target.
* bfloat16 mode: inputs, weights and activations are rounded to bfloat16
  (round to nearest, ties to even, from FP32), products are exact and sums
  are FP32; gradients of the pre-activations are rounded to bfloat16 before
  the weight-gradient and input-gradient products.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 17
K_IN = 32
HIDDEN = 256
N_TENORS = 50
N_FACTORS = 3
# Product codes (the library's numbering) in one-hot order.
SURROGATE_PRODUCTS = (0, 1, 4, 5)
JL_ANN = 1

F_AGE, F_TERM, F_PROD, F_LOGAMT, F_PREM, F_RATE, F_PCA, F_SHOCK, F_STATE, F_AGE2 = (
    0, 1, 2, 6, 7, 8, 9, 12, 13, 16)

GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


# ---------------------------------------------------------------------------
# Rounding
# ---------------------------------------------------------------------------
def bf16(x):
    """Round FP32 values to the nearest bfloat16 (ties to even); returns FP32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


# ---------------------------------------------------------------------------
# Activation
# ---------------------------------------------------------------------------
def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + GELU_A * x ** 3)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    t = np.tanh(GELU_C * (x + GELU_A * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * x * x)


# ---------------------------------------------------------------------------
# Curve features
# ---------------------------------------------------------------------------
def zero_rates(v):
    """Zero rates at the 50 annual tenors of discount curves v[..., n_steps]."""
    v = np.asarray(v, dtype=np.float64)
    n_steps = v.shape[-1]
    cum = np.cumsum(np.log(v), axis=-1)
    out = np.empty(v.shape[:-1] + (N_TENORS,))
    for T in range(1, N_TENORS + 1):
        m = min(12 * T, n_steps)
        out[..., T - 1] = -(12.0 / m) * cum[..., m - 1]
    return out


def short_rate(v):
    return -12.0 * np.log(np.asarray(v, dtype=np.float64)[..., 0])


def fit_pca(z):
    """Mean curve and the three leading eigenvectors [50][3] of curves z[n][50]."""
    z = np.asarray(z, dtype=np.float64).reshape(-1, N_TENORS)
    zbar = z.mean(axis=0)
    d = z - zbar
    cov = d.T @ d / z.shape[0]
    w, e = np.linalg.eigh(cov)
    order = np.argsort(w)[::-1][:N_FACTORS]
    E = e[:, order].copy()
    for j in range(N_FACTORS):
        if E[np.argmax(np.abs(E[:, j])), j] < 0:
            E[:, j] = -E[:, j]
    return zbar, E, w[order]


def scenario_features(v_node_scen, shock, zbar, E):
    """Raw scenario features [n][5] (short rate, 3 factors, shock) of curves [n][n_steps]."""
    v = np.asarray(v_node_scen, dtype=np.float64)
    z = zero_rates(v)
    out = np.empty((v.shape[0], 5))
    out[:, 0] = short_rate(v)
    out[:, 1:4] = (z - zbar) @ E
    out[:, 4] = shock
    return out


def patterned(pf):
    """Annuities with a payment pattern (escalation or annual payment): outside
    the surrogate's domain, whose features describe level payments only."""
    esc = getattr(pf, "escalation", None)
    ann = getattr(pf, "annual", None)
    out = np.zeros(pf.n, bool)
    if esc is not None:
        out |= np.asarray(esc) > 0.0
    if ann is not None:
        out |= np.asarray(ann) == 1
    return out


def product_signature(pf):
    """Per one-hot product: (table of life 1, table of life 2 or -1, annuity
    timing or -1) of the training policies, which must be unique; None for a
    product absent from training.  Features carry neither tables nor timing,
    so other combinations are outside the model's domain."""
    sig = []
    level = ~patterned(pf)
    for code in SURROGATE_PRODUCTS:
        sel = (pf.product == code) & level
        if not sel.any():
            sig.append(None)
            continue
        t2 = pf.table2[sel] if code == JL_ANN else np.full(sel.sum(), -1)
        tm = pf.timing[sel] if code in (0, 1) else np.full(sel.sum(), -1)
        combos = set(zip(pf.table1[sel].tolist(), t2.tolist(), tm.tolist()))
        if len(combos) != 1:
            raise ValueError(f"product {code}: several (table, timing) combinations")
        sig.append(combos.pop())
    return sig


def policy_features(pf, node, node_step, signature=None):
    """Raw policy features [n][9]: columns 0-7 and 16 of the feature vector
    (age, term, one-hot x4, log amount, premium rate, age2), and whether the
    policy's product (and, given a signature, its tables and timing) is in
    the model's domain (level payments only)."""
    n = pf.n
    out = np.zeros((n, 9))
    shift = node * node_step
    out[:, 0] = (pf.age1_m + shift) / 12.0
    out[:, 1] = (pf.term_m - shift) / 12.0
    for j, code in enumerate(SURROGATE_PRODUCTS):
        out[:, 2 + j] = (pf.product == code).astype(np.float64)
    out[:, 6] = np.log(pf.amount)
    out[:, 7] = 12.0 * pf.premium / pf.amount
    out[:, 8] = np.where(pf.product == JL_ANN, (pf.age2_m + shift) / 12.0, 0.0)
    supported = np.isin(pf.product, SURROGATE_PRODUCTS) & ~patterned(pf)
    if signature is not None:
        for j, code in enumerate(SURROGATE_PRODUCTS):
            sel = pf.product == code
            if signature[j] is None:
                supported &= ~sel
                continue
            t1, t2, tm = signature[j]
            bad = pf.table1 != t1
            if t2 >= 0:
                bad |= pf.table2 != t2
            if tm >= 0:
                bad |= pf.timing != tm
            supported &= ~(sel & bad)
    return out, supported


def assemble(pol_row, scen_row, state):
    x = np.zeros(N_FEAT)
    x[0:8] = pol_row[0:8]
    x[F_RATE:F_RATE + 5] = scen_row
    x[F_STATE + state] = 1.0
    x[F_AGE2] = pol_row[8]
    return x


# ---------------------------------------------------------------------------
# Training samples
# ---------------------------------------------------------------------------
def samples(workload, node_begin, node_count, scen_begin, scen_count, node_step, r_all, zbar, E):
    """Rows (node-major, then scenario, policy, state) of features and targets.

    r_all[node][policy][scen][4] are the exact reserves of every state (from
    ``oracle.reserves``).  Rows: every live supported policy, states 0-2 for
    joint-life annuities and state 0 otherwise."""
    b, pf = workload.basis, workload.portfolio
    X, T = [], []
    for kr in range(node_count):
        k = node_begin + kr
        pol, ok = policy_features(pf, k, node_step)
        shock = b.shock[k] if b.shock is not None else 1.0
        sc = scenario_features(b.v[k, scen_begin:scen_begin + scen_count], shock, zbar, E)
        for s in range(scen_count):
            for i in range(pf.n):
                if not ok[i] or pf.term_m[i] - k * node_step <= 0:
                    continue
                states = (0, 1, 2) if pf.product[i] == JL_ANN else (0,)
                for j in states:
                    X.append(assemble(pol[i], sc[s], j))
                    T.append(r_all[kr, i, s, j] / pf.amount[i])
    return np.array(X).reshape(-1, N_FEAT), np.array(T)


def node_samples(workload, node_begin, node_count, scen_begin, scen_count, node_step, r_all, zbar, E):
    """Rows (node-major, then policy) of the node-level model: the policy
    features, the node's scenario features averaged over its scenarios and
    state 0; the target is the policy's state-0 reserve averaged over the
    node's scenarios, per unit amount.  r_all as for ``samples``."""
    b, pf = workload.basis, workload.portfolio
    X, T = [], []
    for kr in range(node_count):
        k = node_begin + kr
        pol, ok = policy_features(pf, k, node_step)
        shock = b.shock[k] if b.shock is not None else 1.0
        sc = scenario_features(b.v[k, scen_begin:scen_begin + scen_count], shock, zbar, E)
        nsc = np.array([math.fsum(sc[:, j]) / scen_count for j in range(5)])
        for i in range(pf.n):
            if not ok[i] or pf.term_m[i] - k * node_step <= 0:
                continue
            X.append(assemble(pol[i], nsc, 0))
            T.append(math.fsum(r_all[kr, i, :, 0]) / scen_count / pf.amount[i])
    return np.array(X).reshape(-1, N_FEAT), np.array(T)


def normalisation(X, t):
    mu = X.mean(axis=0)
    sd = np.sqrt(((X - mu) ** 2).mean(axis=0))
    sd = np.where(sd > 0, sd, 1.0)
    tmu, tsd = np.zeros(4), np.ones(4)
    for j in range(4):
        sel = X[:, F_PROD + j] == 1.0
        if sel.any():
            tmu[j] = t[sel].mean()
            s = np.sqrt(((t[sel] - tmu[j]) ** 2).mean())
            tsd[j] = s if s > 0 else 1.0
    return mu, sd, X.min(axis=0), X.max(axis=0), tmu, tsd


def product_index(X):
    """One-hot product slot (0..3) of each row."""
    return np.argmax(np.asarray(X)[:, F_PROD:F_PROD + 4], axis=1)


def standardise_target(X, t, tmu, tsd):
    j = product_index(X)
    return f32((np.asarray(t, np.float64) - tmu[j]) / tsd[j])


def standardise(X, mu, sd):
    """Standardised features as FP32, zero-padded to 32 inputs."""
    z = np.zeros((X.shape[0], K_IN), dtype=np.float32)
    z[:, :N_FEAT] = f32((X - mu) / sd)
    return z


def in_range(X, lo, hi):
    return np.all((X >= lo) & (X <= hi), axis=1)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
def forward(p, z, quant=True):
    """Prediction y[n] of the standardised target and the saved activations.

    quant=True: the bfloat16 mode; quant=False: every value kept in FP64
    (the rounding points become the identity)."""
    if quant:
        q = bf16
        acc = f32
    else:
        q = acc = lambda a: np.asarray(a, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    xq = q(z)
    W1, W2, W3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    z1 = acc(xq.astype(np.float64) @ W1.astype(np.float64) + p["b1"])
    a1 = q(acc(gelu(z1)))
    z2 = acc(a1.astype(np.float64) @ W2.astype(np.float64) + p["b2"])
    a2 = q(acc(gelu(z2)))
    y = acc(a2.astype(np.float64) @ W3.astype(np.float64) + p["b3"])
    return y, dict(xq=xq, z1=z1, a1=a1, z2=z2, a2=a2, W1=W1, W2=W2, W3=W3)


def loss(p, z, t, quant=True):
    y, _ = forward(p, z, quant)
    return float(np.mean((np.asarray(y, np.float64) - t) ** 2))


def backward(p, z, t, quant=True, keep=False):
    """Gradients of the mean squared error with respect to every parameter
    (and, with keep, the forward and backward intermediates as a third value)."""
    if quant:
        q = bf16
        acc = f32
    else:
        q = acc = lambda a: np.asarray(a, dtype=np.float64)
    y, s = forward(p, z, quant)
    n = z.shape[0]
    d = lambda a: np.asarray(a, dtype=np.float64)
    dy = acc(2.0 * (d(y) - t) / n)
    g = {}
    g["b3"] = acc(np.sum(d(dy)))
    g["W3"] = acc(d(s["a2"]).T @ d(dy))
    dz2 = acc(np.outer(d(dy), d(s["W3"])) * gelu_grad(s["z2"]))
    dz2q = q(dz2)
    g["b2"] = acc(d(dz2q).sum(axis=0))
    g["W2"] = acc(d(s["a1"]).T @ d(dz2q))
    da1 = d(dz2q) @ d(s["W2"]).T
    dz1 = acc(da1 * gelu_grad(s["z1"]))
    dz1q = q(dz1)
    g["b1"] = acc(d(dz1q).sum(axis=0))
    g["W1"] = acc(d(s["xq"]).T @ d(dz1q))
    if keep:
        s.update(y=y, dy=dy, dz2=dz2, dz2q=dz2q, da1=da1, dz1=dz1, dz1q=dz1q)
        return g, y, s
    return g, y


# ---------------------------------------------------------------------------
# Rounding-error bookkeeping for parity tests of the bfloat16 kernels
# ---------------------------------------------------------------------------
U32 = 2.0 ** -24          # unit roundoff of FP32


def gamma(n):
    """gamma_n = n u / (1 - n u), u the FP32 unit roundoff: an n-term FP32
    sum in any order differs from the exact sum by at most gamma_{n-1} times
    the sum of the absolute terms (Higham, Accuracy and Stability of
    Numerical Algorithms, 2002, Sec. 4.2)."""
    return n * U32 / (1.0 - n * U32)


def abs_sums(p, s, n_rows):
    """Sums of absolute terms of every FP32 accumulation in forward and
    backward (s = the intermediates of ``backward(..., keep=True)``):
    z1, z2, y and da1 per row and unit; and, per gradient element, the sum
    of the absolute terms it adds up (the scale of its accumulation error)."""
    d = lambda a: np.abs(np.asarray(a, dtype=np.float64))
    out = {}
    out["z1"] = d(s["xq"]) @ d(s["W1"]) + d(p["b1"])
    out["z2"] = d(s["a1"]) @ d(s["W2"]) + d(p["b2"])
    out["y"] = d(s["a2"]) @ d(s["W3"]) + abs(float(p["b3"]))
    out["da1"] = d(s["dz2q"]) @ d(s["W2"]).T
    g = {}
    g["b3"] = float(np.sum(d(s["dy"])))
    g["W3"] = d(s["a2"]).T @ d(s["dy"])
    g["b2"] = d(s["dz2q"]).sum(axis=0)
    g["W2"] = d(s["a1"]).T @ d(s["dz2q"])
    g["b1"] = d(s["dz1q"]).sum(axis=0)
    g["W1"] = d(s["xq"]).T @ d(s["dz1q"])
    out["grad"] = g
    return out


def bf16_boundary_distance(x):
    """Distance of each FP32 value to the nearest point where its bfloat16
    rounding changes (the midpoint between the two neighbouring bfloat16
    values), as FP64; zeros and values already in bfloat16 are far from it."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    a = np.abs(x)
    lo_bits = a.view(np.uint32) & np.uint32(0xFFFF0000)
    lo = lo_bits.view(np.float32).astype(np.float64)
    hi = (lo_bits + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    a64 = a.astype(np.float64)
    d = np.abs(a64 - 0.5 * (lo + hi))
    # just above a power of two the boundary below lo is closer (smaller units below)
    has_prev = lo_bits >= np.uint32(0x10000)
    prev = np.where(has_prev, lo_bits - np.uint32(0x10000), lo_bits).view(np.float32).astype(np.float64)
    below = np.where(has_prev, a64 - 0.5 * (prev + lo), np.inf)
    return np.minimum(d, below)


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in FP32 (step counts from 1); returns new (p, m, v)."""
    c1 = np.float32(1.0 / (1.0 - beta1 ** step))
    c2 = np.float32(1.0 / (1.0 - beta2 ** step))
    b1, b2 = np.float32(beta1), np.float32(beta2)
    o1, o2 = np.float32(1.0 - beta1), np.float32(1.0 - beta2)
    lr, eps = np.float32(lr), np.float32(eps)
    out_p, out_m, out_v = {}, {}, {}
    for k in p:
        gk = np.asarray(g[k], np.float32)
        mk = b1 * np.asarray(m[k], np.float32) + o1 * gk
        vk = b2 * np.asarray(v[k], np.float32) + o2 * gk * gk
        out_p[k] = np.asarray(p[k], np.float32) - lr * (mk * c1) / (np.sqrt(vk * c2) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v


PARAM_SHAPES = (("W1", (K_IN, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
                ("b2", (HIDDEN,)), ("W3", (HIDDEN,)), ("b3", ()))


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k, _ in PARAM_SHAPES])


def unflatten(vec):
    out, o = {}, 0
    for k, shp in PARAM_SHAPES:
        size = int(np.prod(shp)) if shp else 1
        out[k] = np.asarray(vec[o:o + size], np.float32).reshape(shp) if shp else np.float32(vec[o])
        o += size
    return out


N_PARAMS = sum(int(np.prod(s)) if s else 1 for _, s in PARAM_SHAPES)


def predict_reserves(p, X, amount, mu, sd, tmu, tsd):
    """Reserve predictions in FP64 from raw features X (bfloat16 mode)."""
    y, _ = forward(p, standardise(X, mu, sd), quant=True)
    j = product_index(X)
    return amount * (np.asarray(y, np.float64) * tsd[j] + tmu[j])
