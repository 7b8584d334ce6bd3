"""Seeded synthetic inputs for the reserve recurrence.

This module only draws and shapes inputs: mortality tables, discount
curves, portfolios and the sampling recipe for surrogate training.  It holds
none of the valuation arithmetic (no discounting of cash flows, no transition
matrices, no reserves); both the CPU oracle and the GPU library consume what
it returns, as plain NumPy arrays.

The paper states that mortality and interest may come from any model that
yields the one-step quantities when needed (Sec. 3.7.2, 3.7.3) and evaluates
its method on its own synthetic annuity data (Sec. 5), which is not
published.  The recipes here stand in for those data:

* mortality: Gompertz-Makeham force mu(x) = A + B c^x (A=5e-4, B=7.5e-5,
  c=1.1), integrated exactly over each month to give the monthly death
  probability q by attained age in whole months; q = 1 from age 120 on
  (the paper's limiting age, Sec. 4.1.1); per-table loadings multiply q and
  are capped at 1;
* interest: flat 3 % effective per year, or the Vasicek short rate
  (a=0.1, b=0.03, sigma=0.01) simulated with the exact Gaussian transition of
  (r, integral of r) over each month; the one-step discount factor is
  exp(-integral of r over the month);
* portfolios: the mixes described in the module-level ``config_*`` builders.

Product codes are an interface value shared by convention with the library
header and the oracle (each side keeps its own copy of the numbers).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ----------------------------------------------------------------------------
# Interface values (input format): product codes and annuity timing.
# ----------------------------------------------------------------------------
SL_ANN = 0        # single-life annuity (2-state model, Sec. 4.1.1)
JL_ANN = 1        # joint-life annuity (4-state model, Sec. 4.2.1 b)
REV_ANN = 2       # reversionary annuity to the second life (Sec. 4.2.1 a)
LS_ANN = 3        # last-survivor annuity (Sec. 4.2.1 c)
TERM = 4          # term assurance (3-state model, Sec. 4.1.3)
ENDOW = 5         # pure endowment (Sec. 4.1.2)
ENDOW_ASSUR = 6   # endowment assurance: term assurance + pure endowment
N_PRODUCTS = 7    # products with closed-form cash flows (0..6)
CF_TABLE = 7      # single life, cash flows amount x cf[row][t] from a table (Sec. 4.6)
JL_ENDOW = 8      # two-life pure endowment: SA at maturity if both alive (Sec. 4.2.2)
JL_ASSUR1 = 9     # two-life term assurance, SA on the first death (9-state model, Sec. 4.2.3)
JL_ASSUR2 = 10    # two-life term assurance, SA on the second death (Sec. 4.2.3)
TWO_LIFE_INS = (JL_ENDOW, JL_ASSUR1, JL_ASSUR2)
MARKOV = 11       # one life on an uploaded Markov model (table1 = model; Sec. 4.5)
TWO_LIFE = (JL_ANN, REV_ANN, LS_ANN, 8, 9, 10)   # with the two-life endowment and assurances
JL3_ANN = 12      # joint-life annuity on three lives (2^3 = 8 states, Sec. 4.3)
LS3_ANN = 13      # last-survivor annuity on three lives (Sec. 4.3)
THREE_LIFE = (JL3_ANN, LS3_ANN)

ADVANCE = 0       # annuity paid at the start of each month (f = 0)
ARREARS = 1       # annuity paid at the end of each month (f = 1)
FRACTIONAL = 2    # annuity paid at the basis's fraction f of each month (0 < f < 1)

GM_A, GM_B, GM_C = 5e-4, 7.5e-5, 1.1
LIMIT_AGE_M = 1440   # 120 years in months
VAS_A, VAS_B, VAS_SIGMA, VAS_R0 = 0.1, 0.03, 0.01, 0.03
DT = 1.0 / 12.0


# ----------------------------------------------------------------------------
# Mortality basis
# ----------------------------------------------------------------------------
def gm_monthly_q(n_ages: int, loading: float = 1.0, A: float = GM_A,
                 B: float = GM_B, c: float = GM_C,
                 limit_m: int = LIMIT_AGE_M) -> np.ndarray:
    """Monthly death probability by attained age in whole months.

    q(a) = 1 - exp(-int_{a/12}^{(a+1)/12} mu(s) ds) with mu(s) = A + B c^s,
    whose integral is A/12 + (B / ln c) c^{a/12} (c^{1/12} - 1).  The loading
    multiplies q and the result is capped at 1; ages >= limit_m die surely.
    """
    a = np.arange(n_ages, dtype=np.float64)
    x = a / 12.0
    H = A / 12.0 + (B / math.log(c)) * np.power(c, x) * (c ** (1.0 / 12.0) - 1.0)
    q = -np.expm1(-H)
    q = np.minimum(1.0, loading * q)
    q[np.arange(n_ages) >= limit_m] = 1.0
    return q


def mortality_tables(n_ages: int, loadings) -> np.ndarray:
    """Stack of GM tables, one per loading: shape [n_tables, n_ages]."""
    return np.stack([gm_monthly_q(n_ages, lam) for lam in loadings])


# ----------------------------------------------------------------------------
# Interest basis
# ----------------------------------------------------------------------------
def flat_v(n_steps: int, annual_rate: float = 0.03) -> np.ndarray:
    """One-step (monthly) discount factors for a flat effective annual rate."""
    return np.full(n_steps, (1.0 + annual_rate) ** (-1.0 / 12.0))


def vasicek_paths(rng: np.random.Generator, n_paths: int, n_steps: int,
                  r0, a: float = VAS_A, b: float = VAS_B,
                  sigma: float = VAS_SIGMA, dt: float = DT):
    """Exact simulation of the Vasicek short rate and its monthly integral.

    Returns (v, r): v[p, t] = exp(-int_t^{t+dt} r) and r[p, t] for
    t = 0..n_steps (r[:, 0] = r0).  The pair (r_{t+dt}, int r) is jointly
    Gaussian given r_t (Glasserman, Monte Carlo Methods in Financial
    Engineering, Sec. 3.3); it is sampled with two independent normals.
    """
    r0 = np.broadcast_to(np.asarray(r0, dtype=np.float64), (n_paths,))
    e = math.exp(-a * dt)
    mr_coef = e
    var_r = sigma ** 2 * (1.0 - e * e) / (2.0 * a)
    var_y = (sigma ** 2 / a ** 2) * (dt - 2.0 * (1.0 - e) / a + (1.0 - e * e) / (2.0 * a))
    cov = (sigma ** 2 / (2.0 * a ** 2)) * (1.0 - e) ** 2
    sd_r = math.sqrt(var_r)
    sd_y = math.sqrt(var_y)
    rho = cov / (sd_r * sd_y)
    sd_y_perp = sd_y * math.sqrt(max(0.0, 1.0 - rho * rho))
    r = np.empty((n_paths, n_steps + 1))
    y = np.empty((n_paths, n_steps))
    r[:, 0] = r0
    for t in range(n_steps):
        z = rng.standard_normal((2, n_paths))
        rt = r[:, t]
        y[:, t] = b * dt + (rt - b) * (1.0 - e) / a + rho * sd_y * z[0] + sd_y_perp * z[1]
        r[:, t + 1] = b + (rt - b) * mr_coef + sd_r * z[0]
    return np.exp(-y), r


def vasicek_zcb(T: float, r0: float, a: float = VAS_A, b: float = VAS_B,
                sigma: float = VAS_SIGMA) -> float:
    """Vasicek zero-coupon bond price P(0, T) (closed form)."""
    Bt = (1.0 - math.exp(-a * T)) / a
    lnA = (Bt - T) * (a * a * b - 0.5 * sigma * sigma) / (a * a) - sigma * sigma * Bt * Bt / (4.0 * a)
    return math.exp(lnA - Bt * r0)


# ----------------------------------------------------------------------------
# Portfolios
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Portfolio:
    product: np.ndarray   # int32 [n]
    age1_m: np.ndarray    # int32 [n] attained age of life 1 at node 0 (months)
    age2_m: np.ndarray    # int32 [n] attained age of life 2 (two-life products)
    term_m: np.ndarray    # int32 [n] remaining term at node 0 (months)
    table1: np.ndarray    # int32 [n] mortality table of life 1
    table2: np.ndarray    # int32 [n] mortality table of life 2
    timing: np.ndarray    # int32 [n] annuity timing (ADVANCE / ARREARS)
    amount: np.ndarray    # float64 [n] annual annuity amount or sum assured
    premium: np.ndarray   # float64 [n] level monthly premium, paid in advance
    # Annuity payment pattern (None: monthly, level):
    escalation: np.ndarray | None = None   # float64 [n] rate e, payments x (1+e) at each anniversary
    anniv_m: np.ndarray | None = None      # int32 [n] months from node 0 to the first anniversary, 1..12
    annual: np.ndarray | None = None       # int32 [n] 1: one payment of `amount` per anniversary
    # Cash-flow tables (CF_TABLE policies): policy i pays amount[i] x cf[cf_row[i]][T]
    # at the end of month T after node 0 if alive.
    cf_row: np.ndarray | None = None       # int32 [n]
    cf: np.ndarray | None = None           # float64 [n_rows][cf_len]
    # Uploaded Markov models (MARKOV policies, table1 = model): (w, c) with
    # w [models][ages][m][m] monthly one-step matrices (row = state at the
    # start of the month) and c [models][m] benefits per unit amount.
    markov: tuple | None = None
    # Life 3 of the three-life annuities (None when there are none).
    age3_m: np.ndarray | None = None       # int32 [n]
    table3: np.ndarray | None = None       # int32 [n]

    @property
    def n(self) -> int:
        return int(self.product.shape[0])

    def subset(self, idx) -> "Portfolio":
        d = {f.name: (None if getattr(self, f.name) is None
                      else np.ascontiguousarray(getattr(self, f.name)[idx]))
             for f in dataclasses.fields(self) if f.name not in ("cf", "markov")}
        d["cf"] = None if self.cf is None else self.cf.copy()   # rows are shared
        d["markov"] = self.markov
        return Portfolio(**d)

    def scaled(self, factor: float) -> "Portfolio":
        d = {f.name: (None if getattr(self, f.name) is None else getattr(self, f.name).copy())
             for f in dataclasses.fields(self)}
        d["amount"] = d["amount"] * factor
        d["premium"] = d["premium"] * factor
        return Portfolio(**d)


@dataclasses.dataclass
class Basis:
    q: np.ndarray           # float64 [n_tables, n_ages] monthly q by attained age (months)
    v: np.ndarray           # float64 [n_nodes, n_scen, n_steps] one-step discount factors
    shock: np.ndarray | None = None   # float64 [n_nodes] mortality multiplier or None
    frac: float = 0.0                 # payment point of FRACTIONAL annuities within the month

    @property
    def n_nodes(self) -> int:
        return int(self.v.shape[0])

    @property
    def n_scen(self) -> int:
        return int(self.v.shape[1])

    @property
    def n_steps(self) -> int:
        return int(self.v.shape[2])


@dataclasses.dataclass
class Workload:
    name: str
    basis: Basis
    portfolio: Portfolio
    node_step_m: int = 12
    note: str = ""


def _lognormal(rng, mean, sigma, size):
    """Lognormal with the given arithmetic mean and log-scale sd sigma."""
    mu = math.log(mean) - 0.5 * sigma * sigma
    return rng.lognormal(mu, sigma, size)


# Loadings on q per table: annuitants, term assurance, endowments.
TABLE_ANNUITANT, TABLE_TERM, TABLE_ENDOW = 0, 1, 2
C2_LOADINGS = (0.80, 1.20, 1.00)


def _premiums(rng, product, age1_m, term_m, sa):
    """Level monthly premiums by a simple rating rule (not a valuation).

    Term assurance: sum assured times the GM force of mortality at the age
    half way through the term, over 12, times U(0.9, 1.3).  Endowments:
    sum assured over the number of months, times U(0.6, 0.95).  Annuities
    are single-premium (no premiums after the valuation date).
    """
    n = product.shape[0]
    prem = np.zeros(n)
    u = rng.uniform(0.0, 1.0, n)
    mid_age = (age1_m + 0.5 * term_m) / 12.0
    mu_mid = (GM_A + GM_B * np.power(GM_C, mid_age)) * C2_LOADINGS[TABLE_TERM]
    is_term = product == TERM
    prem[is_term] = sa[is_term] * mu_mid[is_term] / 12.0 * (0.9 + 0.4 * u[is_term])
    is_end = (product == ENDOW) | (product == ENDOW_ASSUR)
    prem[is_end] = sa[is_end] / term_m[is_end] * (0.6 + 0.35 * u[is_end])
    return prem


def portfolio_single_life_annuities(rng, n: int, term_m: int = 300,
                                    age_lo_y: int = 60, age_hi_y: int = 80,
                                    mean_amount: float = 1.0e4,
                                    sigma: float = 0.5,
                                    table: int = 0,
                                    timing: int = ARREARS) -> Portfolio:
    """Level single-life annuities, monthly, ages uniform in whole months."""
    age = rng.integers(age_lo_y * 12, age_hi_y * 12, n, endpoint=True).astype(np.int32)
    amt = _lognormal(rng, mean_amount, sigma, n)
    z = np.zeros(n, np.int32)
    return Portfolio(product=np.full(n, SL_ANN, np.int32), age1_m=age,
                     age2_m=z.copy(), term_m=np.full(n, term_m, np.int32),
                     table1=np.full(n, table, np.int32), table2=np.full(n, table, np.int32),
                     timing=np.full(n, timing, np.int32), amount=amt,
                     premium=np.zeros(n))


def portfolio_mixed(rng, n: int, mix=(0.4, 0.2, 0.2, 0.2),
                    products=(SL_ANN, JL_ANN, TERM, ENDOW),
                    age_lo_y: int = 20, age_hi_y: int = 85,
                    term_lo_m: int = 60, term_hi_m: int = 600) -> Portfolio:
    """Mixed portfolio: shares ``mix`` of ``products`` (exact counts, shuffled)."""
    counts = np.floor(np.asarray(mix) * n).astype(int)
    counts[0] += n - counts.sum()
    product = np.concatenate([np.full(c, p, np.int32) for c, p in zip(counts, products)])
    rng.shuffle(product)
    age1 = rng.integers(age_lo_y * 12, age_hi_y * 12, n, endpoint=True).astype(np.int32)
    age2 = rng.integers(age_lo_y * 12, age_hi_y * 12, n, endpoint=True).astype(np.int32)
    term = rng.integers(term_lo_m, term_hi_m, n, endpoint=True).astype(np.int32)
    theta = _lognormal(rng, 1.0e4, 0.5, n)
    sa = _lognormal(rng, 1.0e5, 0.8, n)
    is_ann = np.isin(product, (SL_ANN, JL_ANN, REV_ANN, LS_ANN))
    amount = np.where(is_ann, theta, sa)
    table = np.full(n, TABLE_ANNUITANT, np.int32)
    table[product == TERM] = TABLE_TERM
    table[(product == ENDOW) | (product == ENDOW_ASSUR)] = TABLE_ENDOW
    premium = _premiums(rng, product, age1, term, sa)
    is_two = np.isin(product, TWO_LIFE)
    age2 = np.where(is_two, age2, 0).astype(np.int32)
    return Portfolio(product=product, age1_m=age1, age2_m=age2, term_m=term,
                     table1=table, table2=table.copy(),
                     timing=np.full(n, ARREARS, np.int32), amount=amount,
                     premium=premium)


def max_attained_age(p: Portfolio) -> int:
    a = int((p.age1_m + p.term_m).max(initial=0))
    two = np.isin(p.product, TWO_LIFE + THREE_LIFE)
    if two.any():
        a = max(a, int((p.age2_m[two] + p.term_m[two]).max()))
    three = np.isin(p.product, THREE_LIFE)
    if three.any():
        a = max(a, int((p.age3_m[three] + p.term_m[three]).max()))
    return a


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
def config_c1(seed: int = 1001) -> Workload:
    """1,000 single-life level annuities, monthly in arrears, ages 60-80,
    300 steps, GM mortality, flat 3 %, one scenario."""
    rng = np.random.default_rng(seed)
    pf = portfolio_single_life_annuities(rng, 1000)
    n_steps = 300
    q = mortality_tables(max(max_attained_age(pf) + 1, 1), (1.0,))
    v = flat_v(n_steps)[None, None, :]
    return Workload("C1: 1,000 single-life annuities x 1 flat scenario, 300 monthly steps",
                    Basis(q=q, v=v), pf)


def config_c2(seed: int = 1002, n: int = 100_000) -> Workload:
    """Mixed portfolio: 40 % SL, 20 % JL, 20 % term, 20 % endowments; ages
    20-85, terms 60-600 months; one flat 3 % scenario."""
    rng = np.random.default_rng(seed)
    pf = portfolio_mixed(rng, n)
    n_steps = 600
    q = mortality_tables(max_attained_age(pf) + 1, C2_LOADINGS)
    v = flat_v(n_steps)[None, None, :]
    return Workload(f"C2: {n:,}-policy mixed portfolio x 1 flat scenario, 60-600 monthly steps",
                    Basis(q=q, v=v), pf)


def config_c3(seed: int = 1003, n: int = 10_000, n_scen: int = 1000,
              scen_seed: int = 2003, n_steps: int = 600) -> Workload:
    """Nested brute force: the C2 policy laws x Vasicek inner scenarios."""
    rng = np.random.default_rng(seed)
    pf = portfolio_mixed(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, C2_LOADINGS)
    srng = np.random.default_rng(scen_seed)
    v, _ = vasicek_paths(srng, n_scen, n_steps, VAS_R0)
    return Workload(f"C3: {n:,} mixed policies x {n_scen:,} Vasicek scenarios, 60-600 monthly steps",
                    Basis(q=q, v=v[None]), pf)


def config_c3a(seed: int = 1013, n: int = 10_000, n_scen: int = 1000,
               scen_seed: int = 2013) -> Workload:
    """C1-law single-life annuities x Vasicek scenarios, 300 steps."""
    rng = np.random.default_rng(seed)
    pf = portfolio_single_life_annuities(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, (1.0,))
    srng = np.random.default_rng(scen_seed)
    v, _ = vasicek_paths(srng, n_scen, 300, VAS_R0)
    return Workload(f"C3a: {n:,} single-life annuities x {n_scen:,} Vasicek scenarios, 300 steps",
                    Basis(q=q, v=v[None]), pf)


# Representative annuity portfolio (Sec. 5.3, Table 2): tables by sex.
TABLE_MALE, TABLE_FEMALE = 0, 1
REP_LOADINGS = (1.0, 0.6)          # female q = 0.6 x male q (a reading: the paper gives no table)
REP_COMPOSITION = ((SL_ANN, 300_000), (JL_ANN, 50_000), (REV_ANN, 100_000), (LS_ANN, 50_000))
REP_AGE_LO_Y, REP_AGE_HI_Y = 57, 67
REP_N_STEPS = LIMIT_AGE_M - REP_AGE_LO_Y * 12     # 756: to age 120 from the youngest age


def portfolio_representative(rng, n: int = 500_000) -> Portfolio:
    """Annuities of a recently retired cohort (Sec. 5.3): products in the
    proportions of Table 2 (exact counts for n = 500,000); attained ages
    uniform over [57, 67] years in whole months, both lives of two-life
    policies from the same law; life 1 male with probability 0.75, life 2 of
    the other sex; inception uniform over the year before the valuation date,
    so the next anniversary is U{1..12} months away; 80 % pay monthly, 20 %
    once a year on the anniversary; the amount of each payment is lognormal
    with mean 5.0 and sd 1.5; 95 % level, the rest escalating at 3, 4.25 or
    5 % on each anniversary.  Payments fall at month ends (arrears), no
    premiums remain, and every policy runs to the limiting age of 120 of its
    younger life (q = 1 from there)."""
    total = sum(c for _, c in REP_COMPOSITION)
    counts = np.array([c * n // total for _, c in REP_COMPOSITION])
    counts[0] += n - counts.sum()
    product = np.concatenate([np.full(c, p, np.int32) for (p, _), c in zip(REP_COMPOSITION, counts)])
    rng.shuffle(product)
    two = np.isin(product, TWO_LIFE)
    age1 = rng.integers(REP_AGE_LO_Y * 12, REP_AGE_HI_Y * 12, n, endpoint=True).astype(np.int32)
    age2 = rng.integers(REP_AGE_LO_Y * 12, REP_AGE_HI_Y * 12, n, endpoint=True).astype(np.int32)
    age2 = np.where(two, age2, 0).astype(np.int32)
    male = rng.uniform(size=n) < 0.75
    table1 = np.where(male, TABLE_MALE, TABLE_FEMALE).astype(np.int32)
    table2 = np.where(two, np.where(male, TABLE_FEMALE, TABLE_MALE), table1).astype(np.int32)
    youngest = np.where(two, np.minimum(age1, age2), age1)
    term = (LIMIT_AGE_M - youngest).astype(np.int32)
    annual = (rng.uniform(size=n) < 0.20).astype(np.int32)
    sd_log = math.sqrt(math.log1p((1.5 / 5.0) ** 2))
    per_payment = _lognormal(rng, 5.0, sd_log, n)
    amount = np.where(annual == 1, per_payment, 12.0 * per_payment)
    rates = np.array([0.03, 0.0425, 0.05])
    esc = np.where(rng.uniform(size=n) < 0.05, rates[rng.integers(0, 3, n)], 0.0)
    anniv = rng.integers(1, 13, n).astype(np.int32)
    return Portfolio(product=product, age1_m=age1, age2_m=age2, term_m=term, table1=table1,
                     table2=table2, timing=np.full(n, ARREARS, np.int32), amount=amount,
                     premium=np.zeros(n), escalation=esc, anniv_m=anniv, annual=annual)


def config_rep(seed: int = 1006, n: int = 500_000, n_scen: int = 1000,
               scen_seed: int = 2006) -> Workload:
    """The representative 500,000-annuity portfolio x Vasicek inner scenarios
    over the 756 monthly steps to the limiting age."""
    rng = np.random.default_rng(seed)
    pf = portfolio_representative(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, REP_LOADINGS)
    srng = np.random.default_rng(scen_seed)
    v, _ = vasicek_paths(srng, n_scen, REP_N_STEPS, VAS_R0)
    return Workload(f"representative portfolio: {n:,} annuities (Table 2 mix, 5 % escalating, "
                    f"20 % annual) x {n_scen:,} Vasicek scenarios, 756 monthly steps",
                    Basis(q=q, v=v[None]), pf)


def outer_path(rng, n_nodes: int, node_step_m: int = 12):
    """One outer Vasicek path observed every node_step_m months: r at nodes."""
    _, r = vasicek_paths(rng, 1, n_nodes * node_step_m, VAS_R0)
    return r[0, ::node_step_m][:n_nodes].copy()


def config_c4(seed: int = 1004, n: int = 10_000, n_nodes: int = 60,
              n_inner: int = 500, scen_seed: int = 2004,
              shock_seed: int = 3004, n_steps: int = 600,
              node_step_m: int = 12) -> Workload:
    """Full nested valuation: one outer path, annual nodes, inner Vasicek
    scenarios from each node's short rate, a mortality shock per node."""
    rng = np.random.default_rng(seed)
    pf = portfolio_mixed(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, C2_LOADINGS)
    srng = np.random.default_rng(scen_seed)
    r_nodes = outer_path(srng, n_nodes, node_step_m)
    v = np.empty((n_nodes, n_inner, n_steps))
    for k in range(n_nodes):
        v[k], _ = vasicek_paths(srng, n_inner, n_steps, r_nodes[k])
    shock = np.random.default_rng(shock_seed).normal(1.0, 0.05, n_nodes)
    return Workload(f"C4: {n:,} mixed policies x {n_nodes} annual nodes x {n_inner} inner Vasicek scenarios",
                    Basis(q=q, v=v, shock=shock), pf, node_step_m=node_step_m,
                    note=f"outer short rates {r_nodes[:3]}...")


def random_small(rng, n: int, n_steps: int, n_scen: int = 1, n_nodes: int = 1,
                 products=tuple(range(N_PRODUCTS)), n_tables: int = 2,
                 random_q: bool = True, shock: bool = False) -> Workload:
    """Small random case for parity: random q tables and random v."""
    age_hi = 900
    n_ages = age_hi + n_steps + 1
    if random_q:
        q = rng.uniform(0.0, 0.08, (n_tables, n_ages))
        q[:, rng.integers(0, n_ages, 5)] = 0.0
    else:
        q = mortality_tables(n_ages, [1.0 + 0.1 * i for i in range(n_tables)])
    v = rng.uniform(0.990, 1.0005, (n_nodes, n_scen, n_steps))
    product = rng.choice(np.asarray(products, np.int32), n).astype(np.int32)
    age1 = rng.integers(0, age_hi, n).astype(np.int32)
    age2 = rng.integers(0, age_hi, n).astype(np.int32)
    term = rng.integers(1, n_steps, n, endpoint=True).astype(np.int32)
    t1 = rng.integers(0, n_tables, n).astype(np.int32)
    t2 = rng.integers(0, n_tables, n).astype(np.int32)
    timing = rng.integers(0, 2, n).astype(np.int32)
    amount = rng.uniform(0.5, 2.0, n) * 1000.0
    premium = rng.uniform(0.0, 5.0, n)
    sh = rng.normal(1.0, 0.2, n_nodes) if shock else None
    pf = Portfolio(product=product, age1_m=age1, age2_m=age2, term_m=term,
                   table1=t1, table2=t2, timing=timing, amount=amount,
                   premium=premium)
    if any(p in THREE_LIFE for p in products):
        pf.age3_m = rng.integers(0, age_hi, n).astype(np.int32)
        pf.table3 = rng.integers(0, n_tables, n).astype(np.int32)
    return Workload("random small", Basis(q=q, v=v, shock=sh), pf)


# ----------------------------------------------------------------------------
# Surrogate inputs
# ----------------------------------------------------------------------------
def surrogate_training_workload(seed: int = 1005, n: int = 5000, n_nodes: int = 20,
                                n_scen: int = 100, n_steps: int = 600,
                                shock_sd: float = 0.05, horizon_y: float = 60.0) -> Workload:
    """Training inputs for the reserve surrogate: C2-law policies; each node is
    an independent draw of an inner short rate from the outer Vasicek law at a
    uniform horizon in [0, horizon_y] years, a mortality shock N(1, shock_sd)
    and n_scen inner scenarios from that rate.  Nodes share the valuation date
    (use node_step_m = 0)."""
    rng = np.random.default_rng(seed)
    pf = portfolio_mixed(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, C2_LOADINGS)
    T = rng.uniform(0.0, horizon_y, n_nodes)
    m = VAS_B + (VAS_R0 - VAS_B) * np.exp(-VAS_A * T)
    sd = VAS_SIGMA * np.sqrt((1.0 - np.exp(-2.0 * VAS_A * T)) / (2.0 * VAS_A))
    r0 = m + sd * rng.standard_normal(n_nodes)
    v = np.empty((n_nodes, n_scen, n_steps))
    for k in range(n_nodes):
        v[k], _ = vasicek_paths(rng, n_scen, n_steps, r0[k])
    shock = rng.normal(1.0, shock_sd, n_nodes)
    return Workload(f"surrogate training: {n:,} C2-law policies x {n_nodes} nodes x {n_scen} scenarios",
                    Basis(q=q, v=v, shock=shock), pf, node_step_m=0,
                    note=f"node short rates {np.round(r0[:4], 4)}...")


def node_training_workload(seed: int = 1007, n: int = 5000, n_nodes: int = 120,
                           node_step_m: int = 6, n_scen: int = 32, n_steps: int = 600,
                           shock_sd: float = 0.05) -> Workload:
    """Training inputs for the node-level surrogate: C2-law policies at nodes
    node_step_m months apart (policies age and terms shorten with the node);
    node k draws its own inner short rate from the outer Vasicek law at its
    horizon, a mortality shock N(1, shock_sd) and n_scen inner scenarios, so
    the rate is not tied to the node's time."""
    rng = np.random.default_rng(seed)
    pf = portfolio_mixed(rng, n)
    q = mortality_tables(max_attained_age(pf) + 1, C2_LOADINGS)
    T = np.arange(n_nodes) * node_step_m / 12.0
    m = VAS_B + (VAS_R0 - VAS_B) * np.exp(-VAS_A * T)
    sd = VAS_SIGMA * np.sqrt((1.0 - np.exp(-2.0 * VAS_A * T)) / (2.0 * VAS_A))
    r0 = m + sd * rng.standard_normal(n_nodes)
    v = np.empty((n_nodes, n_scen, n_steps))
    for k in range(n_nodes):
        v[k], _ = vasicek_paths(rng, n_scen, n_steps, r0[k])
    shock = rng.normal(1.0, shock_sd, n_nodes)
    return Workload(f"node-level surrogate training: {n:,} C2-law policies x {n_nodes} nodes "
                    f"({node_step_m} months apart) x {n_scen} scenarios",
                    Basis(q=q, v=v, shock=shock), pf, node_step_m=node_step_m)


def random_mlp_params(rng, n_feat: int = 17, k_in: int = 32, hidden: int = 256,
                      bias_sd: float = 0.1) -> dict:
    """Random surrogate weights: W1 [k_in][hidden] (rows >= n_feat zero),
    b1, W2 [hidden][hidden], b2, W3 [hidden], b3 (FP32)."""
    W1 = np.zeros((k_in, hidden), np.float32)
    W1[:n_feat] = rng.normal(0.0, 1.0 / np.sqrt(n_feat), (n_feat, hidden))
    return {"W1": W1,
            "b1": rng.normal(0.0, bias_sd, hidden).astype(np.float32),
            "W2": rng.normal(0.0, 1.0 / np.sqrt(hidden), (hidden, hidden)).astype(np.float32),
            "b2": rng.normal(0.0, bias_sd, hidden).astype(np.float32),
            "W3": rng.normal(0.0, 1.0 / np.sqrt(hidden), hidden).astype(np.float32),
            "b3": np.float32(rng.normal(0.0, bias_sd))}


def with_cash_flow_tables(rng, pf: Portfolio, frac: float = 0.3, n_rows: int = 5,
                          cf_len: int | None = None) -> Portfolio:
    """Copy of pf in which a share `frac` of the policies become CF_TABLE
    policies (one life: table1, age1) drawing on `n_rows` random tables of
    cash flows per unit amount: some rows level, some increasing, some with
    a single lump, some signed."""
    n = pf.n
    out = pf.subset(np.arange(n))
    L = int(pf.term_m.max()) if cf_len is None else cf_len
    t = np.arange(L)
    shapes = [np.full(L, 1.0 / 12.0), (1.0 + t) / 12.0, np.where(t == L // 2, 5.0, 0.0),
              rng.uniform(-0.2, 1.0, L), np.where(t % 12 == 11, 1.0, 0.0)]
    cf = np.stack([shapes[r % len(shapes)] * rng.uniform(0.5, 2.0) for r in range(n_rows)])
    pick = rng.uniform(size=n) < frac
    out.product = np.where(pick, CF_TABLE, pf.product).astype(np.int32)
    out.cf_row = rng.integers(0, n_rows, n).astype(np.int32)
    out.cf = cf
    out.age2_m = np.where(pick, 0, pf.age2_m).astype(np.int32)
    return out


def phi_models(n_ages: int, loadings=(1.0, 1.3), recovery: float = 0.08,
               incidence_scale: float = 0.3) -> tuple:
    """Permanent-health-insurance models (Sec. 4.5: a reversible state model,
    not upper triangular): states healthy, sick, dead; monthly sickness
    incidence proportional to the GM death probability, recovery at a fixed
    monthly rate, sick lives dying at twice the healthy rate; benefit
    1/12 of the amount for each month ending sick.  One model per loading."""
    q = mortality_tables(n_ages, loadings)
    w = np.zeros((len(loadings), n_ages, 3, 3))
    for m in range(len(loadings)):
        qh = q[m]
        inc = np.minimum(incidence_scale * np.sqrt(qh), 0.5)
        qs = np.minimum(2.0 * qh, 1.0)
        w[m, :, 0, 2] = qh
        w[m, :, 0, 1] = (1.0 - qh) * inc
        w[m, :, 0, 0] = 1.0 - qh - (1.0 - qh) * inc
        w[m, :, 1, 2] = qs
        w[m, :, 1, 0] = (1.0 - qs) * recovery
        w[m, :, 1, 1] = 1.0 - qs - (1.0 - qs) * recovery
        w[m, :, 2, 2] = 1.0
    c = np.tile(np.array([0.0, 1.0 / 12.0, 0.0]), (len(loadings), 1))
    return w, c


def with_markov_policies(rng, pf: Portfolio, models: tuple, frac: float = 0.3) -> Portfolio:
    """Copy of pf in which a share `frac` of the policies become MARKOV
    policies on `models` (table1 drawn among the models), keeping their age,
    term, amount and premium."""
    out = pf.subset(np.arange(pf.n))
    pick = rng.uniform(size=pf.n) < frac
    out.product = np.where(pick, MARKOV, pf.product).astype(np.int32)
    out.table1 = np.where(pick, rng.integers(0, models[0].shape[0], pf.n), pf.table1).astype(np.int32)
    out.age2_m = np.where(pick, 0, pf.age2_m).astype(np.int32)
    if out.escalation is not None:            # payment patterns are for annuities only
        out.escalation = np.where(pick, 0.0, out.escalation)
    if out.annual is not None:
        out.annual = np.where(pick, 0, out.annual).astype(np.int32)
    out.markov = models
    return out


def with_payment_patterns(rng, pf: Portfolio, frac_escalating: float = 0.5,
                          frac_annual: float = 0.5,
                          rates=(0.03, 0.0425, 0.05)) -> Portfolio:
    """Copy of pf whose annuities get random payment patterns: an anniversary
    month U{1..12}, escalation at one of `rates` for frac_escalating of them
    and annual payment for frac_annual; escalating or annual annuities carry
    no premium (single-premium annuities)."""
    n = pf.n
    out = pf.subset(np.arange(n))
    is_ann = np.isin(pf.product, (SL_ANN, JL_ANN, REV_ANN, LS_ANN))
    esc = np.where(is_ann & (rng.uniform(size=n) < frac_escalating),
                   np.asarray(rates)[rng.integers(0, len(rates), n)], 0.0)
    annual = (is_ann & (rng.uniform(size=n) < frac_annual)).astype(np.int32)
    out.escalation = esc.astype(np.float64)
    out.anniv_m = rng.integers(1, 13, n).astype(np.int32)
    out.annual = annual
    out.premium = np.where((esc > 0) | (annual == 1), 0.0, pf.premium)
    return out
