"""GPU parity for annuity payment patterns (escalation on policy
anniversaries, annual payment) and the representative annuity portfolio
(Sec. 5.3, Table 2), through the C ABI against the CPU oracle.

Same bar as the level products: FP64 reserves within 1e-10 of max(|r|,
gross PV) per valuation and totals within 1e-10 of the summed gross PV.
The representative portfolio at its full size (500,000 annuities x 1,000
Vasicek scenarios x 756 steps) is checked on sampled outputs in the launch
configuration the benchmark times."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import RTOL, assert_reserves_close, assert_states_close, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ANNUITIES = (synth.SL_ANN, synth.JL_ANN, synth.REV_ANN, synth.LS_ANN)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_1757_amd as rr
    return rr


@pytest.fixture()
def ctx(rr):
    c = rr.Context(0)
    yield c
    c.close()


def patterned_workload(seed, n, n_steps, n_scen, n_nodes, products=tuple(range(7)), node_step=7):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True,
                           products=products)
    pf = synth.with_payment_patterns(rng, w.portfolio, 0.5, 0.4)
    return synth.Workload("patterned", w.basis, pf, node_step_m=node_step)


def compare(ctx, w, all_states=True, node0=0, nnode=None, scen0=0, nscen=None):
    b, pf = w.basis, w.portfolio
    nnode = b.n_nodes - node0 if nnode is None else nnode
    nscen = b.n_scen - scen0 if nscen is None else nscen
    out = ctx.alloc_outputs(nnode, nscen, all_states=all_states)
    ctx.reserve_recurrence(node0, nnode, scen0, nscen, w.node_step_m, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(b, pf, node0, nnode, scen0, nscen, w.node_step_m)
    if all_states:
        assert_states_close(to_np(out["r0"]), ref["r_all"], ref["gross"])
    else:
        assert_reserves_close(to_np(out["r0"]), ref["r_all"][..., 0], ref["gross"])
    err = np.abs(to_np(out["totals"]) - ref["totals"])
    assert np.all(err <= RTOL * np.maximum(ref["gross_totals"], 1e-300)), err.max()
    return out, ref


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (32, 1), (4, 2),
                                 (8, 2), (16, 2), (2, 4), (4, 4), (8, 4), (16, 4)])
def test_patterns_mixed_with_level_policies(ctx, K, J):
    """Every product; half the annuities escalate, 40 % pay annually; three
    nodes 7 months apart with shocks; ragged tiles and scenario blocks."""
    w = patterned_workload(500 + K + 7 * J, n=400, n_steps=100, n_scen=2 * K + 3, n_nodes=3)
    assert (w.portfolio.escalation > 0).sum() > 20 and w.portfolio.annual.sum() > 20
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(1, K)
    ctx.set_option(8, J)
    _say(f"patterns K={K} J={J}")
    compare(ctx, w)


@pytest.mark.parametrize("product", ANNUITIES)
def test_patterns_each_annuity_all_states(ctx, product):
    w = patterned_workload(600 + product, n=150, n_steps=200, n_scen=9, n_nodes=2,
                           products=(product,), node_step=12)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    _say(f"patterns product {product}")
    compare(ctx, w)


def test_pattern_paths(ctx):
    """Reserve at every step for one node and scenario (K = 1 path mode)."""
    w = patterned_workload(700, n=120, n_steps=150, n_scen=3, n_nodes=2, products=ANNUITIES,
                           node_step=12)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("pattern paths")
    for node, scen in ((0, 0), (1, 2)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))        # every entry must be written
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_level_patterns_bitwise_equal_plain(ctx):
    """Anniversaries on level policies change nothing: same tiles, same bits."""
    rng = np.random.default_rng(710)
    w = synth.random_small(rng, n=300, n_steps=90, n_scen=17, n_nodes=2, shock=True)
    b, pf = w.basis, w.portfolio
    lv = pf.subset(np.arange(pf.n))
    lv.escalation = np.zeros(pf.n)
    lv.anniv_m = rng.integers(1, 13, pf.n).astype(np.int32)
    lv.annual = np.zeros(pf.n, np.int32)
    ctx.basis_upload(b.q, b.v, b.shock)
    res = []
    for p in (pf, lv):
        ctx.portfolio_upload(p)
        out = ctx.alloc_outputs(2, b.n_scen, all_states=True)
        ctx.reserve_recurrence(0, 2, 0, b.n_scen, 12, out)
        torch.cuda.synchronize()
        res.append((to_np(out["r0"]), to_np(out["totals"])))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])


def test_representative_portfolio_small_all_steps(ctx):
    """3,000 policies of the Sec. 5.3 law, 24 Vasicek scenarios, every
    output checked (756 monthly steps to the limiting age)."""
    w = synth.config_rep(n=3000, n_scen=24)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    _say("representative 3,000 x 24")
    compare(ctx, w)


def test_representative_portfolio_full_size_sampled(ctx):
    """500,000 annuities x 1,000 scenarios in the benchmark's launch
    configuration (autotuned, totals and the tail statistic): two scenario
    totals over the whole portfolio and sampled reserves against the oracle."""
    import os
    threads = int(os.environ.get("ORACLE_THREADS", min(os.cpu_count() or 1, 16)))
    w = synth.config_rep()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("representative 500,000 x 1,000")
    out = ctx.alloc_outputs(1, b.n_scen, r0=False, stats=True)
    ctx.reserve_recurrence(0, 1, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    tot = to_np(out["totals"])[0]
    st = to_np(out["stats"])[0]
    k = int(np.ceil(0.005 * b.n_scen))
    assert st[1] == np.sort(tot)[::-1][k - 1]
    for s in (0, 777):
        _say(f"  oracle total of scenario {s}")
        ref = oracle.reserves(b, pf, 0, 1, s, 1, 12, n_threads=threads)
        assert abs(tot[s] - ref["totals"][0, 0]) <= RTOL * ref["gross_totals"][0, 0]
    # sampled reserves in a window of scenarios (r0 written)
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(pf.n, 400, replace=False))
    win = ctx.alloc_outputs(1, 8, all_states=True)
    ctx.reserve_recurrence(0, 1, 500, 8, 12, win)
    torch.cuda.synchronize()
    got = to_np(win["r0"])[:, idx]
    ref = oracle.reserves(b, pf.subset(idx), 0, 1, 500, 8, 12, n_threads=threads)
    assert_states_close(got, ref["r_all"], ref["gross"])


# ---------------------------------------------------------------------------
# Cash-flow tables (RR_CF_TABLE), alone and beside pattern and level tiles
# ---------------------------------------------------------------------------
def table_workload(seed, n, n_steps, n_scen, n_nodes, node_step=7, frac=0.3):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True)
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=frac, n_rows=7)
    pf = synth.with_payment_patterns(rng, pf, 0.4, 0.3)
    return synth.Workload("tables", w.basis, pf, node_step_m=node_step)


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (32, 1), (4, 2),
                                 (8, 2), (16, 2), (2, 4), (4, 4), (8, 4), (16, 4)])
def test_cash_flow_tables_with_patterns_and_level(ctx, K, J):
    w = table_workload(800 + K + 7 * J, n=420, n_steps=100, n_scen=2 * K + 5, n_nodes=3)
    assert (w.portfolio.product == synth.CF_TABLE).sum() > 80
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(1, K)
    ctx.set_option(8, J)
    _say(f"tables K={K} J={J}")
    compare(ctx, w)


def test_cash_flow_table_paths(ctx):
    w = table_workload(900, n=150, n_steps=160, n_scen=3, n_nodes=2, node_step=12, frac=0.5)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("table paths")
    for node, scen in ((0, 1), (1, 2)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_cash_flow_tables_only_full_steps(ctx):
    """A portfolio of table policies only (600-month tables, 200 policies
    spanning four tiles and a ragged tail), every output against the oracle."""
    rng = np.random.default_rng(901)
    w = synth.random_small(rng, n=200, n_steps=600, n_scen=9, n_nodes=1, products=(0,))
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=1.0, n_rows=11, cf_len=600)
    w = synth.Workload("tables only", w.basis, pf)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(pf)
    _say("tables only")
    compare(ctx, w)


# ---------------------------------------------------------------------------
# Two-life endowment and first/second-death assurances (Sec. 4.2.2, 4.2.3)
# ---------------------------------------------------------------------------
TWO_LIFE_INS = (synth.JL_ENDOW, synth.JL_ASSUR1, synth.JL_ASSUR2)


@pytest.mark.parametrize("product", TWO_LIFE_INS)
def test_two_life_insurance_all_states(ctx, product):
    rng = np.random.default_rng(1000 + product)
    w = synth.random_small(rng, n=200, n_steps=150, n_scen=11, n_nodes=2, shock=True,
                           products=(product,))
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    _say(f"two-life product {product}")
    compare(ctx, w)


@pytest.mark.parametrize("K,J", [(1, 1), (4, 1), (16, 1), (32, 1), (8, 2), (16, 2), (2, 4), (8, 4),
                                 (16, 4)])
def test_every_product_together(ctx, K, J):
    """All eleven products, payment patterns and cash-flow tables in one
    portfolio, three nodes with shocks."""
    rng = np.random.default_rng(1100 + K + 7 * J)
    w = synth.random_small(rng, n=600, n_steps=90, n_scen=2 * K + 1, n_nodes=3, shock=True,
                           products=tuple(range(7)) + TWO_LIFE_INS)
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.1, n_rows=4)
    pf = synth.with_payment_patterns(rng, pf, 0.5, 0.3)
    w = synth.Workload("all products", w.basis, pf, node_step_m=7)
    assert set(np.unique(pf.product)) == set(range(11))
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(pf)
    ctx.set_option(1, K)
    ctx.set_option(8, J)
    _say(f"every product K={K} J={J}")
    compare(ctx, w)


def test_two_life_insurance_paths(ctx):
    rng = np.random.default_rng(1200)
    w = synth.random_small(rng, n=90, n_steps=140, n_scen=2, n_nodes=2, shock=True,
                           products=TWO_LIFE_INS)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("two-life insurance paths")
    for node, scen in ((0, 0), (1, 1)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


# ---------------------------------------------------------------------------
# Policies on uploaded Markov models (Sec. 4.5)
# ---------------------------------------------------------------------------
def markov_workload(seed, n, n_steps, n_scen, n_nodes, models=None, frac=0.4, node_step=7):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True,
                           products=tuple(range(7)) + TWO_LIFE_INS)
    n_ages = w.basis.q.shape[1]
    if models is None:
        models = synth.phi_models(n_ages)
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.1, n_rows=3)
    pf = synth.with_payment_patterns(rng, pf, 0.4, 0.3)
    pf = synth.with_markov_policies(rng, pf, models, frac=frac)
    return synth.Workload("markov", w.basis, pf, node_step_m=node_step)


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (8, 1), (16, 1), (32, 1), (8, 2), (4, 4), (16, 4)])
def test_markov_policies_with_every_other_kind(ctx, K, J):
    w = markov_workload(1300 + K + 7 * J, n=500, n_steps=90, n_scen=2 * K + 3, n_nodes=3)
    assert (w.portfolio.product == synth.MARKOV).sum() > 100
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.markov_upload(*w.portfolio.markov)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(1, K)
    ctx.set_option(8, J)
    _say(f"markov K={K} J={J}")
    compare(ctx, w)


def test_random_four_state_models_all_states(ctx):
    rng = np.random.default_rng(1400)
    n_ages = 900 + 120 + 1
    raw = rng.uniform(0.0, 1.0, (3, n_ages, 4, 4))
    raw[:, :, 3, :] = [0.0, 0.0, 0.0, 1.0]
    W = raw / raw.sum(axis=3, keepdims=True)
    c = rng.uniform(-1.0, 2.0, (3, 4))
    w = markov_workload(1401, n=200, n_steps=120, n_scen=9, n_nodes=2, models=(W, c), frac=1.0,
                        node_step=12)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.markov_upload(W, c)
    ctx.portfolio_upload(w.portfolio)
    _say("random 4-state models")
    compare(ctx, w)
    # paths at two nodes
    b, pf = w.basis, w.portfolio
    for node, scen in ((0, 3), (1, 8)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_markov_invalid_uploads(ctx, rr):
    w = markov_workload(1500, n=50, n_steps=60, n_scen=2, n_nodes=1)
    b, pf = w.basis, w.portfolio
    W, c = pf.markov
    ctx.basis_upload(b.q, b.v, b.shock)
    with pytest.raises(rr.RRError, match="need rr_markov_upload"):
        ctx.portfolio_upload(pf)
    bad = W.copy(); bad[0, 5, 1, 0] += 0.01
    with pytest.raises(rr.RRError, match="row 1 sums"):
        ctx.markov_upload(bad, c)
    bad = W.copy(); bad[1, 7, 0, 0] = -0.1; bad[1, 7, 0, 1] += 0.1
    with pytest.raises(rr.RRError, match="not a probability"):
        ctx.markov_upload(bad, c)
    cb = c.copy(); cb[0, 1] = np.nan
    with pytest.raises(rr.RRError, match="benefit"):
        ctx.markov_upload(W, cb)
    with pytest.raises(rr.RRError, match="n_states"):
        ctx.markov_upload(np.zeros((1, 10, 10, 10)), np.zeros((1, 10)))
    ctx.markov_upload(W, c)
    pf2 = pf.subset(np.arange(pf.n))
    i = int(np.flatnonzero(pf2.product == synth.MARKOV)[0])
    pf2.table1[i] = W.shape[0]
    with pytest.raises(rr.RRError, match=f"policy {i} model"):
        ctx.portfolio_upload(pf2)
    ctx.portfolio_upload(pf)
    ctx.markov_upload(W, c)                      # new models: the portfolio is dropped
    out = ctx.alloc_outputs(1, 2)
    with pytest.raises(rr.RRError):
        ctx.reserve_recurrence(0, 1, 0, 2, 12, out)


# ---------------------------------------------------------------------------
# Fractional payment timing (annuities paid at the basis's fraction f)
# ---------------------------------------------------------------------------
def frac_workload(seed, n, n_steps, n_scen, n_nodes, f=0.35, node_step=7):
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True,
                           products=tuple(range(7)) + TWO_LIFE_INS)
    pf = w.portfolio
    ann = np.isin(pf.product, (synth.SL_ANN, synth.JL_ANN))
    pf.timing = np.where(ann & (rng.uniform(size=pf.n) < 0.6), synth.FRACTIONAL, pf.timing).astype(np.int32)
    w.basis.frac = f
    return synth.Workload("fractional", w.basis, pf, node_step_m=node_step)


@pytest.mark.parametrize("K,J", [(1, 1), (4, 1), (16, 1), (32, 1), (8, 2), (16, 4)])
def test_fractional_timing_with_other_products(ctx, K, J):
    w = frac_workload(1600 + K + 7 * J, n=400, n_steps=100, n_scen=2 * K + 3, n_nodes=3)
    assert (w.portfolio.timing == synth.FRACTIONAL).sum() > 20
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock, frac=w.basis.frac)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(1, K)
    ctx.set_option(8, J)
    _say(f"fractional K={K} J={J}")
    compare(ctx, w)


def test_fractional_paths_and_regenerated_curves(ctx):
    w = frac_workload(1700, n=150, n_steps=120, n_scen=2, n_nodes=2, f=0.6, node_step=12)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock, frac=0.6)
    ctx.portfolio_upload(pf)
    _say("fractional paths")
    for node, scen in ((0, 0), (1, 1)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")
    # device-generated curves: v^f follows every regeneration
    A, Bm, Sg, DT = synth.VAS_A, synth.VAS_B, synth.VAS_SIGMA, 1.0 / 12.0
    ctx.basis_generate_vasicek(b.q, 20, b.n_steps, [0.03, 0.05], A, Bm, Sg, DT, (4, 4),
                               shock=b.shock, frac=0.6)
    ctx.portfolio_upload(pf)
    for key, r0 in (((4, 4), [0.03, 0.05]), ((5, 6), [0.02, 0.04])):
        ctx.curves_generate_vasicek(r0, A, Bm, Sg, DT, key)
        ov, _ = oracle.vasicek_curves(A, Bm, Sg, DT, r0, 20, b.n_steps, key)
        gb = synth.Basis(q=b.q, v=ov, shock=b.shock, frac=0.6)
        out = ctx.alloc_outputs(2, 20, all_states=False)
        ctx.reserve_recurrence(0, 2, 0, 20, 12, out)
        torch.cuda.synchronize()
        ref = oracle.reserves(gb, pf, 0, 2, 0, 20, 12)
        assert_reserves_close(to_np(out["r0"]), ref["r_all"][..., 0], ref["gross"])


def test_fractional_invalid(ctx, rr):
    w = frac_workload(1800, n=60, n_steps=60, n_scen=2, n_nodes=1)
    b, pf = w.basis, w.portfolio
    with pytest.raises(rr.RRError, match="frac must be"):
        ctx.basis_upload(b.q, b.v, b.shock, frac=1.0)
    ctx.basis_upload(b.q, b.v, b.shock)                 # no fraction
    with pytest.raises(rr.RRError, match="needs a basis with frac"):
        ctx.portfolio_upload(pf)
    ctx.basis_upload(b.q, b.v, b.shock, frac=0.35)
    bad = pf.subset(np.arange(pf.n))
    i = int(np.flatnonzero(bad.product == synth.TERM)[0])
    bad.timing[i] = synth.FRACTIONAL
    with pytest.raises(rr.RRError, match=f"policy {i}: fractional timing needs"):
        ctx.portfolio_upload(bad)
    ctx.portfolio_upload(pf)
    with pytest.raises(rr.RRError, match="fractional timing"):
        ctx.node_expected_reserves(0, 1, 0, 2, 12)
    ctx.basis_upload(b.q, b.v, b.shock)                 # a basis without the fraction drops it
    out = ctx.alloc_outputs(1, 2)
    with pytest.raises(rr.RRError):
        ctx.reserve_recurrence(0, 1, 0, 2, 12, out)


# ---------------------------------------------------------------------------
# Uploaded models of five to nine states (Sec. 4.5; the 9-state two-life
# model of Sec. 4.2.3 as a table)
# ---------------------------------------------------------------------------
def nine_state_tables(q, gap, benefit):
    """The 9-state two-life assurance model by the attained age x of life 1,
    life 2 being x + gap (Kronecker product of the 3-state life models)."""
    n_ages = q.shape[1] - gap
    W = np.zeros((1, n_ages, 9, 9))
    for x in range(n_ages):
        W[0, x] = oracle.build_w(2, 3, [q[0, x], q[1, x + gap]])
    return W, np.asarray([benefit], np.float64)


@pytest.mark.parametrize("model", [synth.JL_ASSUR1, synth.JL_ASSUR2])
def test_nine_state_upload_equals_two_life_assurance(ctx, model):
    """The same policies as built-in first- or second-death assurances and as
    MARKOV policies on the uploaded 9-state table: equal state-0 reserves
    (1e-13), both against the oracle."""
    rng = np.random.default_rng(1700 + model)
    gap, S, n = 60, 240, 150
    q = synth.mortality_tables(1500, [1.0, 1.3])
    benefit = {synth.JL_ASSUR1: [0, 1, 0, 1, 1, 0, 0, 0, 0],
               synth.JL_ASSUR2: [0, 0, 0, 0, 1, 1, 0, 1, 0]}[model]
    W, c = nine_state_tables(q, gap, benefit)
    ages = rng.integers(300, 1100, n).astype(np.int32)
    common = dict(age1_m=np.concatenate([ages, ages]), age2_m=np.concatenate([ages + gap, ages]),
                  term_m=np.full(2 * n, S, np.int32), table1=np.concatenate([np.zeros(n, np.int32),
                                                                             np.zeros(n, np.int32)]),
                  table2=np.ones(2 * n, np.int32), timing=np.ones(2 * n, np.int32),
                  amount=np.tile(rng.uniform(1e3, 1e5, n), 2), premium=np.tile(rng.uniform(0, 50, n), 2))
    pf = synth.Portfolio(product=np.array([model] * n + [synth.MARKOV] * n, np.int32), **common)
    pf.markov = (W, c)
    v = rng.uniform(0.995, 1.0, (2, 9, S))
    w = synth.Workload("nine states", synth.Basis(q=q, v=v, shock=np.array([1.0, 1.04])), pf)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.markov_upload(W, c)
    ctx.portfolio_upload(pf)
    _say(f"nine-state table vs built-in {model}")
    out = ctx.alloc_outputs(1, 9, all_states=True)
    ctx.reserve_recurrence(0, 1, 0, 9, 12, out)
    torch.cuda.synchronize()
    got = to_np(out["r0"])
    ref = oracle.reserves(w.basis, pf, 0, 1, 0, 9, 12)
    assert_states_close(got, ref["r_all"], ref["gross"])
    built, up = got[0, :n, :, 0], got[0, n:, :, 0]
    scale = np.maximum(np.abs(built), ref["gross"][0, :n])
    assert np.all(np.abs(up - built) <= 1e-13 * scale)


@pytest.mark.parametrize("m,K", [(5, 8), (9, 1), (9, 4), (9, 16), (7, 32)])
def test_large_random_markov_models(ctx, rr, m, K):
    """Random reversible models of m states beside every other kind of
    tile, every state slot, two nodes; paths for K = 1."""
    rng = np.random.default_rng(1800 + m + K)
    n_ages = 900 + 90 + 1
    raw = rng.uniform(0.0, 1.0, (2, n_ages, m, m))
    raw[:, :, m - 1, :] = 0.0
    raw[:, :, m - 1, m - 1] = 1.0
    W = raw / raw.sum(axis=3, keepdims=True)
    c = rng.uniform(-1.0, 2.0, (2, m))
    w = markov_workload(1801 + m, n=400, n_steps=90, n_scen=2 * K + 3, n_nodes=2, models=(W, c),
                        frac=0.3, node_step=12)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.markov_upload(W, c)
    ctx.portfolio_upload(pf)
    ctx.set_option(rr.OPT_BLOCK_K, K)
    _say(f"random {m}-state models K={K}")
    compare(ctx, w)
    if K == 1:
        for node, scen in ((0, 2), (1, 4)):
            po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
            po["path"].fill_(float("nan"))
            ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
            torch.cuda.synchronize()
            path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
            ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
            gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
            assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


# ---------------------------------------------------------------------------
# Three lives (Sec. 4.3)
# ---------------------------------------------------------------------------
THREE = (synth.JL3_ANN, synth.LS3_ANN)


def three_life_workload(seed, n, n_steps, n_scen, n_nodes, node_step=7, products=None):
    rng = np.random.default_rng(seed)
    products = products or THREE + (synth.SL_ANN, synth.JL_ANN, synth.LS_ANN, synth.TERM,
                                     synth.JL_ASSUR2)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True,
                           products=products, n_tables=3)
    pf = synth.with_payment_patterns(rng, w.portfolio, 0.3, 0.2)
    three = np.isin(pf.product, THREE)
    pf.premium = np.where(three & (rng.uniform(size=pf.n) < 0.5), 0.0, pf.premium)
    return synth.Workload("three lives", w.basis, pf, node_step_m=node_step)


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (4, 1), (8, 2), (16, 1), (16, 4), (32, 1)])
def test_three_life_annuities_with_other_kinds(ctx, rr, K, J):
    """Joint-life and last-survivor annuities on three lives (advance and
    arrears, with and without premiums) beside level, patterned and
    two-life tiles; three nodes with shocks, every state slot."""
    w = three_life_workload(1900 + K + 7 * J, n=400, n_steps=90, n_scen=2 * K + 3, n_nodes=3)
    assert np.isin(w.portfolio.product, THREE).sum() > 60
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(rr.OPT_BLOCK_K, K)
    ctx.set_option(rr.OPT_BLOCK_J, J)
    _say(f"three lives K={K} J={J}")
    compare(ctx, w)


def test_three_life_paths_and_long_terms(ctx):
    w = three_life_workload(1990, n=120, n_steps=300, n_scen=3, n_nodes=2, node_step=12,
                            products=THREE)
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("three-life paths")
    compare(ctx, w)
    for node, scen in ((0, 0), (1, 2)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_three_life_invalid(ctx, rr):
    rng = np.random.default_rng(1995)
    w = synth.random_small(rng, n=20, n_steps=50, n_scen=2, products=THREE)
    ctx.basis_upload(w.basis.q, w.basis.v)
    bad = w.portfolio.subset(np.arange(20))
    bad.age3_m = None
    with pytest.raises(rr.RRError, match="age3_m"):
        ctx.portfolio_upload(bad)
    bad = w.portfolio.subset(np.arange(20))
    bad.timing[3] = synth.FRACTIONAL
    with pytest.raises(rr.RRError):
        ctx.portfolio_upload(bad)
    bad = w.portfolio.subset(np.arange(20))
    bad.escalation = np.zeros(20)
    bad.escalation[4] = 0.03
    bad.premium[4] = 0.0
    with pytest.raises(rr.RRError, match="policy 4"):
        ctx.portfolio_upload(bad)
