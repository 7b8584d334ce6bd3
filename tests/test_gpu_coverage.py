"""GPU parity for configurations the other parity tests do not reach.

* Survival tables read from device memory.  A workgroup stages the tables in
  LDS when they fit in 64 KiB (8,192 doubles); bases with more tables or
  longer tables run the kernel instances that read them from device memory
  instead.  These tests use such bases with every product, payment
  patterns, cash-flow tables, uploaded Markov models and fractional timing,
  over every launch shape, and check every valuation against the oracle.
* The full-size nested valuation (10,000 policies x 60 annual nodes x 500
  inner scenarios) in the launch configuration the benchmark times: every
  valuation and every total of three whole nodes against the oracle, and
  those nodes' mean and 1-in-200 statistic against the oracle's own totals.
* The headline workload (10,000 policies x 1,000 scenarios) in full: all
  10^7 valuations, the totals and the statistics against the oracle.
* Every one of the 30,000 totals of the full nested valuation, and every
  node's mean and 1-in-200 total, against the oracle's reduced mode (pinned
  to its dense mode at 1e-13), within 1e-10 of the sum of |r| per total.

Bar: FP64 reserves within 1e-10 of max(|r|, gross PV) per valuation, totals
within 1e-10 of the summed gross PV."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import RTOL, assert_reserves_close, assert_states_close, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TWO_LIFE_INS = (synth.JL_ENDOW, synth.JL_ASSUR1, synth.JL_ASSUR2)
ALL_LIFE_PRODUCTS = tuple(range(7)) + TWO_LIFE_INS
LDS_TABLE_DOUBLES = 8192


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


def compare(ctx, w, all_states=True):
    b, pf = w.basis, w.portfolio
    out = ctx.alloc_outputs(b.n_nodes, b.n_scen, all_states=all_states)
    ctx.reserve_recurrence(0, b.n_nodes, 0, b.n_scen, w.node_step_m, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(b, pf, 0, b.n_nodes, 0, b.n_scen, w.node_step_m)
    if all_states:
        assert_states_close(to_np(out["r0"]), ref["r_all"], ref["gross"])
    else:
        assert_reserves_close(to_np(out["r0"]), ref["r_all"][..., 0], ref["gross"])
    err = np.abs(to_np(out["totals"]) - ref["totals"])
    assert np.all(err <= RTOL * np.maximum(ref["gross_totals"], 1e-300)), err.max()
    return out, ref


def wide_basis_workload(seed, n, n_steps, n_scen, n_nodes, n_tables=10, node_step=7,
                        markov=True, frac=0.0, products=ALL_LIFE_PRODUCTS):
    """Every product on n_tables random tables (more than LDS holds), with
    cash-flow tables, payment patterns and permanent-health Markov policies."""
    rng = np.random.default_rng(seed)
    w = synth.random_small(rng, n=n, n_steps=n_steps, n_scen=n_scen, n_nodes=n_nodes, shock=True,
                           products=products, n_tables=n_tables)
    assert w.basis.q.size > LDS_TABLE_DOUBLES
    pf = synth.with_cash_flow_tables(rng, w.portfolio, frac=0.1, n_rows=4)
    pf = synth.with_payment_patterns(rng, pf, 0.4, 0.3)
    if frac > 0.0:
        level_ann = np.isin(pf.product, (synth.SL_ANN, synth.JL_ANN)) & (pf.escalation == 0) & (pf.annual == 0)
        pick = level_ann & (rng.uniform(size=pf.n) < 0.6)
        pf.timing = np.where(pick, synth.FRACTIONAL, pf.timing).astype(np.int32)
        w.basis.frac = frac
    if markov:
        pf = synth.with_markov_policies(rng, pf, synth.phi_models(w.basis.q.shape[1]), frac=0.15)
    return synth.Workload("wide basis", w.basis, pf, node_step_m=node_step)


def upload(ctx, w):
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock, frac=getattr(b, "frac", 0.0) or 0.0)
    if getattr(pf, "markov", None) is not None:
        ctx.markov_upload(*pf.markov)
    ctx.portfolio_upload(pf)


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (32, 1), (4, 2),
                                 (8, 2), (16, 2), (2, 4), (4, 4), (8, 4), (16, 4)])
def test_tables_in_device_memory_every_kind(ctx, rr, K, J):
    """Ten random tables (over 10,000 doubles): every product, patterns,
    cash-flow tables and Markov tiles over every (K, J) shape."""
    w = wide_basis_workload(2000 + K + 7 * J, n=500, n_steps=90, n_scen=2 * K + 3, n_nodes=3)
    pf = w.portfolio
    assert set(np.unique(pf.product)) == set(range(12))
    upload(ctx, w)
    ctx.set_option(rr.OPT_BLOCK_K, K)
    ctx.set_option(rr.OPT_BLOCK_J, J)
    _say(f"device-memory tables K={K} J={J}")
    compare(ctx, w)
    assert ctx.get_option(rr.OPT_LAST_TABLES_LDS) == 0
    assert ctx.get_option(rr.OPT_LAST_K) == K and ctx.get_option(rr.OPT_LAST_J) == J


def test_tables_in_device_memory_gm_long_terms(ctx, rr):
    """Eight Gompertz-Makeham tables to 1,501 ages (12,008 doubles), terms to
    600 months, autotuned launch; state-0 outputs."""
    rng = np.random.default_rng(2100)
    w = synth.random_small(rng, n=700, n_steps=600, n_scen=20, n_nodes=2, shock=True,
                           products=ALL_LIFE_PRODUCTS, n_tables=8, random_q=False)
    assert w.basis.q.size > LDS_TABLE_DOUBLES
    w = synth.Workload("gm tables", w.basis, w.portfolio, node_step_m=12)
    upload(ctx, w)
    _say("device-memory GM tables, 600 steps")
    compare(ctx, w, all_states=False)
    assert ctx.get_option(rr.OPT_LAST_TABLES_LDS) == 0


def test_tables_in_device_memory_fractional(ctx, rr):
    w = wide_basis_workload(2200, n=600, n_steps=100, n_scen=19, n_nodes=2, frac=0.37, markov=False,
                            products=tuple(range(7)))
    assert (w.portfolio.timing == synth.FRACTIONAL).sum() > 20
    upload(ctx, w)
    ctx.set_option(rr.OPT_BLOCK_K, 8)
    _say("device-memory tables, fractional timing")
    compare(ctx, w)
    assert ctx.get_option(rr.OPT_LAST_TABLES_LDS) == 0


@pytest.mark.parametrize("K,J", [(16, 1), (16, 2), (8, 2)])
def test_tables_in_device_memory_curve_ring(ctx, rr, K, J):
    """The curve-ring instances with the tables in device memory (level
    single- and joint-life annuities)."""
    rng = np.random.default_rng(2300 + K + J)
    w = synth.random_small(rng, n=400, n_steps=80, n_scen=2 * K + 5, n_nodes=2, shock=True,
                           products=(synth.SL_ANN, synth.JL_ANN), n_tables=12)
    upload(ctx, w)
    ctx.set_option(rr.OPT_BLOCK_K, K)
    ctx.set_option(rr.OPT_BLOCK_J, J)
    ctx.set_option(rr.OPT_WG_PER_CU, 1)
    ctx.set_option(rr.OPT_CURVE_RING, 1)
    _say(f"device-memory tables, curve ring K={K} J={J}")
    compare(ctx, w)
    assert ctx.get_option(rr.OPT_LAST_RING) == 1
    assert ctx.get_option(rr.OPT_LAST_TABLES_LDS) == 0


def test_tables_in_device_memory_paths(ctx, rr):
    w = wide_basis_workload(2400, n=150, n_steps=120, n_scen=3, n_nodes=2, node_step=12)
    b, pf = w.basis, w.portfolio
    upload(ctx, w)
    _say("device-memory tables, paths")
    for node, scen in ((0, 1), (1, 2)):
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=node, node_step=12)
        po["path"].fill_(float("nan"))
        ctx.reserve_recurrence(node, 1, scen, 1, 12, po)
        torch.cuda.synchronize()
        assert ctx.get_option(rr.OPT_LAST_TABLES_LDS) == 0
        path, off = oracle.reserve_paths(b, pf, node=node, scen=scen, node_step=12)
        ref = oracle.reserves(b, pf, node, 1, scen, 1, 12)
        gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
        assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_c4_full_size_three_nodes_every_valuation(ctx, rr):
    """10,000 mixed policies x 60 annual nodes x 500 inner scenarios, one
    autotuned launch with r0, totals and statistics (the benchmark's
    outputs plus r0).  Nodes 0, 29 and 47 are checked whole against the
    oracle: every valuation, every total, the mean and the 1-in-200 total."""
    w = synth.config_c4()
    b, pf = w.basis, w.portfolio
    upload(ctx, w)
    out = ctx.alloc_outputs(b.n_nodes, b.n_scen, stats=True)
    _say("C4 full size with r0")
    ctx.reserve_recurrence(0, b.n_nodes, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    stats = to_np(out["stats"])
    tot = to_np(out["totals"])
    for node in (0, 29, 47):
        live = int((pf.term_m - 12 * node > 0).sum())
        _say(f"  node {node}: {live} live policies x {b.n_scen} scenarios")
        ref = oracle.reserves(b, pf, node, 1, 0, b.n_scen, 12)
        got = to_np(out["r0"][node:node + 1])
        assert_reserves_close(got, ref["r_all"][..., 0], ref["gross"])
        err = np.abs(tot[node:node + 1] - ref["totals"])
        assert np.all(err <= RTOL * np.maximum(ref["gross_totals"], 1e-300)), err.max()
        mean, q = oracle.node_stats(ref["totals"])
        gsum = float(ref["gross_totals"].mean())
        assert abs(stats[node, 0] - mean[0]) <= RTOL * gsum, (stats[node, 0], mean[0])
        assert abs(stats[node, 1] - q[0]) <= RTOL * float(ref["gross_totals"].max()), (stats[node, 1], q[0])
        assert live > 0


def test_c3_full_size_every_valuation(ctx, rr):
    """The headline workload in the benchmark's launch configuration
    (autotuned, r0 + totals + statistics): all 10,000 x 1,000 valuations,
    every total and the 1-in-200 total against the oracle."""
    w = synth.config_c3()
    b, pf = w.basis, w.portfolio
    upload(ctx, w)
    out = ctx.alloc_outputs(1, b.n_scen, stats=True)
    _say("C3 full size, every valuation")
    ctx.reserve_recurrence(0, 1, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(b, pf, 0, 1, 0, b.n_scen, 12)
    assert_reserves_close(to_np(out["r0"]), ref["r_all"][..., 0], ref["gross"])
    err = np.abs(to_np(out["totals"]) - ref["totals"])
    assert np.all(err <= RTOL * ref["gross_totals"]), err.max()
    mean, q = oracle.node_stats(ref["totals"])
    st = to_np(out["stats"])[0]
    gsum = float(ref["gross_totals"].max())
    assert abs(st[0] - mean[0]) <= RTOL * gsum and abs(st[1] - q[0]) <= RTOL * gsum


def test_c4_full_size_every_total(ctx, rr):
    w = synth.config_c4()
    b, pf = w.basis, w.portfolio
    upload(ctx, w)
    out = ctx.alloc_outputs(b.n_nodes, b.n_scen, r0=False, stats=True)
    _say("C4 full size, every total")
    ctx.reserve_recurrence(0, b.n_nodes, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    red = oracle.reserves_reduced(b, pf, 0, b.n_nodes, 0, b.n_scen, 12, want_r=False)
    tot = to_np(out["totals"])
    scale = red["abs_totals"]
    live = scale > 0
    assert np.all(tot[~live] == 0.0)
    err = np.abs(tot - red["totals"])
    assert np.all(err[live] <= RTOL * scale[live]), float((err[live] / scale[live]).max())
    mean, q = oracle.node_stats(red["totals"])
    st = to_np(out["stats"])
    smax = scale.max(axis=1)
    assert np.all(np.abs(st[:, 0] - mean) <= RTOL * smax + 0.0)
    assert np.all(np.abs(st[:, 1] - q) <= RTOL * smax + 0.0)
