"""GPU parity: the HIP recurrence (through the C ABI) against the CPU oracle.

FP64 reserves must agree within 1e-10 of max(|r|, gross PV) per valuation and
within 1e-10 of the summed gross PV for portfolio totals.  Sizes span several
tiles of 64 policies with a ragged last tile, several scenario blocks with a
ragged last block, several nodes with mortality shocks; the full-size
configurations are checked on sampled outputs."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import RTOL, assert_reserves_close, assert_states_close, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def run_and_compare(ctx, w, node0=0, nnode=None, scen0=0, nscen=None, K=None, all_states=True,
                    check_totals=True):
    b, pf = w.basis, w.portfolio
    nnode = b.n_nodes - node0 if nnode is None else nnode
    nscen = b.n_scen - scen0 if nscen is None else nscen
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    if K is not None:
        ctx.set_option(1, K)
    out = ctx.alloc_outputs(nnode, nscen, all_states=all_states)
    ctx.reserve_recurrence(node0, nnode, scen0, nscen, w.node_step_m, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(b, pf, node0, nnode, scen0, nscen, w.node_step_m)
    g = to_np(out["r0"])
    gross = ref["gross"]
    if all_states:
        assert_states_close(g, ref["r_all"], gross)
    else:
        assert_reserves_close(g, ref["r_all"][..., 0], gross)
    if check_totals:
        tol = RTOL * np.maximum(ref["gross_totals"], 1e-300)
        err = np.abs(to_np(out["totals"]) - ref["totals"])
        assert np.all(err <= tol), (err.max(), tol.min())
    return out, ref


@pytest.mark.parametrize("K,J", [(1, 1), (2, 1), (4, 1), (8, 1), (16, 1), (32, 1), (4, 2),
                                 (8, 2), (16, 2), (2, 4), (4, 4), (8, 4)])
def test_all_products_random_small(ctx, K, J):
    rng = np.random.default_rng(100 + K + 7 * J)
    w = synth.random_small(rng, n=450, n_steps=90, n_scen=37, n_nodes=3, shock=True)
    ctx.set_option(8, J)
    _say(f"random small K={K} J={J}")
    run_and_compare(ctx, w, K=K)


@pytest.mark.parametrize("K,J", [(2, 1), (4, 1), (8, 1), (16, 1), (4, 2), (8, 2), (16, 2), (2, 4),
                                 (4, 4), (8, 4), (16, 4)])
def test_even_scenario_count_state0_rows(ctx, K, J):
    """State-0 outputs only, an even scenario count with a ragged last block."""
    rng = np.random.default_rng(300 + K + 7 * J)
    w = synth.random_small(rng, n=333, n_steps=80, n_scen=2 * K + 6 if K > 2 else 10, n_nodes=2,
                           shock=True)
    ctx.set_option(8, J)
    _say(f"even scenarios K={K} J={J}")
    run_and_compare(ctx, w, K=K, all_states=False)


@pytest.mark.parametrize("product", list(range(7)))
def test_each_product_with_gm_tables(ctx, product):
    rng = np.random.default_rng(product)
    w = synth.random_small(rng, n=130, n_steps=240, n_scen=5, n_nodes=2,
                           products=(product,), random_q=False, shock=True)
    _say(f"product {product}")
    run_and_compare(ctx, w)


def test_scenario_and_node_windows(ctx):
    rng = np.random.default_rng(5)
    w = synth.random_small(rng, n=200, n_steps=72, n_scen=70, n_nodes=5, shock=True)
    _say("windows")
    run_and_compare(ctx, w, node0=2, nnode=2, scen0=13, nscen=41, K=16)
    run_and_compare(ctx, w, node0=4, nnode=1, scen0=69, nscen=1, K=32)


def test_c1_full_with_path(ctx, rr):
    w = synth.config_c1()
    _say("C1 full")
    out, ref = run_and_compare(ctx, w, all_states=False)
    po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=0)
    ctx.reserve_recurrence(0, 1, 0, 1, 12, po)
    torch.cuda.synchronize()
    path, off = oracle.reserve_paths(w.basis, w.portfolio)
    gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
    assert_reserves_close(to_np(po["path"]), path, np.maximum(gross, 0), what="path")


def test_path_at_a_later_node_with_expired_policies(ctx):
    """Path mode at node 2 (24 months on): expired policies own one entry,
    which must be written as 0; the buffer starts as NaN."""
    rng = np.random.default_rng(77)
    w = synth.random_small(rng, n=200, n_steps=60, n_scen=2, n_nodes=3, shock=True)
    b, pf = w.basis, w.portfolio
    assert (pf.term_m <= 24).sum() > 20
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("path at node 2")
    po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=2, node_step=12)
    po["path"].fill_(float("nan"))
    ctx.reserve_recurrence(2, 1, 1, 1, 12, po)
    torch.cuda.synchronize()
    path, off = oracle.reserve_paths(b, pf, node=2, scen=1, node_step=12)
    ref = oracle.reserves(b, pf, 2, 1, 1, 1, 12)
    gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
    got = to_np(po["path"])
    assert not np.isnan(got).any()
    assert_reserves_close(got, path, np.maximum(gross, 0), what="path")


def test_path_every_term_1_to_80(ctx):
    """Path mode with every term from 1 to 80 months across all products:
    the kernel writes paths out in aligned blocks of 16 steps, so this
    covers blocks that are partial at the top, that end exactly at S and
    that hold one step.  The buffer starts as NaN; every entry must match."""
    rng = np.random.default_rng(91)
    w = synth.random_small(rng, n=1280, n_steps=80, n_scen=2, n_nodes=1, shock=True)
    b, pf = w.basis, w.portfolio
    pf.term_m[:] = (np.arange(len(pf.term_m)) % 80 + 1).astype(np.int32)
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("path, terms 1..80")
    po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=0)
    po["path"].fill_(float("nan"))
    ctx.reserve_recurrence(0, 1, 1, 1, 12, po)
    torch.cuda.synchronize()
    path, off = oracle.reserve_paths(b, pf, node=0, scen=1, node_step=12)
    ref = oracle.reserves(b, pf, 0, 1, 1, 1, 12)
    gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
    got = to_np(po["path"])
    assert not np.isnan(got).any()
    assert_reserves_close(got, path, np.maximum(gross, 0), what="path")


def test_many_tiles_chunked_totals(ctx):
    """Over 512 tiles with a wide scenario range: the totals are summed in
    tile chunks, then the chunks in order; every total against the oracle."""
    rng = np.random.default_rng(78)
    w = synth.random_small(rng, n=40_000, n_steps=24, n_scen=70, n_nodes=2, shock=True)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    _say("chunked totals, 40,000 policies")
    out = ctx.alloc_outputs(2, 70, r0=False, stats=True)
    ctx.reserve_recurrence(0, 2, 0, 70, 12, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(w.basis, w.portfolio, 0, 2, 0, 70, 12)
    err = np.abs(to_np(out["totals"]) - ref["totals"])
    assert np.all(err <= RTOL * np.maximum(ref["gross_totals"], 1e-300)), err.max()


def test_c2_full_r0_totals_and_path(ctx):
    w = synth.config_c2()
    _say("C2 full")
    out, ref = run_and_compare(ctx, w, all_states=False)
    po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=0)
    ctx.reserve_recurrence(0, 1, 0, 1, 12, po)
    torch.cuda.synchronize()
    path, off = oracle.reserve_paths(w.basis, w.portfolio)
    gross = np.repeat(ref["gross"][0, :, 0], np.diff(off))
    assert_reserves_close(to_np(po["path"]), path, gross, what="path")


def test_c3_full_size_sampled(ctx):
    """10,000 mixed policies x 1,000 Vasicek scenarios x up to 600 steps, in the
    launch configuration the benchmark times; oracle on sampled scenarios."""
    w = synth.config_c3()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    ctx.set_option(1, 0)
    out = ctx.alloc_outputs(1, b.n_scen)
    _say("C3 full size")
    ctx.reserve_recurrence(0, 1, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    r0 = to_np(out["r0"])
    tot = to_np(out["totals"])
    for s in (0, 517, 999):
        ref = oracle.reserves(b, pf, 0, 1, s, 1)
        assert_reserves_close(r0[:, :, s:s + 1], ref["r_all"][..., 0], ref["gross"])
        assert abs(tot[0, s] - ref["totals"][0, 0]) <= RTOL * ref["gross_totals"][0, 0]
    # sampled single valuations across all scenarios
    rng = np.random.default_rng(1)
    idx = rng.choice(pf.n, 40, replace=False)
    sub = pf.subset(idx)
    ref = oracle.reserves(b, sub, 0, 1, 0, b.n_scen)
    assert_reserves_close(r0[:, idx, :], ref["r_all"][..., 0], ref["gross"])


def test_c4_full_size_sampled(ctx):
    """60 annual nodes x 500 inner scenarios with per-node mortality shocks;
    totals and per-node statistics checked at sampled nodes."""
    w = synth.config_c4()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    ctx.set_option(1, 0)
    out = ctx.alloc_outputs(b.n_nodes, b.n_scen, r0=False, stats=True)
    _say("C4 full size")
    ctx.reserve_recurrence(0, b.n_nodes, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    tot = to_np(out["totals"])
    stats = to_np(out["stats"])
    for node in (0, 23, 47, 59):
        for s in (0, 499):
            ref = oracle.reserves(b, pf, node, 1, s, 1)
            assert abs(tot[node, s] - ref["totals"][0, 0]) <= RTOL * max(ref["gross_totals"][0, 0], 1e-300)
    mean, q = oracle.node_stats(tot)
    np.testing.assert_allclose(stats[:, 0], mean, rtol=1e-12, atol=0)
    np.testing.assert_array_equal(stats[:, 1], q)
    # all policies expire before node 50 of a 600-month book? (terms <= 600)
    live = [(pf.term_m - 12 * k > 0).sum() for k in range(b.n_nodes)]
    for k in range(b.n_nodes):
        if live[k] == 0:
            assert np.all(tot[k] == 0.0)


def test_c4_node_valuations_sampled(ctx):
    w = synth.config_c4(n=700, n_nodes=8, n_inner=40)
    _say("C4 small all valuations")
    run_and_compare(ctx, w, all_states=False)


def test_deterministic_and_invariant_to_tuning(ctx):
    rng = np.random.default_rng(77)
    w = synth.random_small(rng, n=333, n_steps=120, n_scen=100, n_nodes=2, shock=True)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    results = []
    for K, J, wg, xcd, graph in [(8, 1, 2, 1, 1), (8, 1, 2, 1, 1), (4, 1, 1, 0, 0), (16, 1, 4, 1, 0),
                                 (32, 1, 2, 0, 1), (1, 1, 1, 1, 1), (2, 1, 8, 1, 1), (8, 2, 2, 1, 1),
                                 (16, 2, 3, 1, 0), (4, 4, 2, 0, 1), (8, 4, 1, 1, 1)]:
        ctx.set_option(1, K)
        ctx.set_option(8, J)
        ctx.set_option(2, wg)
        ctx.set_option(5, xcd)
        ctx.set_option(3, graph)
        _say(f"tuning K={K} J={J} wg={wg} xcd={xcd} graph={graph}")
        out = ctx.alloc_outputs(2, 100, all_states=True)
        for _ in range(2):
            ctx.reserve_recurrence(0, 2, 0, 100, 12, out)
        torch.cuda.synchronize()
        results.append((to_np(out["r0"]), to_np(out["totals"])))
    for r, t in results[1:]:
        assert np.array_equal(r, results[0][0])
    # totals sum tile partials in a fixed order for a given shape
    for r, t in results[1:]:
        assert np.array_equal(t, results[0][1])


def test_graph_replays_match_eager(ctx):
    rng = np.random.default_rng(8)
    w = synth.random_small(rng, n=500, n_steps=100, n_scen=64, n_nodes=1)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    ctx.set_option(1, 8)
    ctx.set_option(2, 2)
    ctx.set_option(3, 0)
    eager = ctx.alloc_outputs(1, 64, stats=True)
    ctx.reserve_recurrence(0, 1, 0, 64, 12, eager)
    torch.cuda.synchronize()
    ctx.set_option(3, 1)
    out = ctx.alloc_outputs(1, 64, stats=True)
    for rep in range(4):
        for v in out.values():
            v.zero_()
        ctx.reserve_recurrence(0, 1, 0, 64, 12, out)
        torch.cuda.synchronize()
        for k in ("r0", "totals", "stats"):
            assert torch.equal(out[k], eager[k]), (rep, k)


def test_edge_cases(ctx, rr):
    q = synth.gm_monthly_q(1500)[None]
    v = np.full((2, 3, 120), 1.03 ** (-1 / 12))
    ctx.basis_upload(q, v)
    # empty portfolio: totals and stats are zero
    empty = synth.Portfolio(*(np.zeros(0, np.int32),) * 7, np.zeros(0), np.zeros(0))
    ctx.portfolio_upload(empty)
    out = ctx.alloc_outputs(2, 3, stats=True)
    out["totals"].fill_(7.0)
    ctx.reserve_recurrence(0, 2, 0, 3, 12, out)
    torch.cuda.synchronize()
    assert torch.all(out["totals"] == 0) and torch.all(out["stats"] == 0)
    # single policies at the extremes of term and age
    pf = synth.Portfolio(product=np.array([0, 4, 5, 6, 1, 3], np.int32),
                         age1_m=np.array([0, 1379, 700, 1000, 500, 1200], np.int32),
                         age2_m=np.array([0, 0, 0, 0, 1379, 1379], np.int32),
                         term_m=np.array([1, 120, 1, 120, 120, 13], np.int32),
                         table1=np.zeros(6, np.int32), table2=np.zeros(6, np.int32),
                         timing=np.array([1, 1, 1, 1, 0, 0], np.int32),
                         amount=np.array([1200.0, 1e5, 1e4, 2e4, 600.0, 600.0]),
                         premium=np.array([0.0, 20.0, 5.0, 50.0, 0.0, 0.0]))
    from synth import Basis, Workload
    w = Workload("edges", Basis(q=q, v=v), pf)
    run_and_compare(ctx, w)
    # node where every policy has expired (node_step 120)
    out = ctx.alloc_outputs(1, 3, all_states=True)
    ctx.reserve_recurrence(1, 1, 0, 3, 120, out)
    torch.cuda.synchronize()
    assert torch.all(out["r0"] == 0) and torch.all(out["totals"] == 0)


def test_invalid_calls_raise(ctx, rr):
    q = synth.gm_monthly_q(1500)[None]
    v = np.full((1, 2, 100), 0.99)
    with pytest.raises(rr.RRError) as e:
        ctx.reserve_recurrence(0, 1, 0, 1, 12)
    assert e.value.code == rr.RR_ESTATE
    ctx.basis_upload(q, v)
    w = synth.random_small(np.random.default_rng(0), n=10, n_steps=100)
    bad = w.portfolio.subset(np.arange(10))
    bad.table1[:] = 0
    bad.table2[:] = 0
    bad.term_m[4] = 101
    with pytest.raises(rr.RRError) as e:
        ctx.portfolio_upload(bad)
    assert e.value.code == rr.RR_EINVAL and "policy 4" in str(e.value)
    with pytest.raises(rr.RRError):
        ctx.basis_upload(q, -v)
    bad.term_m[4] = 50
    bad.age1_m[:] = 100
    bad.age2_m[:] = 100
    ctx.portfolio_upload(bad)
    with pytest.raises(rr.RRError) as e:
        ctx.reserve_recurrence(0, 1, 1, 2, 12)          # scenario range outside
    assert e.value.code == rr.RR_EINVAL
    small = {"path": torch.empty(5, dtype=torch.float64, device="cuda")}
    with pytest.raises(rr.RRError) as e:
        ctx.reserve_recurrence(0, 1, 0, 1, 12, small)
    assert e.value.code == rr.RR_ERANGE
    with pytest.raises(rr.RRError):
        ctx.set_option(1, 3)
    # a basis that no longer covers the portfolio drops it
    ctx.basis_upload(q[:, :120], v)
    with pytest.raises(rr.RRError) as e:
        ctx.reserve_recurrence(0, 1, 0, 1, 12)
    assert e.value.code == rr.RR_ESTATE
