"""GPU parity of the curve-ring kernel instances (level single- and joint-life
portfolios): the scenario discount factors reach the recurrence through a
per-wavefront LDS ring instead of scalar loads.  The arithmetic is the same
sequence of operations as the scalar-load instances, so besides the oracle
bar (1e-10 of the gross value) the two must agree bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import RTOL, assert_reserves_close, to_np
from tests.test_gpu_parity import run_and_compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RING_SHAPES = [(16, 1), (16, 2), (8, 2)]
SCALAR_PRODUCTS = (0, 1, 4, 5, 6, 8, 9)   # single-life and joint-life scalar-reserve models
OPT_K, OPT_WG, OPT_J, OPT_RING, OPT_LAST_RING = 1, 2, 8, 11, 12


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


def _pin(ctx, K, J, wg, ring):
    ctx.set_option(OPT_K, K)
    ctx.set_option(OPT_J, J)
    ctx.set_option(OPT_WG, wg)
    ctx.set_option(OPT_RING, ring)


@pytest.mark.parametrize("K,J", RING_SHAPES)
def test_ring_random_small_all_states(ctx, K, J):
    """Several chunks of 16 steps plus a partial one, ragged heads, shocks,
    three nodes, a ragged last scenario block."""
    rng = np.random.default_rng(900 + K + 7 * J)
    w = synth.random_small(rng, n=450, n_steps=100, n_scen=37, n_nodes=3, shock=True,
                           products=SCALAR_PRODUCTS)
    _pin(ctx, K, J, 2, 1)
    _say(f"ring random small K={K} J={J}")
    run_and_compare(ctx, w, K=K)
    assert ctx.get_option(OPT_LAST_RING) == 1


@pytest.mark.parametrize("K,J", RING_SHAPES)
def test_ring_bitwise_equals_scalar_loads(ctx, K, J):
    rng = np.random.default_rng(950 + K + 7 * J)
    w = synth.random_small(rng, n=300, n_steps=160, n_scen=70, n_nodes=2, shock=True,
                           products=SCALAR_PRODUCTS)
    b = w.basis
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(w.portfolio)
    res = []
    for ring in (0, 1):
        _pin(ctx, K, J, 2, ring)
        _say(f"ring bitwise K={K} J={J} ring={ring}")
        out = ctx.alloc_outputs(2, b.n_scen, all_states=True)
        ctx.reserve_recurrence(0, 2, 0, b.n_scen, 12, out)
        torch.cuda.synchronize()
        assert ctx.get_option(OPT_LAST_RING) == ring
        res.append((to_np(out["r0"]), to_np(out["totals"])))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_ring_skipped_for_vector_models(ctx):
    """A portfolio with reversionary annuities has vector tiles: the ring
    instances do not run them, so a pinned ring launch falls back."""
    rng = np.random.default_rng(5)
    w = synth.random_small(rng, n=200, n_steps=60, n_scen=20, n_nodes=1, products=(0, 2, 3))
    _pin(ctx, 16, 2, 2, 1)
    _say("ring with vector tiles")
    run_and_compare(ctx, w, K=16)
    assert ctx.get_option(OPT_LAST_RING) == 0


def test_ring_c4_small_nodes(ctx):
    """Nodes 0..7 of a small C4 book (terms up to 600 months, node shift 12k):
    long chunk sequences, expired policies at later nodes."""
    w = synth.config_c4(n=700, n_nodes=8, n_inner=40)
    _pin(ctx, 16, 2, 2, 1)
    _say("ring C4 small")
    run_and_compare(ctx, w, K=16, all_states=False)
    assert ctx.get_option(OPT_LAST_RING) == 1


def test_ring_c3_full_size_sampled(ctx):
    """The headline workload (10,000 mixed policies x 1,000 scenarios) with
    the ring pinned, sampled against the oracle."""
    w = synth.config_c3()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _pin(ctx, 16, 2, 2, 1)
    out = ctx.alloc_outputs(1, b.n_scen)
    _say("ring C3 full size")
    ctx.reserve_recurrence(0, 1, 0, b.n_scen, 12, out)
    torch.cuda.synchronize()
    assert ctx.get_option(OPT_LAST_RING) == 1
    r0 = to_np(out["r0"])
    tot = to_np(out["totals"])
    for s in (0, 511, 999):
        ref = oracle.reserves(b, pf, 0, 1, s, 1)
        assert_reserves_close(r0[:, :, s:s + 1], ref["r_all"][..., 0], ref["gross"])
        assert abs(tot[0, s] - ref["totals"][0, 0]) <= RTOL * ref["gross_totals"][0, 0]
    rng = np.random.default_rng(2)
    idx = rng.choice(pf.n, 40, replace=False)
    ref = oracle.reserves(b, pf.subset(idx), 0, 1, 0, b.n_scen)
    assert_reserves_close(r0[:, idx, :], ref["r_all"][..., 0], ref["gross"])


@pytest.mark.parametrize("K,J,wg", [(16, 4, 1), (8, 2, 2), (4, 1, 3)])
def test_queue_modes_bitwise(ctx, K, J, wg):
    """Plain longest-first queues, dealt windows, and windows taken by whole
    workgroups (one atomic per window, partial windows at queue ends, queue
    switching) give the same results bit for bit, equal to the oracle."""
    rng = np.random.default_rng(40 + K + J)
    w = synth.random_small(rng, n=700, n_steps=120, n_scen=53, n_nodes=3, shock=True)
    b = w.basis
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(w.portfolio)
    res = []
    for mode in (0, 1, 2, 2, -1):
        ctx.set_option(OPT_K, K)
        ctx.set_option(OPT_J, J)
        ctx.set_option(OPT_WG, wg)
        ctx.set_option(14, mode)
        _say(f"queue mode {mode} K={K} J={J} wg={wg}")
        out = ctx.alloc_outputs(3, b.n_scen, all_states=True)
        ctx.reserve_recurrence(0, 3, 0, b.n_scen, 12, out)
        torch.cuda.synchronize()
        res.append((to_np(out["r0"]), to_np(out["totals"])))
    for r, t in res[1:]:
        assert np.array_equal(r, res[0][0])
        assert np.array_equal(t, res[0][1])
    ref = oracle.reserves(b, w.portfolio, 0, 3, 0, b.n_scen, 12)
    from tests._helpers import assert_states_close
    assert_states_close(res[0][0], ref["r_all"], ref["gross"])


def test_scheduling_options_validated(ctx, rr):
    """Out-of-range values of the scheduling options are rejected; the
    read-only options report the last launch."""
    for opt, bad in ((OPT_RING, 2), (OPT_RING, -2), (14, 3), (14, -2)):
        with pytest.raises(rr.RRError) as e:
            ctx.set_option(opt, bad)
        assert e.value.code == rr.RR_EINVAL
    assert ctx.get_option(OPT_RING) == 0          # curve ring off by default
    assert ctx.get_option(14) == -1               # window mode chosen by the autotuner
    assert ctx.get_option(13) == 1                # lane spread on
    assert ctx.get_option(10) == 4                # term bucket, months
    rng = np.random.default_rng(3)
    w = synth.random_small(rng, n=200, n_steps=60, n_scen=40, n_nodes=1, products=SCALAR_PRODUCTS)
    _say("scheduling options")
    run_and_compare(ctx, w)
    assert ctx.get_option(rr.OPT_LAST_WINDOWS) in (0, 1)
    assert ctx.get_option(OPT_LAST_RING) == 0
