"""GPU parity of the device-generated Vasicek scenarios (through the C ABI)
against the oracle's generator, and of reserves valued on them.

The curves agree within 1e-13 relative (v) and 1e-14 absolute (r): both sides
draw the same Philox blocks bit for bit; the transcendental functions and the
fused multiply-adds of the device differ from the host's in the last bits."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import RTOL, assert_reserves_close, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

A, B, SIG, DT = synth.VAS_A, synth.VAS_B, synth.VAS_SIGMA, 1.0 / 12.0


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


def check_curves(gv, gr, ov, orr):
    np.testing.assert_allclose(gv, ov, rtol=1e-13, atol=0)
    np.testing.assert_allclose(gr, orr, rtol=0, atol=1e-14)


@pytest.mark.parametrize("sigma", [SIG, 0.0, 0.05])
def test_curves_match_oracle(ctx, sigma):
    r0 = [0.03, 0.05, 0.01]
    key = (7, 9)
    _say(f"curves sigma={sigma}")
    gv, gr = ctx.vasicek_curves(70, 130, r0, A, B, sigma, DT, key)
    torch.cuda.synchronize()
    ov, orr = oracle.vasicek_curves(A, B, sigma, DT, r0, 70, 130, key)
    check_curves(to_np(gv), to_np(gr), ov, orr)


def test_curves_full_c3_size(ctx):
    """1,000 scenarios x 600 monthly steps, every value."""
    key = (2003, 1)
    _say("curves 1,000 x 600")
    gv, gr = ctx.vasicek_curves(1000, 600, [synth.VAS_R0], A, B, SIG, DT, key)
    torch.cuda.synchronize()
    ov, orr = oracle.vasicek_curves(A, B, SIG, DT, [synth.VAS_R0], 1000, 600, key)
    check_curves(to_np(gv), to_np(gr), ov, orr)


def reserves_on_generated(ctx, w, r0, key, nscen):
    """Reserves from a device-generated basis vs the oracle on its own curves."""
    b, pf = w.basis, w.portfolio
    ov, _ = oracle.vasicek_curves(A, B, SIG, DT, r0, nscen, b.n_steps, key)
    out = ctx.alloc_outputs(len(r0), nscen, all_states=False, stats=True)
    ctx.reserve_recurrence(0, len(r0), 0, nscen, w.node_step_m, out)
    torch.cuda.synchronize()
    ref = oracle.reserves(synth.Basis(q=b.q, v=ov, shock=b.shock), pf, 0, len(r0), 0, nscen,
                          w.node_step_m)
    assert_reserves_close(to_np(out["r0"]), ref["r_all"][..., 0], ref["gross"])
    err = np.abs(to_np(out["totals"]) - ref["totals"])
    assert np.all(err <= RTOL * np.maximum(ref["gross_totals"], 1e-300))
    return out


def test_generated_basis_reserves_and_in_place_regeneration(ctx):
    rng = np.random.default_rng(31)
    w = synth.random_small(rng, n=300, n_steps=120, n_scen=1, n_nodes=2, shock=True,
                           random_q=False)
    b = w.basis
    r0a, keya = [0.03, 0.045], (11, 12)
    r0b, keyb = [0.02, 0.06], (13, 14)
    ctx.basis_generate_vasicek(b.q, 45, b.n_steps, r0a, A, B, SIG, DT, keya, shock=b.shock)
    ctx.portfolio_upload(w.portfolio)
    _say("generated basis")
    first = reserves_on_generated(ctx, w, r0a, keya, 45)
    first_r0 = to_np(first["r0"]).copy()
    _say("regenerated in place")
    ctx.curves_generate_vasicek(r0b, A, B, SIG, DT, keyb)
    reserves_on_generated(ctx, w, r0b, keyb, 45)
    # several regenerations and graph replays in a row, back to the first curves
    for _ in range(3):
        ctx.curves_generate_vasicek(r0b, A, B, SIG, DT, keyb)
        ctx.curves_generate_vasicek(r0a, A, B, SIG, DT, keya)
        again = ctx.alloc_outputs(2, 45, all_states=False, stats=True)
        ctx.reserve_recurrence(0, 2, 0, 45, w.node_step_m, again)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(again["r0"]), first_r0)


def test_invalid_generator_calls(ctx, rr):
    q = synth.gm_monthly_q(400)[None]
    with pytest.raises(rr.RRError, match="no basis"):
        ctx.curves_generate_vasicek([0.03], A, B, SIG, DT, (1, 2))
    for kw, msg in ((dict(a=0.0), "a must be"), (dict(sigma=-0.01), "sigma must be"),
                    (dict(dt=0.0), "dt must be"), (dict(b=float("nan")), "b must be")):
        args = dict(a=A, b=B, sigma=SIG, dt=DT)
        args.update(kw)
        with pytest.raises(rr.RRError, match=msg):
            ctx.basis_generate_vasicek(q, 10, 50, [0.03], key=(1, 2), **args)
    with pytest.raises(rr.RRError, match="r0"):
        ctx.basis_generate_vasicek(q, 10, 50, [float("inf")], A, B, SIG, DT, (1, 2))
    with pytest.raises(rr.RRError, match="n_nodes, n_scen and n_steps"):
        ctx.vasicek_curves(0, 50, [0.03], A, B, SIG, DT, (1, 2))
    ctx.basis_generate_vasicek(q, 10, 50, [0.03], A, B, SIG, DT, (1, 2))
    with pytest.raises(rr.RRError, match="r0"):
        ctx.curves_generate_vasicek([float("nan")], A, B, SIG, DT, (1, 2))
