"""The allocation-free recurrence entry point (rr_reserve_recurrence_noalloc)
against rr_reserve_recurrence: same kernels, same launch shape, so the same
bits, on two calls in a row (the second smaller, so the static scratch holds
the first call's contents), from two contexts that share the device's
scratch, and against the oracle at the FP64 parity bound."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import assert_states_close, to_np

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


def outputs(ctx, nnode, nscen, totals=True):
    o = ctx.alloc_outputs(nnode, nscen, all_states=True, totals=totals, stats=True)
    for v in o.values():
        v.fill_(float("nan"))
    return o


def same(a, b, what):
    for k in a:
        assert torch.equal(a[k], b[k]), (what, k)


def test_noalloc_matches_the_allocating_entry_point(rr):
    rng = np.random.default_rng(4100)
    big = synth.random_small(rng, n=450, n_steps=90, n_scen=37, n_nodes=3, shock=True,
                             products=tuple(range(7)) + (8, 9, 10))
    small = synth.random_small(rng, n=70, n_steps=40, n_scen=5, n_nodes=2, shock=True)
    c1, c2 = rr.Context(0), rr.Context(0)
    try:
        # call 1: the big case; the allocating call autotunes, the
        # allocation-free one then runs the shape it chose
        b, pf = big.basis, big.portfolio
        c1.basis_upload(b.q, b.v, b.shock)
        c1.portfolio_upload(pf)
        _say("big case: 450 policies x 3 nodes x 37 scenarios")
        ref = c1.reserve_recurrence(0, 3, 0, 37, 12, outputs(c1, 3, 37))
        got = c1.reserve_recurrence_noalloc(0, 3, 0, 37, 12, outputs(c1, 3, 37))
        torch.cuda.synchronize()
        same(got, ref, "big")
        orc = oracle.reserves(b, pf, 0, 3, 0, 37, 12)
        assert_states_close(to_np(got["r0"]), orc["r_all"], orc["gross"])
        # call 2, smaller, from another context on the same device: the
        # scratch still holds call 1's lists and partials; statistics
        # without totals use the scratch for the totals too
        b2, pf2 = small.basis, small.portfolio
        c2.basis_upload(b2.q, b2.v, b2.shock)
        c2.portfolio_upload(pf2)
        _say("small case: 70 policies x 2 nodes x 5 scenarios, no totals output")
        ref2 = c2.reserve_recurrence(0, 2, 0, 5, 12, outputs(c2, 2, 5, totals=False))
        got2 = c2.reserve_recurrence_noalloc(0, 2, 0, 5, 12, outputs(c2, 2, 5, totals=False))
        torch.cuda.synchronize()
        same(got2, ref2, "small")
        orc2 = oracle.reserves(b2, pf2, 0, 2, 0, 5, 12)
        assert_states_close(to_np(got2["r0"]), orc2["r_all"], orc2["gross"])
        # the first context again, a sub-range, untuned shape: the default
        # shape (K = 16, J = 2, one workgroup per CU), against the
        # allocating call pinned to it
        _say("sub-range with the default shape")
        got3 = c1.reserve_recurrence_noalloc(1, 2, 3, 30, 12, outputs(c1, 2, 30))
        torch.cuda.synchronize()
        assert c1.get_option(rr.OPT_LAST_K) == 16 and c1.get_option(rr.OPT_LAST_J) == 2
        c1.set_option(rr.OPT_BLOCK_K, 16)
        c1.set_option(rr.OPT_BLOCK_J, 2)
        c1.set_option(rr.OPT_WG_PER_CU, 1)
        ref3 = c1.reserve_recurrence(1, 2, 3, 30, 12, outputs(c1, 2, 30))
        torch.cuda.synchronize()
        same(got3, ref3, "default shape")
        # repeated calls give the same bits (counters re-armed every call)
        got4 = c1.reserve_recurrence_noalloc(1, 2, 3, 30, 12, outputs(c1, 2, 30))
        torch.cuda.synchronize()
        same(got4, ref3, "repeat")
    finally:
        c1.close()
        c2.close()


def test_noalloc_rejects_paths_and_oversized_runs(rr):
    ctx = rr.Context(0)
    try:
        q = synth.gm_monthly_q(1500)[None]
        v = np.full((1, 14_000, 2), 1.03 ** (-1 / 12))
        ctx.basis_upload(q, v)
        rng = np.random.default_rng(4200)
        w = synth.random_small(rng, n=40_000, n_steps=2, products=(0,))
        pf = w.portfolio
        pf.table1[:] = 0
        pf.age1_m[:] = rng.integers(0, 1400, pf.n)
        ctx.portfolio_upload(pf)
        po = ctx.alloc_outputs(1, 1, r0=False, totals=False, path_node=0)
        with pytest.raises(rr.RRError) as e:
            ctx.reserve_recurrence_noalloc(0, 1, 0, 1, 12, po)
        assert e.value.code == rr.RR_EINVAL
        # 625 tiles x 14,000 scenarios of partial totals: over 64 MiB
        big = ctx.alloc_outputs(1, 14_000, r0=False)
        with pytest.raises(rr.RRError) as e:
            ctx.reserve_recurrence_noalloc(0, 1, 0, 14_000, 12, big)
        assert e.value.code == rr.RR_ERANGE and "MiB" in str(e.value)
        # without totals there is nothing to hold per tile: it runs
        r0 = ctx.alloc_outputs(1, 2_000, r0=True, totals=False)
        ctx.reserve_recurrence_noalloc(0, 1, 0, 2_000, 12, r0)
        ref = ctx.reserve_recurrence(0, 1, 0, 2_000, 12, ctx.alloc_outputs(1, 2_000, totals=False))
        torch.cuda.synchronize()
        assert torch.equal(r0["r0"], ref["r0"])
    finally:
        ctx.close()
