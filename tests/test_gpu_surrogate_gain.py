"""What the trained surrogate gains over the method without it.

The surrogate is trained on the GPU (samples from the exact recurrence on the
surrogate training workload) and inferred over the 10,000-policy x 1,000
Vasicek-scenario workload.  Its scenario-averaged portfolio reserve is judged
by the CPU oracle's exact reserves and compared with a non-learned proxy of
the same inputs and similar cost: the exact reserve on the base curve (the
scenarios' mean log discount factors) adjusted to first order along the
first principal component of the curves.  The surrogate must be within 1e-3
of the exact average and closer than the proxy.  Per-scenario and 1-in-200 errors and the speed
ratio over the exact batched recurrence are reported, not asserted."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TRAIN = dict(seed=1005, n=5000, n_nodes=20, n_scen=100)
EPOCHS, BATCH, LR = 24, 8192, 2e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def base_and_bumps(v, e1, h):
    """Base curve (mean log v over scenarios) and the curves whose zero rates
    move by +-h e1 at the 50 annual tenors (piecewise-flat monthly forwards
    within each year)."""
    logv = np.log(v).mean(axis=0)
    T = np.arange(1, mlp.N_TENORS + 1)
    dz = h * e1
    df = T * dz - np.concatenate([[0.0], (T[:-1]) * dz[:-1]])
    dlog = np.repeat(-df / 12.0, 12)[: v.shape[1]]
    return np.exp(np.stack([logv, logv + dlog, logv - dlog]))


def test_surrogate_beats_first_order_proxy():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_1757_amd as rr
    threads = int(os.environ.get("ORACLE_THREADS", min(os.cpu_count() or 1, 16)))
    tw = synth.surrogate_training_workload(**TRAIN)
    w = synth.config_c3()
    b, pf = w.basis, w.portfolio

    _say("train")
    c = rr.Context(0)
    try:
        c.basis_upload(tw.basis.q, tw.basis.v, tw.basis.shock)
        c.portfolio_upload(tw.portfolio)
        rep = c.surrogate_train(node_step=0, epochs=EPOCHS, batch=BATCH, lr=LR, lr_final=LR * 5e-3,
                                holdout=0.01, seed=11)
        _say(f"  {rep}")
        c.basis_upload(b.q, b.v, b.shock)
        c.portfolio_upload(pf)
        out = c.alloc_outputs(1, b.n_scen, r0=False, stats=True)
        c.surrogate_infer(0, 1, 0, b.n_scen, 12, out)
        torch.cuda.synchronize()
        sur = out["totals"].cpu().numpy()[0]
        _say(f"  inference {out['report']}")
        # speed ratio over the exact batched recurrence (same outputs)
        ex = c.alloc_outputs(1, b.n_scen, r0=False, stats=True)
        timings = {}
        for name, fn in (("exact", lambda: c.reserve_recurrence(0, 1, 0, b.n_scen, 12, ex)),
                         ("surrogate", lambda: c.surrogate_infer(0, 1, 0, b.n_scen, 12, out,
                                                                 report=False))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                fn()
            torch.cuda.synchronize()
            timings[name] = (time.perf_counter() - t0) / 10
        _say(f"  exact {timings['exact'] * 1e3:.3f} ms, surrogate {timings['surrogate'] * 1e3:.3f} ms, "
             f"speed ratio {timings['exact'] / timings['surrogate']:.3f}")
    finally:
        c.close()

    _say("oracle")
    exact = oracle.reserves(b, pf, 0, 1, 0, b.n_scen, 12, want_gross=False, n_threads=threads)["totals"][0]
    zbar, E, _ = mlp.fit_pca(mlp.zero_rates(tw.basis.v.reshape(-1, tw.basis.n_steps)))
    h = 1e-3
    curves = base_and_bumps(b.v[0], E[:, 0], h)
    zb = mlp.zero_rates(curves)
    assert np.allclose(zb[1] - zb[0], h * E[:, 0], atol=1e-12)
    R = oracle.reserves(synth.Basis(q=b.q, v=curves[None]), pf, 0, 1, 0, 3, 12,
                        want_gross=False, n_threads=threads)["totals"][0]
    grad = (R[1] - R[2]) / (2 * h)
    f1 = (mlp.zero_rates(b.v[0]) - zbar) @ E[:, 0]
    f1b = (zb[0] - zbar) @ E[:, 0]
    proxy = R[0] + grad * (f1 - f1b)

    mean_exact = exact.mean()
    err_sur = abs(sur.mean() - mean_exact) / abs(mean_exact)
    err_proxy = abs(proxy.mean() - mean_exact) / abs(mean_exact)
    k = int(np.ceil(0.005 * b.n_scen))
    q = lambda x: np.sort(x)[::-1][k - 1]
    _say(f"  scenario-averaged portfolio reserve {mean_exact:.6e}: surrogate rel err {err_sur:.3e}, "
         f"proxy rel err {err_proxy:.3e}")
    _say(f"  per-scenario rms rel err: surrogate {np.sqrt(np.mean(((sur - exact) / exact) ** 2)):.3e}, "
         f"proxy {np.sqrt(np.mean(((proxy - exact) / exact) ** 2)):.3e}")
    _say(f"  1-in-200 total rel err: surrogate {(q(sur) - q(exact)) / q(exact):.3e}, "
         f"proxy {(q(proxy) - q(exact)) / q(exact):.3e}")
    assert err_sur <= 1e-3
    assert err_sur < err_proxy
