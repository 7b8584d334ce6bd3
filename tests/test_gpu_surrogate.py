"""GPU parity of the reserve surrogate against the surrogate oracle
(oracle/mlp.py): the bfloat16 MFMA forward pass, the gradients, the Adam
step, the features and range flags, fused inference with the exact fallback,
training, and the gain over a non-learned proxy.

Tolerances.  Both sides round the same bfloat16 operands and accumulate in
FP32 in different orders, so pre-activations differ by about 1e-6 relative;
an activation within that distance of a bfloat16 rounding boundary rounds
the other way (one bfloat16 unit, 2^-8 relative) on one side only.  Such
flips are rare: most outputs agree to FP32 rounding, a few differ by a
flip's effect.  The checks therefore bound the median error at the FP32
level, the error of 99 % of outputs at 1e-3 of the output scale and every
error at 2e-2 of it.  Rows the exact fallback computes meet the FP64 bound
of the recurrence (1e-10 of the gross value)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests._helpers import RTOL, to_np

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


def assert_flip_tolerant(got, ref, scale, what):
    err = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64)) / scale
    med, q99, mx = np.median(err), np.quantile(err, 0.99), err.max()
    _say(f"{what}: median {med:.2e} q99 {q99:.2e} max {mx:.2e}")
    assert med <= 2e-5, (what, med)
    assert q99 <= 1e-3, (what, q99)
    assert mx <= 2e-2, (what, mx)


def neutral_model(rng, params):
    """A blob around random weights with identity standardisation."""
    import paper_1401_1757_amd as rr
    E, _ = np.linalg.qr(rng.normal(size=(mlp.N_TENORS, 3)))
    return rr.pack_surrogate_blob(mlp.flatten(params), np.zeros(17), np.ones(17),
                                  np.full(17, -1e9), np.full(17, 1e9), np.zeros(4), np.ones(4),
                                  np.zeros(mlp.N_TENORS), E.T, np.full((4, 3), -1))


def random_rows(rng, n):
    z = np.zeros((n, mlp.K_IN), np.float32)
    z[:, :mlp.N_FEAT] = rng.normal(0, 1, (n, mlp.N_FEAT))
    return z


# ---------------------------------------------------------------------------
# Layers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4099])
def test_forward_matches_bf16_oracle(ctx, rr, n):
    rng = np.random.default_rng(10 + n)
    p = synth.random_mlp_params(rng)
    ctx.surrogate_set_weights(neutral_model(rng, p))
    z = random_rows(rng, n)
    _say(f"forward n={n}")
    y = to_np(ctx.surrogate_forward(torch.from_numpy(z).cuda()))
    ref, _ = mlp.forward(p, z, quant=True)
    scale = max(float(np.sqrt(np.mean(np.square(ref)))), 1e-3)
    assert_flip_tolerant(y, ref, scale, f"forward n={n}")


@pytest.mark.parametrize("n", [64, 700, 8192])
def test_gradients_match_bf16_oracle(ctx, rr, n):
    rng = np.random.default_rng(20 + n)
    p = synth.random_mlp_params(rng)
    ctx.surrogate_set_weights(neutral_model(rng, p))
    z = random_rows(rng, n)
    t = rng.normal(0, 1, n).astype(np.float32)
    _say(f"gradients n={n}")
    g, loss = ctx.surrogate_gradients(torch.from_numpy(z).cuda(), torch.from_numpy(t).cuda())
    g = to_np(g)
    gref, yref = mlp.backward(p, z, t, quant=True)
    lref = float(np.mean((np.asarray(yref, np.float64) - t) ** 2))
    assert abs(float(to_np(loss)[0]) - lref) <= 1e-4 * lref
    g64, _ = mlp.backward({k: np.asarray(v, np.float64) for k, v in p.items()}, z, t, quant=False)
    gg = mlp.unflatten(g)
    for k, _ in mlp.PARAM_SHAPES:
        a = np.ravel(gg[k]).astype(np.float64)
        b = np.ravel(gref[k]).astype(np.float64)
        c = np.ravel(g64[k]).astype(np.float64)
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        rel64 = np.linalg.norm(a - c) / max(np.linalg.norm(c), 1e-30)
        _say(f"  {k}: vs bf16 oracle {rel:.2e}, vs fp64 oracle {rel64:.2e}")
        assert rel <= 5e-3, (k, rel)
        assert rel64 <= 5e-2, (k, rel64)
    assert np.all(gg["W1"][mlp.N_FEAT:] == 0.0)   # padded inputs


def test_adam_step_matches_oracle(ctx, rr):
    rng = np.random.default_rng(30)
    p = synth.random_mlp_params(rng)
    m = {k: rng.normal(0, 1e-3, np.shape(v)).astype(np.float32) for k, v in p.items()}
    v = {k: rng.uniform(0, 1e-6, np.shape(x)).astype(np.float32) for k, x in p.items()}
    for d in (m, v):
        d["W1"][mlp.N_FEAT:] = 0
    blob = rr.pack_surrogate_blob(mlp.flatten(p), np.zeros(17), np.ones(17), np.full(17, -1.0),
                                  np.ones(17), np.zeros(4), np.ones(4), np.zeros(50), np.eye(3, 50),
                                  np.full((4, 3), -1), adam_m=mlp.flatten(m), adam_v=mlp.flatten(v),
                                  adam_step=4)
    ctx.surrogate_set_weights(blob)
    g = {k: rng.normal(0, 1e-3, np.shape(x)).astype(np.float32) for k, x in p.items()}
    ctx.surrogate_adam_step(torch.from_numpy(mlp.flatten(g)).cuda(), 3e-4)
    got = rr.unpack_surrogate_blob(ctx.surrogate_get_weights())
    assert got["adam_step"] == 5
    rp, rm, rv = mlp.adam(p, g, m, v, 5, 3e-4)
    # FP32 rounding of each update (the device may fuse a multiply and an
    # add): a few units in the last place of the terms that are summed.
    fm, fv, fg = (np.abs(mlp.flatten(d)).astype(np.float64) for d in (m, v, g))
    scales = {"params": np.abs(mlp.flatten(p)).astype(np.float64) + 3e-4,
              "m": 0.9 * fm + 0.1 * fg, "v": 0.999 * fv + 0.001 * fg * fg}
    for name, a, b in (("params", got["params"], mlp.flatten(rp)), ("m", got["adam_m"], mlp.flatten(rm)),
                       ("v", got["adam_v"], mlp.flatten(rv))):
        err = np.abs(a.astype(np.float64) - b) / (scales[name] + 1e-30)
        assert err.max() <= 5e-7, (name, err.max())


# ---------------------------------------------------------------------------
# Features, flags and inference against the oracle
# ---------------------------------------------------------------------------
def oracle_model(seed=40, n=400, n_nodes=8, n_scen=8):
    """Standardisation, box, components and signature fitted by the oracle on
    a small training workload (node_step 0)."""
    tw = synth.surrogate_training_workload(seed=seed, n=n, n_nodes=n_nodes, n_scen=n_scen)
    b, pf = tw.basis, tw.portfolio
    ref = oracle.reserves(b, pf, 0, n_nodes, 0, n_scen, 0)
    zbar, E, _ = mlp.fit_pca(mlp.zero_rates(b.v.reshape(-1, b.n_steps)))
    X, T = mlp.samples(tw, 0, n_nodes, 0, n_scen, 0, ref["r_all"], zbar, E)
    mu, sd, lo, hi, tmu, tsd = mlp.normalisation(X, T)
    sig = mlp.product_signature(pf)
    sig_arr = np.array([s if s is not None else (-1, -1, -1) for s in sig])
    return dict(mu=mu, sd=sd, lo=lo, hi=hi, tmu=tmu, tsd=tsd, zbar=zbar, E=E, sig=sig,
                sig_arr=sig_arr, X=X, T=T, workload=tw, ref=ref)


@pytest.fixture(scope="module")
def omodel():
    return oracle_model()


def parity_workload(seed=41, n=300, n_nodes=2, n_scen=40):
    """C2-law policies plus out-of-domain ones, Vasicek scenarios, shocks."""
    rng = np.random.default_rng(seed)
    pf = synth.portfolio_mixed(rng, n)
    pf.timing[np.flatnonzero(pf.product == synth.SL_ANN)[0]] = synth.ADVANCE
    pf.product[np.flatnonzero(pf.product == synth.SL_ANN)[1]] = synth.REV_ANN
    pf.age2_m[np.flatnonzero(pf.product == synth.REV_ANN)] = 700
    pf.amount[np.flatnonzero(pf.product == synth.TERM)[0]] *= 1e4   # far outside the box
    pf.term_m[np.flatnonzero(pf.product == synth.ENDOW)[:2]] = 12    # expired at node 1
    # escalating and annual annuities: outside the domain (exact fallback)
    sl = np.flatnonzero(pf.product == synth.SL_ANN)
    pf.escalation = np.zeros(n)
    pf.annual = np.zeros(n, np.int32)
    pf.anniv_m = (np.arange(n) % 12 + 1).astype(np.int32)
    pf.escalation[sl[2]] = 0.05
    pf.annual[sl[3]] = 1
    q = synth.mortality_tables(synth.max_attained_age(pf) + 1, synth.C2_LOADINGS)
    v = np.empty((n_nodes, n_scen, 600))
    for k in range(n_nodes):
        v[k], _ = synth.vasicek_paths(rng, n_scen, 600, 0.03 + 0.01 * k)
    v[0, 3] = v[0, 3] ** 3      # a scenario far outside the training curves
    shock = np.linspace(1.0, 1.02, n_nodes)
    return synth.Workload("surrogate parity", synth.Basis(q=q, v=v, shock=shock), pf)


def blob_of(rr, om, params):
    return rr.pack_surrogate_blob(mlp.flatten(params), om["mu"], om["sd"], om["lo"], om["hi"],
                                  om["tmu"], om["tsd"], om["zbar"], om["E"].T, om["sig_arr"])


def oracle_flags(om, w, node_step):
    b, pf = w.basis, w.portfolio
    pflag = np.zeros((b.n_nodes, pf.n), np.int32)
    sflag = np.zeros((b.n_nodes, b.n_scen), np.int32)
    praw = np.zeros((b.n_nodes, pf.n, 9))
    sraw = np.zeros((b.n_nodes, b.n_scen, 5))
    pidx = list(range(8)) + [16]
    for k in range(b.n_nodes):
        pol, ok = mlp.policy_features(pf, k, node_step, om["sig"])
        praw[k] = pol
        inbox = np.all((pol >= om["lo"][pidx]) & (pol <= om["hi"][pidx]), axis=1)
        pflag[k] = np.where(pf.term_m - k * node_step <= 0, 2, np.where(ok & inbox, 1, 0))
        sc = mlp.scenario_features(b.v[k], b.shock[k], om["zbar"], om["E"])
        sraw[k] = sc
        st = np.array([1.0, 0.0, 0.0])
        sflag[k] = (np.all((sc >= om["lo"][8:13]) & (sc <= om["hi"][8:13]), axis=1) &
                    np.all((st >= om["lo"][13:16]) & (st <= om["hi"][13:16])))
    return praw, sraw, pflag, sflag


def test_features_and_flags_match_oracle(ctx, rr, omodel):
    rng = np.random.default_rng(42)
    p = synth.random_mlp_params(rng)
    w = parity_workload()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    ctx.surrogate_set_weights(blob_of(rr, omodel, p))
    _say("features")
    f = ctx.surrogate_features(node_step=12)
    praw, sraw, pflag, sflag = oracle_flags(omodel, w, 12)
    np.testing.assert_allclose(to_np(f["pol"]), praw, rtol=1e-14, atol=0)
    np.testing.assert_allclose(to_np(f["scen"]), sraw, rtol=1e-12, atol=1e-13)
    assert np.array_equal(to_np(f["pflag"]), pflag)
    assert np.array_equal(to_np(f["sflag"]), sflag)
    assert (pflag == 0).sum() >= 5 and (pflag == 2).sum() >= 1 and (sflag == 0).sum() >= 1
    sl = np.flatnonzero(pf.product == synth.SL_ANN)
    assert np.all(pflag[:, sl[2:4]] == 0)     # patterned annuities


def test_infer_matches_oracle_with_fallback(ctx, rr, omodel):
    rng = np.random.default_rng(43)
    p = synth.random_mlp_params(rng)
    w = parity_workload()
    b, pf = w.basis, w.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    ctx.surrogate_set_weights(blob_of(rr, omodel, p))
    _say("infer with fallback")
    out = ctx.alloc_outputs(b.n_nodes, b.n_scen, stats=True)
    ctx.surrogate_infer(0, b.n_nodes, 0, b.n_scen, 12, out)
    tot_only = ctx.alloc_outputs(b.n_nodes, b.n_scen, r0=False, stats=True)
    ctx.surrogate_infer(0, b.n_nodes, 0, b.n_scen, 12, tot_only)
    torch.cuda.synchronize()
    got = to_np(out["r0"])
    ref = oracle.reserves(b, pf, 0, b.n_nodes, 0, b.n_scen, 12)
    exact = ref["r_all"][..., 0]
    praw, sraw, pflag, sflag = oracle_flags(omodel, w, 12)
    net = (pflag[:, :, None] == 1) & (sflag[:, None, :] == 1)
    fb = (pflag[:, :, None] == 0) | ((pflag[:, :, None] == 1) & (sflag[:, None, :] == 0))
    expired = np.broadcast_to(pflag[:, :, None] == 2, net.shape)
    assert out["report"]["n_in_range"] == int(net.sum())
    assert out["report"]["n_fallback"] == int(fb.sum())
    # exact rows
    scale = np.maximum(np.abs(exact), ref["gross"])
    assert np.all(np.abs(got - exact)[fb] <= RTOL * scale[fb])
    assert np.all(got[expired] == 0.0)
    # network rows
    pred = np.zeros_like(exact)
    for k in range(b.n_nodes):
        for i in range(pf.n):
            if pflag[k, i] != 1:
                continue
            X = np.array([mlp.assemble(praw[k, i], sraw[k, s], 0) for s in range(b.n_scen)])
            pred[k, i] = mlp.predict_reserves(p, X, pf.amount[i], omodel["mu"], omodel["sd"],
                                              omodel["tmu"], omodel["tsd"])
    slot = np.select([pf.product == c for c in mlp.SURROGATE_PRODUCTS], [0, 1, 2, 3], 0)
    ys = (pf.amount * omodel["tsd"][slot])[None, :, None] * np.ones_like(exact)
    assert_flip_tolerant(got[net] / ys[net], pred[net] / ys[net], 1.0, "inference rows")
    # totals: the sum of the rows, with or without r0 written
    tot = to_np(out["totals"])
    live = ~expired
    assert np.allclose(tot, np.where(live, got, 0.0).sum(axis=1), rtol=1e-12, atol=1e-6)
    assert np.array_equal(tot, to_np(tot_only["totals"]))
    assert np.array_equal(to_np(out["stats"]), to_np(tot_only["stats"]))
    st = to_np(out["stats"])
    for k in range(b.n_nodes):
        assert st[k, 1] == np.sort(tot[k])[::-1][int(np.ceil(0.005 * b.n_scen)) - 1]


# ---------------------------------------------------------------------------
# Training
# ---------------------------------------------------------------------------
def test_training_fits_and_matches_oracle_statistics(ctx, rr, omodel):
    tw = omodel["workload"]
    b, pf = tw.basis, tw.portfolio
    ctx.basis_upload(b.q, b.v, b.shock)
    ctx.portfolio_upload(pf)
    _say("train small")
    rep = ctx.surrogate_train(0, b.n_nodes, 0, b.n_scen, 0, epochs=30, batch=256, lr=3e-3,
                              lr_final=1e-4, holdout=0.1, seed=5)
    _say(f"  {rep}")
    assert rep["n_samples"] == omodel["X"].shape[0]
    assert rep["n_train"] % 256 == 0 and rep["n_train"] + rep["n_holdout"] == rep["n_samples"]
    assert rep["final_loss"] < 0.05 * rep["first_loss"]
    assert rep["holdout_loss"] < 0.05
    got = rr.unpack_surrogate_blob(ctx.surrogate_get_weights())
    for k in ("mu", "sd", "tsd"):
        np.testing.assert_allclose(got[k], omodel[k], rtol=1e-9, atol=1e-12)
    # target means carry the output calibration reported by training
    cal = np.asarray(rep["calibration"], np.float64)
    assert np.all(np.abs(cal) < 0.05)
    np.testing.assert_allclose(got["tmu"] - got["tsd"] * cal, omodel["tmu"], rtol=0,
                               atol=1e-6 * float(np.max(omodel["tsd"])))
    np.testing.assert_allclose(got["lo"], omodel["lo"], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(got["hi"], omodel["hi"], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(got["zbar"], omodel["zbar"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(got["evec"], omodel["E"].T, atol=1e-7)
    assert np.array_equal(got["signature"], omodel["sig_arr"])
    assert got["adam_step"] == rep["steps"]
    # the blob reloads into another context and predicts the same
    z = torch.from_numpy(random_rows(np.random.default_rng(1), 500)).cuda()
    y1 = to_np(ctx.surrogate_forward(z))
    c2 = rr.Context(0)
    try:
        c2.surrogate_set_weights(ctx.surrogate_get_weights())
        y2 = to_np(c2.surrogate_forward(z))
    finally:
        c2.close()
    assert np.array_equal(y1, y2)


def test_training_and_inference_are_deterministic(rr, omodel):
    """Every reduction runs in a fixed order: the same seed gives the same
    model bit for bit, and inference repeats bit for bit."""
    tw = omodel["workload"]
    b, pf = tw.basis, tw.portfolio
    blobs, outs = [], []
    for _ in range(2):
        c = rr.Context(0)
        try:
            c.basis_upload(b.q, b.v, b.shock)
            c.portfolio_upload(pf)
            c.surrogate_train(0, b.n_nodes, 0, b.n_scen, 0, epochs=3, batch=512, lr=2e-3,
                              lr_final=1e-4, holdout=0.05, seed=9)
            blobs.append(c.surrogate_get_weights())
            o = c.alloc_outputs(b.n_nodes, b.n_scen, stats=True)
            c.surrogate_infer(0, b.n_nodes, 0, b.n_scen, 0, o)
            torch.cuda.synchronize()
            outs.append({k: to_np(v) for k, v in o.items() if k != "report"})
        finally:
            c.close()
    assert blobs[0] == blobs[1]
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_invalid_surrogate_calls(ctx, rr):
    w = parity_workload(n=64, n_nodes=1, n_scen=4)
    ctx.basis_upload(w.basis.q, w.basis.v, w.basis.shock)
    ctx.portfolio_upload(w.portfolio)
    with pytest.raises(rr.RRError) as e:
        ctx.surrogate_infer(0, 1, 0, 4, 12)
    assert e.value.code == rr.RR_ESTATE
    with pytest.raises(rr.RRError) as e:
        ctx.surrogate_set_weights(b"RRSURR01" + bytes(100))
    assert e.value.code == rr.RR_EINVAL
    with pytest.raises(rr.RRError) as e:
        ctx.surrogate_train(0, 1, 0, 4, 0, epochs=1, batch=100)
    assert e.value.code == rr.RR_EINVAL
    with pytest.raises(rr.RRError) as e:   # several tables within one product
        w.portfolio.table1[np.flatnonzero(w.portfolio.product == synth.TERM)[0]] = 0
        ctx.portfolio_upload(w.portfolio)
        ctx.surrogate_train(0, 1, 0, 4, 0, epochs=1, batch=64)
    assert e.value.code == rr.RR_EINVAL
