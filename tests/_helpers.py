"""Shared helpers for the GPU parity tests (not collected by pytest)."""
import numpy as np

# Tolerance on FP64 reserves: per valuation |gpu - oracle| <= RTOL * max(|oracle|, G)
# with G = PV(benefits) + PV(premiums) from the oracle; totals against the
# sum of G over the portfolio.
RTOL = 1e-10


def assert_reserves_close(gpu, orc, gross, rtol=RTOL, what="r0"):
    gpu = np.asarray(gpu)
    orc = np.asarray(orc)
    gross = np.asarray(gross)
    assert gpu.shape == orc.shape, (gpu.shape, orc.shape)
    scale = np.maximum(np.abs(orc), gross)
    bad = np.abs(gpu - orc) > rtol * scale
    if bad.any():
        idx = np.argwhere(bad)[:5]
        det = [(tuple(i), gpu[tuple(i)], orc[tuple(i)], scale[tuple(i)]) for i in idx]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside {rtol} gross-relative: {det}")


def assert_states_close(gpu4, orc4, gross, rtol=RTOL):
    """All four state slots; every slot is scaled by the policy's state-0 gross PV."""
    g = np.asarray(gross)[..., None]
    scale = np.maximum(np.abs(orc4), g)
    bad = np.abs(np.asarray(gpu4) - orc4) > rtol * scale
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"states: {bad.sum()} outside tolerance at {idx.tolist()}")


def to_np(t):
    return t.detach().cpu().numpy()
