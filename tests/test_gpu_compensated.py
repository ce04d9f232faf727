"""The compensated moment sums (VL_PAIRWISE_COMPENSATED OR-ed into the precision of
pairwise_stats) against the FP64 oracle, through the C ABI.

The flag changes how the two sample means of Eq. 2 are summed (Kahan-compensated per lane,
FP64 across the wave and the chunks), not how each sample's terms are evaluated (FP32), so the
element-wise bars are those of the plain sums (tests/test_gpu_parity.py: the per-term bound);
the measured errors of both forms are printed side by side.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import varlingam as O
import parity as PA

pytestmark = pytest.mark.gpu

TOL_HX = 1e-6
TOL_HR = 2e-6
TOL_S = 6e-6


@pytest.fixture(scope="module")
def api():
    from paper_2409_05500_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _api


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _residuals(m, n, seed):
    rng = np.random.default_rng(seed)
    mix = np.eye(m) + 0.3 * np.tril(rng.normal(size=(m, m)), -1)
    return (rng.laplace(size=(n, m)) @ mix.T).astype(np.float32)


def _compare(api, dev, E32):
    oHx, oHr, oS = O.pairwise_stats(E32.astype(np.float64))
    Ed = _dev(E32, dev)
    out = {}
    for comp in (False, True):
        Hx, Hr, S, Cov = [t.cpu().numpy() for t in api.pairwise_stats(Ed, "mixed",
                                                                      compensated=comp)]
        out[comp] = (Hx, Hr, S, Cov)
        print(f"  compensated={comp}: max|dHx| {np.abs(Hx - oHx).max():.2e} "
              f"max|dHr| {np.abs(Hr - oHr).max():.2e} max|dS| {np.abs(S - oS).max():.2e}",
              flush=True)
    Hx, Hr, S, Cov = out[True]
    np.testing.assert_allclose(Hx, oHx, rtol=0, atol=TOL_HX)
    np.testing.assert_allclose(Hr, oHr, rtol=0, atol=TOL_HR)
    np.testing.assert_allclose(S, oS, rtol=0, atol=TOL_S)
    assert np.array_equal(S, -S.T) and np.all(np.diag(S) == 0.0)
    # the flag leaves the covariance and Hx alone
    assert np.array_equal(Cov, out[False][3]) and np.array_equal(Hx, out[False][0])
    return S, oS


@pytest.mark.parametrize("m,n", [(2, 50), (5, 64), (13, 255), (37, 1234), (65, 2049)])
def test_compensated_ragged_shapes(api, dev, m, n):
    print(f"compensated m={m} n={n}", flush=True)
    _compare(api, dev, _residuals(m, n, 3 * m + n))


def test_compensated_medium_workload_order(api, dev):
    inst = synth.make_instance(synth.MEDIUM, 0)
    _, _, E = O.fit_var(inst.X_parity, 1)
    print(f"compensated {synth.MEDIUM.name}", flush=True)
    S, oS = _compare(api, dev, E.astype(np.float32))
    order, _ = api.approx_order(_dev(S, dev))
    assert PA.order_violations(order.cpu().numpy(), oS) == []


def test_compensated_near_collinear_pairs(api, dev):
    """The listed near-collinear micro-tiles go through the FP64-residual kernel, which writes
    FP64 partials in this mode."""
    print("compensated near-collinear", flush=True)
    _compare(api, dev, synth.near_collinear(3000, 29, [0.99, 0.9999, 0.999999]))


def test_compensated_long_lane_sums_sampled(api, dev):
    """m = 400, n = 40000: four chunks of about 10^4 samples, ~158 a lane, where the rounding
    of a plain running sum is largest; sampled pairs against the oracle's per-pair moments."""
    m, n = 400, 40000
    rng = np.random.default_rng(5)
    mix = np.eye(m) + 0.3 * np.tril(rng.normal(size=(m, m)), -1)
    E32 = (rng.standard_t(4, size=(n, m)) @ mix.T).astype(np.float32)
    E64 = E32.astype(np.float64)
    Ed = _dev(E32, dev)
    pairs = [(int(i), int(j)) for i, j in rng.integers(0, m, (24, 2)) if i != j]
    pairs += [(m - 1, 0), (m - 2, m - 1)]
    ref = {p: O.entropy_from_moments(*O.pair_moments(E64, *p)) for p in pairs}
    for comp in (False, True):
        Hr = api.pairwise_stats(Ed, "mixed", compensated=comp)[1].cpu().numpy()
        err = max(abs(Hr[i, j] - ref[(i, j)]) for i, j in pairs)
        print(f"  compensated={comp}: max|dHr| over {len(pairs)} pairs {err:.2e}", flush=True)
        assert err <= TOL_HR


def test_compensated_deterministic_and_noalloc(api, dev):
    E = _dev(_residuals(41, 3000, 8), dev)
    a = api.pairwise_stats(E, "mixed", compensated=True)
    b = api.pairwise_stats(E, "mixed", compensated=True)
    c = api.pairwise_stats_noalloc(E, "mixed", compensated=True)
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y) and torch.equal(x, z)


def test_compensated_fitter(api, dev):
    """The whole fit with the compensated precompute (Fitter): the order passes the oracle's
    walk and B0 / B_tau match the oracle's at the 1e-5 bar."""
    wl = synth.MEDIUM
    inst = synth.make_instance(wl, 0)
    print(f"compensated fit {wl.name}", flush=True)
    res = O.fit(inst.X_parity, wl.p)
    X = _dev(inst.X32, dev)
    f = api.Fitter(wl.n, wl.m, wl.p, "mixed", dev, compensated=True)
    f.run(X)
    f.check()
    order = f.order.cpu().numpy()
    assert PA.order_violations(order, res["S"]) == []
    if np.array_equal(order, res["order"]):
        B0_ref, Bl_ref = res["B0"], res["B_lags"]
    else:
        B0_ref, Bl_ref = O.estimate_B(res["E"], order, res["M"])
    assert PA.b_rel_error(f.B0.cpu().numpy(), B0_ref) <= PA.B_TOL_FP32
    assert PA.b_rel_error(f.B_lags.cpu().numpy(), Bl_ref) <= PA.B_TOL_FP32
