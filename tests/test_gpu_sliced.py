"""VL_PREC_SLICED (the three GEMM-shaped products from int8 slices, the Ozaki scheme) against
the FP64 oracle and against the FP64-MFMA products of VL_PREC_MIXED, through the C ABI.

Bounds: each product term carries at most 2^-39 of 2^(e_a + e_b), the two vectors' power-of-two
scales (e = the exponent of the vector's largest magnitude), so a covariance entry over n
samples, divided by n, is within 2^-39 2^(e_i + e_j) of the exact one (FP64 rounding besides).
The VAR coefficients and E are held to the bars of the FP64 products (test_gpu_parity.py): the
Gram's error, ~1e-10 relative here, moves them far less than those bars.
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


def _exponent(v):
    """e with |v| < 2^e for every entry (the slices' power-of-two scale)."""
    mx = float(np.abs(v).max())
    return int(np.frexp(mx)[1]) if mx > 0 else 0


@pytest.mark.parametrize("wl,seed", [(synth.SMALL, 0), (synth.SMALL, 4), (synth.MEDIUM, 0),
                                     (synth.FINANCE, 0)])
def test_var_fit_sliced_parity(api, dev, wl, seed):
    print(f"sliced var fit {wl.name} seed {seed}", flush=True)
    inst = synth.make_instance(wl, seed)
    oM, oc, oE = O.fit_var(inst.X_parity, wl.p)
    X = _dev(inst.X32, dev)
    M, c, E = [t.cpu().numpy() for t in api.fit_var(X, wl.p, "sliced")]
    eM = np.max(np.abs(M - oM)) / max(1.0, np.abs(oM).max())
    print(f"  M rel err {eM:.1e}, max|dE| {np.abs(E - oE).max():.1e}", flush=True)
    assert eM <= 1e-7
    assert np.max(np.abs(c - oc)) <= 1e-7 * max(1.0, np.abs(inst.X_parity).max())
    assert np.max(np.abs(E - oE)) <= 2.0 ** -23 * np.abs(oE).max() + 1e-7
    # the FP64-MFMA products of MIXED: the same fit to well within those bars
    Mm, cm, Em = [t.cpu().numpy() for t in api.fit_var(X, wl.p, "mixed")]
    dM = np.max(np.abs(M - Mm)) / max(1.0, np.abs(Mm).max())
    print(f"  vs mixed: M rel {dM:.1e}, E max diff {np.abs(E - Em).max():.1e}", flush=True)
    assert dM <= 1e-8


@pytest.mark.parametrize("m,n", [(2, 50), (5, 64), (13, 255), (37, 1234), (65, 2049),
                                 (130, 3001)])
def test_pairwise_sliced_covariance(api, dev, m, n):
    """Ragged shapes (tiles of 64, K padded to 32): the covariance within the slice bound of
    the exact one, and Hx, Hr, S at the bars of the FP64 covariance."""
    print(f"sliced pairwise m={m} n={n}", flush=True)
    rng = np.random.default_rng(m + 7 * n)
    mix = np.eye(m) + 0.3 * np.tril(rng.normal(size=(m, m)), -1)
    E32 = (rng.laplace(size=(n, m)) @ mix.T + rng.normal(0, 5, m)).astype(np.float32)
    E64 = E32.astype(np.float64)
    Hx, Hr, S, Cov = [t.cpu().numpy() for t in api.pairwise_stats(_dev(E32, dev), "sliced")]
    oCov = np.cov(E64.T, bias=True)
    Ec = E64 - E64.mean(0)
    ex = np.array([_exponent(Ec[:, i]) for i in range(m)])
    bound = 2.0 ** (-39 + ex[:, None] + ex[None, :]) + 1e-15 * np.abs(oCov).max()
    ratio = float((np.abs(Cov - oCov) / bound).max())
    print(f"  covariance error / slice bound {ratio:.3f}", flush=True)
    assert ratio <= 1.0
    assert np.array_equal(Cov, Cov.T)
    oHx, oHr, oS = O.pairwise_stats(E64)
    np.testing.assert_allclose(Hx, oHx, rtol=0, atol=TOL_HX)
    np.testing.assert_allclose(Hr, oHr, rtol=0, atol=TOL_HR)
    np.testing.assert_allclose(S, oS, rtol=0, atol=TOL_S)


@pytest.mark.parametrize("wl,seed", [(synth.SMALL, 2), (synth.MEDIUM, 0)])
def test_fit_sliced_end_to_end(api, dev, wl, seed):
    """Order walked on the oracle's S, B0 / B_tau at the 1e-5 bar."""
    inst = synth.make_instance(wl, seed)
    res = O.fit(inst.X_parity, wl.p)
    g = api.fit(_dev(inst.X32, dev), wl.p, "sliced")
    order = g.order.cpu().numpy()
    assert PA.order_violations(order, res["S"]) == []
    if np.array_equal(order, res["order"]):
        B0_ref, Bl_ref = res["B0"], res["B_lags"]
    else:
        B0_ref, Bl_ref = O.estimate_B(res["E"], order, res["M"])
    e0 = PA.b_rel_error(g.B0.cpu().numpy(), B0_ref)
    e1 = PA.b_rel_error(g.B_lags.cpu().numpy(), Bl_ref)
    print(f"sliced fit {wl.name}: B0 {e0:.1e} B_lags {e1:.1e}", flush=True)
    assert e0 <= PA.B_TOL_FP32 and e1 <= PA.B_TOL_FP32


def test_sliced_deterministic_and_fitter(api, dev):
    """Bit-identical repeats (int32 sums do not depend on the order of the K loop) and the same
    result through the preallocated Fitter."""
    wl = synth.MEDIUM
    X = _dev(synth.make_instance(wl, 1).X32, dev)
    a = api.fit(X, wl.p, "sliced")
    b = api.fit(X, wl.p, "sliced")
    assert torch.equal(a.B0, b.B0) and torch.equal(a.S, b.S) and torch.equal(a.M, b.M)
    f = api.Fitter(wl.n, wl.m, wl.p, "sliced", dev)
    f.run(X)
    f.check()
    assert torch.equal(f.B0, a.B0) and torch.equal(f.order, a.order)
