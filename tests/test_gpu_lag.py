"""GPU parity of the VAR lag-order selection (varlingam_select_lag) against the FP64 oracle
(oracle.varlingam.select_lag): ln det Sigma_p, AIC and BIC for every p = 1 .. p_max on the common
sample, and the selected orders.

Tolerance: the GPU forms the Gram matrices from exact products of the FP32 data with FP64 sums,
factors in FP64 and takes ln det from the factor of T Sigma_p = Yc^T Yc - sum_tau W_tau^T W_tau,
so each entry carries ~cond(G) 1e-16 relative error; ln det moves by about m times that.  1e-8
absolute is far above it and far below what a dropped lag block or a wrong sample range costs
(>= 1e-4 on these series).  The selected p must match unless the oracle's own criterion gap
between its best and the GPU's pick is below 1e-9."""
import numpy as np
import pytest
import torch

import synth
from oracle import varlingam as O

pytestmark = pytest.mark.gpu
TOL = 1e-8


@pytest.fixture(scope="module")
def api():
    from paper_2409_05500_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _api


def _check(api, X32, p_max):
    ref = O.select_lag(X32.astype(np.float64), p_max)
    ld, aic, bic, (pa, pb) = api.select_lag(torch.from_numpy(X32).cuda(), p_max)
    ld, aic, bic = (t.cpu().numpy() for t in (ld, aic, bic))
    err = max(np.abs(ld - ref["logdet"]).max(), np.abs(aic - ref["aic"]).max(),
              np.abs(bic - ref["bic"]).max())
    print(f"  max |err| {err:.2e}; p_aic {pa} ({ref['p_aic']}), p_bic {pb} ({ref['p_bic']})",
          flush=True)
    assert err <= TOL
    assert ref["aic"][pa - 1] - ref["aic"].min() <= 1e-9
    assert ref["bic"][pb - 1] - ref["bic"].min() <= 1e-9


CASES = [("m10_n1000", synth.make_instance(synth.SMALL, 0).X32, 4),
         ("m100_n5000", synth.make_instance(synth.MEDIUM, 0).X32, 3),
         ("m37_n2100_p2", synth.make_custom(37, 2100, 2, "t4", 3, edge_prob=0.1, w_lo=0.1,
                                            w_hi=0.4).X32, 5),
         ("m65_n900", synth.make_custom(65, 900, 1, "laplace", 4, edge_prob=0.05, w_lo=0.1,
                                        w_hi=0.5).X32, 2)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_select_lag_matches_oracle(api, case):
    name, X32, p_max = case
    print(f"lag selection {name} p_max={p_max}", flush=True)
    _check(api, np.ascontiguousarray(X32), p_max)


def test_select_lag_univariate_and_strided(api):
    rng = np.random.default_rng(3)
    x = np.zeros(1500)
    for t in range(2, 1500):
        x[t] = 0.5 * x[t - 1] - 0.3 * x[t - 2] + rng.laplace()
    _check(api, x[:, None].astype(np.float32), 4)
    # a strided view (ldx > m): the first 7 columns of a 9-column array
    X = synth.make_custom(9, 1200, 1, "uniform", 6).X32
    ref = O.select_lag(X[:, :7].astype(np.float64), 3)
    ld, _, _, _ = api.select_lag(torch.from_numpy(X).cuda()[:, :7], 3)
    assert np.abs(ld.cpu().numpy() - ref["logdet"]).max() <= TOL


def test_select_lag_recovers_the_generating_order(api):
    inst = synth.make_custom(6, 8000, 2, "laplace", 8, edge_prob=0.2, w_lo=0.1, w_hi=0.4)
    _, _, _, (pa, pb) = api.select_lag(torch.from_numpy(inst.X32).cuda(), 4)
    assert pb == 2 and pa >= 2
