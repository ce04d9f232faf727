"""Pins of the pruning oracle (adaptive lasso on B0 / B_tau, LARS-lasso path, BIC knot)."""
import math

import numpy as np
import pytest
from scipy.stats import norm
from sklearn.linear_model import lars_path

import synth
from oracle import prune as P
from oracle import varlingam as O


def _correlated_problem(seed, T=60, d=10):
    """Strongly correlated columns: paths with variables leaving and re-entering."""
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(T, d)) @ (0.9 * rng.normal(size=(d, d)))
    y = Z[:, :3] @ rng.normal(size=3) + 2.0 * rng.normal(size=T)
    return Z - Z.mean(0), y - y.mean()


SEEDS = range(12)


def test_paths_exercise_the_lasso_modification():
    leaves = sum(sum(e == -1 for e, _ in P.lars_lasso_path(*_correlated_problem(s))["events"])
                 for s in SEEDS)
    assert leaves >= 10


@pytest.mark.parametrize("seed", SEEDS)
def test_kkt_conditions_at_every_knot(seed):
    """Each knot is the lasso solution at lambda = max_j |z_j^T r|: every nonzero coefficient
    has z_j^T r = lambda sign(beta_j), every other |z_j^T r| <= lambda."""
    Z, y = _correlated_problem(seed)
    path = P.lars_lasso_path(Z, y)
    lam0 = np.abs(Z.T @ y).max()
    for b in path["knots"]:
        c = Z.T @ (y - Z @ b)
        lam = np.abs(c).max()
        nz = b != 0
        if nz.any():
            assert np.abs(c[nz] - lam * np.sign(b[nz])).max() <= 1e-9 * lam0


@pytest.mark.parametrize("seed", SEEDS)
def test_knots_match_scikit_learn_lars_lasso(seed):
    Z, y = _correlated_problem(seed)
    path = P.lars_lasso_path(Z, y)
    alphas, _, coefs = lars_path(Z, y, method="lasso")
    K = np.array(path["knots"]).T
    assert K.shape == coefs.shape
    assert np.abs(K - coefs).max() <= 1e-9 * np.abs(coefs).max()
    lams = [np.abs(Z.T @ (y - Z @ b)).max() for b in path["knots"]]
    np.testing.assert_allclose(np.array(lams) / len(y), alphas, rtol=1e-9, atol=1e-12)


def test_path_ends_at_least_squares():
    for seed in (0, 3, 7):
        Z, y = _correlated_problem(seed, T=200, d=15)
        path = P.lars_lasso_path(Z, y)
        assert path["events"][-1] == (0, -1)
        ols = np.linalg.lstsq(Z, y, rcond=None)[0]
        assert np.abs(path["knots"][-1] - ols).max() <= 1e-10 * np.abs(ols).max()


def test_one_regressor_closed_form():
    """d = 1: knots 0 and the OLS slope; BIC keeps the regressor iff -T ln(1 - R^2) > ln T."""
    rng = np.random.default_rng(3)
    T = 400
    for scale in (0.0, 0.05, 0.1, 0.2, 1.0):
        z = rng.normal(size=T)
        y = scale * z + rng.normal(size=T)
        z, y = z - z.mean(), y - y.mean()
        path = P.lars_lasso_path(z[:, None], y)
        slope = (z @ y) / (z @ z)
        assert len(path["knots"]) == 2 and abs(path["knots"][1][0] - slope) < 1e-13 * abs(slope)
        r2 = (z @ y) ** 2 / ((z @ z) * (y @ y))
        keep = -T * math.log(1 - r2) > math.log(T)
        assert P.bic_select(z[:, None], y, path["knots"])["knot"] == (1 if keep else 0)


def test_bic_is_the_gaussian_likelihood_criterion():
    """-2 ln L of the residuals under N(0, RSS/T), summed sample by sample with an independent
    density routine, plus df ln T equals the oracle's BIC plus T (1 + ln 2 pi)."""
    Z, y = _correlated_problem(4, T=80)
    path = P.lars_lasso_path(Z, y)
    sel = P.bic_select(Z, y, path["knots"])
    T = len(y)
    for b, bic in zip(path["knots"], sel["bic"]):
        r = y - Z @ b
        ll = norm.logpdf(r, scale=math.sqrt(r @ r / T)).sum()
        df = np.count_nonzero(b)
        assert abs(-2 * ll + df * math.log(T) - (bic + T * (1 + math.log(2 * math.pi)))) < 1e-8


def test_design_reproduces_the_unpruned_estimates():
    """OLS of each variable on its lag-0 predecessors and all lags is exactly (B0, B_tau) of
    the fit (Frisch-Waugh), which is what makes |b| the adaptive weights."""
    inst = synth.make_custom(6, 3000, 2, "laplace", 2, edge_prob=0.4, w_lo=0.2, w_hi=0.6)
    ref = O.fit(inst.X_parity, 2)
    for pos in range(6):
        y, Z, cols = P.regression_design(inst.X_parity, 2, ref["order"], pos)
        i = int(ref["order"][pos])
        b = np.linalg.lstsq(Z, y, rcond=None)[0]
        want = [ref["B0"][i, v] if t == 0 else ref["B_lags"][t - 1][i, v] for t, v in cols]
        np.testing.assert_allclose(b, want, rtol=0, atol=1e-10)


def test_scale_invariance():
    """Adaptive weights with exponent 1: rescaling series v by D_v maps the pruned matrices to
    D_i B_ij / D_j, with the same zeros."""
    inst = synth.make_custom(5, 1500, 1, "uniform", 5, edge_prob=0.4, w_lo=0.1, w_hi=0.5)
    X = inst.X_parity
    ref = O.fit(X, 1)
    D = np.array([0.3, 2.0, 7.0, 1.0, 0.05])
    a = P.prune(X, 1, ref["order"], ref["B0"], ref["B_lags"])
    S = D[:, None] / D[None, :]
    b = P.prune(X * D, 1, ref["order"], ref["B0"] * S, ref["B_lags"] * S)
    assert np.array_equal(a["B0"] != 0, b["B0"] != 0)
    assert np.array_equal(a["B_lags"] != 0, b["B_lags"] != 0)
    np.testing.assert_allclose(b["B0"], a["B0"] * S, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(b["B_lags"], a["B_lags"] * S, rtol=1e-9, atol=1e-12)


def test_zero_weight_column_is_left_out():
    inst = synth.make_custom(5, 1200, 1, "laplace", 6, edge_prob=0.5, w_lo=0.2, w_hi=0.6)
    ref = O.fit(inst.X_parity, 1)
    order = ref["order"]
    i, j = int(order[4]), int(order[1])
    B0 = ref["B0"].copy()
    B0[i, j] = 0.0
    out = P.prune(inst.X_parity, 1, order, B0, ref["B_lags"])
    assert out["B0"][i, j] == 0.0
    assert out["info"][4]["d"] == 4 + 5 - 1


def test_recovers_the_true_contemporaneous_support():
    """Long series, true order: the pruned B0 has exactly the generating edges, and the lag
    entries with |B_tau| >= 0.1 survive."""
    for seed in (1, 2):
        inst = synth.make_custom(6, 20000, 1, "uniform", seed, edge_prob=0.3, w_lo=0.3,
                                 w_hi=0.8)
        X = inst.X_parity
        M, _, E = O.fit_var(X, 1)
        B0, Bl = O.estimate_B(E, inst.perm, M)
        out = P.prune(X, 1, inst.perm, B0, Bl)
        assert np.array_equal(out["B0"] != 0, inst.B0 != 0), seed
        big = np.abs(inst.B_lags) >= 0.1
        assert np.all(out["B_lags"][big] != 0)
        assert np.abs(out["B0"] - inst.B0).max() < 0.05


def test_intercept_absorbs_constant_offsets():
    """The regressions carry an intercept: adding a constant to every series changes nothing."""
    inst = synth.make_custom(5, 1500, 2, "laplace", 9, edge_prob=0.4, w_lo=0.2, w_hi=0.6)
    X = inst.X_parity
    ref = O.fit(X, 2)
    a = P.prune(X, 2, ref["order"], ref["B0"], ref["B_lags"])
    b = P.prune(X + 40.0 * np.arange(1, 6), 2, ref["order"], ref["B0"], ref["B_lags"])
    assert np.array_equal(a["B0"] != 0, b["B0"] != 0)
    np.testing.assert_allclose(b["B0"], a["B0"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(b["B_lags"], a["B_lags"], rtol=0, atol=1e-9)


def test_duplicate_column_is_excluded():
    """A column equal to an active one cannot enter (its Schur complement is 0): the knots are
    those of the path without it, and its coefficient stays 0."""
    rng = np.random.default_rng(1)
    Z = rng.normal(size=(300, 8))
    y = Z[:, :3] @ np.array([1.0, -0.5, 0.3]) + rng.laplace(size=300)
    Z, y = Z - Z.mean(0), y - y.mean()
    a = P.lars_lasso_path(Z, y)
    b = P.lars_lasso_path(np.hstack([Z, Z[:, [1]]]), y)
    Ka, Kb = np.array(a["knots"]), np.array(b["knots"])
    assert Ka.shape[0] == Kb.shape[0]
    assert np.abs(Kb[:, :8] - Ka).max() <= 1e-12 * np.abs(Ka).max()
    assert np.all(Kb[:, 8] == 0.0)
