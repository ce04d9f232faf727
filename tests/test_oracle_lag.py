"""Pins of the oracle's VAR lag-order selection (AIC / BIC over p = 1 .. p_max on the common
sample t = p_max .. n-1, maximum-likelihood residual covariance)."""
import math

import numpy as np
from scipy.stats import multivariate_normal

import synth
from oracle import varlingam as O


def _var_series(m, n, p, seed, radius=0.5):
    """A stable VAR(p) with Laplace shocks (direct simulation, no generator reuse)."""
    rng = np.random.default_rng(seed)
    A = [rng.normal(0, 0.2, (m, m)) for _ in range(p)]
    comp = np.zeros((m * p, m * p))
    comp[:m] = np.hstack(A)
    comp[m:, :-m] = np.eye(m * (p - 1))
    rad = max(abs(np.linalg.eigvals(comp)))
    A = [a * radius / rad for a in A]
    x = np.zeros((n + 500, m))
    for t in range(p, n + 500):
        x[t] = sum(A[k] @ x[t - 1 - k] for k in range(p)) + rng.laplace(size=m)
    return x[500:]


def test_univariate_closed_form():
    """m = 1, p = 1: the ML residual variance of a regression on one lag with intercept is
    var(y) (1 - corr(y, y_lag)^2) with population moments over the common sample."""
    x = _var_series(1, 2000, 1, 0)
    r = O.select_lag(x, 3)
    y, z = x[3:, 0], x[2:-1, 0]
    rho = np.corrcoef(y, z)[0, 1]
    var = np.mean((y - y.mean()) ** 2) * (1 - rho ** 2)
    assert abs(r["logdet"][0] - math.log(var)) < 1e-11


def test_gaussian_likelihood_brute_force():
    """-2/T times the Gaussian log-likelihood of the residuals under their ML covariance,
    summed sample by sample with an independent density routine, equals
    ln det Sigma_p + m (1 + ln 2 pi) for every p (so AIC / BIC differ from the classical
    criteria by a constant only)."""
    x = _var_series(3, 800, 2, 1)
    p_max = 3
    r = O.select_lag(x, p_max)
    T = len(x) - p_max
    for p in range(1, p_max + 1):
        Y = x[p_max:]
        Z = np.hstack([x[p_max - tau: len(x) - tau] for tau in range(1, p + 1)] + [np.ones((T, 1))])
        E = Y - Z @ np.linalg.lstsq(Z, Y, rcond=None)[0]
        Sig = E.T @ E / T
        ll = sum(multivariate_normal.logpdf(E[t], mean=np.zeros(3), cov=Sig) for t in range(T))
        assert abs(-2.0 * ll / T - (r["logdet"][p - 1] + 3 * (1 + math.log(2 * math.pi)))) < 1e-9


def test_nested_models_never_fit_worse():
    x = _var_series(4, 600, 2, 2)
    ld = O.select_lag(x, 5)["logdet"]
    assert np.all(np.diff(ld) <= 1e-12)


def test_scale_invariance():
    x = _var_series(3, 700, 1, 3)
    D = np.array([0.5, 3.0, 11.0])
    a, b = O.select_lag(x, 4), O.select_lag(x * D, 4)
    np.testing.assert_allclose(b["logdet"] - a["logdet"], 2 * np.sum(np.log(D)), atol=1e-10)
    assert (a["p_aic"], a["p_bic"]) == (b["p_aic"], b["p_bic"])


def test_bic_recovers_the_generating_lag_order():
    for p_true, seed in ((1, 4), (2, 5), (3, 6)):
        x = _var_series(3, 20000, p_true, seed)
        r = O.select_lag(x, 5)
        assert r["p_bic"] == p_true, (p_true, r["bic"])
        assert r["p_aic"] >= p_true            # AIC does not under-fit on long series


def test_white_noise_picks_the_smallest_lag():
    x = np.random.default_rng(7).laplace(size=(5000, 4))
    assert O.select_lag(x, 4)["p_bic"] == 1


def test_generator_series():
    inst = synth.make_custom(6, 8000, 2, "laplace", 8, edge_prob=0.2, w_lo=0.1, w_hi=0.4)
    assert O.select_lag(inst.X_parity, 4)["p_bic"] == 2


def test_penalty_per_lag_matches_the_likelihood_ratio_degrees_of_freedom():
    """Wilks: when the extra lag is superfluous, T (ln det Sigma_p - ln det Sigma_{p+1}) is
    asymptotically chi-square with one degree of freedom per added coefficient.  Its Monte
    Carlo mean over VAR(1) series fixes that count (m^2 = 9 here, against m = 3 or 2 m^2), and
    the criteria's increments per lag must be 2 (AIC) and ln T (BIC) times it, over T."""
    m, n, R = 3, 600, 300
    drops, d_aic, d_bic = [], [], []
    for r in range(R):
        res = O.select_lag(_var_series(m, n, 1, 1000 + r), 2)
        T = n - 2
        drops.append(T * (res["logdet"][0] - res["logdet"][1]))
        d_aic.append(T * ((res["aic"][1] - res["logdet"][1]) - (res["aic"][0] - res["logdet"][0])))
        d_bic.append(T * ((res["bic"][1] - res["logdet"][1]) - (res["bic"][0] - res["logdet"][0])))
    dof = float(np.mean(drops))          # chi2_9: mean 9, standard error sqrt(18 / R) = 0.25
    assert abs(dof - m * m) < 1.2, dof
    assert abs(np.mean(d_aic) - 2 * dof) < 2.4
    assert abs(np.mean(d_bic) - math.log(n - 2) * dof) < 1.2 * math.log(n - 2)
