"""Pins of the oracle's VAR fit and B estimation (Sec. 2.1 and the B0 estimator of Sec. 4)."""
import numpy as np
import pytest

import synth
from oracle import varlingam as O


def test_var_residuals_orthogonal_to_regressors():
    inst = synth.make_custom(5, 800, 2, "laplace", 0)
    M, c, E = O.fit_var(inst.X_parity, 2)
    _, Z = O.var_design(inst.X_parity, 2)
    G = Z.T @ E
    assert np.max(np.abs(G)) < 1e-8 * np.max(np.abs(Z)) * np.max(np.abs(E)) * len(E)
    assert np.max(np.abs(E.mean(axis=0))) < 1e-12       # intercept -> zero-mean residuals


def test_var_normal_equations_route_agrees():
    inst = synth.make_custom(6, 1500, 2, "uniform", 1)
    M, c, E = O.fit_var(inst.X_parity, 2)
    Y, Z = O.var_design(inst.X_parity, 2)
    coef = np.linalg.solve(Z.T @ Z, Z.T @ Y)              # independent route
    np.testing.assert_allclose(M[0], coef[:6].T, atol=1e-10)
    np.testing.assert_allclose(M[1], coef[6:12].T, atol=1e-10)
    np.testing.assert_allclose(c, coef[12], atol=1e-10)


def test_ar1_closed_form():
    rng = np.random.default_rng(5)
    x = np.zeros(3000)
    for t in range(1, 3000):
        x[t] = 0.6 * x[t - 1] + rng.laplace()
    M, c, E = O.fit_var(x[:, None], 1)
    y, z = x[1:], x[:-1]
    slope = np.sum((z - z.mean()) * (y - y.mean())) / np.sum((z - z.mean()) ** 2)
    assert abs(M[0, 0, 0] - slope) < 1e-12
    assert abs(c[0] - (y.mean() - slope * z.mean())) < 1e-12


def test_var_recovers_reduced_form_on_long_series():
    inst = synth.make_custom(4, 60000, 1, "laplace", 3)
    M, _, _ = O.fit_var(inst.X_parity, 1)
    A = np.linalg.inv(np.eye(4) - inst.B0)
    np.testing.assert_allclose(M[0], A @ inst.B_lags[0], atol=0.03)


def test_var_shape_errors():
    with pytest.raises(ValueError):
        O.fit_var(np.random.default_rng(0).normal(size=(6, 5)), 1)    # n - p <= m p + 1
    x = np.random.default_rng(0).normal(size=(100, 2))
    with pytest.raises(ValueError):
        O.fit_var(np.column_stack([x, x[:, :1]]), 1)                   # singular design


def test_b0_ols_identity_and_triangularity():
    inst = synth.make_instance(synth.SMALL, 2)
    res = O.fit(inst.X_parity, 1)
    E, B0, order = res["E"], res["B0"], res["order"]
    Sigma = np.cov(E.T, bias=True)
    D = (np.eye(10) - B0) @ Sigma @ (np.eye(10) - B0).T
    off = D - np.diag(np.diag(D))
    assert np.max(np.abs(off)) < 1e-12            # OLS residuals are mutually uncorrelated
    pos = np.empty(10, int)
    pos[order] = np.arange(10)
    for i in range(10):
        for j in range(10):
            if pos[j] >= pos[i]:
                assert B0[i, j] == 0.0            # strictly lower-triangular in the order


def test_b0_ldl_route_agrees():
    """Second route: LDL^T (via Cholesky) of the order-permuted covariance gives B0 = I - L^-1."""
    inst = synth.make_instance(synth.SMALL, 4)
    res = O.fit(inst.X_parity, 1)
    K = res["order"]
    Sigma = np.cov(res["E"].T, bias=True)[np.ix_(K, K)]
    Lc = np.linalg.cholesky(Sigma)
    L = Lc / np.diag(Lc)[None, :]                 # unit lower-triangular factor
    BK = np.eye(10) - np.linalg.inv(L)
    B0 = np.zeros((10, 10))
    B0[np.ix_(K, K)] = BK
    np.testing.assert_allclose(B0, res["B0"], atol=1e-10)


def test_lag_matrices_structural_identity():
    """B_tau from estimate_B must satisfy the structural VAR equation row by row:
    (I - B0) x(t) - sum_tau B_tau x(t - tau) - (I - B0) c = (I - B0) e(t)."""
    inst = synth.make_custom(5, 400, 2, "uniform", 7)
    X = inst.X_parity
    M, c, E = O.fit_var(X, 2)
    _, _, S = O.pairwise_stats(E)
    order, _ = O.approx_order(S)
    B0, Bl = O.estimate_B(E, order, M)
    I = np.eye(5)
    lhs = X[2:] @ (I - B0).T - X[1:-1] @ Bl[0].T - X[:-2] @ Bl[1].T - (I - B0) @ c
    np.testing.assert_allclose(lhs, E @ (I - B0).T, atol=1e-10)


def test_generator_identity():
    inst = synth.make_custom(5, 200, 2, "uniform", 7)
    A = np.linalg.inv(np.eye(5) - inst.B0)
    for t in range(2):
        np.testing.assert_allclose((np.eye(5) - inst.B0) @ (A @ inst.B_lags[t]),
                                   inst.B_lags[t], atol=1e-12)


def test_b0_recovers_truth_given_true_order_long_series():
    inst = synth.make_custom(5, 50000, 1, "uniform", 6, edge_prob=0.6)
    M, c, E = O.fit_var(inst.X_parity, 1)
    B0, Bl = O.estimate_B(E, inst.perm, M)
    np.testing.assert_allclose(B0, inst.B0, atol=0.03)
    np.testing.assert_allclose(Bl[0], inst.B_lags[0], atol=0.03)


def test_covariance_route_of_b_equals_least_squares():
    """estimate_B_cov (normal equations on the population covariance) against estimate_B (one
    least-squares fit with intercept per variable) on two workloads and a random order."""
    for inst, p in ((synth.make_instance(synth.SMALL, 1), 1),
                    (synth.make_custom(30, 2000, 2, "laplace", 4, edge_prob=0.1), 2)):
        M, _, E = O.fit_var(inst.X_parity, p)
        m = E.shape[1]
        for order in (np.arange(m), np.random.default_rng(m).permutation(m)):
            B0, Bl = O.estimate_B(E, order, M)
            C0, Cl = O.estimate_B_cov(O.population_cov(E), order, M)
            np.testing.assert_allclose(C0, B0, rtol=0, atol=1e-10)
            np.testing.assert_allclose(Cl, Bl, rtol=0, atol=1e-10)


def test_population_cov_divisor():
    rng = np.random.default_rng(0)
    E = rng.normal(size=(500, 4))
    np.testing.assert_allclose(O.population_cov(E), np.cov(E.T, bias=True), atol=1e-14)
