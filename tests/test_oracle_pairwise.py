"""Pins of the oracle's residual (Eq. 1) and pairwise score (Eq. 2, Eq. 3 argument)."""
import math

import numpy as np
import pytest

import synth
from oracle import varlingam as O


def _data(m=6, n=3000, seed=0):
    rng = np.random.default_rng(seed)
    e = rng.laplace(0, 1, (n, m))
    mix = np.eye(m) + np.tril(rng.uniform(-0.6, 0.6, (m, m)), -1)
    return e @ mix.T + rng.normal(0, 3, m)       # correlated, shifted columns


def test_residual_is_orthogonal_and_has_variance_one_minus_rho2():
    X = O.standardize_columns(_data())
    for i in range(X.shape[1]):
        for j in range(X.shape[1]):
            if i == j:
                continue
            r = O.residual(X[:, i], X[:, j])
            rho = np.mean(X[:, i] * X[:, j])
            assert abs(np.mean(r * X[:, j])) < 1e-14           # least-squares normal equation
            assert abs(np.mean(r)) < 1e-14
            assert abs(np.var(r) - (1.0 - rho * rho)) < 1e-13


def test_residual_slope_uses_consistent_moments():
    # regression of x on itself plus independent noise: slope must be exactly the OLS slope
    rng = np.random.default_rng(3)
    xj = rng.normal(size=500)
    xi = 0.7 * xj + rng.normal(size=500)
    slope = np.polyfit(xj, xi, 1)[0]
    r = O.residual(xi, xj)
    np.testing.assert_allclose(xi - r, slope * xj, rtol=1e-10)


def test_standardize_population_moments_and_degenerate():
    v = O.standardize(np.arange(10.0))
    assert abs(v.mean()) < 1e-15 and abs(v.std() - 1.0) < 1e-15   # ddof = 0
    with pytest.raises(ValueError):
        O.standardize(np.ones(10))


def test_score_antisymmetric_zero_diagonal_bitwise():
    _, _, S = O.pairwise_stats(_data())
    assert np.array_equal(S, -S.T)
    assert np.all(np.diag(S) == 0.0)


def test_score_invariant_to_affine_column_maps():
    E = _data()
    _, _, S = O.pairwise_stats(E)
    rng = np.random.default_rng(11)
    a = rng.uniform(0.5, 3, E.shape[1]) * np.where(rng.random(E.shape[1]) < 0.5, -1, 1)
    b = rng.normal(0, 10, E.shape[1])
    _, _, S2 = O.pairwise_stats(E * a + b)
    np.testing.assert_allclose(S2, S, atol=1e-11)


def test_score_permutation_equivariance_bitwise():
    E = _data()
    _, _, S = O.pairwise_stats(E)
    P = np.random.default_rng(5).permutation(E.shape[1])
    _, _, SP = O.pairwise_stats(E[:, P])
    assert np.array_equal(SP, S[np.ix_(P, P)])


def test_score_sign_points_from_cause_to_effect():
    # x -> y with non-Gaussian cause and noise: S[x, y] > 0 (x precedes y)
    rng = np.random.default_rng(2)
    n = 20000
    x = rng.uniform(-1, 1, n)
    y = 0.8 * x + rng.uniform(-1, 1, n)
    _, _, S = O.pairwise_stats(np.column_stack([x, y]))
    assert S[0, 1] > 0.0
    _, _, S = O.pairwise_stats(np.column_stack([y, x]))
    assert S[1, 0] > 0.0


def test_pair_moments_match_matrix():
    E = _data(m=4)
    Hx, Hr, S, mom = O.pairwise_stats(E, return_moments=True)
    for i, j in [(0, 1), (3, 2), (1, 3)]:
        a, b = O.pair_moments(E, i, j)
        assert abs(a - mom["A"][i, j]) < 1e-14 and abs(b - mom["B"][i, j]) < 1e-14
        assert abs(O.entropy_from_moments(a, b) - Hr[i, j]) < 1e-13


def test_degenerate_pair_raises():
    rng = np.random.default_rng(0)
    x = rng.laplace(size=1000)
    with pytest.raises(ValueError):
        O.pairwise_stats(np.column_stack([x, -2.0 * x + 1.0, rng.laplace(size=1000)]))


def test_residual_entropy_by_brute_force_definition():
    """Tiny-n brute force: every quantity recomputed with explicit Python loops."""
    E = _data(m=3, n=64, seed=9)
    Hx, Hr, S = O.pairwise_stats(E)
    n, m = E.shape

    def mean(v):
        return sum(v) / len(v)

    cols = []
    for i in range(m):
        c = [float(E[t, i]) for t in range(n)]
        mu = mean(c)
        sd = math.sqrt(mean([(v - mu) ** 2 for v in c]))
        cols.append([(v - mu) / sd for v in c])

    def H(u):
        a = mean([math.log(math.cosh(v)) for v in u])
        b = mean([v * math.exp(-v * v / 2) for v in u])
        return (1 + math.log(2 * math.pi)) / 2 - 79.047 * (a - 0.37457) ** 2 - 7.4129 * b * b

    for i in range(m):
        assert abs(H(cols[i]) - Hx[i]) < 1e-12
        for j in range(m):
            if i == j:
                continue
            rho = mean([cols[i][t] * cols[j][t] for t in range(n)])
            r = [cols[i][t] - rho * cols[j][t] for t in range(n)]
            mu = mean(r)
            sd = math.sqrt(mean([(v - mu) ** 2 for v in r]))
            assert abs(H([(v - mu) / sd for v in r]) - Hr[i, j]) < 1e-12
    for i in range(m):
        for j in range(m):
            if i != j:
                t_ij = Hx[i] - Hr[i, j]
                t_ji = Hx[j] - Hr[j, i]
                assert abs(S[i, j] - (t_ji - t_ij)) < 1e-13


def test_synth_instance_is_float32_roundtrip():
    inst = synth.make_instance(synth.SMALL, 0)
    assert inst.X32.dtype == np.float32 and inst.X32.shape == (1000, 10)
    assert np.array_equal(inst.X_parity, inst.X32.astype(np.float64))


def test_rows_computed_elsewhere_give_the_same_bits():
    """pairwise_stats with rows handed in (as worker processes compute them) equals the
    serial precompute bit for bit, and a short row list is refused."""
    rng = np.random.default_rng(9)
    E = rng.laplace(size=(700, 6)) @ (np.eye(6) + 0.3 * rng.normal(size=(6, 6)))
    ref = O.pairwise_stats(E)
    X = O.standardize_columns(E)
    rows = [O.pair_row(X, i) for i in reversed(range(6))][::-1]
    out = O.pairwise_stats(E, rows=rows)
    for a, b in zip(ref, out):
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        O.pairwise_stats(E, rows=rows[:5])
