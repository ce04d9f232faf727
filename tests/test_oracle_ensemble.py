"""Pins of the ensemble oracle (rolling windows, residual bootstrap, edge aggregation)."""
import numpy as np

import synth
from oracle import ensemble as EN
from oracle import varlingam as O


def test_identity_resample_reproduces_the_series():
    """Drawing the residual rows in their own order regenerates the observed series (the
    residuals are defined by x(t) = c + sum M_tau x(t - tau) + e(t))."""
    for p in (1, 2, 3):
        inst = synth.make_custom(5, 600, p, "laplace", p, edge_prob=0.4, w_lo=0.2, w_hi=0.6)
        X = inst.X_parity
        M, c, E = O.fit_var(X, p)
        x = EN.simulate_var(M, c, X[:p], E, np.arange(len(E)))
        assert np.abs(x - X).max() <= 1e-9 * np.abs(X).max()


def test_zero_residuals_reach_the_process_mean():
    rng = np.random.default_rng(1)
    m, p = 4, 2
    M = rng.normal(0, 0.15, (p, m, m))
    c = rng.normal(size=m)
    mu = np.linalg.solve(np.eye(m) - M.sum(0), c)
    x = EN.simulate_var(M, c, rng.normal(size=(p, m)), np.zeros((1, m)), np.zeros(400, int))
    assert np.abs(x[-1] - mu).max() <= 1e-10 * np.abs(mu).max()


def test_resample_uses_the_drawn_rows():
    """A single draw repeated: x*(t) - M x*(t-1) - c is that residual row at every step."""
    rng = np.random.default_rng(2)
    M = rng.normal(0, 0.2, (1, 3, 3))
    c = rng.normal(size=3)
    E = rng.normal(size=(10, 3))
    x = EN.simulate_var(M, c, np.zeros((1, 3)), E, np.array([7, 2, 2, 9]))
    for t, j in zip(range(1, 5), (7, 2, 2, 9)):
        np.testing.assert_allclose(x[t] - M[0] @ x[t - 1] - c, E[j], atol=1e-13)


def test_edge_frequency_special_cases():
    rng = np.random.default_rng(3)
    m, p, K = 6, 2, 5
    order = rng.permutation(m)
    B0 = rng.normal(size=(m, m)) * (rng.random((m, m)) < 0.5)
    Bl = rng.normal(size=(p, m, m)) * (rng.random((p, m, m)) < 0.5)
    same = EN.edge_frequency([order] * K, [B0] * K, [Bl] * K, 0.0)
    assert same["count"] == K
    assert np.array_equal(same["P0"], (B0 != 0).astype(float))
    assert np.array_equal(same["P_lags"], (Bl != 0).astype(float))
    pos = np.argsort(order)
    assert np.array_equal(same["P_order"], (pos[None, :] < pos[:, None]).astype(float))
    # two problems with reversed orders: every precedence has probability 1/2
    two = EN.edge_frequency([order, order[::-1]], [B0, -B0], [Bl, Bl], 0.0)
    off = ~np.eye(m, dtype=bool)
    assert np.all(two["P_order"][off] == 0.5) and np.all(np.diag(two["P_order"]) == 0)
    # the threshold is strict, invalid problems are left out
    thr = EN.edge_frequency([order] * 3, [B0, B0 * 0, B0 * 0], [Bl] * 3, 0.0,
                            valid=[True, True, False])
    assert thr["count"] == 2 and np.array_equal(thr["P0"], (B0 != 0) / 2)
    big = EN.edge_frequency([order], [B0], [Bl], float(np.abs(B0).max()))
    assert np.all(big["P0"] == 0)


def test_order_probabilities_of_a_pair_sum_to_one():
    rng = np.random.default_rng(4)
    m, K = 7, 9
    orders = [rng.permutation(m) for _ in range(K)]
    z = np.zeros((K, m, m))
    agg = EN.edge_frequency(orders, z, np.zeros((K, 1, m, m)))
    Po = agg["P_order"]
    off = ~np.eye(m, dtype=bool)
    np.testing.assert_allclose((Po + Po.T)[off], 1.0, atol=1e-15)


def test_rolling_windows_are_the_slices():
    inst = synth.make_custom(4, 1300, 1, "uniform", 5, edge_prob=0.5, w_lo=0.3, w_hi=0.7)
    X = inst.X_parity
    r = EN.rolling_windows(X, 1, 500, 400)
    assert r["starts"] == [0, 400, 800]
    one = O.fit(X[400:900], 1)
    assert np.array_equal(r["orders"][1], one["order"])
    np.testing.assert_allclose(r["B0"][1], one["B0"], atol=1e-12)


def test_bootstrap_recovers_strong_edges():
    """Long strongly non-Gaussian series: every generating B0 edge of magnitude >= 0.3 appears
    in (nearly) every resample, in the generating direction."""
    inst = synth.make_custom(4, 4000, 1, "uniform", 6, edge_prob=0.6, w_lo=0.4, w_hi=0.8)
    X = inst.X_parity
    rng = np.random.default_rng(7)
    idx = rng.integers(0, len(X) - 1, size=(8, len(X) - 1))
    r = EN.bootstrap(X, 1, idx, threshold=0.1)
    assert r["count"] == 8
    strong = np.abs(inst.B0) >= 0.3
    assert strong.any()
    assert np.all(r["P0"][strong] >= 0.875)
    assert np.all(r["P_order"][strong] >= 0.875)
