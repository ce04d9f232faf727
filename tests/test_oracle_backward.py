"""Pins of the reference gradient of the pairwise score (oracle/backward.py)."""
import numpy as np
import pytest
import torch

from oracle import varlingam as O
from oracle import backward as OB


def _data(m, n, seed):
    rng = np.random.default_rng(seed)
    mix = np.eye(m) + 0.4 * np.tril(rng.normal(size=(m, m)), -1)
    return rng.laplace(size=(n, m)) @ mix.T + rng.normal(0, 2, m)


def test_forward_matches_numpy_oracle():
    E = _data(6, 700, 0)
    _, _, S = O.pairwise_stats(E)
    St = OB.score(torch.tensor(E)).numpy()
    np.testing.assert_allclose(St, S, atol=1e-12)


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences_of_the_numpy_oracle(seed):
    m, n = 4, 200
    E = _data(m, n, seed)
    G = np.random.default_rng(seed + 10).normal(size=(m, m))
    g = OB.grad_E(E, G).numpy()
    rng = np.random.default_rng(seed + 20)
    for _ in range(12):
        t, i = int(rng.integers(n)), int(rng.integers(m))
        h = 1e-6 * E[:, i].std()
        Ep, Em = E.copy(), E.copy()
        Ep[t, i] += h
        Em[t, i] -= h
        Lp = np.sum(G * O.pairwise_stats(Ep)[2])
        Lm = np.sum(G * O.pairwise_stats(Em)[2])
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[t, i] - fd) <= 1e-6 * max(1.0, np.abs(g).max()), (t, i, g[t, i], fd)


def test_gradient_invariants():
    m, n = 7, 500
    E = _data(m, n, 3)
    G = np.random.default_rng(4).normal(size=(m, m))
    g = OB.grad_E(E, G).numpy()
    scale = np.abs(g).max()
    # shift invariance of S: every column of dL/dE sums to zero
    assert np.max(np.abs(g.sum(0))) < 1e-12 * n * scale
    # scale invariance: <dL/de_i, e_i - mean> = 0
    Ec = E - E.mean(0)
    assert np.max(np.abs((g * Ec).sum(0))) < 1e-10 * n * scale * np.abs(Ec).max()
    # a symmetric cotangent sees only S + S^T = 0
    gs = OB.grad_E(E, G + G.T).numpy()
    assert np.max(np.abs(gs)) < 1e-12 * scale


@pytest.mark.parametrize("m,n,seed", [(5, 300, 5), (9, 1100, 6)])
def test_column_gradient_matches_autograd(m, n, seed):
    E = _data(m, n, seed)
    G = np.random.default_rng(seed + 1).normal(size=(m, m))
    g = OB.grad_E(E, G).numpy()
    cols = list(range(m))
    gc = OB.grad_E_columns(E, G, cols, block=3)     # several partner blocks
    np.testing.assert_allclose(gc, g[:, cols], rtol=0, atol=1e-11 * np.abs(g).max())


def test_column_scale_bounds_the_gradient_and_ignores_the_sign_of_G():
    """The magnitudes returned with the columns: mag >= |dL/dE| elementwise (it sums the
    absolute sizes of the same terms), and both are unchanged by the sign of G (they see only
    |G - G^T|)."""
    m, n = 6, 400
    E = _data(m, n, 8)
    G = np.random.default_rng(9).normal(size=(m, m))
    g, sc, cs = OB.grad_E_columns(E, G, list(range(m)), with_scale=True)
    assert np.all(sc >= np.abs(g) * (1 - 1e-12))
    g2, sc2, cs2 = OB.grad_E_columns(E, -G, list(range(m)), with_scale=True)
    np.testing.assert_allclose(g2, -g, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(sc2, sc, rtol=1e-12)
    np.testing.assert_allclose(cs2, cs, rtol=1e-12)
    assert np.all(cs > 0)
