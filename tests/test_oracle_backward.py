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
