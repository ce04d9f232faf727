"""Pins of the oracle's Sec. 3 step 5 refinement (the original DirectLiNGAM search replaces
every remaining column by its least-squares residual on the variable just taken)."""
import numpy as np

import synth
from oracle import varlingam as O


def test_refined_columns_satisfy_the_residual_identities():
    """Each refined column is centred, has zero sample covariance with the standardised pick
    and variance 1 - rho^2 (rho from the original columns, computed independently with
    numpy's correlation); the pick's own column and columns outside U are left alone."""
    rng = np.random.default_rng(11)
    n, m = 4000, 5
    X = rng.laplace(size=(n, m)) @ (np.eye(m) + 0.4 * rng.normal(size=(m, m)))
    X0 = X.copy()
    c, U = 2, [0, 2, 3, 4]          # variable 1 was taken earlier: not refined again
    O.refine(X, U, c)
    xc = (X0[:, c] - X0[:, c].mean()) / X0[:, c].std()
    R = np.corrcoef(X0.T)
    for j in (0, 3, 4):
        assert abs(X[:, j].mean()) < 1e-12
        assert abs(np.mean(X[:, j] * xc)) < 1e-12
        assert abs(np.mean(X[:, j] ** 2) - (1.0 - R[j, c] ** 2)) < 1e-12
    np.testing.assert_array_equal(X[:, c], X0[:, c])
    np.testing.assert_array_equal(X[:, 1], X0[:, 1])


def test_refinement_returns_the_hidden_noise():
    """x0 = e0, x1 = 2 e0 + e1 with e1 made exactly orthogonal to e0 in the sample: the
    residual of x1 on the pick x0 is e1 itself up to a positive factor (correlation +1).  A
    regression the wrong way round (x0 on x1) or a flipped sign fails."""
    rng = np.random.default_rng(5)
    n = 3000
    e0 = rng.uniform(-1, 1, n)
    e0 -= e0.mean()
    e1 = rng.laplace(size=n)
    e1 -= e1.mean()
    e1 -= (e1 @ e0) / (e0 @ e0) * e0
    X = np.column_stack([e0, 2.0 * e0 + e1])
    O.refine(X, [0, 1], 0)
    assert abs(np.corrcoef(X[:, 1], e1)[0, 1] - 1.0) < 1e-12


def test_search_step_uses_the_refined_data():
    """After the first pick, the iterative search scores the refined columns: its second pick
    equals the first pick of a fresh search on the data refined by hand with refine()."""
    inst = synth.make_custom(5, 3000, 1, "uniform", 7, edge_prob=0.6, w_lo=0.4, w_hi=0.9)
    _, _, E = O.fit_var(inst.X_parity, 1)
    full = O.directlingam_iterative(E)
    X = E.copy()
    U = list(range(5))
    c = int(full[0])
    U.remove(c)
    O.refine(X, U, c)
    rest = O.directlingam_iterative(X[:, U])
    assert U[int(rest[0])] == int(full[1])
