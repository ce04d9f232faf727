"""Reference gradient of the pairwise score (test infrastructure only; see package doc).

An independent re-implementation of the score in torch (CPU, float64) whose autograd gives
dL/dE for L = <G, S(E)> with an m x m cotangent G.  The forward follows the same steps as
`oracle.varlingam.pairwise_stats` but vectorised over pairs (no code is shared with it):
standardise (Sec. 3 step 1), residual of every ordered pair (Eq. 1) re-standardised,
entropy approximation (Eq. 2), S[i, j] = (Hx[j] + Hr[i, j]) - (Hx[i] + Hr[j, i]).

Pinned by (tests marked "not gpu"): central finite differences of the NumPy oracle's S,
agreement of the forward with the NumPy oracle, and three invariants that hold exactly:
column sums of dL/dE are zero (shift invariance), <dL/de_i, e_i - mean e_i> = 0 (scale
invariance), and a symmetric cotangent gives dL/dE = 0 (S is antisymmetric).
"""
from __future__ import annotations

import math

import torch

K1, K2, GAMMA = 79.047, 7.4129, 0.37457
H_GAUSS = (1.0 + math.log(2.0 * math.pi)) / 2.0


def _log_cosh(u):
    a = u.abs()
    return a + torch.log1p(torch.exp(-2.0 * a)) - math.log(2.0)


def _entropy(u, dim):
    a = _log_cosh(u).mean(dim)
    b = (u * torch.exp(-0.5 * u * u)).mean(dim)
    return H_GAUSS - K1 * (a - GAMMA) ** 2 - K2 * b ** 2


def score(E: torch.Tensor) -> torch.Tensor:
    """S(E) for an n x m float64 tensor (differentiable)."""
    mu = E.mean(0, keepdim=True)
    xc = E - mu
    sd = torch.sqrt((xc * xc).mean(0, keepdim=True))
    X = xc / sd                                         # n x m standardised
    m = X.shape[1]
    Hx = _entropy(X, 0)                                 # m
    xi = X[:, :, None]                                  # n x m x 1  (i)
    xj = X[:, None, :]                                  # n x 1 x m  (j)
    cov = (xi * xj).mean(0)                             # m x m, 1/n moments of standardised data
    var = (xj * xj).mean(0)
    R = xi - (cov / var)[None] * xj                     # r_{i<-j}[t, i, j]
    eye = torch.eye(m, dtype=E.dtype, device=E.device, requires_grad=False)
    Rm = R.mean(0, keepdim=True)
    Rs = torch.sqrt(((R - Rm) ** 2).mean(0, keepdim=True) + eye[None])   # guard the diagonal
    U = (R - Rm) / Rs
    Hr = _entropy(U, 0) * (1.0 - eye)
    S = (Hx[None, :] + Hr) - (Hx[:, None] + Hr.T)
    return S * (1.0 - eye)


def grad_E(E, G) -> torch.Tensor:
    """dL/dE for L = sum(G * S(E)); E n x m, G m x m (numpy or torch), float64 result."""
    Et = torch.as_tensor(E, dtype=torch.float64).clone().requires_grad_(True)
    Gt = torch.as_tensor(G, dtype=torch.float64)
    L = (Gt * score(Et)).sum()
    (g,) = torch.autograd.grad(L, Et)
    return g.detach()
