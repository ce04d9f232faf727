"""Reference gradient of the pairwise score (test infrastructure only; see package doc).

An independent re-implementation of the score in torch (CPU, float64) whose autograd gives
dL/dE for L = <G, S(E)> with an m x m cotangent G.  The forward follows the same steps as
`oracle.varlingam.pairwise_stats` but vectorised over pairs (no code is shared with it):
standardise (Sec. 3 step 1), residual of every ordered pair (Eq. 1) re-standardised,
entropy approximation (Eq. 2), S[i, j] = (Hx[j] + Hr[i, j]) - (Hx[i] + Hr[j, i]).

`grad_E_columns` writes the same gradient out by the chain rule, one column of dL/dE at a
time in O(m n) (for sampled checks at sizes where the autograd graph does not fit in memory).

Pinned by (tests marked "not gpu"): central finite differences of the NumPy oracle's S,
agreement of the forward with the NumPy oracle, and three invariants that hold exactly:
column sums of dL/dE are zero (shift invariance), <dL/de_i, e_i - mean e_i> = 0 (scale
invariance), and a symmetric cotangent gives dL/dE = 0 (S is antisymmetric);
`grad_E_columns` is pinned by agreement with the autograd gradient.
"""
from __future__ import annotations

import math

import numpy as np
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


def grad_E_columns(E, G, cols, block: int = 128, with_scale: bool = False):
    """Columns `cols` of dL/dE (n x len(cols), float64), L = sum(G * S(E)), by the chain rule.

    With `with_scale`, also returns two magnitudes of the sum each element is (same shape),
    carried through the standardisation like the gradient:
      mag   the sum of the absolute sizes of its terms: |alpha| + |beta| per direction
            (|tanh| <= 1, |(1-u^2)e^{-u^2/2}| <= 1), the Hx term, and for the rho chain
            |x_j(t)| / n times the sum over samples of the absolute sizes of R_ij's terms;
      cmag  the same sums with |alpha| + |beta| replaced by (2 k1 + 2 k2) |G_ij - G_ji| / n:
            the change of the element per unit absolute error of the moments A, B that the
            coefficients alpha = -2 k1 (A - gamma) dL/dHr, beta = -2 k2 B dL/dHr are made from.
    A sum of terms each evaluated to a relative accuracy of k units of rounding u, with
    coefficients from moments accurate to dA, differs from the exact sum by at most about
    k u mag + dA cmag (the usual forward error bound of a floating-point sum), whatever the
    cancellation.

    With x the standardised columns (population moments), rho_ij = mean(x_i x_j),
    s_ij = sqrt(1 - rho_ij^2) and u_ij = (x_i - rho_ij x_j) / s_ij (Eq. 1 re-standardised,
    exactly, because x has mean 0 and variance 1), A/B the two moments of Eq. 2:
      dL/dHr_ij = G_ij - G_ji,   dL/dHx_i = sum_k (G_ki - G_ik)
      g_ij(t)   = dL/du_ij(t) = dL/dHr_ij (-2 k1 (A_ij - gamma) tanh u - 2 k2 B_ij (1-u^2)e^{-u^2/2}) / n
      dL/dx_i(t) = sum_j [g_ij(t) - rho_ij g_ji(t)] / s_ij                    (through u)
                 + sum_j R_ij x_j(t) / n                                       (through rho)
                 + dL/dHx_i (-2 k1 (A_i - gamma) tanh x_i - 2 k2 B_i (1-x_i^2)e^{-x_i^2/2}) / n
      R_ij = sum_t g_ij (rho u_ij / s^2 - x_j / s) + g_ji (rho u_ji / s^2 - x_i / s)
      dL/de_i = (dL/dx_i - mean(dL/dx_i) - x_i mean(x_i dL/dx_i)) / sd_i      (standardisation)
    """
    E = np.asarray(E, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n, m = E.shape
    mu = E.mean(0)
    sd = np.sqrt(((E - mu) ** 2).mean(0))
    X = (E - mu) / sd
    Gh = G - G.T
    out = np.empty((n, len(cols)))
    scale = np.empty((n, len(cols)))
    cscale = np.empty((n, len(cols)))

    def log_cosh(u):
        a = np.abs(u)
        return a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)

    def du(u, dA, dB, A, B):
        # derivative of the entropy estimate H(u) (times dL/dH) w.r.t. each sample of u
        al = -2.0 * K1 * (A - GAMMA) * dA
        be = -2.0 * K2 * B * dB
        return (al * np.tanh(u) + be * (1.0 - u * u) * np.exp(-0.5 * u * u)) / n

    def mag(dA, dB, A, B):
        return (np.abs(2.0 * K1 * (A - GAMMA) * dA) + np.abs(2.0 * K2 * B * dB)) / n

    for c, i in enumerate(cols):
        xi = X[:, i]
        dx = np.zeros(n)
        sc = np.zeros(n)
        cs = np.zeros(n)
        for j0 in range(0, m, block):
            js = [j for j in range(j0, min(m, j0 + block)) if j != i]
            if not js:
                continue
            xj = X[:, js]
            rho = (xi[:, None] * xj).mean(0)
            s = np.sqrt(1.0 - rho * rho)
            uij = (xi[:, None] - rho * xj) / s
            uji = (xj - rho * xi[:, None]) / s
            Aij, Bij = log_cosh(uij).mean(0), (uij * np.exp(-0.5 * uij * uij)).mean(0)
            Aji, Bji = log_cosh(uji).mean(0), (uji * np.exp(-0.5 * uji * uji)).mean(0)
            gh = Gh[i, js]
            gij = du(uij, gh, gh, Aij, Bij)
            gji = du(uji, -gh, -gh, Aji, Bji)
            dx += ((gij - rho * gji) / s).sum(1)
            R = (gij * (rho * uij / s ** 2 - xj / s)
                 + gji * (rho * uji / s ** 2 - xi[:, None] / s)).sum(0)
            dx += (xj * R).sum(1) / n
            mij, mji = mag(gh, gh, Aij, Bij), mag(gh, gh, Aji, Bji)
            kc = (2.0 * K1 + 2.0 * K2) * np.abs(gh) / n
            sc += ((mij + np.abs(rho) * mji) / s).sum()
            cs += (kc * (1.0 + np.abs(rho)) / s).sum()
            wij = np.abs(rho * uij / s ** 2 - xj / s).sum(0)          # sum over samples
            wji = np.abs(rho * uji / s ** 2 - xi[:, None] / s).sum(0)
            sc += (np.abs(xj) * (mij * wij + mji * wji)).sum(1) / n
            cs += (np.abs(xj) * (kc * (wij + wji))).sum(1) / n
        Ai, Bi = log_cosh(xi).mean(), (xi * np.exp(-0.5 * xi * xi)).mean()
        ci = Gh[:, i].sum()
        dx += du(xi, ci, ci, Ai, Bi)
        sc += mag(ci, ci, Ai, Bi)
        out[:, c] = (dx - dx.mean() - xi * (dx * xi).mean()) / sd[i]
        ax = np.abs(xi)
        scale[:, c] = (sc + sc.mean() + ax * (sc * ax).mean()) / sd[i]
        cscale[:, c] = (cs + cs.mean() + ax * (cs * ax).mean()) / sd[i]
    return (out, scale, cscale) if with_scale else out
