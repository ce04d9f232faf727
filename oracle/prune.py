"""FP64 oracle of the pruning stage after the VarLiNGAM fit (test infrastructure only: imported
by the tests, the smoke check and the benchmark's CPU baseline, never by the GPU path).

The paper names pruning of the estimated B0 / B_tau as the step after its method and leaves it
unspecified.  Readings taken here (each also listed in the design notes):

* every variable i is regressed, with intercept, on its predecessors in the causal order at
  lag 0 and on all m variables at lags 1..p, over the VAR fit's sample t = p..n-1.  The OLS
  coefficients of that regression are exactly the unpruned B0[i, :] and B_tau[i, :]
  (Frisch-Waugh: the lag-0 part is the regression of e_i on its predecessors' residuals, the lag
  part ((I - B0) M_tau)[i, :]);
* adaptive lasso (Zou 2006) with weight exponent 1: column j of the design is scaled by
  |b_j|, b the unpruned coefficient, and the coefficient recovered as beta_j = |b_j| beta~_j.
  Columns with b_j = 0 are left out.  With exponent 1 the result does not depend on the scale
  of any column or of the target;
* the lasso path is the LARS path with the lasso modification (Efron, Hastie, Johnstone and
  Tibshirani 2004, Sec. 2 and Sec. 3.1), followed from beta = 0 until the active set reaches
  the least-squares fit (every correlation 0), or max_steps steps (default 8 d);
* the knot is chosen by Schwarz's criterion with the maximum-likelihood variance,
  BIC = T ln(RSS / T) + df ln T, df = number of nonzero coefficients (Zou, Hastie and Tibshirani
  2007); knot 0 (all coefficients 0) is a candidate; ties go to the earlier knot;
* numerical rules of the path: a candidate step length must exceed 1e-12 of the full step
  C/A_A (this removes the zero root of a variable that has just left the active set; its other
  root, re-entry with the opposite sign, stays a candidate); a variable whose column is (numerically) in the span of the active ones (Schur complement
  <= 1e-12 of its squared norm) is excluded for the rest of the path; the path stops once
  C <= 1e-12 C_0.

Pinned by (tests marked "not gpu"): the lasso optimality (KKT) conditions at every knot,
agreement of the knots with scikit-learn's lars_path(method="lasso"), the least-squares end of
the path, the closed form of a one-regressor path, BIC as the Gaussian likelihood criterion
(an independent density routine), the Frisch-Waugh identity behind the weights, invariance
under rescaling and under constant offsets, a zero weight leaving its column out, a duplicated
column never entering, and recovery of the true support on long strongly identified series.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_REL = 1e-12      # smallest admissible step, relative to C / A_A
COLLINEAR_REL = 1e-12  # Schur complement below this fraction of the column's squared norm
STOP_REL = 1e-12       # the path ends once C <= STOP_REL * C_0


def lars_lasso_path(Z: np.ndarray, y: np.ndarray, max_steps: int = 0) -> dict:
    """LARS with the lasso modification on a centred design Z (T x d) and centred target y.

    Efron et al. (2004), Sec. 2: with c = Z^T (y - Z beta) the current correlations,
    C = max_j |c_j|, the active set A, s_j = sign(c_j), the signed active design
    Z_A = (s_j z_j)_{j in A}, G_A = Z_A^T Z_A, A_A = (1^T G_A^{-1} 1)^{-1/2},
    w_A = A_A G_A^{-1} 1, u_A = Z_A w_A (the equiangular direction), a = Z^T u_A; the step is
    gamma^ = min+ over j not in A of {(C - c_j) / (A_A - a_j), (C + c_j) / (A_A + a_j)}.
    Sec. 3.1: with d_j = s_j w_Aj and gamma_j = -beta_j / d_j, gamma~ = min over gamma_j > 0;
    if gamma~ < gamma^ the step stops at gamma~ and j~ leaves A.

    Returns the knots (beta after each step, knot 0 = zeros), the events ((+1, j) join,
    (-1, j) leave, (0, -1) last step to the least-squares fit) and, per step, the relative gap
    between the chosen step length and the next candidate (a measure of how close the event
    was to a tie)."""
    Z = np.asarray(Z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    T, d = Z.shape
    cap = max_steps if max_steps > 0 else 8 * d
    beta = np.zeros(d)
    active: list[int] = []
    excluded = np.zeros(d, dtype=bool)
    norms = (Z * Z).sum(0)
    excluded |= norms <= 0.0
    knots = [beta.copy()]
    events: list[tuple[int, int]] = []
    gaps: list[float] = []
    c = Z.T @ y
    if np.all(excluded):
        return {"knots": knots, "events": events, "gaps": gaps}
    cand = np.where(excluded, -np.inf, np.abs(c))
    j0 = int(np.argmax(cand))
    C0 = float(cand[j0])
    if C0 <= 0.0:
        return {"knots": knots, "events": events, "gaps": gaps}
    active.append(j0)
    for _ in range(cap):
        c = Z.T @ (y - Z @ beta)                   # correlations with the current residual
        s = np.sign(c[active])
        C = float(np.max(np.abs(c[active])))
        ZA = Z[:, active] * s
        GA = ZA.T @ ZA
        q = np.linalg.solve(GA, np.ones(len(active)))
        AA = 1.0 / math.sqrt(float(q.sum()))
        w = AA * q
        u = ZA @ w
        a = Z.T @ u
        full = C / AA
        tol = GAMMA_REL * full
        # gamma^ over the inactive, eligible variables
        cands = []
        for j in range(d):
            if j in active or excluded[j]:
                continue
            for num, den in ((C - c[j], AA - a[j]), (C + c[j], AA + a[j])):
                if den != 0.0:
                    g = num / den
                    if np.isfinite(g) and g > tol:
                        cands.append((g, j))
        # gamma~ over the active variables (sign change of a coefficient)
        dj = s * w
        drops = []
        for r, j in enumerate(active):
            if beta[j] != 0.0 and dj[r] != 0.0:
                g = -beta[j] / dj[r]
                if g > tol:
                    drops.append((g, j))
        g_hat, j_hat = min(cands) if cands else (full, -1)
        g_til, j_til = min(drops) if drops else (math.inf, -1)
        allg = sorted([g for g, _ in cands] + [g for g, _ in drops] + ([full] if not cands else []))
        if g_til < g_hat:
            gamma, event = g_til, (-1, j_til)
        elif j_hat >= 0:
            gamma, event = g_hat, (1, j_hat)
        else:
            gamma, event = full, (0, -1)
        gaps.append((allg[1] - allg[0]) / full if len(allg) > 1 else math.inf)
        beta[active] += gamma * dj
        if event[0] == -1:
            beta[event[1]] = 0.0
            active.remove(event[1])
        knots.append(beta.copy())
        events.append(event)
        if event[0] == 0:
            break
        if event[0] == 1:
            k = event[1]
            # Schur complement of the joining column against the active ones
            if active:
                ZA_ = Z[:, active]
                coef = np.linalg.lstsq(ZA_, Z[:, k], rcond=None)[0]
                schur = float(((Z[:, k] - ZA_ @ coef) ** 2).sum())
            else:
                schur = float(norms[k])
            if schur <= COLLINEAR_REL * norms[k]:
                excluded[k] = True
            else:
                active.append(k)
        if C - gamma * AA <= STOP_REL * C0:
            break
        if not active:           # (a lone active coefficient moves monotonically: not reached)
            break
    return {"knots": knots, "events": events, "gaps": gaps}


def bic_select(Z: np.ndarray, y: np.ndarray, knots) -> dict:
    """BIC = T ln(RSS / T) + df ln T over the knots (df = nonzero coefficients); the first
    minimum wins.  Returns the knot index, the criterion values and the gap to the runner-up."""
    T = Z.shape[0]
    bic = []
    for b in knots:
        r = y - Z @ b
        rss = float(r @ r)
        df = int(np.count_nonzero(b))
        bic.append(T * math.log(rss / T) + df * math.log(T))
    bic = np.array(bic)
    k = int(np.argmin(bic))
    rest = np.delete(bic, k)
    return {"knot": k, "bic": bic,
            "gap": float(rest.min() - bic[k]) if rest.size else math.inf}


def regression_design(X: np.ndarray, p: int, order, i_pos: int):
    """Centred target and design of the variable at position i_pos of the order: lag-0
    predecessors first (in order), then lags tau = 1..p, variables 0..m-1 within each lag.
    Returns (y, Z, cols) with cols[j] = (tau, variable) of design column j."""
    X = np.asarray(X, dtype=np.float64)
    n, m = X.shape
    order = [int(v) for v in order]
    i = order[i_pos]
    rows = slice(p, n)
    cols = [(0, v) for v in order[:i_pos]] + [(tau, k) for tau in range(1, p + 1)
                                               for k in range(m)]
    Z = np.stack([X[p - tau: n - tau, k] for tau, k in cols], axis=1) if cols else \
        np.zeros((n - p, 0))
    y = X[rows, i]
    return y - y.mean(), Z - Z.mean(0), cols


def prune(X: np.ndarray, p: int, order, B0: np.ndarray, B_lags: np.ndarray,
          max_steps: int = 0, positions=None) -> dict:
    """Adaptive-lasso pruning of B0 / B_tau (readings in the module header).  Returns the
    pruned B0 (m x m), B_lags (p x m x m) and per variable the path events, the chosen knot, its
    df and the BIC / step-length gaps that tests use to recognise near-ties.  With positions,
    only the variables at those positions of the order are computed (the other rows stay 0
    and info lists the computed ones)."""
    X = np.asarray(X, dtype=np.float64)
    n, m = X.shape
    B0p = np.zeros((m, m))
    Blp = np.zeros((p, m, m))
    info = []
    order = [int(v) for v in order]
    for pos in (range(m) if positions is None else positions):
        i = order[pos]
        y, Z, cols = regression_design(X, p, order, pos)
        b = np.array([B0[i, v] if tau == 0 else B_lags[tau - 1][i, v] for tau, v in cols])
        keep = np.flatnonzero(b != 0.0)
        Zs = Z[:, keep] * np.abs(b[keep])
        path = lars_lasso_path(Zs, y, max_steps)
        sel = bic_select(Zs, y, path["knots"])
        beta = path["knots"][sel["knot"]] * np.abs(b[keep])
        for jj, j in enumerate(keep):
            tau, v = cols[j]
            if tau == 0:
                B0p[i, v] = beta[jj]
            else:
                Blp[tau - 1][i, v] = beta[jj]
        info.append({"var": i, "pos": pos, "d": len(keep), "steps": len(path["events"]),
                     "knot": sel["knot"], "df": int(np.count_nonzero(beta)),
                     "events": [(e, int(keep[j]) if j >= 0 else -1) for e, j in path["events"]],
                     "bic_gap": sel["gap"], "min_step_gap": min(path["gaps"], default=math.inf)})
    return {"B0": B0p, "B_lags": Blp, "info": info}
