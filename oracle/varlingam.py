"""FP64 oracle of the heuristic VarLiNGAM path (test infrastructure only; see package doc).

Everything here follows the paper's text in its own order and notation:

* Sec. 2.1 (VarLiNGAM): fit a VAR model, then run the LiNGAM ordering on its residuals;
  the lag matrices follow from B_tau = (I - B0) M_tau.
* Sec. 3 step 1: standardise each column (mean 0, variance 1; population moments).
* Sec. 3 step 2, Eq. 1: least-squares residual r_{i<-j} = x_i - cov(x_i,x_j)/var(x_j) x_j.
* Sec. 3 step 3, Eq. 2: T_{i<-j} = H(x_i) - H(r_{i<-j}) with an entropy approximation H.
* Sec. 3 step 4, Eq. 3: M_i = sum over remaining j != i of f(T_{i<-j}, T_{j<-i}); the
  variable of maximum overall independence (smallest M) is taken next.
* Sec. 3 step 5: the original algorithm replaces each remaining column by its residual on the
  chosen one (kept here only as a comparator).
* Sec. 4.2 and Alg. 1: the heuristic precomputes H(x_i) (size m) and H(r_{i<-j}) (m x m) once
  from the unaltered data and then runs m lookup-only selection steps.

Readings where the paper is silent (each is also listed in the design notes):
* H is Hyvarinen's (1998) maximum-entropy approximation with G1 = log cosh and
  G2 = u exp(-u^2/2), with the literal constants k1 = 79.047, k2 = 7.4129, gamma = 0.37457
  and H(nu) = (1 + ln 2 pi)/2 for the unit Gaussian;
* the residual is re-standardised before H (the approximation assumes unit variance);
* cov and var in Eq. 1 both use 1/n, so the coefficient is the least-squares slope;
* f(T_{i<-j}, T_{j<-i}) = min(0, T_{j<-i} - T_{i<-j})^2 (pairwise likelihood-ratio measure of
  Hyvarinen & Smith 2013), i.e. M_i = sum_j min(0, S_ij)^2 with S_ij = T_{j<-i} - T_{i<-j};
* j in Eq. 3 runs over the *current* candidate set U; exact ties go to the lowest index;
* "the data matrix X" of Alg. 1 is the VAR residual matrix;
* the VAR model includes an intercept and uses the given lag order p;
* B0 is the least-squares regression (with intercept) of each variable on its predecessors in
  the order; B_tau = (I - B0) M_tau;
* lag-order selection (before the fit; the paper fixes p): every candidate p on the common
  sample t = p_max .. n-1, AIC / BIC of Lutkepohl (2005) with the maximum-likelihood residual
  covariance (divisor T) and p m^2 counted parameters.

Pinned by (tests marked "not gpu"): quadrature population values of H for five laws, the
unit-Gaussian special case, residual orthogonality identities, antisymmetry / invariance /
equivariance of S, a hand-built total-order S, m = 2 identity with the iterative algorithm and
equal first picks for any m, tiny-m agreement with the iterative algorithm, recovery of the
generating order, VAR orthogonality and the AR(1) closed form, the exact OLS identity
(I - B0) Sigma (I - B0)^T diagonal, the generator identity (I - B0) M_tau = B_tau, and for the
lag selection the univariate closed form, nested monotonicity, scale invariance and recovery
of the generating lag order by BIC on long series; the ordering margins by hand-computed values
on a small integer score matrix (the runner-up is not the next pick there); the Sec. 3 step 5
refinement by its exact identities (each refined column is centred, orthogonal to the pick and
has variance 1 - rho^2) and by a sample-orthogonal construction whose refined column is the
hidden noise exactly; estimate_B_cov by agreement with the per-variable least squares.
Parity unpinned: the literal digits of k1 and gamma (pinned by citation of the published
constants only).
"""
from __future__ import annotations

import math

import numpy as np

# Hyvarinen (1998) maximum-entropy approximation constants (as published).
K1 = 79.047
K2 = 7.4129
GAMMA = 0.37457
H_GAUSS = (1.0 + math.log(2.0 * math.pi)) / 2.0   # differential entropy of N(0, 1)


# ---------------------------------------------------------------------------------------------
# Sec. 3 step 1 -- standardisation
# ---------------------------------------------------------------------------------------------
def standardize(v: np.ndarray) -> np.ndarray:
    """Mean 0, variance 1 with population (1/n) moments.  Raises on a constant column."""
    v = np.asarray(v, dtype=np.float64)
    sd = v.std()
    if not sd > 0.0:
        raise ValueError("degenerate column: zero variance")
    return (v - v.mean()) / sd


# ---------------------------------------------------------------------------------------------
# Sec. 3 step 2, Eq. 1 -- pairwise least-squares residual
# ---------------------------------------------------------------------------------------------
def residual(xi: np.ndarray, xj: np.ndarray) -> np.ndarray:
    """r_{i<-j} = x_i - cov(x_i, x_j) / var(x_j) * x_j, both moments with 1/n (Eq. 1)."""
    xi = np.asarray(xi, dtype=np.float64)
    xj = np.asarray(xj, dtype=np.float64)
    cov = np.mean((xi - xi.mean()) * (xj - xj.mean()))
    var = np.mean((xj - xj.mean()) ** 2)
    if not var > 0.0:
        raise ValueError("degenerate column: zero variance")
    return xi - (cov / var) * xj


# ---------------------------------------------------------------------------------------------
# Sec. 3 step 3, Eq. 2 -- entropy approximation and dependence score
# ---------------------------------------------------------------------------------------------
def log_cosh(u: np.ndarray) -> np.ndarray:
    """log cosh u in an overflow-free form: |u| + log(1 + exp(-2|u|)) - log 2."""
    a = np.abs(u)
    return a + np.log1p(np.exp(-2.0 * a)) - math.log(2.0)


def entropy_moments(u: np.ndarray) -> tuple[float, float]:
    """The two sample moments the approximation uses: E[log cosh u], E[u exp(-u^2/2)]."""
    u = np.asarray(u, dtype=np.float64)
    return float(np.mean(log_cosh(u))), float(np.mean(u * np.exp(-0.5 * u * u)))


def entropy_from_moments(a: float, b: float) -> float:
    """H = H(nu) - k1 (E[G1] - gamma)^2 - k2 (E[G2])^2."""
    return H_GAUSS - K1 * (a - GAMMA) ** 2 - K2 * b ** 2


def entropy(u: np.ndarray) -> float:
    """Maximum-entropy approximation of the differential entropy of a standardised sample."""
    return entropy_from_moments(*entropy_moments(u))


def dependence_score(xi: np.ndarray, xj: np.ndarray) -> float:
    """T_{i<-j} = H(x_i) - H(r_{i<-j}) for standardised x_i, x_j (Eq. 2)."""
    return entropy(xi) - entropy(standardize(residual(xi, xj)))


# ---------------------------------------------------------------------------------------------
# Sec. 4.2 steps 1-2 / Alg. 1 precomputation -- E_x (size m) and E_r (m x m) once
# ---------------------------------------------------------------------------------------------
def standardize_columns(E: np.ndarray) -> np.ndarray:
    E = np.asarray(E, dtype=np.float64)
    return np.column_stack([standardize(E[:, i]) for i in range(E.shape[1])])


def pair_row(X: np.ndarray, i: int):
    """Row i of the precompute from the standardised columns X: A[i, j], B[i, j] and
    Hr[i, j] for every j != i (0 on the diagonal), one pair at a time (Eq. 1 residual,
    re-standardised, Eq. 2 moments)."""
    m = X.shape[1]
    A = np.zeros(m)
    B = np.zeros(m)
    Hr = np.zeros(m)
    for j in range(m):
        if i == j:
            continue
        r = residual(X[:, i], X[:, j])
        if not r.std() > 1e-6:       # 1 - rho_ij^2 below 1e-12
            raise ValueError("degenerate pair: residual has (near) zero variance")
        A[j], B[j] = entropy_moments(standardize(r))
        Hr[j] = entropy_from_moments(A[j], B[j])
    return A, B, Hr


def pairwise_stats(E: np.ndarray, return_moments: bool = False, rows=None):
    """Precompute Hx[i] = H(x_i) and Hr[i, j] = H(std(r_{i<-j})) for every ordered pair, and
    the antisymmetric pairwise score S[i, j] = T_{j<-i} - T_{i<-j}
                                            = (Hx[j] + Hr[i, j]) - (Hx[i] + Hr[j, i]).
    S[i, j] > 0 is evidence that i precedes j.  One pair at a time, from scratch.

    With `return_moments`, also returns the per-pair moment matrices A[i, j] =
    E[log cosh u_{i<-j}], B[i, j] = E[u_{i<-j} exp(-u_{i<-j}^2/2)] and Ax, Bx (size m).

    `rows` may hold pair_row(standardize_columns(E), i) for i = 0 .. m-1, computed elsewhere
    (for instance by worker processes, the rows being independent); the result is then
    bit-identical to computing them here.
    """
    X = standardize_columns(E)
    m = X.shape[1]
    Ax = np.empty(m)
    Bx = np.empty(m)
    for i in range(m):
        Ax[i], Bx[i] = entropy_moments(X[:, i])
    Hx = np.array([entropy_from_moments(Ax[i], Bx[i]) for i in range(m)])
    if rows is None:
        rows = [pair_row(X, i) for i in range(m)]
    if len(rows) != m:
        raise ValueError("rows must hold one pair_row result per variable")
    A = np.array([r[0] for r in rows]).reshape(m, m)
    B = np.array([r[1] for r in rows]).reshape(m, m)
    Hr = np.array([r[2] for r in rows]).reshape(m, m)
    S = np.zeros((m, m))
    for i in range(m):
        for j in range(m):
            if i != j:
                S[i, j] = (Hx[j] + Hr[i, j]) - (Hx[i] + Hr[j, i])
    if return_moments:
        return Hx, Hr, S, {"A": A, "B": B, "Ax": Ax, "Bx": Bx}
    return Hx, Hr, S


def pair_moments(E: np.ndarray, i: int, j: int) -> tuple[float, float]:
    """A[i, j], B[i, j] for one ordered pair (for sampled checks at large sizes)."""
    E = np.asarray(E, dtype=np.float64)
    xi = standardize(E[:, i])
    xj = standardize(E[:, j])
    r = residual(xi, xj)
    return entropy_moments(standardize(r))


# ---------------------------------------------------------------------------------------------
# Sec. 4.2 step 3 / Alg. 1 main loop -- lookup-only ordering
# ---------------------------------------------------------------------------------------------
def aggregate_scores(S: np.ndarray, U) -> np.ndarray:
    """M_i over the current candidate set U (Eq. 3 with f = min(0, S_ij)^2), recomputed from
    scratch: M_i = sum_{j in U, j != i} min(0, S[i, j])^2."""
    U = list(U)
    sub = np.asarray(S, dtype=np.float64)[np.ix_(U, U)]
    pen = np.minimum(0.0, sub) ** 2
    np.fill_diagonal(pen, 0.0)
    return pen.sum(axis=1)


def approx_order(S: np.ndarray):
    """Alg. 1: m selection steps over the static score matrix.  Returns (order, margin):
    order[k] = c_k (smallest M; exact ties -> lowest index), margin[k] = second-smallest M
    minus smallest M at step k (+inf when one candidate is left)."""
    m = S.shape[0]
    U = list(range(m))
    order = []
    margin = []
    for _ in range(m):
        M = aggregate_scores(S, U)
        best = int(np.argmin(M))          # argmin returns the first (lowest-index) minimiser
        if len(U) > 1:
            srt = np.sort(M)
            margin.append(float(srt[1] - srt[0]))
        else:
            margin.append(math.inf)
        order.append(U[best])
        del U[best]
    return np.array(order, dtype=np.int64), np.array(margin)


# ---------------------------------------------------------------------------------------------
# Sec. 3 steps 1-5 -- the original iterative DirectLiNGAM ordering (comparator only)
# ---------------------------------------------------------------------------------------------
def directlingam_iterative(E: np.ndarray, k_exact: int | None = None):
    """Original DirectLiNGAM causal-order search: score all pairs on the current data, pick the
    most independent variable, then replace every remaining column by its residual on it
    (Sec. 3 step 5) and repeat.  O(m^3 n).  Returns the order.

    With k_exact, a hybrid: the first k_exact picks as above, then the heuristic of Sec. 4.2 /
    Alg. 1 on the refined data of the remaining variables (one pairwise precompute, lookup-only
    selection).  k_exact = 0 is the heuristic on E; k_exact >= m - 1 the original search."""
    X = np.array(E, dtype=np.float64, copy=True)
    m = X.shape[1]
    U = list(range(m))
    order = []
    while U:
        if len(U) == 1:
            order.append(U.pop())
            break
        if k_exact is not None and len(order) == k_exact:
            _, _, S_rest = pairwise_stats(X[:, U])
            rest, _ = approx_order(S_rest)
            order.extend(U[int(r)] for r in rest)
            break
        Xs = {i: standardize(X[:, i]) for i in U}
        H = {i: entropy(Xs[i]) for i in U}
        Hr = {}
        for i in U:
            for j in U:
                if i != j:
                    Hr[i, j] = entropy(standardize(residual(Xs[i], Xs[j])))
        M = []
        for i in U:
            tot = 0.0
            for j in U:
                if i != j:
                    s = (H[j] + Hr[i, j]) - (H[i] + Hr[j, i])
                    tot += min(0.0, s) ** 2
            M.append(tot)
        best = int(np.argmin(M))
        c = U[best]
        order.append(c)
        del U[best]
        refine(X, U, c)
    return np.array(order, dtype=np.int64)


def refine(X: np.ndarray, U, c: int) -> None:
    """Sec. 3 step 5: after variable c is taken, every remaining column j in U is replaced (in
    place) by the least-squares residual of its standardised data on the standardised x_c,
    x_j <- std(x_j) - rho_jc std(x_c)  (Eq. 1 between standardised columns)."""
    xc = standardize(X[:, c])
    for j in U:
        if j != c:
            X[:, j] = residual(standardize(X[:, j]), xc)


# ---------------------------------------------------------------------------------------------
# Sec. 2.1 -- VAR(p) least-squares fit (the step that feeds the ordering)
# ---------------------------------------------------------------------------------------------
def var_design(X: np.ndarray, p: int):
    """Y = x(t) and Z = [x(t-1), ..., x(t-p), 1] for t = p .. n-1."""
    X = np.asarray(X, dtype=np.float64)
    n, m = X.shape
    Y = X[p:]
    Z = np.hstack([X[p - tau: n - tau] for tau in range(1, p + 1)] + [np.ones((n - p, 1))])
    return Y, Z


def fit_var(X: np.ndarray, p: int):
    """Least-squares VAR(p) with intercept.  Returns (M, c, E) with
    x(t) = sum_tau M[tau-1] x(t - tau) + c + E[t - p]."""
    X = np.asarray(X, dtype=np.float64)
    n, m = X.shape
    if p < 1 or n - p <= m * p + 1:
        raise ValueError("VAR fit needs p >= 1 and n - p > m p + 1")
    Y, Z = var_design(X, p)
    coef, _, rank, _ = np.linalg.lstsq(Z, Y, rcond=None)
    if rank < Z.shape[1]:
        raise ValueError("singular VAR design")
    M = np.stack([coef[(tau - 1) * m: tau * m].T for tau in range(1, p + 1)])
    c = coef[-1].copy()
    E = Y - Z @ coef
    return M, c, E


def select_lag(X: np.ndarray, p_max: int) -> dict:
    """VAR lag-order selection for the fit of Sec. 2.1 (the paper fixes p; this is the step
    before it).  Every p = 1 .. p_max is fitted by least squares with intercept on the same
    sample t = p_max .. n-1 (T = n - p_max rows), and scored with the maximum-likelihood
    residual covariance Sigma_p = E_p^T E_p / T:
        AIC(p) = ln det Sigma_p + 2 p m^2 / T,   BIC(p) = ln det Sigma_p + ln(T) p m^2 / T
    (Lutkepohl 2005, Sec. 4.3; the m intercepts are common to every p and not counted).
    Returns ln det Sigma_p, AIC, BIC (arrays over p) and the p minimising each (lowest p on
    ties)."""
    X = np.asarray(X, dtype=np.float64)
    n, m = X.shape
    if p_max < 1 or n - p_max <= m * p_max + 1:
        raise ValueError("lag selection needs p_max >= 1 and n - p_max > m p_max + 1")
    T = n - p_max
    Y = X[p_max:]
    logdet, aic, bic = [], [], []
    for p in range(1, p_max + 1):
        Z = np.hstack([X[p_max - tau: n - tau] for tau in range(1, p + 1)] + [np.ones((T, 1))])
        coef, _, rank, _ = np.linalg.lstsq(Z, Y, rcond=None)
        if rank < Z.shape[1]:
            raise ValueError("singular VAR design")
        E = Y - Z @ coef
        sign, ld = np.linalg.slogdet(E.T @ E / T)
        if sign <= 0:
            raise ValueError("singular residual covariance")
        logdet.append(ld)
        aic.append(ld + 2.0 * p * m * m / T)
        bic.append(ld + math.log(T) * p * m * m / T)
    aic, bic = np.array(aic), np.array(bic)
    return {"logdet": np.array(logdet), "aic": aic, "bic": bic,
            "p_aic": int(np.argmin(aic)) + 1, "p_bic": int(np.argmin(bic)) + 1}


# ---------------------------------------------------------------------------------------------
# Sec. 4 (B0 estimation) and Sec. 2.1 (lag matrices)
# ---------------------------------------------------------------------------------------------
def estimate_B(E: np.ndarray, order, M: np.ndarray):
    """B0[K_k, K_<k] = least-squares coefficients (with intercept) of e_{K_k} on its
    predecessors; all other entries 0.  B_tau = (I - B0) M_tau."""
    E = np.asarray(E, dtype=np.float64)
    n, m = E.shape
    B0 = np.zeros((m, m))
    order = [int(v) for v in order]
    for k in range(1, m):
        v = order[k]
        preds = order[:k]
        A = np.hstack([E[:, preds], np.ones((n, 1))])
        coef, *_ = np.linalg.lstsq(A, E[:, v], rcond=None)
        B0[v, preds] = coef[:-1]
    Bl = np.stack([(np.eye(m) - B0) @ M[t] for t in range(M.shape[0])])
    return B0, Bl


def estimate_B_cov(Sigma: np.ndarray, order, M: np.ndarray):
    """The same estimator as estimate_B written as normal equations on the population
    covariance Sigma of the residuals (for an OLS with intercept the centred normal equations
    are exactly Sigma_PP b = Sigma_Pv, P = the predecessors of v): B0[v, P] = Sigma_PP^-1
    Sigma_Pv for every v after the first; B_tau = (I - B0) M_tau.  One m x m matrix instead of
    the data, so the larger workloads stay quick."""
    Sigma = np.asarray(Sigma, dtype=np.float64)
    m = Sigma.shape[0]
    B0 = np.zeros((m, m))
    order = [int(v) for v in order]
    for k in range(1, m):
        v = order[k]
        P = order[:k]
        B0[v, P] = np.linalg.solve(Sigma[np.ix_(P, P)], Sigma[P, v])
    Bl = np.stack([(np.eye(m) - B0) @ M[t] for t in range(M.shape[0])])
    return B0, Bl


def population_cov(E: np.ndarray) -> np.ndarray:
    """Covariance of the columns of E with the 1/n divisor."""
    E = np.asarray(E, dtype=np.float64)
    C = E - E.mean(axis=0)
    return C.T @ C / E.shape[0]


# ---------------------------------------------------------------------------------------------
# The whole heuristic fit
# ---------------------------------------------------------------------------------------------
def fit(X: np.ndarray, p: int, b_from_cov: bool = False, rows=None) -> dict:
    """VAR fit -> precompute (Hx, Hr, S) -> Alg. 1 ordering -> B0, B_tau.  `b_from_cov` takes
    B from estimate_B_cov (normal equations on the residual covariance) instead of one
    least-squares fit of the data per variable; `rows` goes to pairwise_stats."""
    M, c, E = fit_var(X, p)
    Hx, Hr, S = pairwise_stats(E, rows=rows)
    order, margin = approx_order(S)
    if b_from_cov:
        B0, Bl = estimate_B_cov(population_cov(E), order, M)
    else:
        B0, Bl = estimate_B(E, order, M)
    return {"M": M, "intercept": c, "E": E, "Hx": Hx, "Hr": Hr, "S": S,
            "order": order, "margin": margin, "B0": B0, "B_lags": Bl}
