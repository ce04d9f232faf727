"""FP64 oracle of the ensemble workloads around the VarLiNGAM fit: rolling windows and the
residual bootstrap, with edge-probability aggregation (test infrastructure only: imported by
the tests and the benchmark's CPU baseline, never by the GPU path).

Readings (the paper uses neither; each is also listed in the design notes):
* rolling windows: window k is rows k*stride .. k*stride + w - 1 of the series, fitted on its
  own (VAR with intercept, ordering, B);
* residual bootstrap of the VAR of Sec. 2.1 (the model-based bootstrap for time series, e.g.
  Lutkepohl 2005, App. D): a resample starts from the first p observed rows and continues
  x*(t) = c + sum_{tau=1..p} M_tau x*(t - tau) + e(idx[t - p]), e the fit's residual rows
  drawn with replacement.  The draws are an input (idx), so any generator can feed them;
* aggregation over the problems whose fit succeeded: P0[i, j] = fraction with
  |B0[i, j]| > threshold, P_tau likewise, and P_order[i, j] = fraction in which j precedes i in
  the causal order.

Pinned by (tests marked "not gpu"): the identity resample (idx = 0, 1, 2, ...) reproduces the
observed series exactly, zero residuals converge to the closed-form process mean
(I - sum M_tau)^{-1} c, the aggregation's special cases (identical problems give 0/1, the order
probabilities of a pair sum to 1, unanimity), and bootstrap recovery of strong edges on a long
series.
"""
from __future__ import annotations

import numpy as np

from . import varlingam as O


def simulate_var(M: np.ndarray, c: np.ndarray, X0: np.ndarray, E: np.ndarray,
                 idx: np.ndarray) -> np.ndarray:
    """One resample of length p + len(idx): rows 0..p-1 are X0, then the VAR recursion driven
    by the residual rows E[idx]."""
    M = np.asarray(M, dtype=np.float64)
    p, m, _ = M.shape
    T = len(idx)
    x = np.zeros((p + T, m))
    x[:p] = np.asarray(X0, dtype=np.float64)[:p]
    E = np.asarray(E, dtype=np.float64)
    for t in range(p, p + T):
        acc = np.array(c, dtype=np.float64) + E[int(idx[t - p])]
        for tau in range(1, p + 1):
            acc = acc + M[tau - 1] @ x[t - tau]
        x[t] = acc
    return x


def edge_frequency(orders, B0s, Bls, threshold: float = 0.0, valid=None) -> dict:
    """Aggregate K fits (orders K x m, B0s K x m x m, Bls K x p x m x m) over the problems with
    valid[k] (default all): edge probabilities with |B| > threshold and order precedence."""
    orders = np.asarray(orders)
    B0s = np.asarray(B0s, dtype=np.float64)
    Bls = np.asarray(Bls, dtype=np.float64)
    K, m = orders.shape
    keep = np.ones(K, dtype=bool) if valid is None else np.asarray(valid, dtype=bool)
    cnt = int(keep.sum())
    P0 = np.zeros((m, m))
    Pl = np.zeros(Bls.shape[1:])
    Po = np.zeros((m, m))
    for k in np.flatnonzero(keep):
        P0 += np.abs(B0s[k]) > threshold
        Pl += np.abs(Bls[k]) > threshold
        pos = np.empty(m, dtype=np.int64)
        pos[orders[k]] = np.arange(m)
        Po += pos[None, :] < pos[:, None]          # [i, j]: j precedes i
    if cnt:
        P0, Pl, Po = P0 / cnt, Pl / cnt, Po / cnt
    return {"P0": P0, "P_lags": Pl, "P_order": Po, "count": cnt}


def fit_all(series, p: int) -> dict:
    """The oracle fit of each series; a failed fit (degenerate data) is marked invalid."""
    orders, B0s, Bls, valid = [], [], [], []
    for X in series:
        X = np.asarray(X, dtype=np.float64)
        m = X.shape[1]
        try:
            r = O.fit(X, p)
            orders.append(np.asarray(r["order"]))
            B0s.append(r["B0"])
            Bls.append(r["B_lags"])
            valid.append(True)
        except (ValueError, np.linalg.LinAlgError):
            orders.append(np.arange(m))
            B0s.append(np.zeros((m, m)))
            Bls.append(np.zeros((p, m, m)))
            valid.append(False)
    return {"orders": np.array(orders), "B0": np.array(B0s), "B_lags": np.array(Bls),
            "valid": np.array(valid)}


def rolling_windows(X: np.ndarray, p: int, window: int, stride: int,
                    threshold: float = 0.0) -> dict:
    X = np.asarray(X, dtype=np.float64)
    starts = list(range(0, X.shape[0] - window + 1, stride))
    fits = fit_all([X[s: s + window] for s in starts], p)
    agg = edge_frequency(fits["orders"], fits["B0"], fits["B_lags"], threshold, fits["valid"])
    return {"starts": starts, **fits, **agg}


def bootstrap(X: np.ndarray, p: int, idx: np.ndarray, threshold: float = 0.0) -> dict:
    """Residual bootstrap with draws idx (R x (n - p), values in 0 .. n - p - 1)."""
    X = np.asarray(X, dtype=np.float64)
    M, c, E = O.fit_var(X, p)
    series = [simulate_var(M, c, X[:p], E, row) for row in np.asarray(idx)]
    fits = fit_all(series, p)
    agg = edge_frequency(fits["orders"], fits["B0"], fits["B_lags"], threshold, fits["valid"])
    return {"series": series, **fits, **agg}
