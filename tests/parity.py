"""Parity helpers shared by the GPU tests and the smoke check (test infrastructure).

* order parity: walk the GPU order; at every step the oracle's aggregate score M over the GPU's
  current candidate set must put the GPU's pick within ORDER_TIE of the minimum (orders may
  differ only where the oracle's own margin is below that); this re-synchronises after an
  allowed near-tie divergence instead of cascading;
* B parity: |b - b_ref| <= tol * max(|b_ref|, 1e-2 * max |B_ref|) elementwise.
"""
from __future__ import annotations

import numpy as np

from oracle import varlingam as O

ORDER_TIE = 1e-9        # the oracle margin below which either pick is correct
B_TOL_FP32 = 1e-5       # relative tolerance of B0 / B_tau (FP32 and mixed paths)
B_TOL_BF16 = 1e-3       # relative tolerance of B0 / B_tau (BF16 Gram path)
# Plain FP32 mode (FP32 MFMA Gram matrices and residual GEMM with FP32 sums, no refinement):
# a sum of n products in FP32 carries a relative error up to ~n u (u = 6e-8; 5e-4 at n = 8000
# in the worst case, ~sqrt(n) u typically), and the least-squares coefficients inherit it
# times the conditioning of the Gram matrix (~10-20 on these laws).  It does not meet
# B_TOL_FP32: measured 4e-5 (m = 10) and 3e-5 (m = 100) on the single-problem path, up to
# 1.1e-3 (m = 256, n = 2600) batched.  Its error is reported against this worst-case bound.
B_TOL_PLAIN = 1e-2


def order_violations(order, S_ref, tie=ORDER_TIE):
    """List of (step, gpu_pick, gap) where the GPU's pick is not an oracle minimiser."""
    m = S_ref.shape[0]
    U = list(range(m))
    bad = []
    for k, c in enumerate(np.asarray(order).tolist()):
        if c not in U:
            bad.append((k, c, np.inf))
            break
        M = O.aggregate_scores(S_ref, U)
        gap = float(M[U.index(c)] - M.min())
        if gap > tie:
            bad.append((k, c, gap))
        U.remove(c)
    if len(U) and not bad:
        bad.append((m, -1, np.inf))
    return bad


def b_rel_error(B, B_ref):
    """max over entries of |B - B_ref| / max(|B_ref|, 1e-2 max|B_ref|)."""
    B = np.asarray(B, dtype=np.float64)
    B_ref = np.asarray(B_ref, dtype=np.float64)
    floor = 1e-2 * max(np.max(np.abs(B_ref)), 1e-300)
    return float(np.max(np.abs(B - B_ref) / np.maximum(np.abs(B_ref), floor)))


def _iterative_walk(order, X, U, steps, tie, bad):
    """The first `steps` picks of a GPU order checked with the oracle's arithmetic on its current
    data X (columns U), which is then refined with the GPU's pick (Sec. 3 step 5)."""
    for k, c in enumerate(np.asarray(order).tolist()[:steps]):
        if c not in U:
            bad.append((k, c, np.inf))
            return False
        if len(U) == 1:
            U.remove(c)
            return True
        Xs = {i: O.standardize(X[:, i]) for i in U}
        H = {i: O.entropy(Xs[i]) for i in U}
        Hr = {(i, j): O.entropy(O.standardize(O.residual(Xs[i], Xs[j])))
              for i in U for j in U if i != j}
        M = {i: sum(min(0.0, (H[j] + Hr[i, j]) - (H[i] + Hr[j, i])) ** 2 for j in U if j != i)
             for i in U}
        gap = float(M[c] - min(M.values()))
        if gap > tie:
            bad.append((k, c, gap))
        U.remove(c)
        O.refine(X, U, c)
    return True


def iterative_order_violations(order, E, tie=ORDER_TIE):
    """Walk a GPU order of the original iterative DirectLiNGAM search (Sec. 3 steps 1-5) with
    the oracle's arithmetic: at each step the oracle's aggregates on its current data must put
    the GPU's pick within `tie` of their minimum; the oracle's data is then refined with the
    GPU's pick.  Returns the list of (step, gpu_pick, gap) that fail."""
    X = np.array(E, dtype=np.float64, copy=True)
    U = list(range(X.shape[1]))
    bad = []
    _iterative_walk(order, X, U, X.shape[1], tie, bad)
    return bad


def hybrid_order_violations(order, E, k_exact, tie=ORDER_TIE):
    """A GPU hybrid order: its first k_exact picks walked as in iterative_order_violations,
    the rest checked with order_violations against the oracle's precompute of its data refined
    with the GPU's picks."""
    X = np.array(E, dtype=np.float64, copy=True)
    U = list(range(X.shape[1]))
    bad = []
    if not _iterative_walk(order, X, U, k_exact, tie, bad) or len(U) < 2:
        return bad
    rest = np.asarray(order).tolist()[k_exact:]
    if sorted(rest) != sorted(U):
        return bad + [(k_exact, -1, np.inf)]
    _, _, S_rest = O.pairwise_stats(X[:, U])
    local = [U.index(v) for v in rest]
    return bad + [(k_exact + s, v, g) for s, v, g in order_violations(local, S_rest, tie)]
