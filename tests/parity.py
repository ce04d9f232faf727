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
