"""Oracle fits of the full-size workloads, computed by worker processes while the other tests
run (test infrastructure).

The precompute of an m = 400, n = 10 000 series takes the plain oracle tens of seconds per
seed on one core.  Its rows are independent, so a pool of worker processes computes them with
the oracle's own pair_row(); the test process then assembles the fit with
oracle.varlingam.pairwise_stats(E, rows=...), which is bit-identical to the serial oracle.

The pool is forked when collection ends, before any test has touched the GPU: the workers
never use it.  The series and the oracle's VAR fits are made in the parent before the fork, so
the workers inherit the standardised residuals instead of receiving them.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import synth
from oracle import varlingam as O

# (workload name, seed) pairs the full-size tests use
JOBS = [("m400_n10000_p2_t4", s) for s in (0, 1, 2)]
ROWS_PER_TASK = 20

_pool = None
_pending: dict = {}
_done: dict = {}
_inputs: dict = {}       # (name, seed) -> standardised oracle residuals


def _rows(key, i0: int, i1: int):
    X = _inputs[key]
    return i0, [O.pair_row(X, i) for i in range(i0, min(i1, X.shape[1]))]


def start(workers: int | None = None) -> None:
    """Generate the series and the oracle's VAR fits here, then fork the pool (the workers
    inherit them) and queue every job's rows.  No-op when already started."""
    global _pool
    if _pool is not None:
        return
    for key in JOBS:
        if key not in _inputs:
            inst = synth.make_instance(*key)
            _, _, E = O.fit_var(inst.X_parity, inst.workload.p)
            _inputs[key] = O.standardize_columns(E)
    if workers is None:
        workers = max(1, min(8, (os.cpu_count() or 2) - 2))
    _pool = mp.get_context("fork").Pool(workers)
    for key in JOBS:
        m = _inputs[key].shape[1]
        _pending[key] = [_pool.apply_async(_rows, (key, i0, i0 + ROWS_PER_TASK))
                         for i0 in range(0, m, ROWS_PER_TASK)]


def stop() -> None:
    global _pool
    if _pool is not None:
        _pool.terminate()
        _pool.join()
        _pool = None
    _pending.clear()


def fit(name: str, seed: int, timeout: float = 900.0) -> dict:
    """The oracle's whole fit of one full-size series (B from the residual covariance, the
    same estimator as the per-variable least squares), plus its residual covariance.  Prints
    a line while it waits for the workers."""
    key = (name, seed)
    if key in _done:
        return _done[key]
    inst = synth.make_instance(name, seed)
    rows = None
    if key in _pending:
        got = {}
        pending = _pending.pop(key)
        t0 = time.time()
        for r in pending:
            while not r.ready():
                r.wait(20.0)
                if time.time() - t0 > timeout:
                    raise TimeoutError(f"oracle rows of {key} not ready after {timeout} s")
                print(f"  oracle {key}: {sum(q.ready() for q in pending)} of {len(pending)} "
                      f"row blocks done", flush=True)
            i0, rs = r.get()
            for k, row in enumerate(rs):
                got[i0 + k] = row
        rows = [got[i] for i in range(len(got))]
    res = O.fit(inst.X_parity, inst.workload.p, b_from_cov=True, rows=rows)
    res["Cov"] = O.population_cov(res["E"])
    res["X32"] = inst.X32
    _done[key] = res
    return res
