"""Seeded synthetic VAR-LiNGAM time series: the input generator shared by tests and bench.

This module only *generates inputs*.  It holds none of the method's arithmetic (no
standardisation, pairwise residual, entropy, ordering or regression), so the CPU oracle and
the GPU path can both draw from it without sharing any computation.

Data-generating process (the structural VAR-LiNGAM model of Sec. 2.1 of the paper, with the
contemporaneous DAG B0 and lag matrices B_tau):

    x(t) = B0 x(t) + sum_{tau=1..p} B_tau x(t - tau) + e(t)
         = (I - B0)^{-1} ( sum_tau B_tau x(t - tau) + e(t) )

* a hidden permutation pi fixes the causal order; B0 is strictly lower-triangular in pi order:
  each pair pi_a -> pi_b (a < b) gets an edge with probability q, weight sign(+-1) * U[lo, hi];
* each B_tau has i.i.d. N(0, 0.2^2) entries, rescaled to a target spectral radius;
* e(t) is i.i.d., unit variance: uniform[-sqrt3, sqrt3], Laplace(0, 1/sqrt2) or Student-t(4)/sqrt2;
* x(t < 0) = 0, 1000 burn-in samples are discarded; if the reduced-form companion matrix has
  spectral radius >= 0.95, every B_tau is scaled by 0.9 / radius once (flag `rescaled`).

All draws come from numpy's PCG64 seeded by `SeedSequence(seed)`, in a fixed order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

BURN_IN = 1000


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: shape, DAG density, weight range, lag radius and noise law."""

    name: str
    m: int            # variables
    n: int            # samples kept (after burn-in)
    p: int            # VAR lag order
    edge_prob: float  # probability of each allowed B0 edge
    w_lo: float       # |B0 weight| lower bound
    w_hi: float       # |B0 weight| upper bound
    lag_radius: float  # target spectral radius of each B_tau
    noise: str        # 'uniform' | 'laplace' | 't4'
    dtype: str        # precision the series is handed over in: 'f64' or 'f32'


# The five workloads the library is checked and measured on.
SMALL = Workload("m10_n1000_p1_uniform", 10, 1000, 1, 0.3, 0.2, 0.8, 0.5, "uniform", "f64")
MEDIUM = Workload("m100_n5000_p1_laplace", 100, 5000, 1, 0.05, 0.1, 0.5, 0.5, "laplace", "f32")
FINANCE = Workload("m400_n10000_p2_t4", 400, 10000, 2, 0.02, 0.05, 0.4, 0.4, "t4", "f32")
LARGE = Workload("m1000_n50000_p1_laplace", 1000, 50000, 1, 0.005, 0.1, 0.5, 0.5, "laplace", "f32")
WORKLOADS = {w.name: w for w in (SMALL, MEDIUM, FINANCE, LARGE)}

# Batched workload: 256 independent instances, uneven shapes.
BATCH_COUNT = 256
BATCH_M_RANGE = (20, 200)
BATCH_N_RANGE = (500, 8000)


@dataclass
class Instance:
    """A generated series plus its ground truth."""

    workload: Workload
    seed: int
    X64: np.ndarray          # n x m float64 series
    B0: np.ndarray           # m x m, true contemporaneous matrix (row = effect, col = cause)
    B_lags: np.ndarray       # p x m x m, true lag matrices
    perm: np.ndarray         # true causal order (pi): perm[0] is the most exogenous variable
    rescaled: bool = False
    extra: dict = field(default_factory=dict)

    @property
    def X32(self) -> np.ndarray:
        """The series rounded to float32 (what the GPU receives), C-contiguous n x m."""
        return np.ascontiguousarray(self.X64.astype(np.float32))

    @property
    def X_parity(self) -> np.ndarray:
        """float32-rounded values upcast to float64: what the oracle consumes for parity."""
        return self.X32.astype(np.float64)


def _noise(rng: np.random.Generator, kind: str, size) -> np.ndarray:
    if kind == "uniform":
        return rng.uniform(-math.sqrt(3.0), math.sqrt(3.0), size)
    if kind == "laplace":
        return rng.laplace(0.0, 1.0 / math.sqrt(2.0), size)
    if kind == "t4":
        return rng.standard_t(4.0, size) / math.sqrt(2.0)
    raise ValueError(f"unknown noise law {kind!r}")


def _spectral_radius(a: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(a)))) if a.size else 0.0


def _companion(mats: np.ndarray) -> np.ndarray:
    p, m, _ = mats.shape
    c = np.zeros((m * p, m * p))
    c[:m, :] = np.concatenate(list(mats), axis=1)
    if p > 1:
        c[m:, : m * (p - 1)] = np.eye(m * (p - 1))
    return c


def _draw_model(rng: np.random.Generator, w: Workload, m: int):
    perm = rng.permutation(m)
    B0 = np.zeros((m, m))
    for b in range(1, m):
        has = rng.random(b) < w.edge_prob
        signs = np.where(rng.random(b) < 0.5, -1.0, 1.0)
        mags = rng.uniform(w.w_lo, w.w_hi, b)
        for a in np.nonzero(has)[0]:
            B0[perm[b], perm[a]] = signs[a] * mags[a]
    lags = np.empty((w.p, m, m))
    for tau in range(w.p):
        raw = rng.normal(0.0, 0.2, (m, m))
        r = _spectral_radius(raw)
        lags[tau] = raw * (w.lag_radius / r) if r > 0 else raw
    return perm, B0, lags


def _simulate(rng, w: Workload, m: int, n: int, B0, lags):
    A = np.linalg.inv(np.eye(m) - B0)
    red = np.einsum("ij,tjk->tik", A, lags)          # reduced-form lag matrices
    rescaled = False
    rad = _spectral_radius(_companion(red))
    if rad >= 0.95:
        lags = lags * (0.9 / rad)
        red = red * (0.9 / rad)
        rescaled = True
    total = n + BURN_IN
    shocks = _noise(rng, w.noise, (total, m)) @ A.T   # A e(t) for every t
    x = np.zeros((total, m))
    p = w.p
    for t in range(total):
        acc = shocks[t].copy()
        for tau in range(1, p + 1):
            if t - tau >= 0:
                acc += red[tau - 1] @ x[t - tau]
        x[t] = acc
    return np.ascontiguousarray(x[BURN_IN:]), lags, rescaled


def make_instance(workload: Workload | str, seed: int = 0) -> Instance:
    """Generate one seeded instance of `workload` (a Workload or its name)."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    perm, B0, lags = _draw_model(rng, w, w.m)
    X, lags, rescaled = _simulate(rng, w, w.m, w.n, B0, lags)
    return Instance(w, seed, X, B0, lags, perm, rescaled)


def make_custom(m: int, n: int, p: int = 1, noise: str = "uniform", seed: int = 0,
                edge_prob: float = 0.3, w_lo: float = 0.2, w_hi: float = 0.8,
                lag_radius: float = 0.5) -> Instance:
    """Generate an instance of an ad-hoc shape (tests: ragged sizes, tiny m, etc.)."""
    w = Workload(f"custom_m{m}_n{n}_p{p}_{noise}", m, n, p, edge_prob, w_lo, w_hi,
                 lag_radius, noise, "f32")
    return make_instance(w, seed)


def batch_shapes(seed: int = 0, count: int = BATCH_COUNT):
    """The (m, n, noise) tuples of the batched workload, drawn from one seeded stream."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    ms = rng.integers(BATCH_M_RANGE[0], BATCH_M_RANGE[1] + 1, count)
    ns = rng.integers(BATCH_N_RANGE[0], BATCH_N_RANGE[1] + 1, count)
    kinds = np.where(rng.random(count) < 0.5, "uniform", "laplace")
    return [(int(a), int(b), str(c)) for a, b, c in zip(ms, ns, kinds)]


def make_batch(seed: int = 0, count: int = BATCH_COUNT) -> list[Instance]:
    """The batched workload: `count` independent instances of uneven (m, n), p = 1,
    q = 0.1, weights +-[0.1, 0.5], lag radius 0.5, uniform or Laplace noise (50/50)."""
    shapes = batch_shapes(seed, count)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for b, (m, n, kind) in enumerate(shapes):
        w = Workload(f"batch{b}_m{m}_n{n}_p1_{kind}", m, n, 1, 0.1, 0.1, 0.5, 0.5, kind, "f32")
        rng = np.random.default_rng(children[b])
        perm, B0, lags = _draw_model(rng, w, m)
        X, lags, rescaled = _simulate(rng, w, m, n, B0, lags)
        out.append(Instance(w, seed, X, B0, lags, perm, rescaled, {"index": b}))
    return out


def near_collinear(n: int, seed: int, rhos) -> np.ndarray:
    """n x (2 len(rhos) + 2) float32 series of i.i.d. rows: for each rho a pair of columns
    (z0, rho z0 + sqrt(1 - rho^2) z1) with Laplace, uniform and centred exponential noise in
    turn, then one Laplace and one uniform column unrelated to the rest.  Pairs near |rho| = 1
    are the near-collinear edge case of the pairwise residual."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    cols = []
    for k, r in enumerate(rhos):
        if k % 3 == 0:
            z0, z1 = rng.laplace(size=n), rng.laplace(size=n)
        elif k % 3 == 1:
            z0, z1 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        else:
            z0, z1 = rng.exponential(size=n) - 1.0, rng.exponential(size=n) - 1.0
        cols += [z0, r * z0 + math.sqrt(1.0 - r * r) * z1]
    cols += [rng.laplace(size=n), rng.uniform(-1, 1, n)]
    return np.ascontiguousarray(np.column_stack(cols).astype(np.float32))
