"""Torch-facing wrappers of the C ABI: they allocate outputs and workspace as CUDA (HIP)
tensors, pass raw device pointers and the current stream, and check the status codes.
All arithmetic happens in the HIP library."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import PREC, check, lib


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _prec(prec) -> int:
    if isinstance(prec, int):
        return prec
    return PREC[prec]


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 256-byte aligned blocks (512 in practice)
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


class DeviceStatus:
    """The int32 status word the kernels write; read() synchronises and raises on error."""

    def __init__(self, device):
        self.t = torch.zeros(1, dtype=torch.int32, device=device)

    @property
    def ptr(self) -> int:
        return self.t.data_ptr()

    def read(self, where: str) -> None:
        code = int(self.t.item())
        check(code, where)


def _require(t: torch.Tensor, dtype, name: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 2 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")


def fit_var(X: torch.Tensor, p: int, prec="mixed", status: "DeviceStatus | None" = None):
    """VAR(p) least-squares fit with intercept.  X: n x m float32 device tensor.
    Returns (M [p, m, m] f64, intercept [m] f64, E [n-p, m] f32)."""
    _require(X, torch.float32, "X")
    n, m = X.shape
    dev = X.device
    M = torch.empty((p, m, m), dtype=torch.float64, device=dev)
    c = torch.empty(m, dtype=torch.float64, device=dev)
    E = torch.empty((n - p, m), dtype=torch.float32, device=dev)
    nb = lib.varlingam_fit_var_workspace_bytes(n, m, p, _prec(prec))
    ws = _workspace(nb, dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_fit_var(X.data_ptr(), n, m, X.stride(0), p, _prec(prec), M.data_ptr(),
                                c.data_ptr(), E.data_ptr(), E.stride(0), ws.data_ptr(),
                                ws.numel(), st.ptr, _stream_ptr(dev)), "varlingam_fit_var")
    if status is None:
        st.read("varlingam_fit_var")
    return M, c, E


def select_lag(X: torch.Tensor, p_max: int, status: "DeviceStatus | None" = None):
    """VAR lag-order selection over p = 1 .. p_max on the common sample t = p_max .. n-1:
    (logdet [p_max], aic [p_max], bic [p_max]) f64 and (p_AIC, p_BIC)."""
    _require(X, torch.float32, "X")
    n, m = X.shape
    dev = X.device
    logdet = torch.empty(p_max, dtype=torch.float64, device=dev)
    aic = torch.empty(p_max, dtype=torch.float64, device=dev)
    bic = torch.empty(p_max, dtype=torch.float64, device=dev)
    best = torch.empty(2, dtype=torch.int32, device=dev)
    ws = _workspace(lib.varlingam_select_lag_workspace_bytes(n, m, p_max), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_select_lag(X.data_ptr(), n, m, X.stride(0), p_max, logdet.data_ptr(),
                                   aic.data_ptr(), bic.data_ptr(), best.data_ptr(),
                                   ws.data_ptr(), ws.numel(), st.ptr, _stream_ptr(dev)),
          "varlingam_select_lag")
    if status is None:
        st.read("varlingam_select_lag")
    b = best.cpu().tolist()
    return logdet, aic, bic, (int(b[0]), int(b[1]))


def _pairwise_prec(prec, compensated: bool) -> int:
    return _prec(prec) | (_lib.PAIRWISE_COMPENSATED if compensated else 0)


def pairwise_stats(E: torch.Tensor, prec="mixed", status: "DeviceStatus | None" = None,
                   compensated: bool = False):
    """Hx [m], Hr [m, m], S [m, m], Cov [m, m] (all f64) from the n_eff x m residuals.
    compensated: Kahan-compensated moment sums with FP64 partials (VL_PAIRWISE_COMPENSATED)."""
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    prec = _pairwise_prec(prec, compensated)
    Hx = torch.empty(m, dtype=torch.float64, device=dev)
    Hr = torch.empty((m, m), dtype=torch.float64, device=dev)
    S = torch.empty((m, m), dtype=torch.float64, device=dev)
    Cov = torch.empty((m, m), dtype=torch.float64, device=dev)
    nb = lib.pairwise_stats_workspace_bytes(n_eff, m, _prec(prec))
    ws = _workspace(nb, dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.pairwise_stats(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec), Hx.data_ptr(),
                             Hr.data_ptr(), S.data_ptr(), Cov.data_ptr(), ws.data_ptr(),
                             ws.numel(), st.ptr, _stream_ptr(dev)), "pairwise_stats")
    if status is None:
        st.read("pairwise_stats")
    return Hx, Hr, S, Cov


def pairwise_stats_noalloc(E: torch.Tensor, prec="mixed", status: "DeviceStatus | None" = None,
                           out=None, compensated: bool = False):
    """pairwise_stats through the entry point that takes no workspace (the library's static
    per-GPU scratch).  `out` may hold preallocated (Hx, Hr, S, Cov) f64 device tensors, so that
    the call itself allocates nothing."""
    prec = _pairwise_prec(prec, compensated)
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    if out is None:
        out = (torch.empty(m, dtype=torch.float64, device=dev),
               torch.empty((m, m), dtype=torch.float64, device=dev),
               torch.empty((m, m), dtype=torch.float64, device=dev),
               torch.empty((m, m), dtype=torch.float64, device=dev))
    Hx, Hr, S, Cov = out
    for t, shape in zip(out, ((m,), (m, m), (m, m), (m, m))):
        if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or \
                not t.is_contiguous():
            raise ValueError("out must be contiguous f64 device tensors (m), (m, m) x 3")
    st = status if status is not None else DeviceStatus(dev)
    check(lib.pairwise_stats_noalloc(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec),
                                     Hx.data_ptr(), Hr.data_ptr(), S.data_ptr(), Cov.data_ptr(),
                                     st.ptr, _stream_ptr(dev)), "pairwise_stats_noalloc")
    if status is None:
        st.read("pairwise_stats_noalloc")
    return Hx, Hr, S, Cov


def pairwise_stats_save(E: torch.Tensor, prec="mixed", status: "DeviceStatus | None" = None):
    """pairwise_stats plus the block of forward statistics the backward can reuse:
    (Hx, Hr, S, Cov, saved) with saved [3 m^2 + 3 m] f64."""
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    Hx = torch.empty(m, dtype=torch.float64, device=dev)
    Hr = torch.empty((m, m), dtype=torch.float64, device=dev)
    S = torch.empty((m, m), dtype=torch.float64, device=dev)
    Cov = torch.empty((m, m), dtype=torch.float64, device=dev)
    saved = torch.empty(lib.pairwise_stats_saved_doubles(m), dtype=torch.float64, device=dev)
    ws = _workspace(lib.pairwise_stats_workspace_bytes(n_eff, m, _prec(prec)), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.pairwise_stats_save(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec),
                                  Hx.data_ptr(), Hr.data_ptr(), S.data_ptr(), Cov.data_ptr(),
                                  saved.data_ptr(), ws.data_ptr(), ws.numel(), st.ptr,
                                  _stream_ptr(dev)), "pairwise_stats_save")
    if status is None:
        st.read("pairwise_stats_save")
    return Hx, Hr, S, Cov, saved


def pairwise_stats_backward(E: torch.Tensor, G: torch.Tensor, prec="mixed",
                            status: "DeviceStatus | None" = None,
                            saved: "torch.Tensor | None" = None) -> torch.Tensor:
    """dE = d<G, S(E)>/dE (n_eff x m f32) for the m x m f64 cotangent G of the score matrix;
    `saved` (from pairwise_stats_save on the same E) skips the forward recompute."""
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    G = G.to(device=dev, dtype=torch.float64).contiguous()
    if G.shape != (m, m):
        raise ValueError(f"G must be {m} x {m}, got {tuple(G.shape)}")
    if saved is not None and (saved.dtype != torch.float64 or not saved.is_cuda or
                              saved.numel() != lib.pairwise_stats_saved_doubles(m)):
        raise ValueError("saved must be the f64 device block of pairwise_stats_save")
    dE = torch.empty((n_eff, m), dtype=torch.float32, device=dev)
    nb = lib.pairwise_stats_backward_workspace_bytes(n_eff, m, _prec(prec))
    ws = _workspace(nb, dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.pairwise_stats_backward(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec),
                                      saved.data_ptr() if saved is not None else None,
                                      G.data_ptr(), dE.data_ptr(), dE.stride(0), ws.data_ptr(),
                                      ws.numel(), st.ptr, _stream_ptr(dev)),
          "pairwise_stats_backward")
    if status is None:
        st.read("pairwise_stats_backward")
    return dE


def edge_influence(E: torch.Tensor, i: int, j: int, prec="mixed",
                   saved: "torch.Tensor | None" = None) -> torch.Tensor:
    """Per-sample influence of the residuals on one edge direction: dS[i, j]/dE (n_eff x m
    f32), the backward with a one-hot cotangent.  Row t, column k: how S[i, j] (positive when
    the data favour j -> i over i -> j) moves with e_k(t)."""
    m = E.shape[1]
    if not (0 <= i < m and 0 <= j < m):
        raise ValueError(f"edge ({i}, {j}) outside 0 .. {m - 1}")
    G = torch.zeros((m, m), dtype=torch.float64, device=E.device)
    G[i, j] = 1.0
    return pairwise_stats_backward(E, G, prec, saved=saved)


class PairwiseScore(torch.autograd.Function):
    """S = score(E) with a backward through the HIP gradient kernels; the forward keeps the
    O(m^2) block of statistics the backward needs (no recompute of the moments)."""

    @staticmethod
    def forward(ctx, E, prec="mixed"):
        ctx.prec = prec
        _, _, S, _, saved = pairwise_stats_save(E.detach(), prec)
        ctx.save_for_backward(E, saved)
        return S

    @staticmethod
    def backward(ctx, G):
        E, saved = ctx.saved_tensors
        return pairwise_stats_backward(E.detach(), G, ctx.prec, saved=saved), None


def pairwise_score(E: torch.Tensor, prec="mixed") -> torch.Tensor:
    """Differentiable S(E) (m x m f64) for an n_eff x m f32 device tensor."""
    return PairwiseScore.apply(E, prec)


def approx_order(S: torch.Tensor, status: "DeviceStatus | None" = None):
    """(order [m] int32, margin [m] f64) from the m x m score matrix."""
    _require(S, torch.float64, "S")
    m = S.shape[0]
    dev = S.device
    order = torch.empty(m, dtype=torch.int32, device=dev)
    margin = torch.empty(m, dtype=torch.float64, device=dev)
    ws = _workspace(lib.approx_order_workspace_bytes(m), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.approx_order(S.contiguous().data_ptr(), m, order.data_ptr(), margin.data_ptr(),
                           ws.data_ptr(), ws.numel(), st.ptr, _stream_ptr(dev)), "approx_order")
    if status is None:
        st.read("approx_order")
    return order, margin


# The largest |S - S_oracle| the FP32-moment scores of pairwise_stats showed on any workload
# tested (6.1e-7), rounded up: the default error bound of the certified ordering.
CERT_EPS_S = 1e-6


def approx_order_certified(E: torch.Tensor, S: torch.Tensor, eps_S: float = CERT_EPS_S,
                           status: "DeviceStatus | None" = None):
    """Alg. 1 on S with every step the bound eps_S cannot settle re-decided on FP64 scores
    recomputed from E (n_eff x m f32, the data S came from).  S (m x m f64) is updated in
    place.  Returns (order [m] int32, margin [m] f64, refined [m] int32 flags, rows refined).
    Synchronises the stream."""
    _require(E, torch.float32, "E")
    _require(S, torch.float64, "S")
    n_eff, m = E.shape
    dev = E.device
    if not S.is_contiguous() or tuple(S.shape) != (m, m):
        raise ValueError("S must be a contiguous m x m f64 device tensor")
    order = torch.empty(m, dtype=torch.int32, device=dev)
    margin = torch.empty(m, dtype=torch.float64, device=dev)
    refined = torch.empty(m, dtype=torch.int32, device=dev)
    ws = _workspace(lib.approx_order_certified_workspace_bytes(n_eff, m), dev)
    st = status if status is not None else DeviceStatus(dev)
    nref = C.c_int64(0)
    check(lib.approx_order_certified(E.data_ptr(), n_eff, m, E.stride(0), S.data_ptr(),
                                     float(eps_S), order.data_ptr(), margin.data_ptr(),
                                     refined.data_ptr(), C.byref(nref), ws.data_ptr(),
                                     ws.numel(), st.ptr, _stream_ptr(dev)),
          "approx_order_certified")
    if status is None:
        st.read("approx_order_certified")
    return order, margin, refined, int(nref.value)


def order_iterative(E: torch.Tensor, prec="mixed", status: "DeviceStatus | None" = None):
    """(order [m] int32, margin [m] f64) of the original iterative DirectLiNGAM search on the
    n_eff x m residuals (the pairwise scores recomputed on the updated data at every step)."""
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    order = torch.empty(m, dtype=torch.int32, device=dev)
    margin = torch.empty(m, dtype=torch.float64, device=dev)
    ws = _workspace(lib.varlingam_order_iterative_workspace_bytes(n_eff, m, _prec(prec)), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_order_iterative(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec),
                                        order.data_ptr(), margin.data_ptr(), ws.data_ptr(),
                                        ws.numel(), st.ptr, _stream_ptr(dev)),
          "varlingam_order_iterative")
    if status is None:
        st.read("varlingam_order_iterative")
    return order, margin


def order_hybrid(E: torch.Tensor, k_exact: int, prec="mixed",
                 status: "DeviceStatus | None" = None):
    """(order [m] int32, margin [m] f64): the original search's first k_exact picks, then the
    heuristic's lookup-only ordering of the remaining variables on their refined data."""
    _require(E, torch.float32, "E")
    n_eff, m = E.shape
    dev = E.device
    order = torch.empty(m, dtype=torch.int32, device=dev)
    margin = torch.empty(m, dtype=torch.float64, device=dev)
    ws = _workspace(lib.varlingam_order_hybrid_workspace_bytes(n_eff, m, _prec(prec)), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_order_hybrid(E.data_ptr(), n_eff, m, E.stride(0), _prec(prec), k_exact,
                                     order.data_ptr(), margin.data_ptr(), ws.data_ptr(),
                                     ws.numel(), st.ptr, _stream_ptr(dev)),
          "varlingam_order_hybrid")
    if status is None:
        st.read("varlingam_order_hybrid")
    return order, margin


def estimate_B(Cov: torch.Tensor, M: torch.Tensor, order: torch.Tensor,
               status: "DeviceStatus | None" = None):
    """(B0 [m, m], B_lags [p, m, m]) f64 from the residual covariance, VAR matrices and order."""
    _require(Cov, torch.float64, "Cov")
    m = Cov.shape[0]
    p = M.shape[0] if M is not None else 0
    dev = Cov.device
    B0 = torch.zeros((m, m), dtype=torch.float64, device=dev)
    Bl = torch.empty((max(p, 1), m, m), dtype=torch.float64, device=dev)
    ws = _workspace(lib.estimate_B_workspace_bytes(m, p), dev)
    st = status if status is not None else DeviceStatus(dev)
    Mp = M.contiguous().data_ptr() if p > 0 else None
    check(lib.estimate_B(Cov.contiguous().data_ptr(), Mp, order.contiguous().data_ptr(), m, p,
                         B0.data_ptr(), Bl.data_ptr() if p > 0 else None, ws.data_ptr(),
                         ws.numel(), st.ptr, _stream_ptr(dev)), "estimate_B")
    if status is None:
        st.read("estimate_B")
    return B0, Bl[:p]


def prune(X: torch.Tensor, p: int, order: torch.Tensor, B0: torch.Tensor, B_lags: torch.Tensor,
          max_steps: int = 0, status: "DeviceStatus | None" = None):
    """Adaptive-lasso pruning of (B0, B_lags) on the series X (n x m float32) of the fit:
    (B0 [m, m], B_lags [p, m, m]) f64 with exact zeros, and info [m, 3] int32 (path steps,
    chosen knot, nonzeros) per variable."""
    _require(X, torch.float32, "X")
    n, m = X.shape
    dev = X.device
    B0o = torch.empty((m, m), dtype=torch.float64, device=dev)
    Blo = torch.empty((p, m, m), dtype=torch.float64, device=dev)
    info = torch.empty((m, 3), dtype=torch.int32, device=dev)
    ws = _workspace(lib.varlingam_prune_workspace_bytes(n, m, p, max_steps), dev)
    st = status if status is not None else DeviceStatus(dev)
    K = order.to(torch.int32).contiguous()
    B0c = B0.to(torch.float64).contiguous()
    Blc = B_lags.to(torch.float64).contiguous()
    check(lib.varlingam_prune(X.data_ptr(), n, m, X.stride(0), p, K.data_ptr(), B0c.data_ptr(),
                              Blc.data_ptr(), max_steps, B0o.data_ptr(), Blo.data_ptr(),
                              info.data_ptr(),
                              ws.data_ptr(), ws.numel(), st.ptr, _stream_ptr(dev)),
          "varlingam_prune")
    if status is None:
        st.read("varlingam_prune")
    return B0o, Blo, info


def probe_rates(device="cuda:0") -> dict:
    """Measured issue rates of this GPU (varlingam_probe_rates): FP32 exp2 per second, FP32
    FMA flop/s and FP64 MFMA flop/s."""
    dev = torch.device(device)
    ws = _workspace(lib.varlingam_probe_workspace_bytes(), dev)
    out = (C.c_double * 3)()
    check(lib.varlingam_probe_rates(out, ws.data_ptr(), ws.numel(), _stream_ptr(dev)),
          "varlingam_probe_rates")
    return {"exp2_per_s": out[0], "fp32_fma_flops": out[1], "fp64_mfma_flops": out[2]}


@dataclass
class FitResult:
    M: torch.Tensor
    intercept: torch.Tensor
    E: torch.Tensor
    Hx: torch.Tensor
    Hr: torch.Tensor
    S: torch.Tensor
    Cov: torch.Tensor
    order: torch.Tensor
    margin: torch.Tensor
    B0: torch.Tensor
    B_lags: torch.Tensor


def fit(X: torch.Tensor, p: int, prec="mixed", verify: bool = True) -> FitResult:
    """The whole heuristic VarLiNGAM on the device: VAR fit -> pairwise precompute ->
    ordering -> B0 and B_tau, enqueued back to back on the current stream.  With `verify`, the
    four status words are read (one synchronisation) at the end."""
    dev = X.device
    st = [DeviceStatus(dev) for _ in range(4)]
    M, c, E = fit_var(X, p, prec, status=st[0])
    Hx, Hr, S, Cov = pairwise_stats(E, prec, status=st[1])
    order, margin = approx_order(S, status=st[2])
    B0, Bl = estimate_B(Cov, M, order, status=st[3])
    if verify:
        for s, name in zip(st, ("varlingam_fit_var", "pairwise_stats", "approx_order",
                                "estimate_B")):
            s.read(name)
    return FitResult(M, c, E, Hx, Hr, S, Cov, order, margin, B0, Bl)


class Fitter:
    """Preallocated outputs and one shared workspace for repeated fits of one shape: run(X)
    enqueues the four stages on the current stream with no host allocation and no
    synchronisation; check() reads the four status words."""

    STAGES = ("varlingam_fit_var", "pairwise_stats", "approx_order", "estimate_B")

    def __init__(self, n: int, m: int, p: int, prec="mixed", device="cuda:0",
                 compensated: bool = False):
        """compensated: the precompute's moment sums with Kahan compensation (the
        VL_PAIRWISE_COMPENSATED flag on its pairwise_stats call)."""
        dev = torch.device(device)
        self.n, self.m, self.p, self.prec, self.dev = n, m, p, _prec(prec), dev
        self.pw_prec = _pairwise_prec(prec, compensated)
        f64 = dict(dtype=torch.float64, device=dev)
        self.M = torch.empty((p, m, m), **f64)
        self.intercept = torch.empty(m, **f64)
        self.E = torch.empty((n - p, m), dtype=torch.float32, device=dev)
        self.Hx = torch.empty(m, **f64)
        self.Hr = torch.empty((m, m), **f64)
        self.S = torch.empty((m, m), **f64)
        self.Cov = torch.empty((m, m), **f64)
        self.order = torch.empty(m, dtype=torch.int32, device=dev)
        self.margin = torch.empty(m, **f64)
        self.B0 = torch.empty((m, m), **f64)
        self.B_lags = torch.empty((p, m, m), **f64)
        need = max(lib.varlingam_fit_var_workspace_bytes(n, m, p, self.prec),
                   lib.pairwise_stats_workspace_bytes(n - p, m, self.pw_prec),
                   lib.approx_order_workspace_bytes(m), lib.estimate_B_workspace_bytes(m, p))
        if need == 0:
            raise ValueError(f"unsupported shape n={n} m={m} p={p}")
        self.ws = _workspace(need, dev)
        self.status = torch.zeros(4, dtype=torch.int32, device=dev)

    def run(self, X: torch.Tensor) -> None:
        _require(X, torch.float32, "X")
        if tuple(X.shape) != (self.n, self.m):
            raise ValueError(f"X must be {self.n} x {self.m}")
        n, m, p, pr = self.n, self.m, self.p, self.prec
        s = _stream_ptr(self.dev)
        ws, nb = self.ws.data_ptr(), self.ws.numel()
        st = self.status.data_ptr()
        check(lib.varlingam_fit_var(X.data_ptr(), n, m, X.stride(0), p, pr, self.M.data_ptr(),
                                    self.intercept.data_ptr(), self.E.data_ptr(), m, ws, nb, st,
                                    s), "varlingam_fit_var")
        check(lib.pairwise_stats(self.E.data_ptr(), n - p, m, m, self.pw_prec,
                                 self.Hx.data_ptr(), self.Hr.data_ptr(), self.S.data_ptr(),
                                 self.Cov.data_ptr(), ws, nb, st + 4, s), "pairwise_stats")
        check(lib.approx_order(self.S.data_ptr(), m, self.order.data_ptr(),
                               self.margin.data_ptr(), ws, nb, st + 8, s), "approx_order")
        check(lib.estimate_B(self.Cov.data_ptr(), self.M.data_ptr(), self.order.data_ptr(), m, p,
                             self.B0.data_ptr(), self.B_lags.data_ptr(), ws, nb, st + 12, s),
              "estimate_B")

    def check(self) -> None:
        for code, name in zip(self.status.cpu().tolist(), self.STAGES):
            check(int(code), name)


@dataclass
class BatchResult:
    M: torch.Tensor
    intercept: torch.Tensor
    E: torch.Tensor
    S: torch.Tensor
    order: torch.Tensor
    margin: torch.Tensor
    B0: torch.Tensor
    B_lags: torch.Tensor


class BatchFitter:
    """Many problems of uneven (n, m) through the whole path with one kernel launch per stage
    (varlingam_fit_batched).  Inputs and outputs are preallocated per problem; the plan is
    bound to one workspace once.  load() copies new series in, run() enqueues the fit on the
    current stream (no allocation, no synchronisation: it may be captured in a graph),
    check() reads the per-problem status words."""

    def __init__(self, shapes, p: int = 1, prec="mixed", device="cuda:0"):
        dev = torch.device(device)
        self.dev, self.p, self.prec = dev, p, _prec(prec)
        f64 = dict(dtype=torch.float64, device=dev)
        self.X, self.results = [], []
        desc = (_lib.VlInstance * len(shapes))()
        for b, (n, m) in enumerate(shapes):
            X = torch.zeros((n, m), dtype=torch.float32, device=dev)
            r = BatchResult(M=torch.empty((p, m, m), **f64), intercept=torch.empty(m, **f64),
                            E=torch.empty((n - p, m), dtype=torch.float32, device=dev),
                            S=torch.empty((m, m), **f64),
                            order=torch.empty(m, dtype=torch.int32, device=dev),
                            margin=torch.empty(m, **f64), B0=torch.empty((m, m), **f64),
                            B_lags=torch.empty((p, m, m), **f64))
            self.X.append(X)
            self.results.append(r)
            d = desc[b]
            d.X, d.n, d.m, d.ldx, d.p = X.data_ptr(), n, m, m, p
            d.M, d.intercept, d.E, d.lde = r.M.data_ptr(), r.intercept.data_ptr(), \
                r.E.data_ptr(), m
            d.S, d.order, d.margin = r.S.data_ptr(), r.order.data_ptr(), r.margin.data_ptr()
            d.B0, d.Blag = r.B0.data_ptr(), r.B_lags.data_ptr()
        handle = C.c_void_p()
        check(lib.varlingam_batch_create(desc, len(shapes), self.prec, C.byref(handle)),
              "varlingam_batch_create")
        self._h = handle
        self.ws = _workspace(lib.varlingam_batch_workspace_bytes(handle), dev)
        self.status = torch.zeros(len(shapes), dtype=torch.int32, device=dev)
        check(lib.varlingam_batch_bind(handle, self.ws.data_ptr(), self.ws.numel(),
                                       _stream_ptr(dev)), "varlingam_batch_bind")

    def __len__(self):
        return len(self.X)

    def load(self, Xs) -> None:
        for dst, src in zip(self.X, Xs):
            dst.copy_(torch.as_tensor(src, dtype=torch.float32), non_blocking=False)

    def run(self) -> None:
        check(lib.varlingam_fit_batched(self._h, self.ws.data_ptr(), self.status.data_ptr(),
                                        _stream_ptr(self.dev)), "varlingam_fit_batched")

    def autotune(self) -> int:
        """Choose the pairwise chunk length per (m, n) bucket by timing whole fits on the loaded
        data (cached per device and bucket, also on disk); returns the length of the bucket
        with the most problems."""
        check(lib.varlingam_batch_autotune(self._h, self.ws.data_ptr(), self.ws.numel(),
                                           self.status.data_ptr(), _stream_ptr(self.dev)),
              "varlingam_batch_autotune")
        return lib.varlingam_batch_chunk_len(self._h)

    @property
    def chunk_len(self) -> int:
        return lib.varlingam_batch_chunk_len(self._h)

    def chunk_lens(self) -> list:
        """The pairwise chunk length of every problem."""
        return [lib.varlingam_batch_chunk_len_of(self._h, b) for b in range(len(self.X))]

    def check(self) -> list:
        """Per-problem status codes (0 = ok); synchronises."""
        return [int(v) for v in self.status.cpu().tolist()]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.varlingam_batch_destroy(h)
            self._h = None


def var_simulate(M: torch.Tensor, intercept: torch.Tensor, X0: torch.Tensor, E: torch.Tensor,
                 idx: torch.Tensor, out: "torch.Tensor | None" = None,
                 status: "DeviceStatus | None" = None) -> torch.Tensor:
    """Residual-bootstrap series of a fitted VAR: (R, p + T, m) float32 from M [p, m, m],
    intercept [m] (f64), the first p rows X0 [p, m], a residual pool E [n_e, m] (f32) and the
    draws idx [R, T] (int32, rows of E)."""
    p, m, _ = M.shape
    R, T = idx.shape
    dev = M.device
    if out is None:
        out = torch.empty((R, p + T, m), dtype=torch.float32, device=dev)
    assert out.shape == (R, p + T, m) and out.stride(2) == 1 and out.stride(1) == m
    Mc, cc = M.contiguous(), intercept.contiguous()
    Ic = idx.to(torch.int32).contiguous()
    _require(X0, torch.float32, "X0")
    _require(E, torch.float32, "E")
    ws = _workspace(lib.varlingam_var_simulate_workspace_bytes(m, p), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_var_simulate(Mc.data_ptr(), cc.data_ptr(), m, p, X0.data_ptr(),
                                     X0.stride(0), E.data_ptr(), E.shape[0], E.stride(0),
                                     Ic.data_ptr(), R, T, out.data_ptr(), m, out.stride(0),
                                     ws.data_ptr(), ws.numel(), st.ptr, _stream_ptr(dev)),
          "varlingam_var_simulate")
    if status is None:
        st.read("varlingam_var_simulate")
    return out


def edge_frequency(orders: torch.Tensor, B0s: torch.Tensor, B_lags: torch.Tensor,
                   threshold: float = 0.0, problem_status: "torch.Tensor | None" = None,
                   status: "DeviceStatus | None" = None):
    """Aggregate K fits: (P0 [m, m], P_lags [p, m, m], P_order [m, m]) f64 and the number of
    problems used (status VL_OK)."""
    K, m = orders.shape
    p = B_lags.shape[1] if B_lags is not None else 0
    dev = orders.device
    f64 = dict(dtype=torch.float64, device=dev)
    P0, Pl, Po = torch.empty((m, m), **f64), torch.empty((max(p, 1), m, m), **f64), \
        torch.empty((m, m), **f64)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    Oc = orders.to(torch.int32).contiguous()
    Bc = B0s.contiguous()
    Lc = B_lags.contiguous() if p > 0 else None
    Sc = problem_status.to(torch.int32).contiguous() if problem_status is not None else None
    ws = _workspace(lib.varlingam_edge_frequency_workspace_bytes(K, m), dev)
    st = status if status is not None else DeviceStatus(dev)
    check(lib.varlingam_edge_frequency(Oc.data_ptr(), Bc.data_ptr(),
                                       Lc.data_ptr() if p > 0 else None, K, m, p,
                                       float(threshold),
                                       Sc.data_ptr() if Sc is not None else None, P0.data_ptr(),
                                       Pl.data_ptr() if p > 0 else None, Po.data_ptr(),
                                       cnt.data_ptr(), ws.data_ptr(), ws.numel(), st.ptr,
                                       _stream_ptr(dev)), "varlingam_edge_frequency")
    if status is None:
        st.read("varlingam_edge_frequency")
    return P0, Pl[:p], Po, int(cnt.item())


class EnsembleFitter:
    """K fits of one dataset's problems (equal n, m, p) on the batched path: rolling windows or
    bootstrap resamples.  The inputs are views into caller buffers (a window of a series, a
    resample of a stack), so nothing is copied; outputs are stacked: order [K, m], B0 [K, m, m],
    B_lags [K, p, m, m], M, intercept, E.  run() enqueues the batched fit and the aggregation
    on the current stream without synchronising."""

    def __init__(self, views, p: int = 1, prec="mixed", threshold: float = 0.0):
        K = len(views)
        n, m = views[0].shape
        dev = views[0].device
        self.views, self.p, self.prec, self.threshold = list(views), p, _prec(prec), threshold
        f64 = dict(dtype=torch.float64, device=dev)
        self.M = torch.empty((K, p, m, m), **f64)
        self.intercept = torch.empty((K, m), **f64)
        self.E = torch.empty((K, n - p, m), dtype=torch.float32, device=dev)
        self.order = torch.empty((K, m), dtype=torch.int32, device=dev)
        self.B0 = torch.empty((K, m, m), **f64)
        self.B_lags = torch.empty((K, p, m, m), **f64)
        desc = (_lib.VlInstance * K)()
        for k, X in enumerate(views):
            assert X.shape == (n, m) and X.dtype == torch.float32 and X.stride(1) == 1
            d = desc[k]
            d.X, d.n, d.m, d.ldx, d.p = X.data_ptr(), n, m, X.stride(0), p
            d.M, d.intercept = self.M[k].data_ptr(), self.intercept[k].data_ptr()
            d.E, d.lde = self.E[k].data_ptr(), m
            d.S, d.margin = None, None
            d.order, d.B0, d.Blag = self.order[k].data_ptr(), self.B0[k].data_ptr(), \
                self.B_lags[k].data_ptr()
        handle = C.c_void_p()
        check(lib.varlingam_batch_create(desc, K, self.prec, C.byref(handle)),
              "varlingam_batch_create")
        self._h = handle
        self.ws = _workspace(lib.varlingam_batch_workspace_bytes(handle), dev)
        self.status = torch.zeros(K, dtype=torch.int32, device=dev)
        check(lib.varlingam_batch_bind(handle, self.ws.data_ptr(), self.ws.numel(),
                                       _stream_ptr(dev)), "varlingam_batch_bind")
        self.agg_status = DeviceStatus(dev)
        self.P0 = self.P_lags = self.P_order = None
        self.count = None

    def run(self) -> None:
        check(lib.varlingam_fit_batched(self._h, self.ws.data_ptr(), self.status.data_ptr(),
                                        _stream_ptr(self.status.device)), "varlingam_fit_batched")

    def aggregate(self):
        """(P0, P_lags, P_order, count) over the problems that succeeded."""
        self.P0, self.P_lags, self.P_order, self.count = edge_frequency(
            self.order, self.B0, self.B_lags, self.threshold, self.status)
        return self.P0, self.P_lags, self.P_order, self.count

    def check(self) -> list:
        return [int(v) for v in self.status.cpu().tolist()]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib.varlingam_batch_destroy(h)
            self._h = None


def rolling_windows(X: torch.Tensor, p: int, window: int, stride: int, threshold: float = 0.0,
                    prec="mixed") -> EnsembleFitter:
    """Fit every window X[k stride : k stride + window] (no copies) and aggregate."""
    _require(X, torch.float32, "X")
    starts = list(range(0, X.shape[0] - window + 1, stride))
    ef = EnsembleFitter([X[s: s + window] for s in starts], p, prec, threshold)
    ef.starts = starts
    ef.run()
    ef.aggregate()
    return ef


def bootstrap(X: torch.Tensor, p: int, idx, threshold: float = 0.0, prec="mixed"):
    """Residual bootstrap: fit the VAR of X, regenerate one series per row of the draws idx
    (R x (n - p), rows of the residual matrix), fit every resample on the batched path and
    aggregate.  Returns the EnsembleFitter (its views are the resampled series)."""
    _require(X, torch.float32, "X")
    n, m = X.shape
    M, c, E = fit_var(X, p, prec)
    idx = torch.as_tensor(idx, dtype=torch.int32).to(X.device)
    series = var_simulate(M, c, X[:p].contiguous(), E, idx)
    ef = EnsembleFitter(list(series), p, prec, threshold)
    ef.series = series
    ef.run()
    ef.aggregate()
    return ef


def fit_batched(Xs, p: int = 1, prec="mixed", autotune: bool = False):
    """Fit every series in Xs (a list of n_b x m_b arrays or tensors) in one batched pass.
    Returns (results, status codes)."""
    dev = torch.device("cuda:0")
    bf = BatchFitter([tuple(x.shape) for x in Xs], p, prec, dev)
    bf.load(Xs)
    if autotune:
        bf.autotune()
    bf.run()
    return bf.results, bf.check()
