"""Heuristic VarLiNGAM hot path on MI355X (gfx950): VAR fit, one-time pairwise entropy
precompute, lookup-only causal ordering and B estimation, as hand-written HIP kernels behind a
C ABI (include/varlingam.h).

`import paper_2409_05500_amd` loads nothing; the HIP library is loaded on first use of the
API (`paper_2409_05500_amd.api`), which raises if libvarlingam.so has not been built.
"""
_API = ("fit", "fit_var", "pairwise_stats", "approx_order", "estimate_B", "FitResult", "Fitter",
        "DeviceStatus", "pairwise_stats_backward", "pairwise_stats_save", "pairwise_score",
        "PairwiseScore", "BatchFitter", "fit_batched", "order_iterative", "order_hybrid",
        "select_lag", "prune", "var_simulate", "edge_frequency", "EnsembleFitter",
        "rolling_windows", "bootstrap", "edge_influence")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
