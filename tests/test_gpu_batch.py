"""GPU parity of the batched fit (varlingam_fit_batched, through the C ABI) against the FP64
oracle, problem by problem, with the single-problem protocol: order identical except where the
oracle's own margin is below 1e-9 (parity.order_violations), B0 / B_tau within 1e-5 relative
(parity.b_rel_error, floor 1e-2 max|B|), S within the pairwise tolerance 6e-6 (see
test_gpu_parity.py for its derivation)."""
import numpy as np
import pytest
import torch

import synth
from oracle import varlingam as O
import parity as PA

pytestmark = pytest.mark.gpu

TOL_S = 6e-6


@pytest.fixture(scope="module")
def api():
    from paper_2409_05500_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _api


def _instances(spec, seed0=0):
    """spec: list of (m, n, p, noise); edges q = 0.1, weights +-[0.1, 0.5] (the batched
    workload's law)."""
    return [synth.make_custom(m, n, p, noise, seed=seed0 + k, edge_prob=0.1, w_lo=0.1, w_hi=0.5)
            for k, (m, n, p, noise) in enumerate(spec)]


_ORACLE = {}


def _oracle_fit(inst, p):
    key = (inst.workload.name, inst.seed, p)
    if key not in _ORACLE:
        _ORACLE[key] = O.fit(inst.X_parity, p)
    return _ORACLE[key]


def _check_problem(res, inst, p, tol=PA.B_TOL_FP32, tol_s=TOL_S):
    ref = _oracle_fit(inst, p)
    S = res.S.cpu().numpy()
    assert np.array_equal(S, -S.T)
    assert np.max(np.abs(S - ref["S"])) <= tol_s
    order = res.order.cpu().numpy()
    assert sorted(order.tolist()) == list(range(inst.X32.shape[1]))
    assert PA.order_violations(order, ref["S"]) == []
    if np.array_equal(order, ref["order"]):
        B0_ref, Bl_ref = ref["B0"], ref["B_lags"]
    else:
        B0_ref, Bl_ref = O.estimate_B(ref["E"], order, ref["M"])
    e0 = PA.b_rel_error(res.B0.cpu().numpy(), B0_ref)
    e1 = PA.b_rel_error(res.B_lags.cpu().numpy(), Bl_ref)
    assert e0 <= tol and e1 <= tol, (e0, e1)
    assert PA.b_rel_error(res.M.cpu().numpy(), ref["M"]) <= tol
    return e0, e1


SPEC = [(2, 300, 1, "uniform"), (3, 257, 1, "laplace"), (20, 1000, 1, "uniform"),
        (63, 700, 1, "laplace"), (64, 1500, 1, "uniform"), (65, 2100, 1, "laplace"),
        (40, 1200, 2, "uniform"), (130, 3000, 1, "laplace"), (200, 4000, 1, "uniform"),
        (128, 2600, 2, "laplace"), (256, 2600, 1, "uniform")]


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_batch_matches_oracle(api, prec):
    insts = _instances(SPEC)
    # problems with different p go in separate batches (one p per batch in this binding)
    for p in (1, 2):
        sel = [(k, s) for k, s in enumerate(SPEC) if s[2] == p]
        print(f"batch prec={prec} p={p}: {[s[:2] for _, s in sel]}", flush=True)
        results, status = api.fit_batched([insts[k].X32 for k, _ in sel], p, prec)
        assert status == [0] * len(sel)
        tol = PA.B_TOL_FP32 if prec == "mixed" else PA.B_TOL_PLAIN
        for (k, s), r in zip(sel, results):
            e = _check_problem(r, insts[k], p, tol=tol)
            print(f"  m={s[0]} n={s[1]}: B rel err {e[0]:.1e} {e[1]:.1e}", flush=True)


def test_batch_matches_single_problem_path(api):
    insts = _instances(SPEC[:9], seed0=40)
    sel = [i for i, s in zip(insts, SPEC[:9]) if s[2] == 1]
    results, status = api.fit_batched([i.X32 for i in sel], 1, "mixed")
    assert status == [0] * len(sel)
    for inst, r in zip(sel, results):
        g = api.fit(torch.from_numpy(inst.X32).cuda(), 1, "mixed")
        # same kernel bodies; the Gram matrices (no split-K) and the pairwise moments (another
        # sample chunking, so other FP32 partial sums) are summed in another order: both are
        # within TOL_S of the oracle, hence within 2 TOL_S of each other
        assert np.max(np.abs(r.S.cpu().numpy() - g.S.cpu().numpy())) <= 2 * TOL_S
        np.testing.assert_allclose(r.E.cpu().numpy(), g.E.cpu().numpy(), rtol=0, atol=1e-5)


def test_batch_near_collinear_pairs(api):
    """Problems whose residuals hold pairs at rho = 0.99 ... 0.999999 (the collinear path of
    the batched moment stage) next to an ordinary one: S of each against the oracle's."""
    Xs = [synth.near_collinear(n, 50 + n, [0.99, 0.9999, 0.999999, 0.999])
          for n in (600, 3000)]
    plain = _instances([(12, 900, 1, "laplace")], seed0=3)[0]
    results, status = api.fit_batched(Xs + [plain.X32], 1, "mixed")
    assert status == [0, 0, 0]
    for X, r in zip(Xs + [plain.X32], results):
        ref = O.fit(X.astype(np.float64), 1, b_from_cov=True)
        S = r.S.cpu().numpy()
        assert np.array_equal(S, -S.T)
        ds = float(np.max(np.abs(S - ref["S"])))
        print(f"  near-collinear batch m={X.shape[1]} n={X.shape[0]}: max|dS| {ds:.2e}",
              flush=True)
        assert ds <= TOL_S


def test_batch_error_isolation(api):
    spec = [(10, 600, 1, "uniform"), (12, 800, 1, "laplace"), (9, 500, 1, "uniform")]
    insts = _instances(spec, seed0=7)
    Xs = [i.X32.copy() for i in insts]
    Xs[1][:, 4] = 2.5                                     # a constant series
    results, status = api.fit_batched(Xs, 1, "mixed")
    assert status[1] != 0 and status[0] == 0 and status[2] == 0
    for k in (0, 2):
        _check_problem(results[k], insts[k], 1)


def test_batch_deterministic_and_graph_replay(api):
    """Capture the batched fit in a graph; replay it on new data three times with eager work
    in between, every replay against an eager fit of the same data."""
    spec = [(15, 900, 1, "uniform"), (33, 1300, 1, "laplace"), (70, 2000, 1, "uniform")]
    a = _instances(spec, seed0=11)
    b = _instances(spec, seed0=21)
    bf = api.BatchFitter([i.X32.shape for i in a], 1, "mixed")
    bf.load([i.X32 for i in a])
    bf.run()
    first = [r.S.clone() for r in bf.results]
    bf.run()
    assert all(torch.equal(x, r.S) for x, r in zip(first, bf.results))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bf.run()                                          # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        bf.run()
    for rep, data in enumerate([b, a, b]):
        bf.load([i.X32 for i in data])
        bf.run()                                          # eager reference
        torch.cuda.synchronize()
        eager = [(r.S.clone(), r.order.clone(), r.B0.clone()) for r in bf.results]
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert bf.check() == [0, 0, 0]
        for (S, o, B0), r in zip(eager, bf.results):
            assert torch.equal(S, r.S) and torch.equal(o, r.order) and torch.equal(B0, r.B0), rep


def test_batch_autotune_keeps_results(api):
    spec = [(50, 3000, 1, "laplace"), (90, 5000, 1, "uniform"), (30, 800, 1, "laplace")]
    insts = _instances(spec, seed0=31)
    bf = api.BatchFitter([i.X32.shape for i in insts], 1, "mixed")
    bf.load([i.X32 for i in insts])
    chunk = bf.autotune()
    assert chunk in (512, 1024, 2048, 4096, 8192)
    bf.run()
    assert bf.check() == [0, 0, 0]
    for r, inst in zip(bf.results, insts):
        _check_problem(r, inst, 1)


def _read_tune(path):
    out = {}
    for line in open(path):
        k, v = line.split()
        out[k] = int(v)
    return out


def test_batch_autotune_per_bucket_cache(api, tmp_path, monkeypatch):
    """Per-bucket chunk lengths: the search writes one cache line per (device, precision,
    bucket) of the batch, every problem runs at its bucket's length, the mixed layout keeps the
    results, and a fresh process that finds all buckets in the file takes them as they are
    (no timing: the forced values below are not what the search chose)."""
    import json
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("VL_TUNE_CACHE", str(cache))
    # buckets (m class, n class): (0, 1), (2, 2), (3, 3)
    spec = [(24, 1500, 1, "laplace"), (100, 3000, 1, "uniform"), (140, 5000, 1, "laplace")]
    insts = _instances(spec, seed0=61)
    shapes = [i.X32.shape for i in insts]
    bf = api.BatchFitter(shapes, 1, "mixed")
    bf.load([i.X32 for i in insts])
    bf.autotune()
    lens = bf.chunk_lens()
    cands = (512, 1024, 2048, 4096, 8192)
    assert all(c in cands for c in lens)
    entries = _read_tune(cache)
    buckets = [f":p1:b{b}" for b in (1, 10, 15)]
    keys = [next(k for k in entries if k.endswith(sfx)) for sfx in buckets]
    assert [entries[k] for k in keys] == lens
    bf.run()
    assert bf.check() == [0, 0, 0]
    for r, inst in zip(bf.results, insts):
        _check_problem(r, inst, 1)
    # a fresh process reads forced values from the file and times nothing
    forced = [1024 if c != 1024 else 4096 for c in lens]
    cache2 = tmp_path / "tune2.txt"
    cache2.write_text("".join(f"{k} {v}\n" for k, v in zip(keys, forced)))
    before = cache2.read_text()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import json, sys; sys.path.insert(0, %r); "
            "from paper_2409_05500_amd import api; import torch; "
            "bf = api.BatchFitter(%r, 1, 'mixed'); bf.autotune(); "
            "print(json.dumps(bf.chunk_lens()))" % (root, [tuple(x) for x in shapes]))
    env = dict(os.environ, VL_TUNE_CACHE=str(cache2))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert json.loads(out.stdout.strip().splitlines()[-1]) == forced
    assert cache2.read_text() == before


def test_batch_full_workload_sampled(api):
    """The 256-problem workload (m in [20, 200], n in [500, 8000], uniform / Laplace):
    every problem checked for structure, four problems recomputed by the oracle."""
    insts = synth.make_batch(0)
    print(f"batch of {len(insts)}", flush=True)
    results, status = api.fit_batched([i.X32 for i in insts], 1, "mixed")
    assert status == [0] * len(insts)
    for r, inst in zip(results, insts):
        m = inst.X32.shape[1]
        S = r.S.cpu().numpy()
        assert np.array_equal(S, -S.T) and np.all(np.isfinite(S))
        assert sorted(r.order.cpu().numpy().tolist()) == list(range(m))
    ms = [i.X32.shape[1] for i in insts]
    for k in sorted({int(np.argmin(ms)), int(np.argmax(ms)), 17, 200}):
        print(f"  oracle check of problem {k} (m={ms[k]})", flush=True)
        _check_problem(results[k], insts[k], 1)
