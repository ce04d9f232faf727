"""pairwise_stats_noalloc (the entry point without a workspace, on the library's static
per-GPU scratch) against pairwise_stats on the same inputs: the same kernels and the same
launch plan, so the outputs must agree bit for bit.  Two calls in a row, the second smaller,
then the first size again (the scratch keeps the last call's contents)."""
import numpy as np
import pytest
import torch

import synth
from oracle import varlingam as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2409_05500_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return _api


def _residuals(name, seed):
    inst = synth.make_instance(name, seed)
    _, _, E = O.fit_var(inst.X_parity, inst.workload.p)
    return E.astype(np.float32)


def test_noalloc_matches_pairwise_stats(api):
    dev = torch.device("cuda:0")
    cases = [("m400_n10000_p2_t4", 0), ("m100_n5000_p1_laplace", 1), ("m400_n10000_p2_t4", 2)]
    for name, seed in cases:
        E = torch.from_numpy(_residuals(name, seed)).to(dev)
        print(f"noalloc {name} seed {seed}", flush=True)
        for prec in ("mixed", "fp32"):
            ref = api.pairwise_stats(E, prec)
            got = api.pairwise_stats_noalloc(E, prec)
            for a, b in zip(ref, got):
                assert torch.equal(a, b), (name, prec)


def test_noalloc_preallocated_outputs_and_size_limit(api):
    from paper_2409_05500_amd._lib import VarLiNGAMError, VL_ERR_WORKSPACE, lib
    dev = torch.device("cuda:0")
    E = torch.from_numpy(synth.make_custom(23, 777, 1, "laplace", 4).X32[1:]).to(dev)
    m = E.shape[1]
    out = (torch.empty(m, dtype=torch.float64, device=dev),
           *(torch.empty((m, m), dtype=torch.float64, device=dev) for _ in range(3)))
    got = api.pairwise_stats_noalloc(E, "mixed", out=out)
    assert all(g is o for g, o in zip(got, out))
    ref = api.pairwise_stats(E, "mixed")
    assert all(torch.equal(a, b) for a, b in zip(ref, got))
    # a size whose workspace exceeds the static scratch is refused before any launch
    big_n = 1 << 19
    assert lib.pairwise_stats_workspace_bytes(big_n, 64, 1) > lib.pairwise_stats_noalloc_max_bytes()
    with pytest.raises(VarLiNGAMError) as ei:
        api.pairwise_stats_noalloc(torch.empty((big_n, 64), dtype=torch.float32, device=dev))
    assert ei.value.code == VL_ERR_WORKSPACE


def test_noalloc_host_checks_without_launch():
    """Host-side refusals of the workspace-free entry point (no device work is enqueued)."""
    from paper_2409_05500_amd import _lib as L
    FAKE = 0x10000
    na = L.lib.pairwise_stats_noalloc
    assert L.lib.pairwise_stats_noalloc_max_bytes() == 64 << 20
    assert na(None, 100, 4, 4, 1, FAKE, FAKE, FAKE, None, FAKE, None) == L.VL_ERR_INVALID_ARG
    assert na(FAKE, 100, 1, 1, 1, FAKE, FAKE, FAKE, None, FAKE, None) == L.VL_ERR_SHAPE
    assert na(FAKE, 100, 4, 3, 1, FAKE, FAKE, FAKE, None, FAKE, None) == L.VL_ERR_INVALID_ARG
    assert na(FAKE, 100, 4, 4, 7, FAKE, FAKE, FAKE, None, FAKE, None) == L.VL_ERR_INVALID_ARG
    assert na(FAKE, 1 << 19, 64, 64, 1, FAKE, FAKE, FAKE, None, FAKE, None) == \
        L.VL_ERR_WORKSPACE
