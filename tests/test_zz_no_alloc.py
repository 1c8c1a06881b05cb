"""The allocation-free resampling entry point against the handle-based one:
bitwise equal ancestors on two calls in a row (the second with fewer
particles, so stale scratch from the first call must not leak into it), the
size limit rejected before any device work, and a non-finite input marked
with -1 ancestors."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as oa
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return oa


def _weights(rng, n, spread):
    lw = rng.normal(scale=spread, size=n)
    lw[rng.random(n) < 0.05] = -np.inf
    lw[0] = 0.0  # at least one finite weight
    return lw


def test_noalloc_matches_resample_two_calls(oa):
    rng = np.random.default_rng(20240812)
    dev = torch.device("cuda", 0)
    for n, spread, u in ((300_001, 3.0, 0x9E3779B9), (4_097, 1.5, 12345)):
        lw = torch.tensor(_weights(rng, n, spread), dtype=torch.float64, device=dev)
        ref = oa.resample(lw, u)
        anc = torch.full((n,), -7, dtype=torch.int32, device=dev)
        oa.resample_noalloc(lw, u, anc)
        torch.cuda.synchronize()
        a, r = anc.cpu().numpy(), ref.cpu().numpy()
        print(f"noalloc N={n}: {np.count_nonzero(a != r)} mismatches", flush=True)
        np.testing.assert_array_equal(a, r)
        assert a.min() >= 0 and a.max() < n


def test_noalloc_limits(oa):
    dev = torch.device("cuda", 0)
    big = oa.api.NOALLOC_MAX_N + 1
    L = oa.api._load()
    lw = torch.zeros(4, dtype=torch.float64, device=dev)
    anc = torch.zeros(4, dtype=torch.int32, device=dev)
    code = L.oasmc_resample_noalloc(big, ctypes.c_void_p(lw.data_ptr()), 0,
                                    ctypes.c_void_p(anc.data_ptr()), None)
    assert code == oa.api.EINVAL
    assert b"static scratch" in L.oasmc_last_error()
    lw = torch.full((1000,), -np.inf, dtype=torch.float64, device=dev)
    anc = torch.zeros(1000, dtype=torch.int32, device=dev)
    oa.resample_noalloc(lw, 5, anc)
    torch.cuda.synchronize()
    assert (anc.cpu().numpy() == -1).all()
