"""The closed-form targets' ell and grad ell as the sweeps evaluate them,
in every built lane layout (1 to 16 lanes per particle, 4 to 24 coordinates
per lane), against the oracle's binary64 evaluation at the same binary32
states.  The mixture cases cover padded component blocks (K not a multiple
of 4), the lane-owned exponentials and the gathered weights of multi-lane
particles, and K up to 16; states are drawn near the components, between
them and far out in the tails (where the log-sum-exp's maximum dominates).

Both sides compute in binary64 from the same inputs; they differ only in
the order of the sums (lane groups vs a sequential loop) and in the last bit
of exp and log, so the tolerance is a few hundred ulps of the terms' scale."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import gpu_problem, oracle_problem
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu

SHAPES = [(1, 4), (1, 8), (1, 12), (1, 16), (1, 20), (1, 24), (2, 16), (4, 8), (8, 4), (4, 16),
          (8, 8), (8, 16), (16, 8), (16, 16)]


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _states(rng, params, family, d, N):
    """Thirds: near a component / the mean, between components, far out."""
    centre = params["means"] if family == "gmm" else params["mu"][None, :]
    k = rng.integers(0, centre.shape[0], N)
    x = centre[k] + 0.3 * rng.standard_normal((N, d))
    m = N // 3
    if family == "gmm" and centre.shape[0] > 1:
        k2 = rng.integers(0, centre.shape[0], m)
        x[m:2 * m] = 0.5 * (centre[k[m:2 * m]] + centre[k2])
    x[2 * m:] = 6.0 * rng.standard_normal((N - 2 * m, d))
    return x.astype(np.float32)


def _check(oa, family, d, params, shapes, N=150, seed=0, ref_mean=None, ref_sigma2=2.0):
    rng = np.random.default_rng(seed)
    x = _states(rng, params, family, d, N)
    P = oracle_problem(family, d, params, ref_sigma2, ref_mean=ref_mean)
    ref = [orc.ell(P, x[i]) for i in range(N)]
    e_ref = np.array([v for v, _ in ref])
    g_ref = np.stack([g for _, g in ref])
    prob = gpu_problem(oa, family, params, ref_sigma2, ref_mean=ref_mean)
    xt = torch.tensor(x, device="cuda")
    for lpp, dpl in shapes:
        if lpp * dpl < d:
            continue
        ell, grad = oa.target_eval(prob, xt, lpp, dpl)
        ell, grad = ell.cpu().numpy(), grad.cpu().numpy()
        # scale of the terms: the reference's quadratic and the largest exponent
        scale = 1.0 + np.abs(e_ref) + np.sum((x.astype(np.float64)) ** 2, 1) / ref_sigma2
        err = np.abs(ell - e_ref) / scale
        assert err.max() < 1e-13, (lpp, dpl, int(err.argmax()), err.max())
        gs = 1.0 + np.abs(g_ref).max(1, keepdims=True) + np.abs(x).max(1, keepdims=True) / ref_sigma2
        gerr = np.abs(grad - g_ref) / gs
        assert gerr.max() < 1e-12, (lpp, dpl, np.unravel_index(gerr.argmax(), gerr.shape),
                                    gerr.max())


@pytest.mark.parametrize("d,K", [(6, 1), (6, 3), (20, 4), (20, 5), (40, 6), (60, 16), (100, 8),
                                 (100, 13), (200, 16), (256, 7)])
def test_mixture_every_shape(oa, d, K):
    rng = np.random.default_rng(100 * d + K)
    params = wl.random_gmm(rng, d, K)
    _check(oa, "gmm", d, params, SHAPES, seed=d + K)


@pytest.mark.parametrize("d", [3, 10, 33, 128, 256])
def test_gaussian_every_shape(oa, d):
    rng = np.random.default_rng(d)
    params = wl.random_gauss(rng, d)
    ref_mean = (0.5 * rng.standard_normal(d)).astype(np.float32)
    _check(oa, "gauss", d, params, SHAPES, seed=d, ref_mean=ref_mean, ref_sigma2=1.5)


def test_default_shape_and_ragged_tiles(oa):
    """lpp = dpl = 0 takes the sweep's default shape; N not a multiple of the
    particles per wave (the tail lane groups evaluate zeros and write nothing)."""
    rng = np.random.default_rng(5)
    params = wl.random_gmm(rng, 60, 16)
    _check(oa, "gmm", 60, params, [(0, 0)], N=67, seed=3)


def test_unid(oa):
    P = orc.Problem(family=orc.FAM_UNID, d=2, binom_n=1e11, binom_k=1e10, box=10.0)
    prob = oa.Problem.unid(1e11, 1e10, 10.0)
    rng = np.random.default_rng(2)
    x0 = rng.uniform(0.02, 10, 200)
    x = np.stack([x0, (0.1 + 3e-6 * rng.standard_normal(200)) / x0], 1).astype(np.float32)
    x[:20, 0] = 11.0  # outside the reference's support
    ell, grad = oa.target_eval(prob, torch.tensor(x, device="cuda"))
    ell = ell.cpu().numpy()
    ref = np.array([orc.ell(P, x[i])[0] for i in range(len(x))])
    np.testing.assert_array_equal(np.isinf(ell), np.isinf(ref))
    fin = np.isfinite(ref)
    np.testing.assert_allclose(ell[fin], ref[fin], rtol=1e-9, atol=1e-9)
    assert np.all(grad.cpu().numpy() == 0.0)


def test_rejects_bad_shapes(oa):
    rng = np.random.default_rng(1)
    params = wl.random_gmm(rng, 40, 4)
    prob = gpu_problem(oa, "gmm", params, 1.0)
    x = torch.zeros((4, 40), device="cuda")
    with pytest.raises(oa.OasmcError):
        oa.target_eval(prob, x, 1, 24)   # 24 < d
    with pytest.raises(oa.OasmcError):
        oa.target_eval(prob, x, 3, 16)   # not a built shape
