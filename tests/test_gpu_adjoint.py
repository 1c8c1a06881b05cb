"""GPU parity of the pathwise gradient of log Z_hat (mixture target, MALA,
decisions held fixed) against the oracle's forward-mode derivative.  Both run
the same chain under common random numbers; the GPU reverse pass recomputes
16-step segments from checkpoints."""
import numpy as np
import pytest
import torch

import oracle as orc
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _case(oa, d, K, N, T, seed, ref_s2=9.0):
    rng = np.random.default_rng(d * 100 + K + N)
    p = wl.random_gmm(rng, d, K)
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)), [1.0]])
    eps = 0.6 / np.sqrt(1 + 4 * beta[1:])
    gp = oa.Problem.gmm(p["means"], p["log_scales"], ref_s2)
    lz_g, g_g = oa.logZ_backward(gp, N, beta, eps, seed, round_k=2)
    op = orc.Problem(family=orc.FAM_GMM, d=d, means=p["means"], log_scales=p["log_scales"],
                     ref_sigma2=ref_s2)
    lz_o, g_o = orc.logZ_grad(op, orc.Opts(move=orc.MOVE_MALA, state_f32=1), N, beta, eps, seed,
                              round_k=2)
    return lz_g, g_g, lz_o, g_o, p, beta, eps


@pytest.mark.parametrize("d,K,N,T", [(20, 4, 300, 40), (5, 2, 129, 33), (30, 3, 70, 17),
                                     (3, 1, 1, 16)])
def test_gradient_matches_oracle(oa, d, K, N, T):
    lz_g, g_g, lz_o, g_o, *_ = _case(oa, d, K, N, T, seed=d + T)
    assert abs(lz_g - lz_o) < 1e-9
    np.testing.assert_allclose(g_g, g_o, rtol=1e-8, atol=1e-8 * np.abs(g_o).max())


def test_autograd_function(oa):
    rng = np.random.default_rng(3)
    p = wl.random_gmm(rng, 6, 2)
    m = torch.tensor(p["means"], device="cuda", requires_grad=True)
    s = torch.tensor(p["log_scales"], device="cuda", requires_grad=True)
    beta = np.linspace(0, 1, 21)
    lz = oa.LogZ.apply(m, s, 4.0, 200, beta, 0.3, 5)
    (2.0 * lz).backward()
    gp = oa.Problem.gmm(p["means"], p["log_scales"], 4.0)
    lz2, g = oa.logZ_backward(gp, 200, beta, 0.3, 5)
    assert abs(float(lz.detach()) - lz2) == 0.0
    np.testing.assert_allclose(m.grad.cpu().numpy().ravel(), 2 * g[:12], rtol=1e-6)
    np.testing.assert_allclose(s.grad.cpu().numpy(), 2 * g[12:], rtol=1e-6)


def test_full_size_gradient(oa):
    """The differentiation workload at full size: K = 4 means in d = 20 drawn
    from N(0, 4 I), log-scales 0, eta = N(0, 9 I), N = 8192, T = 256 MALA steps
    with checkpoints every 16; the whole gradient against the oracle."""
    w = wl.gmm4_d20()
    T = 256
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = w.eps0 / np.sqrt(1 + 8 * beta[1:])
    gp = oa.Problem.gmm(w.params["means"], w.params["log_scales"], w.ref_sigma2)
    lz_g, g_g = oa.logZ_backward(gp, w.N, beta, eps, 17)
    op = orc.Problem(family=orc.FAM_GMM, d=w.d, means=w.params["means"],
                     log_scales=w.params["log_scales"], ref_sigma2=w.ref_sigma2)
    lz_o, g_o = orc.logZ_grad(op, orc.Opts(move=orc.MOVE_MALA, state_f32=1), w.N, beta, eps, 17)
    assert abs(lz_g - lz_o) < 1e-8
    np.testing.assert_allclose(g_g, g_o, rtol=1e-7, atol=1e-7 * np.abs(g_o).max())
