"""Edge cases and error paths of the C ABI on the GPU: sizes beyond what a
kernel is built for, degenerate schedules and parameters, and the smallest
inputs (one particle, one step, d = 1) against the oracle.  Every rejected
call must raise before any device work and leave the handle usable."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import compare_round, gpu_problem, oracle_problem
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def test_unsupported_sizes_raise(oa):
    rng = np.random.default_rng(0)
    big = gpu_problem(oa, "gauss", wl.random_gauss(rng, 257), 1.0)       # d > 256
    with pytest.raises(oa.OasmcError):
        oa.asmc(big, 8, np.linspace(0, 1, 3), 0.1, 1)
    X, y, _ = wl.logreg_data(50, 257, 1)
    with pytest.raises(oa.OasmcError):                                    # logistic d > 256
        oa.asmc(oa.Problem.logreg(X, y), 8, np.linspace(0, 1, 3), 0.1, 1, move="mala")
    mix = gpu_problem(oa, "gmm", wl.random_gmm(rng, 4, 17), 1.0)         # K > 16
    with pytest.raises(oa.OasmcError):
        oa.asmc(mix, 8, np.linspace(0, 1, 3), 0.1, 1)
    X, y, _ = wl.logreg_data(50, 10, 1)
    with pytest.raises(oa.OasmcError):                                    # logistic + RWMH
        oa.asmc(oa.Problem.logreg(X, y), 8, np.linspace(0, 1, 3), 0.1, 1, move="rwmh")


def test_bad_schedules_and_parameters_raise(oa):
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    with pytest.raises(oa.OasmcError):                                    # beta_0 != 0
        oa.asmc(gp, 8, np.array([0.1, 0.5, 1.0]), 0.1, 1)
    with pytest.raises(oa.OasmcError):                                    # beta_T != 1
        oa.asmc(gp, 8, np.array([0.0, 0.5, 0.9]), 0.1, 1)
    with pytest.raises(oa.OasmcError):                                    # no step
        oa.asmc(gp, 8, np.array([0.0]), 0.1, 1)
    with pytest.raises(oa.OasmcError):                                    # NaN step size
        oa.asmc(gp, 8, np.linspace(0, 1, 4), np.nan, 1)
    with pytest.raises(oa.OasmcError):                                    # rho outside (0, 1)
        oa.zja(gp, 64, 1.5, 10, 0.1, 1, move="rwmh")
    with pytest.raises(oa.OasmcError):                                    # K < 1 copies
        oa.pt(gp, 0, np.linspace(0, 1, 4), 0.1, 8, 1)
    x = torch.zeros((0, 10), device="cuda")
    with pytest.raises(oa.OasmcError):                                    # no states
        oa.target_eval(gp, x)
    # the handle still works after the rejected calls
    r = oa.asmc(gp, 8, np.linspace(0, 1, 4), 0.1, 1)
    assert np.isfinite(r["logZ"])


def test_one_particle_one_step_d1(oa):
    """The smallest pass: N = 1, T = 1, d = 1, against the oracle bit for bit."""
    params = dict(mu=np.array([0.7], dtype=np.float32), sigma2=0.5)
    gp = gpu_problem(oa, "gauss", params, 1.0)
    beta = np.array([0.0, 1.0])
    g = oa.asmc(gp, 1, beta, 0.4, 3, move="mala", accept_bits=True)
    op = oracle_problem("gauss", 1, params, 1.0)
    o = orc.asmc(op, orc.Opts(move=orc.MOVE_MALA, state_f32=1), 1, beta, 0.4, 3, traces=True)
    compare_round(g, o, 1, 1)


@pytest.mark.parametrize("N", [1, 31, 32, 33, 63, 64, 65])
@pytest.mark.parametrize("d", [20, 70])
def test_tile_boundaries_logreg(oa, N, d):
    """Logistic regression with N at and around one tile: 64 particles of the
    64-column layout (d = 20), 32 of the panel layout (d = 70); trajectories,
    weights and log Z_hat against the oracle within the measured contraction
    error (the same check as the logistic-regression parity tests)."""
    from test_gpu_logreg import _check, _eps, _round
    n, T = 300, 3
    X, y, beta, g, o = _round(oa, n, d, N, T, seed=N + d)
    _check(oa, X, y, g, o, T, np.arange(N), _eps(beta, n, d))
