"""GPU parity of the pieces of the paper's GPU comparison against the oracle:
the Unid target, the alternating three-scale RWMH kernel (on every family and
with resampling), and the ZJA online CESS-adaptive AIS (its schedule, moments
and log Z_hat)."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import ORC_MOVE, compare_round, first_flips, gpu_problem, oracle_problem, \
    unpack_bits
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu
MOVES = dict(ORC_MOVE, rwmh3=orc.MOVE_RWMH3)


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _unid_pair(oa, n, k):
    return (oa.Problem.unid(n, k), orc.Problem(family=orc.FAM_UNID, d=2, binom_n=n, binom_k=k,
                                                box=10.0))


@pytest.mark.parametrize("n,k,move,N,T", [(1e11, 1e10, "rwmh3", 300, 24), (1e4, 5e3, "rwmh", 1000, 9),
                                          (1e4, 5e3, "rwmh3", 65, 16)])
def test_unid_round_matches_oracle(oa, n, k, move, N, T):
    gp, op = _unid_pair(oa, n, k)
    beta = np.linspace(0, 1, T + 1) ** 4
    eps = np.full(T, 0.5)
    g = oa.asmc(gp, N, beta, eps, 11, move=move, accept_bits=True)
    o = orc.asmc(op, orc.Opts(move=MOVES[move], state_f32=1), N, beta, eps, 11, traces=True)
    assert o["status"] == 0
    compare_round(g, o, T, N, rtol_lw=1e-9)


@pytest.mark.parametrize("family,d,N,T,K", [("gauss", 10, 200, 12, 0), ("gmm", 40, 90, 8, 4),
                                            ("gmm", 100, 50, 6, 8)])
def test_three_scale_kernel_matches_oracle(oa, family, d, N, T, K):
    rng = np.random.default_rng(d + N)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = np.full(T, 0.05)
    gp = gpu_problem(oa, family, params, 1.5)
    g = oa.asmc(gp, N, beta, eps, 3, move="rwmh3", accept_bits=True)
    op = oracle_problem(family, d, params, 1.5)
    o = orc.asmc(op, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), N, beta, eps, 3, traces=True)
    compare_round(g, o, T, N)


@pytest.mark.parametrize("trigger,flags", [("ess", None), ("fixed", [0, 1, 0, 1, 1, 0, 0, 0])])
def test_three_scale_kernel_with_resampling(oa, trigger, flags):
    T, N = 8, 400
    rng = np.random.default_rng(8)
    params = wl.random_gauss(rng, 6)
    params["mu"] = params["mu"] * 3
    params["sigma2"] = 0.05
    beta = np.linspace(0, 1, T + 1) ** 2
    gp = gpu_problem(oa, "gauss", params, 2.0)
    kw = {} if flags is None else dict(resample_at=np.array(flags, dtype=np.int32))
    g = oa.asmc(gp, N, beta, 0.1, 6, move="rwmh3", resample_=True, trigger=trigger, nu=0.5,
                accept_bits=True, **kw)
    op = oracle_problem("gauss", 6, params, 2.0)
    okw = {} if flags is None else dict(resample_at=np.array(flags, dtype=np.uint8))
    o = orc.asmc(op, orc.Opts(move=orc.MOVE_RWMH3, resample=1, trigger=0 if flags is None else 3,
                              nu=0.5, state_f32=1, **okw), N, beta, 0.1, 6, traces=True)
    assert o["n_resample"] >= 1 and g["n_resample"] == o["n_resample"]
    np.testing.assert_array_equal(g["resampled"], o["resampled"])
    compare_round(g, o, T, N)


def _zja_compare(g, o, N):
    """Same number of steps, schedule and moments to the bisection's rounding
    (the last halvings compare log CESS with rho at the level of binary64
    roundoff of two differently ordered sums), and final states of the
    particles whose decisions followed the oracle's."""
    assert g["T"] == o["T"]
    np.testing.assert_allclose(g["beta"], o["beta"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=1e-7, atol=1e-7)
    assert abs(g["logZ"] - o["logZ"]) < 1e-6
    xg = g["x"].cpu().numpy().astype(np.float64)
    same = np.all(xg == o["x"], axis=1)
    assert same.mean() > 0.99, same.mean()


@pytest.mark.parametrize("N,rho", [(2048, 0.95), (777, 0.9)])
def test_zja_gaussian_matches_oracle(oa, N, rho):
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    g = oa.zja(gp, N, rho, 300, 0.2, 5, move="rwmh3")
    op = oracle_problem("gauss", 10, w.params, 1.0)
    o = orc.zja(op, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), N, rho, 300, 0.2, 5)
    assert o["status"] == 0 and 5 < o["T"] < 300
    _zja_compare(g, o, N)


def test_zja_unid_matches_oracle(oa):
    gp, op = _unid_pair(oa, 1e11, 1e10)
    g = oa.zja(gp, 4096, 0.8, 2000, 1.0, 9, move="rwmh3")
    o = orc.zja(op, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), 4096, 0.8, 2000, 1.0, 9)
    assert o["status"] == 0
    _zja_compare(g, o, 4096)


def test_zja_stops_at_tmax_on_gpu(oa):
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    g = oa.zja(gp, 256, 0.999, 40, 0.2, 2, move="rwmh")
    assert g["T"] == 40 and g["beta"][40] == 1.0
