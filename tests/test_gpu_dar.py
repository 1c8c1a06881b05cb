"""GPU parity of the resampling variants with times fixed in advance against
the oracle: SIR (resampling after every step, the per-step path), resampling
at given steps (the segment path: loop-swapped passes between events), and
the round loop with DAR times predicted from the previous round (Sec.
"Effective resample size for deterministic adaptive resampling")."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import ORC_MOVE, compare_round, gpu_problem, oracle_problem
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _params(rng, family, d, K):
    if family == "gauss":
        p = wl.random_gauss(rng, d)
        p["mu"] = p["mu"] * 3  # a concentrated target: weights degenerate quickly
        p["sigma2"] = 0.05
        return p
    return wl.random_gmm(rng, d, K)


def _pair(oa, family, d, move, N, T, K, seed, gpu_kw, orc_kw, slots=0):
    rng = np.random.default_rng(N + 13 * d + T)
    params = _params(rng, family, d, K)
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = np.full(T, 0.3)
    gp = gpu_problem(oa, family, params, 2.0)
    g = oa.asmc(gp, N, beta, eps, seed, move=move, leapfrog=3, resample_=True, nu=0.5,
                accept_bits=True, slots=slots, **gpu_kw)
    op = oracle_problem(family, d, params, 2.0)
    o = orc.asmc(op, orc.Opts(move=ORC_MOVE[move], leapfrog=3, resample=1, nu=0.5, state_f32=1,
                              **orc_kw), N, beta, eps, seed, traces=True)
    assert o["status"] == 0
    return g, o


CASES = [
    # family, d, move, N, T, K
    ("gauss", 4, "rwmh", 300, 9, 0),      # one lane per particle, ragged last tile
    ("gauss", 10, "hmc", 130, 7, 0),
    ("gmm", 20, "mala", 500, 8, 4),       # 4 lanes x 8 coordinates
    ("gmm", 100, "hmc", 70, 6, 5),        # 16 lanes x 8 coordinates, padded block of components
]


@pytest.mark.parametrize("family,d,move,N,T,K", CASES)
def test_sir_matches_oracle(oa, family, d, move, N, T, K):
    """Resampling after every step: the same T - 1 events, ancestors, final
    population, moments, ESS and log Z_hat as the oracle."""
    g, o = _pair(oa, family, d, move, N, T, K, 31, dict(trigger="sir"), dict(trigger=2))
    assert o["n_resample"] == T - 1 and g["n_resample"] == T - 1
    np.testing.assert_array_equal(g["resampled"], o["resampled"])
    np.testing.assert_allclose(g["ess"], o["ess"], rtol=1e-10)
    compare_round(g, o, T, N)


FLAGS = {
    "first_last": lambda T: np.array([1] + [0] * (T - 3) + [1, 0]),
    "consecutive": lambda T: np.array([0, 1, 1, 1] + [0] * (T - 4)),
    "sparse": lambda T: np.array([(t % 3 == 2) for t in range(T - 1)] + [0]),
    "none": lambda T: np.zeros(T, dtype=int),
}


@pytest.mark.parametrize("flags", sorted(FLAGS))
@pytest.mark.parametrize("family,d,move,N,T,K", CASES)
def test_given_times_match_oracle(oa, family, d, move, N, T, K, flags):
    """Resampling at given steps on the segment path (each segment one
    loop-swapped pass from the state the previous one left): same events,
    ancestors, final population, moments and log Z_hat as the oracle."""
    f = FLAGS[flags](T).astype(np.int32)
    g, o = _pair(oa, family, d, move, N, T, K, 57,
                 dict(trigger="fixed", resample_at=f), dict(trigger=3, resample_at=f))
    assert o["n_resample"] == int(f[:-1].sum()) == g["n_resample"]
    np.testing.assert_array_equal(g["resampled"], o["resampled"])
    assert np.all(np.isnan(g["ess"]))  # not streamed between fixed times
    compare_round(g, o, T, N)


def test_given_times_several_tiles_per_slot(oa):
    """The segment path with 3 moment slots for 16 tiles (several tiles folded
    into each slot, and the largest log w merged across them)."""
    T = 8
    f = np.array([0, 1, 0, 0, 1, 1, 0, 0], dtype=np.int32)
    g, o = _pair(oa, "gauss", 6, "rwmh", 1000, T, 0, 5, dict(trigger="fixed", resample_at=f),
                 dict(trigger=3, resample_at=f), slots=3)
    assert g["n_resample"] == o["n_resample"] == 3
    np.testing.assert_array_equal(g["resampled"], o["resampled"])
    compare_round(g, o, T, 1000)


def test_every_step_given_equals_sir_on_gpu(oa):
    """The segment path with every step flagged and the per-step SIR path give
    the same trajectories and ancestors (same arithmetic per particle, in two
    kernels whose binary64 contractions may round differently, so log-weights
    agree to a few ulps; the moments also differ in summation order)."""
    T = 6
    f = np.ones(T, dtype=np.int32)
    rng = np.random.default_rng(3)
    params = wl.random_gmm(rng, 30, 3)
    gp = gpu_problem(oa, "gmm", params, 2.0)
    beta = np.linspace(0, 1, T + 1) ** 2
    kw = dict(move="hmc", leapfrog=3, resample_=True, nu=0.5, accept_bits=True)
    a = oa.asmc(gp, 777, beta, 0.3, 8, trigger="sir", **kw)
    b = oa.asmc(gp, 777, beta, 0.3, 8, trigger="fixed", resample_at=f, **kw)
    assert torch.equal(a["x"], b["x"]) and torch.equal(a["accept_bits"], b["accept_bits"])
    np.testing.assert_allclose(a["lw"].cpu().numpy(), b["lw"].cpu().numpy(), rtol=1e-14, atol=0)
    np.testing.assert_allclose(a["log_g"], b["log_g"], rtol=1e-12, atol=1e-12)
    assert abs(a["logZ"] - b["logZ"]) < 1e-10


def test_round_loop_with_dar_matches_oracle(oa):
    """Alg. 2 with DAR times: the same schedules, step sizes, resampling counts
    and log Z_hat per round as the oracle's round loop."""
    rng = np.random.default_rng(21)
    params = wl.random_gmm(rng, 8, 3)
    gp = gpu_problem(oa, "gmm", params, 4.0)
    kw = dict(budget="double_t", T1=2, T_max=48, eps0=0.8, eps_adapt=True, eps_kappa=3.0,
              accept_target=0.65)
    g = oa.run(gp, 600, 6, seed=4, move="hmc", leapfrog=3, resample_=True, nu=0.5, dar=True, **kw)
    op = oracle_problem("gmm", 8, params, 4.0)
    o = orc.run(op, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, nu=0.5, state_f32=1),
                orc.RunOpts(budget=2, T1=2, Tmax=48, eps_adapt=1, eps0=0.8, eps_kappa=3.0,
                            accept_target=0.65, dar=1), 600, 6, seed=4)
    assert g["rounds_done"] == 6 and o["status"] == 0
    np.testing.assert_array_equal(g["T"], o["T"])
    np.testing.assert_array_equal(g["n_resample"], o["n_resample"])
    assert g["n_resample"][0] == 0 and g["n_resample"][1:].sum() > 0
    np.testing.assert_allclose(g["eps"], o["eps"], rtol=1e-9, atol=0)
    np.testing.assert_allclose(g["beta"], o["beta"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["logZ"], o["logZ"], rtol=0, atol=1e-6)
