"""GPU parity of the closed-form-target sweeps (Gaussian, mixture; RWMH, MALA,
HMC; AIS and adaptive resampling) against the CPU oracle under common random
numbers.  Both sides draw the same Philox words, compute in binary64 from the
same binary32 states, so trajectories agree bit for bit except where an MH
decision sits within rounding of its threshold (excused, see parity_util)."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import ORC_MOVE, first_flips, gpu_problem, oracle_problem, unpack_bits
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu

FLIP_TOL = 1e-9  # |log alpha - log u| below which fp64 rounding may flip a decision


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _compare_round(g, o, T, N, rtol_lw=1e-12, exact=True):
    acc_g = unpack_bits(g["accept_bits"].cpu().numpy(), T)
    excused, bad = first_flips(acc_g, o["accept"], o["margin"], FLIP_TOL)
    assert not bad, f"unexcused MH disagreements (particle, step, margin): {bad[:5]}"
    keep = np.ones(N, dtype=bool)
    for n, _, _ in excused:
        keep[n] = False
    xg = g["x"].cpu().numpy().astype(np.float64)
    lwg = g["lw"].cpu().numpy()
    if exact:
        np.testing.assert_array_equal(xg[keep], o["x"][keep])
    else:
        np.testing.assert_allclose(xg[keep], o["x"][keep], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(lwg[keep], o["lw"][keep], rtol=rtol_lw, atol=rtol_lw)
    if not excused:
        np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(g["accept"], o["acc"], rtol=0, atol=1e-15)
        assert abs(g["logZ"] - o["logZ"]) < 1e-10
    return len(excused)


CASES = [
    # family, d, move, N, T, K
    ("gauss", 10, "rwmh", 200, 20, 0),     # ragged tile (200 = 3*64 + 8), ragged chunk
    ("gauss", 10, "mala", 130, 17, 0),
    ("gauss", 3, "hmc", 64, 9, 0),
    ("gauss", 33, "rwmh", 70, 12, 0),      # 4 lanes per particle
    ("gmm", 20, "mala", 257, 16, 4),
    ("gmm", 5, "hmc", 100, 11, 3),
    ("gmm", 100, "hmc", 40, 8, 8),         # 16 lanes of 8 coordinates per particle
    ("gmm", 150, "rwmh", 33, 6, 2),        # 16 lanes of 16 coordinates
    # mixture exponentials owned by lane k mod LPP: K below, equal to and above LPP
    ("gmm", 30, "mala", 90, 10, 5),        # 2 lanes, 3 components per lane
    ("gmm", 60, "hmc", 50, 7, 16),         # 4 lanes, the largest K
    ("gmm", 128, "mala", 20, 6, 1),        # 16 lanes, one component
    ("gmm", 256, "mala", 24, 5, 3),        # the largest d
    ("gauss", 1, "rwmh", 1, 5, 0),         # a single particle in one dimension
]


@pytest.mark.parametrize("family,d,move,N,T,K", CASES)
def test_ais_round_matches_oracle(oa, family, d, move, N, T, K):
    rng = np.random.default_rng(d * 1000 + N + T)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    ref_mean = rng.normal(size=d).astype(np.float32) * 0.3
    ref_s2 = 1.7
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)), [1.0]])
    eps = rng.uniform(0.2, 0.6, size=T)
    seed = 0xC0FFEE + d
    gp = gpu_problem(oa, family, params, ref_s2, ref_mean)
    g = oa.asmc(gp, N, beta, eps, seed, round_k=3, problem_id=1, move=move, leapfrog=4,
                accept_bits=True)
    op = oracle_problem(family, d, params, ref_s2, ref_mean)
    o = orc.asmc(op, orc.Opts(move=ORC_MOVE[move], leapfrog=4, state_f32=1), N, beta, eps, seed,
                 round_k=3, problem_id=1, traces=True)
    assert o["status"] == 0
    _compare_round(g, o, T, N)


# Several tiles folded into one moment slot (the accumulation branch that the
# default min(#tiles, 2048) slots reach only above 2048 tiles): a slot cap on
# small runs, and one run above 2048 tiles with the default cap.
SLOT_CASES = [
    # family, d, move, N, T, K, slots
    ("gauss", 10, "rwmh", 1000, 9, 0, 3),    # 16 tiles of 64 particles into 3 slots
    ("gauss", 100, "mala", 37, 6, 0, 2),     # 16 lanes per particle, 10 tiles (ragged)
    ("gmm", 20, "mala", 300, 7, 4, 2),       # 4 lanes x 8 coordinates, 19 tiles
    ("gmm", 60, "hmc", 90, 5, 16, 1),        # every tile into one slot
]


@pytest.mark.parametrize("family,d,move,N,T,K,slots", SLOT_CASES)
def test_ais_several_tiles_per_slot(oa, family, d, move, N, T, K, slots):
    rng = np.random.default_rng(d * 77 + N)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)), [1.0]])
    eps = rng.uniform(0.1, 0.4, size=T)
    gp = gpu_problem(oa, family, params, 1.3)
    g = oa.asmc(gp, N, beta, eps, 99, round_k=2, move=move, leapfrog=3, accept_bits=True,
                slots=slots)
    op = oracle_problem(family, d, params, 1.3)
    o = orc.asmc(op, orc.Opts(move=ORC_MOVE[move], leapfrog=3, state_f32=1), N, beta, eps, 99,
                 round_k=2, traces=True)
    assert o["status"] == 0
    _compare_round(g, o, T, N)


def test_ais_above_2048_tiles_matches_oracle(oa):
    """Gaussian d = 100 on 16 lanes per particle (4 particles per tile) with
    N = 8203: 2051 tiles, so the default 2048 slots fold three of them twice.
    At this size the comparison uses the stated tolerances (trajectories
    within 1e-5 relative, decisions excused within 1e-6 of the threshold)
    rather than bitwise equality."""
    rng = np.random.default_rng(8203)
    params = wl.random_gauss(rng, 100)
    T, N = 3, 8203
    beta = np.array([0.0, 0.2, 0.6, 1.0])
    eps = np.full(T, 0.05)
    gp = gpu_problem(oa, "gauss", params, 1.0)
    g = oa.asmc(gp, N, beta, eps, 5, move="rwmh", accept_bits=True)
    op = oracle_problem("gauss", 100, params, 1.0)
    o = orc.asmc(op, orc.Opts(move=orc.MOVE_RWMH, state_f32=1), N, beta, eps, 5, traces=True)
    acc_g = unpack_bits(g["accept_bits"].cpu().numpy(), T)
    excused, bad = first_flips(acc_g, o["accept"], o["margin"], 1e-6)
    assert not bad, bad[:5]
    keep = np.ones(N, dtype=bool)
    keep[[n for n, _, _ in excused]] = False
    xg = g["x"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(xg[keep], o["x"][keep], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(g["lw"].cpu().numpy()[keep], o["lw"][keep], rtol=1e-9, atol=1e-9)
    if not excused:
        np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=1e-10, atol=1e-10)
        assert abs(g["logZ"] - o["logZ"]) < 1e-6


@pytest.mark.parametrize("trigger", ["ess", "cess"])
@pytest.mark.parametrize("family,d,move,N,T,K", [("gauss", 4, "hmc", 300, 12, 0),
                                                 ("gmm", 20, "mala", 2100, 10, 4),
                                                 # 16 lanes x 8 coordinates, K = 5: a
                                                 # padded block of mixture components
                                                 ("gmm", 100, "hmc", 300, 8, 5),
                                                 # > 64 x 256 tiles: several tile records
                                                 # per thread in the first merge level
                                                 ("gauss", 4, "rwmh", 2200000, 3, 0)])
def test_resampling_round_matches_oracle(oa, family, d, move, N, T, K, trigger):
    """Adaptive resampling: same events, same ancestors (integer CDF), same
    final population and log Z_hat."""
    rng = np.random.default_rng(N + d)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    if family == "gauss":  # a concentrated target so that the ESS trigger fires
        params["mu"] = params["mu"] * 3
        params["sigma2"] = 0.05
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = np.full(T, 0.3)
    gp = gpu_problem(oa, family, params, 2.0)
    g = oa.asmc(gp, N, beta, eps, 77, move=move, leapfrog=3, resample_=True, trigger=trigger,
                nu=0.5, accept_bits=True)
    op = oracle_problem(family, d, params, 2.0)
    o = orc.asmc(op, orc.Opts(move=ORC_MOVE[move], leapfrog=3, resample=1,
                              trigger=0 if trigger == "ess" else 1, nu=0.5, state_f32=1), N, beta,
                 eps, 77, traces=True)
    assert o["n_resample"] >= 1 or trigger == "cess"
    np.testing.assert_array_equal(g["resampled"], o["resampled"])
    assert g["n_resample"] == o["n_resample"]
    np.testing.assert_allclose(g["ess"], o["ess"], rtol=1e-10)
    _compare_round(g, o, T, N)


def test_resampler_bit_exact(oa):
    """Integer-CDF systematic resampling: device ancestors equal the oracle's
    on the same log-weights, including ragged block counts and -inf weights."""
    rng = np.random.default_rng(4)
    for N in (1, 7, 2048, 2049, 100003):
        for trial in range(3):
            lw = wl.synthetic_logw(rng, N, scale=4.0)
            if N > 10:
                lw[rng.random(N) < 0.05] = -np.inf
            u = int(rng.integers(0, 2 ** 32))
            a_g = oa.resample(torch.tensor(lw, device="cuda"), u).cpu().numpy()
            a_o = orc.systematic(lw, u)
            np.testing.assert_array_equal(a_g, a_o)


def test_philox_device_matches_oracle(oa):
    rng = np.random.default_rng(9)
    ctr = rng.integers(0, 2 ** 32, size=(500, 4), dtype=np.uint64)
    seed = int(rng.integers(0, 2 ** 63))
    out = oa.philox(seed, torch.tensor(ctr.astype(np.uint32).view(np.int32), device="cuda"))
    out = out.cpu().numpy().view(np.uint32)
    for i in range(ctr.shape[0]):
        ref = orc.philox4x32_10(ctr[i], [seed & 0xFFFFFFFF, seed >> 32])
        np.testing.assert_array_equal(out[i], ref)


def test_round_loop_matches_oracle(oa):
    """Alg. 2 for the d=10 Gaussian target with RWMH at its full size
    (N 128 -> 1024 over 4 rounds, T = 64): every round's schedule, Lambda_hat,
    moments and log Z_hat."""
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    g = oa.run(gp, 128, 4, seed=2024, move="rwmh", budget="double_n", T1=64, eps0=w.eps0)
    op = oracle_problem("gauss", 10, w.params, 1.0)
    o = orc.run(op, orc.Opts(move=orc.MOVE_RWMH, state_f32=1),
                orc.RunOpts(budget=1, T1=64, eps0=w.eps0), 128, 4, seed=2024)
    assert g["rounds_done"] == 4 and o["status"] == 0
    np.testing.assert_array_equal(g["N"], o["N"])
    np.testing.assert_allclose(g["beta"], o["beta"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["Lambda"], o["Lambda"], rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(g["logZ"], o["logZ"], rtol=0, atol=1e-6)


def test_round_loop_step_size_adaptation(oa):
    """Doubling T with adapted HMC step sizes on a mixture: schedules, step
    sizes and log Z_hat per round agree with the oracle."""
    rng = np.random.default_rng(12)
    params = wl.random_gmm(rng, 6, 3)
    gp = gpu_problem(oa, "gmm", params, 4.0)
    kw = dict(budget="double_t", T1=2, T_max=24, eps0=0.8, eps_adapt=True, eps_kappa=3.0,
              accept_target=0.65)
    g = oa.run(gp, 500, 5, seed=5, move="hmc", leapfrog=3, **kw)
    op = oracle_problem("gmm", 6, params, 4.0)
    o = orc.run(op, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, state_f32=1),
                orc.RunOpts(budget=2, T1=2, Tmax=24, eps_adapt=1, eps0=0.8, eps_kappa=3.0,
                            accept_target=0.65), 500, 5, seed=5)
    np.testing.assert_array_equal(g["T"], o["T"])
    np.testing.assert_allclose(g["eps"], o["eps"], rtol=1e-9, atol=0)
    np.testing.assert_allclose(g["beta"], o["beta"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(g["logZ"], o["logZ"], rtol=0, atol=1e-6)


def test_repeat_is_bitwise_identical(oa):
    w = wl.gaussian_d10(N=3000, T=40)
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    beta = np.linspace(0, 1, 41)
    a = oa.asmc(gp, 3000, beta, w.eps0, 1)
    b = oa.asmc(gp, 3000, beta, w.eps0, 1)
    assert torch.equal(a["x"], b["x"]) and torch.equal(a["lw"], b["lw"])
    np.testing.assert_array_equal(a["log_g"], b["log_g"])
    assert a["logZ"] == b["logZ"]


def test_invalid_arguments_raise(oa):
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    with pytest.raises(oa.OasmcError):
        oa.asmc(gp, 10, np.array([0.0, 0.6, 0.5, 1.0]), 0.1, 1)
    with pytest.raises(oa.OasmcError):
        oa.asmc(gp, 0, np.linspace(0, 1, 5), 0.1, 1)
    with pytest.raises(oa.OasmcError):
        oa.asmc(gp, 10, np.linspace(0, 1, 5), -1.0, 1)
