"""GPU parity of final-iteration rejuvenation (Sec. "Computing expectations")
against the oracle: the same resampled starts, chains, end states and
averages, on populations the oracle produced."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import ORC_MOVE, gpu_problem, oracle_problem
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


CASES = [
    # family, d, move, N, T, K
    ("gauss", 10, "rwmh", 300, 20, 0),    # one lane per particle, ragged last tile
    ("gauss", 7, "mala", 65, 12, 0),
    ("gmm", 20, "hmc", 200, 9, 3),        # 4 lanes x 8 coordinates
    ("gmm", 100, "mala", 40, 6, 5),       # 16 lanes x 8 coordinates, padded component block
    ("gauss", 200, "rwmh", 9, 5, 0),      # 16 lanes x 16 coordinates
]


@pytest.mark.parametrize("family,d,move,N,T,K", CASES)
def test_rejuvenation_matches_oracle(oa, family, d, move, N, T, K):
    rng = np.random.default_rng(d * 31 + N)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    op = oracle_problem(family, d, params, 1.5)
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = rng.uniform(0.2, 0.4, size=T)
    opts = orc.Opts(move=ORC_MOVE[move], leapfrog=3, state_f32=1)
    fin = orc.asmc(op, opts, N, beta, eps, 17, round_k=2)
    assert fin["status"] == 0
    o = orc.rejuvenate(op, opts, fin["lw"], fin["x"], T, eps[-1], 17, round_k=2,
                       want_states=True)
    assert o["status"] == 0
    gp = gpu_problem(oa, family, params, 1.5)
    g = oa.rejuvenate(gp, torch.tensor(fin["lw"], device="cuda"),
                      torch.tensor(fin["x"].astype(np.float32), device="cuda"), T, eps[-1], 17,
                      round_k=2, move=move, leapfrog=3, return_states=True)
    np.testing.assert_array_equal(g["x"].cpu().numpy().astype(np.float64), o["x"])
    np.testing.assert_allclose(g["mean"], o["mean"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["second"], o["second"], rtol=1e-12, atol=1e-13)
    assert abs(g["accept"] - o["accept"]) < 1e-15


def test_round_loop_rejuvenation_matches_oracle(oa):
    """Alg. 2 with rejuvenation after every round: each round's averages equal
    the oracle's rejuvenation of the oracle's own round (same schedule and step
    sizes, taken from the oracle's round loop)."""
    w = wl.gaussian_d10()
    gp = gpu_problem(oa, "gauss", w.params, 1.0)
    g = oa.run(gp, 128, 3, seed=2024, move="rwmh", budget="double_n", T1=64, eps0=w.eps0,
               rejuvenate=True)
    op = oracle_problem("gauss", 10, w.params, 1.0)
    opts = orc.Opts(move=orc.MOVE_RWMH, state_f32=1)
    o = orc.run(op, opts, orc.RunOpts(budget=1, T1=64, eps0=w.eps0), 128, 3, seed=2024)
    for k in range(3):
        N, T = int(o["N"][k]), int(o["T"][k])
        fin = orc.asmc(op, opts, N, o["beta"][k][:T + 1], o["eps"][k][:T], 2024, round_k=k + 1)
        rj = orc.rejuvenate(op, opts, fin["lw"], fin["x"], T, o["eps"][k][T - 1], 2024,
                            round_k=k + 1)
        np.testing.assert_allclose(g["rejuv_mean"][k], rj["mean"], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(g["rejuv_second"][k], rj["second"], rtol=1e-9, atol=1e-9)
