"""Launch-shape autotuning of the VALU sweeps: measured shapes hold the
problem's dimension, autotuned passes still match the oracle, and a batch
with autotuning gives the same results as the same problems run one by one
with it (both take the handle's measured shapes)."""
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
    m.autotune(1)
    yield m
    m.autotune(-1)  # later tests use the fixed rule


@pytest.mark.parametrize("family,d,move,N,T,K", [("gauss", 10, "rwmh", 4096, 8, 0),
                                                 ("gmm", 30, "mala", 2048, 6, 4),
                                                 ("gauss", 100, "hmc", 500, 5, 0)])
def test_autotuned_pass_matches_oracle(oa, family, d, move, N, T, K):
    rng = np.random.default_rng(d * 3 + N)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, K)
    gp = gpu_problem(oa, family, params, 1.5)
    lpp, dpl = oa.shape(gp, N, move=move, leapfrog=3)
    assert lpp * dpl >= d and dpl % 4 == 0
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = np.full(T, 0.2)
    g = oa.asmc(gp, N, beta, eps, 21, move=move, leapfrog=3, accept_bits=True)
    op = oracle_problem(family, d, params, 1.5)
    o = orc.asmc(op, orc.Opts(move=ORC_MOVE[move], leapfrog=3, state_f32=1), N, beta, eps, 21,
                 traces=True)
    compare_round(g, o, T, N)


def test_autotuned_batch_equals_one_by_one(oa):
    specs = [s for s in wl.batch_problems(24, seed_offset=9) if s["family"] == "gauss"][:6]
    items = [oa.BatchItem(problem=oa.Problem.gauss(s["params"]["mu"], s["params"]["sigma2"], 1.0),
                          N=min(s["N"], 4096), T=min(s["T"], 64), move="rwmh", eps0=s["eps0"],
                          seed=3, problem_id=i) for i, s in enumerate(specs)]
    b = oa.run_batch(items, 3, use_graph=True)
    for i, it in enumerate(items):
        one = oa.run_batch([it], 3, use_graph=False)
        np.testing.assert_array_equal(b["logZ"][i], one["logZ"][0])
    assert oa.autotune(1) >= 1
