"""GPU parity of parallel tempering (Sec. "Computational duality with
parallel tempering") against the oracle: the same chains, swaps, stepping-stone
estimate, swap rejections, round trips and target-chain averages."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import gpu_problem, oracle_problem
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu
MOVES = {"rwmh": orc.MOVE_RWMH, "mala": orc.MOVE_MALA, "hmc": orc.MOVE_HMC,
         "rwmh3": orc.MOVE_RWMH3}


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


CASES = [
    # family, d, move, K, Np, Tp, kc
    ("gauss", 10, "rwmh", 5, 12, 40, 0),     # one lane per chain, one wave per copy
    ("gauss", 6, "hmc", 3, 70, 20, 0),       # two waves per copy
    ("gmm", 20, "mala", 4, 9, 25, 3),        # 4 lanes x 8 coordinates
    ("gmm", 100, "rwmh3", 2, 20, 10, 5),     # 16 lanes x 8: several waves per copy
]


@pytest.mark.parametrize("family,d,move,K,Np,Tp,kc", CASES)
def test_pt_matches_oracle(oa, family, d, move, K, Np, Tp, kc):
    rng = np.random.default_rng(d * 7 + Np)
    params = wl.random_gauss(rng, d) if family == "gauss" else wl.random_gmm(rng, d, kc)
    beta = np.linspace(0, 1, Np + 1) ** 2
    eps = rng.uniform(0.1, 0.4, size=Np + 1)
    g = oa.pt(gpu_problem(oa, family, params, 1.5), K, beta, eps, Tp, 41, move=move, leapfrog=3)
    o = orc.pt(oracle_problem(family, d, params, 1.5),
               orc.Opts(move=MOVES[move], leapfrog=3, state_f32=1), K, beta, eps, Tp, 41)
    assert o["status"] == 0
    np.testing.assert_allclose(g["ss"], o["ss"], rtol=1e-11, atol=1e-11)
    assert abs(g["logZ"] - o["logZ"]) < 1e-10 * max(1.0, abs(o["logZ"]))
    np.testing.assert_allclose(g["rej"], o["rej"], rtol=1e-12, atol=1e-14)
    assert g["trips"] == o["trips"]
    np.testing.assert_allclose(g["tmean"], o["tmean"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["tsecond"], o["tsecond"], rtol=1e-12, atol=1e-13)


def test_pt_unid_matches_oracle(oa):
    g = oa.pt(oa.Problem.unid(1e4, 5e3), 8, np.linspace(0, 1, 17) ** 4, 0.3, 30, 5, move="rwmh3")
    o = orc.pt(orc.Problem(family=orc.FAM_UNID, d=2, binom_n=1e4, binom_k=5e3, box=10.0),
               orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), 8, np.linspace(0, 1, 17) ** 4, 0.3, 30, 5)
    np.testing.assert_allclose(g["ss"], o["ss"], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g["rej"], o["rej"], rtol=1e-12, atol=1e-14)
    assert g["trips"] == o["trips"]


def test_pt_rejects_too_many_chains(oa):
    rng = np.random.default_rng(1)
    params = wl.random_gmm(rng, 100, 2)
    with pytest.raises(oa.OasmcError):
        oa.pt(gpu_problem(oa, "gmm", params, 1.0), 1, np.linspace(0, 1, 80), 0.1, 2, 1)
