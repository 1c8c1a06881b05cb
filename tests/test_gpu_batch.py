"""Batched runs: many independent problems (mixed families, dimensions and
kernel shapes) in one device-resident enqueue, optionally one hipGraph.  Each
problem's per-round log Z_hat and Lambda_hat_T must equal, bit for bit, a
plain oasmc_run of that problem alone: the same kernels walk the same slots in
the same order, and Alg. 3 runs on the device in both."""
import numpy as np
import pytest
import torch

from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _problem(oa, spec):
    if spec["family"] == "gauss":
        return oa.Problem.gauss(spec["params"]["mu"], spec["params"]["sigma2"], 1.0)
    if spec["family"] == "gmm":
        return oa.Problem.gmm(spec["params"]["means"], spec["params"]["log_scales"], 4.0)
    return oa.Problem.logreg(spec["params"]["X"], spec["params"]["y"], 1.0)


def _plain(oa, prob, spec, rounds, seed, pid):
    T = spec["T"]
    return oa.run(prob, spec["N"], rounds, seed=seed, problem_id=pid, move=spec["move"],
                  leapfrog=3, budget="double_t", T1=max(1, T >> (rounds - 1)), T_max=T,
                  eps0=spec["eps0"], eps_adapt=spec["eps_adapt"], eps_kappa=spec["eps_kappa"],
                  accept_target=0.574, Tcap=T)


def _mixed_specs():
    rng = np.random.default_rng(8)
    specs = []
    for d, N, T in [(5, 100, 8), (10, 256, 16), (33, 300, 12), (70, 130, 8), (150, 65, 4)]:
        specs.append(dict(family="gauss", d=d, N=N, T=T, move="rwmh",
                          params=wl.random_gauss(rng, d), eps0=0.5 / np.sqrt(d), eps_adapt=False,
                          eps_kappa=0.0))
    specs.append(dict(family="gmm", d=20, N=500, T=16, move="mala",
                      params=wl.random_gmm(rng, 20, 4), eps0=0.4, eps_adapt=True, eps_kappa=2.0))
    specs.append(dict(family="gmm", d=6, N=70, T=9, move="hmc",
                      params=wl.random_gmm(rng, 6, 3), eps0=0.3, eps_adapt=True, eps_kappa=1.0))
    # 4 lanes x 16 coordinates, K = 6: per-problem lane-layout means with a
    # padded block of components, read from global memory
    specs.append(dict(family="gmm", d=40, N=130, T=8, move="mala",
                      params=wl.random_gmm(rng, 40, 6), eps0=0.3, eps_adapt=True, eps_kappa=2.0))
    for d, n, N, T in [(7, 300, 64, 8), (50, 1000, 200, 16), (33, 777, 65, 4), (90, 500, 70, 8),
                       (180, 400, 40, 4)]:
        X, y, _ = wl.logreg_data(n, d, n + d)
        specs.append(dict(family="logreg", d=d, N=N, T=T, move="mala", params=dict(X=X, y=y),
                          eps0=0.5 * d ** (-1 / 6), eps_adapt=True, eps_kappa=n / 4))
    return specs


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_plain_runs(oa, use_graph):
    rounds = 3
    specs = _mixed_specs()
    probs = [_problem(oa, s) for s in specs]
    items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], leapfrog=3,
                          eps0=s["eps0"], eps_adapt=s["eps_adapt"], eps_kappa=s["eps_kappa"],
                          seed=1000 + i, problem_id=i) for i, (p, s) in enumerate(zip(probs, specs))]
    b = oa.run_batch(items, rounds, use_graph=use_graph)
    assert np.all(b["status"] == 0)
    for i, (p, s) in enumerate(zip(probs, specs)):
        r = _plain(oa, p, s, rounds, 1000 + i, i)
        np.testing.assert_array_equal(b["logZ"][i], r["logZ"], err_msg=f"problem {i}")
        lam_T = np.array([r["Lambda"][k][r["T"][k]] for k in range(rounds)])
        np.testing.assert_array_equal(b["Lambda_T"][i], lam_T, err_msg=f"problem {i}")


def test_graph_replay_is_identical(oa):
    """The captured batch against the eager enqueue of the same batch: the
    capture's run and two replays, with eager work and synchronisations
    between them, each equal to the eager result (the per-class work counters
    are re-zeroed inside the graph on every replay)."""
    specs = _mixed_specs()[:4]
    probs = [_problem(oa, s) for s in specs]
    items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], eps0=s["eps0"],
                          seed=7, problem_id=i) for i, (p, s) in enumerate(zip(probs, specs))]
    ref = oa.run_batch(items, 2, use_graph=False)
    for rep in range(3):  # capture, then replays of the cached graph
        g = oa.run_batch(items, 2, use_graph=True)
        np.testing.assert_array_equal(g["logZ"], ref["logZ"], err_msg=f"replay {rep}")
        np.testing.assert_array_equal(g["Lambda_T"], ref["Lambda_T"], err_msg=f"replay {rep}")
        e = oa.run_batch(items[:2], 2, use_graph=False)  # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(e["logZ"], ref["logZ"][:2])


def test_full_batch_sampled_against_plain(oa):
    """The 256-problem workload (uneven d, n, N, T; 4 rounds) in one graph;
    sampled problems equal their plain runs and every result is finite."""
    specs = wl.batch_problems()
    probs = [_problem(oa, s) for s in specs]
    items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], eps0=s["eps0"],
                          eps_adapt=s["eps_adapt"], eps_kappa=s["eps_kappa"], seed=99,
                          problem_id=i) for i, (p, s) in enumerate(zip(probs, specs))]
    b = oa.run_batch(items, 4, use_graph=True)
    assert np.all(np.isfinite(b["logZ"]))
    rng = np.random.default_rng(0)
    for i in rng.choice(len(specs), size=4, replace=False):
        s = specs[i]
        r = _plain(oa, probs[i], s, 4, 99, int(i))
        np.testing.assert_array_equal(b["logZ"][i], r["logZ"], err_msg=f"problem {i}")


def test_batch_against_oracle_runs(oa):
    """Batched closed-form problems against the oracle's own Alg. 2 runs (not
    against plain GPU runs): per-round log Z_hat and Lambda_hat_T.  One
    problem (Gaussian d = 150 on 16 lanes per particle, N = 8203, i.e. 2051
    tiles) folds several tiles into a moment slot; the small ones use a slot
    cap of 2.  Tolerances are the stated ones (log Z_hat within 1e-6)."""
    import oracle as orc
    rng = np.random.default_rng(31)
    rounds = 2
    specs = [
        dict(family="gauss", d=150, N=8203, T=4, move="rwmh", params=wl.random_gauss(rng, 150),
             eps0=0.04, eps_adapt=False, eps_kappa=0.0, slots=0),
        dict(family="gauss", d=12, N=700, T=8, move="rwmh", params=wl.random_gauss(rng, 12),
             eps0=0.3, eps_adapt=False, eps_kappa=0.0, slots=2),
        dict(family="gmm", d=20, N=300, T=8, move="mala", params=wl.random_gmm(rng, 20, 4),
             eps0=0.4, eps_adapt=True, eps_kappa=2.0, slots=2),
        dict(family="gmm", d=70, N=90, T=4, move="hmc", params=wl.random_gmm(rng, 70, 5),
             eps0=0.2, eps_adapt=True, eps_kappa=1.0, slots=2),
    ]
    probs = [_problem(oa, s) for s in specs]
    items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], leapfrog=3,
                          eps0=s["eps0"], eps_adapt=s["eps_adapt"], eps_kappa=s["eps_kappa"],
                          seed=500 + i, problem_id=i, slots=s["slots"])
             for i, (p, s) in enumerate(zip(probs, specs))]
    b = oa.run_batch(items, rounds, use_graph=True)
    assert np.all(b["status"] == 0)
    moves = {"rwmh": orc.MOVE_RWMH, "mala": orc.MOVE_MALA, "hmc": orc.MOVE_HMC}
    for i, s in enumerate(specs):
        if s["family"] == "gauss":
            op = orc.Problem(family=orc.FAM_GAUSS, d=s["d"], mu=s["params"]["mu"],
                             sigma2=s["params"]["sigma2"], ref_sigma2=1.0)
        else:
            op = orc.Problem(family=orc.FAM_GMM, d=s["d"], means=s["params"]["means"],
                             log_scales=s["params"]["log_scales"], ref_sigma2=4.0)
        T = s["T"]
        o = orc.run(op, orc.Opts(move=moves[s["move"]], leapfrog=3, state_f32=1),
                    orc.RunOpts(budget=2, T1=max(1, T >> (rounds - 1)), Tmax=T,
                                eps_adapt=int(s["eps_adapt"]), eps0=s["eps0"],
                                eps_kappa=s["eps_kappa"], accept_target=0.574),
                    s["N"], rounds, seed=500 + i, problem_id=i, Tcap=T)
        assert o["status"] == 0
        np.testing.assert_allclose(b["logZ"][i], o["logZ"], rtol=0, atol=1e-6,
                                   err_msg=f"problem {i}")
        lam_T = np.array([o["Lambda"][k][o["T"][k]] for k in range(rounds)])
        np.testing.assert_allclose(b["Lambda_T"][i], lam_T, rtol=1e-6, atol=1e-8,
                                   err_msg=f"problem {i}")


def test_more_kernel_classes_than_one_counter_fill(oa):
    """A batch spanning more than 64 kernel classes (families x moves x lane
    layouts x logistic-regression layouts): the per-class work counters are
    zeroed in fills of 64, and every problem still equals its plain run."""
    rng = np.random.default_rng(64)
    rounds = 2
    specs = []
    # small N: lane layouts (1, 4), (1, 8), (8, 4), (4, 16), (16, 8), (16, 16)
    for fam in ("gauss", "gmm"):
        for move in ("rwmh", "mala", "hmc", "rwmh3"):
            for d in (3, 7, 20, 50, 100, 150):
                params = wl.random_gauss(rng, d) if fam == "gauss" else wl.random_gmm(rng, d, 3)
                specs.append(dict(family=fam, d=d, N=64, T=4, move=move, params=params,
                                  eps0=0.2, eps_adapt=False, eps_kappa=0.0))
    # many particles: one lane of 12 .. 24 coordinates, two lanes of 16
    for d, N in ((12, 131072), (16, 131072), (20, 131072), (24, 131072), (30, 65536)):
        specs.append(dict(family="gauss", d=d, N=N, T=2, move="rwmh",
                          params=wl.random_gauss(rng, d), eps0=0.2, eps_adapt=False,
                          eps_kappa=0.0))
    # logistic regression: the seven 64-column half-widths, the one-panel
    # layout (N >= 4096) and two to four panels
    for d, N in ((7, 64), (15, 64), (22, 64), (31, 64), (39, 64), (50, 64), (60, 64),
                 (20, 4096), (100, 40), (150, 40), (200, 40)):
        X, y, _ = wl.logreg_data(200, d, 3000 + d)
        specs.append(dict(family="logreg", d=d, N=N, T=2, move="mala", params=dict(X=X, y=y),
                          eps0=0.1, eps_adapt=False, eps_kappa=0.0))
    probs = [_problem(oa, s) for s in specs]
    unid = [(oa.Problem.unid(1e4, 2e3, 10.0), mv) for mv in ("rwmh", "rwmh3")]
    valu = {(s["family"], s["move"]) + oa.shape(p, s["N"], move=s["move"], leapfrog=3)
            for p, s in zip(probs, specs) if s["family"] != "logreg"}
    n_logreg_layouts = 11  # half-widths 4 8 12 16 20 25 32, one panel, 2, 3 and 4 panels
    assert len(valu) + n_logreg_layouts + len(unid) > 64
    items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], leapfrog=3,
                          eps0=s["eps0"], seed=70 + i, problem_id=i)
             for i, (p, s) in enumerate(zip(probs, specs))]
    for j, (p, mv) in enumerate(unid):
        items.append(oa.BatchItem(problem=p, N=64, T=4, move=mv, eps0=0.5, seed=900 + j,
                                  problem_id=len(specs) + j))
    b = oa.run_batch(items, rounds, use_graph=True)
    assert np.all(b["status"] == 0)
    for i, (p, s) in enumerate(zip(probs, specs)):
        r = _plain(oa, p, s, rounds, 70 + i, i)
        np.testing.assert_array_equal(b["logZ"][i], r["logZ"], err_msg=f"problem {i}")
