"""Pins of the oracle's parallel tempering (Sec. "Computational duality with
parallel tempering"; appendix on the round trip rate).

What pins it: with the exact kernel the stepping-stone terms of different
temperatures and iterations are independent, so Z_PT is unbiased with the
variance that SIR has with N = T' and T = N' (the duality), in closed form;
swap rejection rates against a numpy Monte Carlo of the closed-form Gaussian
path; Lambda <= sqrt 2 Lambda_PT bound of the paper's proposition on the two
barriers; and the round-trip rate of non-reversible PT on a finite schedule,
1 / (2 + 2 sum_n r_n / (1 - r_n)), including the deterministic Lambda = 0 case
(gamma proportional to eta).
"""
import numpy as np

import closed_forms as cf

LAM_C1 = 9.0033663  # global barrier of the d = 10 target (closed form)


def _gauss(orc, d, mu, s2_tgt, s2_ref=1.0):
    return orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.broadcast_to(mu, (d,)).copy(),
                       sigma2=s2_tgt, ref_sigma2=s2_ref)


def test_stepping_stone_duality_closed_form_variance(orc):
    """Exact kernel: E[Z_PT / Z] = 1 and Var[Z_PT / Z] = prod_n (1 + (e^{D_n} - 1) / (K T')) - 1,
    the SIR variance with the roles of N and T exchanged."""
    d, Np, Tp, K, S = 2, 6, 8, 2, 1500
    mu = np.array([1.5, -1.0])
    P = _gauss(orc, d, mu, 0.3)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.3)
    beta = np.linspace(0, 1, Np + 1)
    D = np.array([cf.discrepancy(beta[n - 1], beta[n], A) for n in range(1, Np + 1)])
    var_th = np.prod(1 + (np.exp(D) - 1) / (K * Tp)) - 1
    lz = np.array([orc.pt(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), K, beta, 0.0, Tp,
                          seed=s)["logZ"] for s in range(S)])
    ratio = np.exp(lz - A(1.0))
    assert abs(ratio.mean() - 1) < 4 * np.sqrt(var_th / S)
    assert abs(ratio.var() / var_th - 1) < 0.2


def test_swap_rejection_matches_gaussian_path(orc):
    """Under the exact kernel the rejection of the swap (n, n+1) is
    1 - E[min(1, exp((b' - b)(V(Y) - V(Y'))))], Y ~ pi_b, Y' ~ pi_b' independent;
    the expectation is taken here by numpy sampling of the closed-form Gaussians."""
    d, Np, Tp, K = 10, 8, 200, 32
    P = _gauss(orc, d, 2.0, 0.25)
    beta = np.linspace(0, 1, Np + 1) ** 2
    r = orc.pt(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), K, beta, 0.0, Tp, seed=4)
    rng = np.random.default_rng(0)

    def draw(b, m):
        lam = (1 - b) + b / 0.25
        mean = (b * 2.0 / 0.25) / lam
        return mean + rng.standard_normal((m, d)) / np.sqrt(lam)

    V = lambda x: -np.sum((x - 2.0) ** 2, 1) / 0.5 + np.sum(x ** 2, 1) / 2.0
    for n in range(Np):
        y, y2 = draw(beta[n], 400000), draw(beta[n + 1], 400000)
        ref = 1 - np.mean(np.minimum(1.0, np.exp((beta[n + 1] - beta[n]) * (V(y) - V(y2)))))
        cnt = K * Tp / 2
        assert abs(r["rej"][n] - ref) < 5 * np.sqrt(ref * (1 - ref) / cnt) + 0.01


def test_communication_barrier_bound_and_round_trips(orc):
    """On a dense schedule the summed rejections estimate Lambda_PT; the
    paper's bound sqrt 2 Lambda_PT <= Lambda holds (Lambda = 9.0034 for the
    d = 10 target, with Lambda / Lambda_PT near sqrt(pi) at this d), and the
    round-trip rate per copy and iteration is that of non-reversible PT on a
    finite schedule, 1 / (2 + 2 sum_n r_n / (1 - r_n)) (1 / (2 + 2 Lambda_PT) in
    the dense limit); long runs, so that the start-up transient (a replica
    needs about (N' + 1) / rate iterations per round trip) stays small."""
    d, Np, Tp, K = 10, 40, 8000, 8
    P = _gauss(orc, d, 2.0, 0.25)
    u = np.linspace(0, 1, Np + 1)
    beta = np.array([cf.phi_star(v, lambda b: cf.delta_gauss(b, 0.0, 1.0, 2.0, 0.25))
                     for v in u[1:-1]])
    beta = np.concatenate([[0.0], beta, [1.0]])
    r = orc.pt(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), K, beta, 0.0, Tp, seed=8)
    lam_pt = r["Lambda_PT"]
    assert np.sqrt(2) * lam_pt <= LAM_C1 * 1.02
    assert 1.5 < LAM_C1 / lam_pt < 1.95
    rate = r["trips"] / (K * Tp)
    rej = r["rej"]
    assert abs(rate / (1 / (2 + 2 * np.sum(rej / (1 - rej)))) - 1) < 0.1


def test_round_trips_without_barrier(orc):
    """gamma proportional to eta (ell constant, Lambda_PT = 0): every swap is
    accepted and each replica sweeps the temperatures deterministically, one
    round trip per 2 (N' + 1) iterations, i.e. T' / 2 per copy."""
    d, Np, Tp, K = 3, 5, 120, 4
    P = _gauss(orc, d, 0.0, 1.0)  # gamma = eta up to the constant
    r = orc.pt(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1), K, np.linspace(0, 1, Np + 1), 0.5,
               Tp, seed=1)
    assert np.all(r["rej"] < 1e-12)  # ell is constant up to rounding
    assert abs(r["trips"] - K * Tp / 2) <= K * (Np + 1)
    assert abs(r["logZ"] - 0.5 * d * np.log(2 * np.pi)) < 1e-9
