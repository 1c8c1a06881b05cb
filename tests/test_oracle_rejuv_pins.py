"""Pins of the oracle's final-iteration rejuvenation (Sec. "Computing
expectations"): resample the final population, run N chains for T steps,
average test functions over the TN states.

What pins it: the identity kernel reduces it to an average over the
resampled particles (the resampler itself is pinned against searchsorted and
the counter layout against the Philox known answers); the exact kernel at
beta = 1 gives iid draws from the target, whose mean and second moment are
closed forms; real MH chains reproduce them within Monte Carlo error; and the
rejuvenated averages beat the final weighted particles, as the paper reports.
"""
import numpy as np
import pytest


def _gauss(orc, d, mu, s2_tgt, s2_ref=1.0):
    return orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.broadcast_to(mu, (d,)).copy(),
                       sigma2=s2_tgt, ref_sigma2=s2_ref)


def _final_population(orc, P, N, T, eps, seed, move):
    beta = np.linspace(0, 1, T + 1) ** 2
    r = orc.asmc(P, orc.Opts(move=move, leapfrog=3, state_f32=1), N, beta, eps, seed)
    assert r["status"] == 0
    return r


def test_identity_kernel_averages_the_resampled_particles(orc):
    """With chains that never move, every chain repeats its resampled start T
    times: the averages are those of x[a_n] with a the systematic ancestors of
    the final weights for the word of step T (particle word 0xFFFFFFFF,
    stream 3).  A wrong event word, ancestors from w_{T-1}, or averages over
    the pre-resampling population fail."""
    d, N, T, seed = 3, 500, 7, 11
    P = _gauss(orc, d, np.array([1.0, -2.0, 0.5]), 0.3)
    fin = _final_population(orc, P, N, T, 0.4, seed, orc.MOVE_RWMH)
    r = orc.rejuvenate(P, orc.Opts(move=orc.MOVE_IDENTITY, state_f32=1), fin["lw"], fin["x"], T,
                       0.4, seed, want_states=True)
    assert r["status"] == 0 and r["accept"] == 1.0
    u = orc.philox4x32_10([0xFFFFFFFF, T, 1, 3 << 24], [seed & 0xFFFFFFFF, seed >> 32])[0]
    a = orc.systematic(fin["lw"], int(u))
    xs = fin["x"][a]
    np.testing.assert_allclose(r["mean"], xs.mean(0), rtol=1e-13)
    np.testing.assert_allclose(r["second"], (xs ** 2).mean(0), rtol=1e-13)
    np.testing.assert_array_equal(r["x"], xs)


def test_exact_kernel_at_beta_one_matches_closed_form(orc):
    """Exact draws from pi_1 = N(mu, s2 I): mean and second moment within a few
    standard errors of mu and mu^2 + s2 (chains at any beta < 1 would shift
    the mean towards eta's)."""
    d, N, T = 4, 400, 50
    mu = np.array([2.0, -1.0, 0.3, 1.5])
    s2 = 0.25
    P = _gauss(orc, d, mu, s2)
    fin = _final_population(orc, P, N, 8, 0.3, 3, orc.MOVE_RWMH)
    r = orc.rejuvenate(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), fin["lw"], fin["x"], T,
                       0.3, 3)
    n = N * T
    assert np.all(np.abs(r["mean"] - mu) < 5 * np.sqrt(s2 / n))
    sd2 = np.sqrt(2 * s2 ** 2 + 4 * mu ** 2 * s2)  # sd of x^2 for x ~ N(mu, s2)
    assert np.all(np.abs(r["second"] - (mu ** 2 + s2)) < 5 * sd2 / np.sqrt(n))


@pytest.mark.parametrize("move,eps", [("rwmh", 0.35), ("mala", 0.3), ("hmc", 0.25)])
def test_mh_chains_match_closed_form(orc, move, eps):
    """pi-invariant MH chains started from the resampled AIS population of the
    d = 10 Gaussian target (mean 2, variance 0.25) reproduce its moments
    within Monte Carlo error (generous for autocorrelation)."""
    d, N, T = 10, 256, 400
    P = _gauss(orc, d, 2.0, 0.25)
    mv = {"rwmh": orc.MOVE_RWMH, "mala": orc.MOVE_MALA, "hmc": orc.MOVE_HMC}[move]
    fin = _final_population(orc, P, N, 256, eps, 5, mv)
    r = orc.rejuvenate(P, orc.Opts(move=mv, leapfrog=3, state_f32=1), fin["lw"], fin["x"], T,
                       eps, 5)
    assert 0.2 < r["accept"] < 1.0
    np.testing.assert_allclose(r["mean"], 2.0, atol=0.05)
    np.testing.assert_allclose(r["second"] - r["mean"] ** 2, 0.25, atol=0.05)


def test_rejuvenation_beats_final_weighted_particles(orc):
    """Over independent seeds, the rejuvenated estimate of E[x] has a smaller
    error than the final weighted particles of a short AIS run (the comparison
    of the appendix on computing expectations)."""
    d, N, T, S = 4, 64, 12, 30
    mu = np.full(d, 1.5)
    P = _gauss(orc, d, mu, 0.2)
    e_w, e_r = [], []
    for s in range(S):
        fin = _final_population(orc, P, N, T, 0.3, 100 + s, orc.MOVE_RWMH)
        W = np.exp(fin["lw"] - fin["lw"].max())
        W /= W.sum()
        e_w.append(np.sum((W @ fin["x"] - mu) ** 2))
        r = orc.rejuvenate(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1), fin["lw"], fin["x"], T,
                           0.3, 100 + s)
        e_r.append(np.sum((r["mean"] - mu) ** 2))
    assert np.mean(e_r) < np.mean(e_w)
