"""Pins of the oracle's deterministic resampling times: SIR (every step), a
given set of times, and the DAR times predicted from a previous round
(Sec. "Effective resample size for deterministic adaptive resampling", eq.
(DAR-times); appendix "Adaptive resampling in the large particle limit").

What pins them: equalities with the adaptive and AIS paths on the same
random numbers (a resampling at given times is the same operation the ESS
trigger performs), the limiting cases the paper states for DAR (no
resampling below exp(-D(B_T)), every step above max_t exp(-D_t)), the event
count implied by eq. (DAR-times), the equal root discrepancies of the
optimised schedule, AR converging to DAR for large N under the exact kernel
(Prop. on AR convergence), and unbiasedness of Z_hat for deterministic
times (Prop. 1).
"""
import numpy as np
import pytest

import closed_forms as cf


def _gauss(orc, d, mu, s2_tgt, s2_ref=1.0):
    return orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.broadcast_to(mu, (d,)).copy(),
                       sigma2=s2_tgt, ref_sigma2=s2_ref)


def _exact_log_g(beta, A):
    """A [3, T] moment block whose D_hat_t equals the closed-form D(beta_{t-1}, beta_t)."""
    T = len(beta) - 1
    lg = np.zeros((3, T))
    lg[2] = [cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1)]
    return lg


def _run(orc, P, N, beta, eps, seed, **kw):
    o = orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, nu=0.5, state_f32=1, **kw)
    r = orc.asmc(P, o, N, beta, eps, seed, traces=True)
    assert r["status"] == 0
    return r


def _same(a, b):
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["lw"], b["lw"])
    np.testing.assert_array_equal(a["accept"], b["accept"])
    np.testing.assert_array_equal(a["log_g"], b["log_g"])
    np.testing.assert_array_equal(a["resampled"], b["resampled"])
    assert a["logZ"] == b["logZ"] and a["n_resample"] == b["n_resample"]


def test_given_times_reproduce_adaptive_sir_and_ais(orc):
    """Resampling at given times is the operation the adaptive trigger performs:
    (i) the ESS trigger's own event times, given back as fixed times, reproduce
    its run bit for bit; (ii) every step flagged equals SIR; (iii) no step
    flagged equals the AIS pass.  A given-times path that resampled before the
    reweight, forgot to reset the weights or to accumulate Z_hat would break
    (i)."""
    d, N, T = 3, 200, 12
    mu = np.array([2.5, -1.0, 0.5])
    P = _gauss(orc, d, mu, 0.1)
    beta = np.linspace(0, 1, T + 1) ** 2
    ar = _run(orc, P, N, beta, 0.3, 7, trigger=0)
    assert 1 <= ar["n_resample"] < T - 1
    fixed = _run(orc, P, N, beta, 0.3, 7, trigger=3,
                 resample_at=ar["resampled"].astype(np.uint8))
    _same(ar, fixed)
    sir = _run(orc, P, N, beta, 0.3, 7, trigger=2)
    assert sir["n_resample"] == T - 1
    allf = _run(orc, P, N, beta, 0.3, 7, trigger=3, resample_at=np.ones(T, np.uint8))
    _same(sir, allf)
    none = _run(orc, P, N, beta, 0.3, 7, trigger=3, resample_at=np.zeros(T, np.uint8))
    ais = orc.asmc(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, state_f32=1), N, beta, 0.3, 7,
                   traces=True)
    np.testing.assert_array_equal(none["x"], ais["x"])
    np.testing.assert_array_equal(none["lw"], ais["lw"])
    np.testing.assert_allclose(none["log_g"], ais["log_g"], rtol=1e-14, atol=1e-14)
    assert abs(none["logZ"] - ais["logZ"]) < 1e-12 and none["n_resample"] == 0


def test_dar_limiting_cases(orc):
    """eq. (DAR-times): no resampling before T when nu <= exp(-D(B_T)) (AIS) and
    resampling at every step when nu > max_t exp(-D(beta_{t-1}, beta_t)) (SIR).
    With the previous round's knots reused (same schedule) the prediction is the
    round's own D_hat exactly, for both interpolants."""
    d = 4
    mu = np.full(d, 1.5)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.3)
    T = 30
    beta = np.linspace(0, 1, T + 1) ** 1.5
    lg = _exact_log_g(beta, A)
    D = lg[2]
    for interp in (0, 1):
        f, Dp, st = orc.dar_times(beta, lg, beta, nu=0.5, interp=interp)
        assert st == 0
        np.testing.assert_allclose(Dp, D, rtol=1e-12, atol=1e-15)
        f, _, _ = orc.dar_times(beta, lg, beta, nu=np.exp(-D.sum()) * 0.999, interp=interp)
        assert f.sum() == 0
        f, _, _ = orc.dar_times(beta, lg, beta, nu=min(np.exp(-D.min()) * 1.0001, 0.999999),
                                interp=interp)
        assert f[:-1].all() and f[-1] == 0


@pytest.mark.parametrize("nu", [0.3, 0.5, 0.8])
def test_dar_event_count_bounds(orc, nu):
    """Between consecutive DAR times the accumulated discrepancy first exceeds
    -log nu at the event and not before; so with R events before T,
    R (-log nu) < D(B_T) <= (R + 1)(-log nu + max_t D_t).  Counting from the
    wrong step, or resetting the sum one step late, breaks the bounds or the
    per-segment checks."""
    d = 8
    mu = np.full(d, 2.5)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.05)
    T = 60
    beta = np.linspace(0, 1, T + 1) ** 2
    lg = _exact_log_g(beta, A)
    f, Dp, _ = orc.dar_times(beta, lg, beta, nu=nu, interp=1)
    thr = -np.log(nu)
    R = int(f.sum())
    assert R >= 2
    assert R * thr < Dp.sum() <= (R + 1) * (thr + Dp.max())
    start = 0
    for t in np.nonzero(f)[0]:  # event after step t + 1
        seg = Dp[start:t + 1]
        assert seg.sum() > thr and seg[:-1].sum() <= thr
        start = t + 1
    assert Dp[start:T - 1].sum() <= thr  # nothing pending before the final step


def test_optimised_schedule_equalises_predicted_discrepancy(orc):
    """On the schedule Alg. 3 builds from the same moments, the predicted root
    discrepancies are all Lambda_hat_T / T' (linear interpolants both ways:
    exactly; monotone cubic both ways: within a few percent), which is the
    equal-spacing property of the optimal schedule; the DAR events are then
    evenly spaced."""
    d = 10
    mu = np.full(d, 2.0)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.25)
    beta = np.linspace(0, 1, 65)
    lg = _exact_log_g(beta, A)
    Tn = 128
    for interp, tol in ((1, 1e-9), (0, 0.08)):
        bn, lam, st = orc.optimise_schedule(beta, lg, Tn, interp=interp)
        assert st == 0
        f, Dp, _ = orc.dar_times(beta, lg, bn, nu=0.95, interp=interp)
        np.testing.assert_allclose(np.sqrt(Dp), lam[-1] / Tn, rtol=tol)
        if interp == 1:
            gaps = np.diff(np.nonzero(f)[0])
            assert gaps.size > 2 and gaps.max() - gaps.min() <= 1


def test_adaptive_resampling_converges_to_dar(orc):
    """Prop. (AR converges to DAR): with the exact kernel and N = 2^14 the ESS
    trigger fires at the DAR times computed from the closed-form
    discrepancies; only an event whose accumulated discrepancy sits within
    the Monte Carlo error of -log nu may move by one step."""
    d, N = 8, 1 << 14
    mu = np.full(d, 2.5)
    P = _gauss(orc, d, mu, 0.05)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.05)
    T = 60
    beta = np.linspace(0, 1, T + 1) ** 2
    lg = _exact_log_g(beta, A)
    f_dar, Dp, _ = orc.dar_times(beta, lg, beta, nu=0.5, interp=1)
    r = orc.asmc(P, orc.Opts(move=orc.MOVE_EXACT, resample=1, trigger=0, nu=0.5, state_f32=0),
                 N, beta, 0.0, seed=3)
    t_ar = np.nonzero(r["resampled"])[0]
    t_dar = np.nonzero(f_dar)[0]
    assert len(t_dar) >= 3
    assert abs(len(t_ar) - len(t_dar)) <= 1
    close = sum(int(a == b) for a, b in zip(t_ar, t_dar))
    assert close >= len(t_dar) - 1
    assert all(abs(int(a) - int(b)) <= 1 for a, b in zip(t_ar, t_dar))


@pytest.mark.parametrize("mode", ["sir", "dar"])
def test_deterministic_times_unbiased(orc, mode):
    """Prop. 1 with deterministic resampling times (every step, or the DAR times
    of the closed-form discrepancies): E[Z_hat] = Z.  Accumulating Z_hat after
    the weight reset, or from w_{t-1} instead of w_{t^-}, biases it."""
    d, N, T, S = 2, 16, 8, 3000
    mu = np.array([2.0, -1.5])
    P = _gauss(orc, d, mu, 0.2)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.2)
    beta = np.linspace(0, 1, T + 1)
    if mode == "sir":
        kw = dict(trigger=2)
    else:
        f, _, _ = orc.dar_times(beta, _exact_log_g(beta, A), beta, nu=0.5, interp=1)
        assert 1 <= f.sum() < T - 1
        kw = dict(trigger=3, resample_at=f)
    lz = np.array([orc.asmc(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, nu=0.5,
                                        state_f32=0, **kw), N, beta, 0.3, seed=s)["logZ"]
                   for s in range(S)])
    ratio = np.exp(lz - A(1.0))
    assert abs(ratio.mean() - 1) < 4.5 * ratio.std() / np.sqrt(S)


def test_run_with_dar_rounds(orc):
    """Alg. 2 with DAR: round 1 resamples at no intermediate step, and round k
    resamples exactly at the times orc_dar_times predicts from round k-1's
    schedule and moments for round k's schedule."""
    d = 6
    mu = np.full(d, 1.5)
    P = _gauss(orc, d, mu, 0.1, s2_ref=2.0)
    o = orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, nu=0.5, state_f32=1)
    ro = orc.RunOpts(budget=2, T1=4, Tmax=64, eps0=0.4, eps_adapt=1, eps_kappa=20.0,
                     accept_target=0.65, dar=1)
    r = orc.run(P, o, ro, 400, 5, seed=9)
    assert r["status"] == 0
    assert r["n_resample"][0] == 0
    for k in range(1, 5):
        Tp, Tk = r["T"][k - 1], r["T"][k]
        f, _, st = orc.dar_times(r["beta"][k - 1][:Tp + 1], r["log_g"][k - 1][:, :Tp],
                                 r["beta"][k][:Tk + 1], nu=0.5, interp=0)
        assert st == 0
        assert r["n_resample"][k] == int(f.sum())
    assert r["n_resample"][1:].sum() > 0
