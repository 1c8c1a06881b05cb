"""Pins of the CPU oracle against things other than itself: published known
answers, closed forms of the linear annealing path for Gaussian targets, a
value the paper prints, library routines for sub-steps (PCHIP, searchsorted),
brute force on tiny inputs and invariants the paper proves (unbiasedness).

Each test names what would fail it (dropped term, wrong sign or index,
transposed operand) in its docstring.
"""
import os

import numpy as np
import pytest
from scipy import interpolate, stats

import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gauss_problem(orc, d, mu, s2_tgt, m_ref=None, s2_ref=1.0):
    return orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.broadcast_to(mu, (d,)).copy(),
                       sigma2=s2_tgt, ref_mean=None if m_ref is None else
                       np.broadcast_to(m_ref, (d,)).copy(), ref_sigma2=s2_ref)


# --------------------------------------------------------------------------- RNG
def test_philox_known_answers(orc):
    """Salmon et al. known-answer vectors: any wrong multiplier, Weyl constant,
    word order or round count fails."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_word_and_counter_layout(orc):
    """The accept uniform is (w0 + 1/2) 2^-32 of the block at the documented
    counter (n, t, round | problem << 16, stream << 24 | substep << 16 | block)."""
    seed = 0x1234_5678_9ABC_DEF0
    w = orc.philox4x32_10([7, 3, 2 | (5 << 16), (2 << 24) | (0 << 16) | 0],
                          [seed & 0xFFFFFFFF, seed >> 32])
    u = orc.uniform(seed, 2, 5, 7, 3, 2, 0)
    assert u == (float(w[0]) + 0.5) / 2.0 ** 32


def test_normals_are_standard_normal(orc):
    """Box-Muller output: KS against N(0,1), moments, and independence of the
    cosine/sine members; a wrong 2 pi, log base or pairing fails."""
    z = np.concatenate([orc.normals(99, 1, 0, n, t, 1, 0, 16)
                        for n in range(400) for t in range(40)])
    assert z.size == 256000
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 0.05
    pairs = z.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5 / np.sqrt(pairs.shape[0])


# --------------------------------------------------------------------------- target algebra
@pytest.mark.parametrize("family", ["gauss", "gmm", "logreg"])
def test_ell_gradient_matches_finite_differences(orc, family):
    """The gradients used by MALA/HMC agree with central differences of ell."""
    rng = np.random.default_rng(3)
    d = 6
    if family == "gauss":
        P = _gauss_problem(orc, d, rng.normal(size=d), 0.3, m_ref=rng.normal(size=d), s2_ref=2.0)
    elif family == "gmm":
        P = orc.Problem(family=orc.FAM_GMM, d=d, means=rng.normal(size=(3, d)),
                        log_scales=np.array([0.0, -0.3, 0.2]), ref_sigma2=4.0)
    else:
        X = rng.normal(size=(30, d))
        y = (rng.random(30) < 0.5).astype(float)
        P = orc.Problem(family=orc.FAM_LOGREG, d=d, X=X, y=y, ref_sigma2=1.0)
    x = rng.normal(size=d)
    v, g = orc.ell(P, x)
    h = 1e-6
    fd = np.array([(orc.ell(P, x + h * e)[0] - orc.ell(P, x - h * e)[0]) / (2 * h)
                   for e in np.eye(d)])
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6)


def test_ell_closed_form_values(orc):
    """ell = log gamma - log eta for each family against an independent numpy/scipy
    evaluation of the densities."""
    rng = np.random.default_rng(5)
    d = 4
    x = rng.normal(size=d)
    mu = rng.normal(size=d)
    P = _gauss_problem(orc, d, mu, 0.7, m_ref=np.ones(d), s2_ref=2.5)
    ref = -np.sum((x - mu) ** 2) / 1.4 - stats.multivariate_normal(np.ones(d), 2.5).logpdf(x)
    assert abs(orc.ell(P, x)[0] - ref) < 1e-12
    means = rng.normal(size=(3, d))
    ls = np.array([0.1, -0.2, 0.0])
    P = orc.Problem(family=orc.FAM_GMM, d=d, means=means, log_scales=ls, ref_sigma2=9.0)
    comp = [-np.sum((x - means[k]) ** 2) / (2 * np.exp(2 * ls[k])) for k in range(3)]
    ref = np.log(np.mean(np.exp(comp))) - stats.multivariate_normal(np.zeros(d), 9.0).logpdf(x)
    assert abs(orc.ell(P, x)[0] - ref) < 1e-11
    X = rng.normal(size=(12, d))
    y = (rng.random(12) < 0.4).astype(float)
    P = orc.Problem(family=orc.FAM_LOGREG, d=d, X=X, y=y)
    z = X @ x
    ref = np.sum(stats.bernoulli.logpmf(y, 1 / (1 + np.exp(-z))))
    assert abs(orc.ell(P, x)[0] - ref) < 1e-11


# --------------------------------------------------------------------------- Alg. 1 vs closed forms
def test_exact_kernel_unbiased_with_closed_form_variance(orc):
    """Exact-sampling kernel on the d=10 Gaussian target: E[Z_hat/Z] = 1 (Prop. 1) and
    N Var[Z_hat/Z] = e^{D(B_T)} - 1 (Thm. 1, AIS) with D from the closed-form A(beta).
    A weight at the post-move state, a wrong Delta beta, or a missing log eta
    normalisation breaks the mean or the variance."""
    d, N, T, S = 10, 64, 64, 1200
    P = _gauss_problem(orc, d, 2.0, 0.25)
    beta = np.linspace(0, 1, T + 1)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    D = sum(cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1))
    var_theory = (np.exp(D) - 1) / N
    logZ = A(1.0)
    assert abs(logZ - 2.2579135264) < 1e-9
    r = np.array([orc.asmc(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), N, beta, 0.0,
                           seed=s)["logZ"] for s in range(S)])
    ratio = np.exp(r - logZ)
    se = np.sqrt(var_theory / S)
    assert abs(ratio.mean() - 1) < 4 * se
    assert abs(ratio.var() / var_theory - 1) < 0.3


def test_identity_kernel_is_importance_sampling(orc):
    """With the identity kernel AIS is importance sampling from eta:
    N Var[Z_hat/Z] = E_eta[(gamma/(Z eta))^2] - 1 in closed form; every step's
    log g is (beta_t - beta_{t-1}) ell of the same point, so log w_T = ell(x_0)."""
    d, N, S = 2, 32, 3000
    mu, s2 = 0.5, 0.8  # s2 < 8/7 keeps the 8th moment of the weight finite
    P = _gauss_problem(orc, d, mu, s2)
    beta = np.linspace(0, 1, 9) ** 2
    # E_eta[(gamma/eta)^2] = exp(A(2)) with the closed form continued to beta = 2
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, np.full(d, mu), s2)
    var_theory = (np.exp(A(2.0) - 2 * A(1.0)) - 1) / N
    r = np.array([orc.asmc(P, orc.Opts(move=orc.MOVE_IDENTITY, state_f32=0), N, beta, 0.0,
                           seed=s)["logZ"] for s in range(S)])
    ratio = np.exp(r - A(1.0))
    assert abs(ratio.mean() - 1) < 4 * np.sqrt(var_theory / S)
    assert abs(ratio.var() / var_theory - 1) < 0.25
    one = orc.asmc(P, orc.Opts(move=orc.MOVE_IDENTITY, state_f32=0), 5, beta, 0.0, seed=1)
    ells = np.array([orc.ell(P, one["x"][j])[0] for j in range(5)])
    np.testing.assert_allclose(one["lw"], ells, rtol=1e-13, atol=1e-13)


def test_moments_estimate_closed_form_discrepancy(orc):
    """D_hat_t from the moments of eq. (CESS) converges to the closed-form
    D(beta_{t-1}, beta_t) under the exact kernel; swapping g_hat_0 and g_hat_2 or
    using w_t instead of w_{t-1} fails.  Also D_hat >= 0 (Cauchy-Schwarz)."""
    d, N, T = 2, 40000, 8
    mu = np.array([1.0, -0.5])
    P = _gauss_problem(orc, d, mu, 0.5)
    beta = np.linspace(0, 1, T + 1)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.5)
    r = orc.asmc(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), N, beta, 0.0, seed=11)
    lg = r["log_g"]
    Dhat = lg[2] - 2 * lg[1] + lg[0]
    Dtrue = np.array([cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1)])
    assert np.all(Dhat >= 0)
    # relative Monte Carlo error of D_hat is about 1% here; 6% is several sigma
    np.testing.assert_allclose(Dhat, Dtrue, rtol=0.06)
    # g_hat_1 / g_hat_0 estimates Z_{beta_t}/Z_{beta_{t-1}}
    inc = lg[1] - lg[0]
    true_inc = np.diff(A(beta))
    np.testing.assert_allclose(inc, true_inc, atol=0.01)


def test_global_barrier_c1_and_schedule_invariance(orc):
    """Lambda_hat_T approaches the closed-form global barrier 9.0033663 of the
    d=10 Gaussian target for two different schedules (Cor. 1: the sum of
    sqrt(D) is schedule invariant up to O(1/T))."""
    d, N, T = 10, 4000, 256
    P = _gauss_problem(orc, d, 2.0, 0.25)
    dl = lambda b: cf.delta_gauss(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    Lam = cf.global_barrier(dl)
    assert abs(Lam - 9.0033663) < 1e-6
    # high-dimensional scaling check of the closed form itself: sqrt(d) times 1-d barrier
    dl1 = lambda b: cf.delta_gauss(b, 0.0, 1.0, 2.0, 0.25)
    assert abs(np.sqrt(d) * cf.global_barrier(dl1) - Lam) < 1e-9
    for beta in (np.linspace(0, 1, T + 1), np.linspace(0, 1, T + 1) ** 2.5):
        r = orc.asmc(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), N, beta, 0.0, seed=5)
        _, lam, st = orc.optimise_schedule(beta, r["log_g"], T)
        assert st == 0
        assert np.all(np.diff(lam) >= 0)
        assert abs(lam[-1] - Lam) < 0.03 * Lam


def test_printed_barrier_isotropic_normal(orc):
    """The paper's printed Lambda_hat = 2.5 for the 5-d annealed normal
    (tab:models) against the oracle's estimate with the exact kernel; the
    closed form is sqrt(5) ln(5)/sqrt(2) = 2.5447."""
    row = [l.split() for l in open(os.path.join(GOLDEN, "isotropic_normal_barrier.txt"))
           if l.strip() and not l.startswith("#")][0]
    d, tau0, tau, printed = int(row[0]), float(row[1]), float(row[2]), float(row[3])
    P = _gauss_problem(orc, d, 0.0, 1.0 / tau, s2_ref=1.0 / tau0)
    T, N = 200, 8000
    beta = np.linspace(0, 1, T + 1)
    r = orc.asmc(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), N, beta, 0.0, seed=2)
    _, lam, _ = orc.optimise_schedule(beta, r["log_g"], T)
    closed = np.sqrt(d) * np.log(tau / tau0) / np.sqrt(2)
    assert abs(lam[-1] - closed) < 0.04
    assert abs(lam[-1] - printed) < 0.1  # printed to two significant figures


def test_gamma_proportional_to_eta_is_exact(orc):
    """gamma = c eta makes every incremental weight constant: log Z_hat = log c
    exactly for every kernel, D_hat = 0, and the moves keep eta invariant."""
    d, N, T = 3, 6000, 12
    s2 = 2.0
    P = _gauss_problem(orc, d, 0.5, s2, m_ref=0.5, s2_ref=s2)
    logc = 0.5 * d * np.log(2 * np.pi * s2)
    beta = np.linspace(0, 1, T + 1)
    for move, eps in ((orc.MOVE_RWMH, 1.5), (orc.MOVE_MALA, 1.2), (orc.MOVE_HMC, 0.7)):
        r = orc.asmc(P, orc.Opts(move=move, leapfrog=4, state_f32=0), N, beta, eps, seed=4)
        assert abs(r["logZ"] - logc) < 1e-12
        Dhat = r["log_g"][2] - 2 * r["log_g"][1] + r["log_g"][0]
        assert np.all(np.abs(Dhat) < 1e-10)
        x = r["x"]
        assert np.all(np.abs(x.mean(0) - 0.5) < 5 * np.sqrt(s2 / N))
        assert np.all(np.abs(x.var(0) / s2 - 1) < 0.08)
        assert 0.2 < r["acc"].mean() < 1.0


@pytest.mark.parametrize("move,eps", [("RWMH", 0.9), ("MALA", 0.6), ("HMC", 0.35)])
def test_mcmc_kernels_unbiased(orc, move, eps):
    """Prop. 1 with real MH kernels: E[Z_hat] = Z only if the kernel leaves
    pi_beta invariant, so a missing MALA proposal correction, a wrong HMC
    kinetic term or a wrong annealed target biases the mean."""
    d, N, T, S = 2, 4, 3, 6000
    P = _gauss_problem(orc, d, np.array([1.5, -1.0]), 0.3, s2_ref=2.0)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 2.0, np.array([1.5, -1.0]), 0.3)
    beta = np.array([0.0, 0.2, 0.55, 1.0])
    mv = getattr(orc, "MOVE_" + move)
    r = np.array([orc.asmc(P, orc.Opts(move=mv, leapfrog=3, state_f32=0), N, beta, eps,
                           seed=s)["logZ"] for s in range(S)])
    ratio = np.exp(r - A(1.0))
    se = ratio.std() / np.sqrt(S)
    assert abs(ratio.mean() - 1) < 4.5 * se
    assert se < 0.05


@pytest.mark.parametrize("trigger", [0, 1])
def test_asmc_resampling_unbiased(orc, trigger):
    """Prop. 1 with adaptive resampling times (ESS and CESS triggers): the
    product over events of mean(w_{tau_r^-}) stays unbiased; resetting weights
    without accumulating Z_hat, or resampling before the reweight, biases it."""
    d, N, T, S = 2, 16, 6, 3000
    mu = np.array([2.0, -1.5])
    P = _gauss_problem(orc, d, mu, 0.2, s2_ref=1.0)
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, mu, 0.2)
    beta = np.linspace(0, 1, T + 1)
    runs = [orc.asmc(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, trigger=trigger,
                                 nu=0.5, state_f32=0), N, beta, 0.3, seed=s)
            for s in range(S)]
    ratio = np.exp(np.array([q["logZ"] for q in runs]) - A(1.0))
    nres = np.array([q["n_resample"] for q in runs])
    assert nres.mean() > 0.5  # the trigger fires in this configuration
    se = ratio.std() / np.sqrt(S)
    assert abs(ratio.mean() - 1) < 4.5 * se


def test_logreg_2d_quadrature(orc):
    """Brute-force quadrature of Z = int eta(x) L(x) dx for a 2-d logistic
    regression against the oracle's AIS estimate (MALA)."""
    rng = np.random.default_rng(7)
    n, d = 25, 2
    X = rng.normal(size=(n, d))
    th = np.array([1.0, -0.5])
    y = (rng.random(n) < 1 / (1 + np.exp(-X @ th))).astype(float)
    g = np.linspace(-6, 6, 801)
    G1, G2 = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([G1.ravel(), G2.ravel()], 1)
    z = pts @ X.T
    ll = np.sum(y * z - np.logaddexp(0, z), axis=1)
    le = stats.multivariate_normal(np.zeros(2), np.eye(2)).logpdf(pts)
    w = np.exp(ll + le - (ll + le).max())
    h = g[1] - g[0]
    logZ = np.log(w.sum() * h * h) + (ll + le).max()
    P = orc.Problem(family=orc.FAM_LOGREG, d=d, X=X, y=y)
    T = 64
    beta = np.linspace(0, 1, T + 1)
    r = [orc.asmc(P, orc.Opts(move=orc.MOVE_MALA, state_f32=0), 2000, beta, 0.5, seed=s)["logZ"]
         for s in range(4)]
    assert abs(np.mean(r) - logZ) < 0.02


def test_gmm_2d_quadrature(orc):
    """Quadrature of the equal-weight mixture's Z against the closed form and
    the oracle's HMC-AIS estimate."""
    d = 2
    means = np.array([[-2.0, 0.0], [2.0, 1.0], [0.0, -2.5]])
    ls = np.array([-0.5, -0.3, -0.7])
    closed = np.log(np.mean([(2 * np.pi * np.exp(2 * s)) ** (d / 2) for s in ls]))
    g = np.linspace(-7, 7, 1401)
    G1, G2 = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([G1.ravel(), G2.ravel()], 1)
    dens = np.mean([np.exp(-np.sum((pts - means[k]) ** 2, 1) / (2 * np.exp(2 * ls[k])))
                    for k in range(3)], axis=0)
    quad = np.log(dens.sum() * (g[1] - g[0]) ** 2)
    assert abs(quad - closed) < 1e-6
    P = orc.Problem(family=orc.FAM_GMM, d=d, means=means, log_scales=ls, ref_sigma2=9.0)
    T = 100
    beta = np.linspace(0, 1, T + 1) ** 2
    r = [orc.asmc(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=5, state_f32=0), 4000, beta, 0.25,
                  seed=s)["logZ"] for s in range(4)]
    assert abs(np.mean(r) - closed) < 0.05


# --------------------------------------------------------------------------- Alg. 3
def test_pchip_matches_library(orc):
    """The monotone interpolant equals scipy's PchipInterpolator (Fritsch-Carlson
    slopes with shape-preserving ends)."""
    rng = np.random.default_rng(0)
    for m in (2, 3, 4, 9, 40):
        xs = np.cumsum(rng.random(m) + 0.01)
        ys = np.cumsum(rng.random(m) * (rng.random(m) < 0.8))
        xq = np.linspace(xs[0], xs[-1], 333)
        ref = interpolate.PchipInterpolator(xs, ys)(xq)
        np.testing.assert_allclose(orc.pchip(xs, ys, xq), ref, rtol=1e-12, atol=1e-12)


def test_schedule_mean_shift_is_identity(orc):
    """Mean-shift example (eta = N(mu0, s^2), pi = N(mu1, s^2)): Lambda = |mu1 - mu0|/s
    and the optimal schedule is the identity, so Alg. 3 fed the exact D of any
    schedule returns the uniform one.  A sign error in the D_hat combination or
    interpolating beta -> Lambda instead of its inverse fails."""
    mu0, mu1, s = -0.3, 1.7, 0.8
    A = lambda b: cf.log_Z_beta(b, mu0, s * s, mu1, s * s)
    for T in (1, 5, 40):
        beta = np.linspace(0, 1, T + 1) ** 3
        D = np.array([cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1)])
        lg = np.stack([np.zeros(T), np.full(T, 0.3), 0.6 + D])
        for T_new in (1, 7, 64):
            bn, lam, st = orc.optimise_schedule(beta, lg, T_new)
            assert st == 0
            np.testing.assert_allclose(bn, np.linspace(0, 1, T_new + 1), atol=1e-9)
            assert abs(lam[-1] - abs(mu1 - mu0) / s) < 1e-9


def test_schedule_reaches_optimal_generator_c1(orc):
    """Alg. 3 with exact D on a fine schedule reproduces phi*(u) = Lambda^{-1}(Lambda u)
    for the d=10 Gaussian target (independent quadrature + root finding)."""
    d = 10
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    dl = lambda b: cf.delta_gauss(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    ref = np.array([cf.phi_star(k / 8, dl) for k in range(9)])
    assert abs(ref[2] - 0.1054253) < 1e-7 and abs(ref[4] - 0.2674865) < 1e-7
    assert abs(ref[6] - 0.5323976) < 1e-7
    err = {}
    for T in (1000, 4000):
        beta = np.linspace(0, 1, T + 1)
        D = np.array([cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1)])
        lg = np.stack([np.zeros(T), np.zeros(T), D])
        bn, lam, st = orc.optimise_schedule(beta, lg, 8)
        assert st == 0
        err[T] = np.abs(bn - ref).max()
    # sqrt(D_t) ~ sqrt(delta(beta_t)) Delta, so Lambda_hat is a Riemann sum with an
    # O(1/T) bias (Cor. 1); the error must shrink like 1/T
    assert err[4000] < 1e-4
    assert err[4000] < 0.35 * err[1000]


def test_schedule_degenerate_cases(orc):
    """D_hat = 0 everywhere gives the uniform schedule; non-finite moments give
    the uniform schedule and a non-finite status; duplicate Lambda knots are
    skipped and the result is strictly increasing with exact endpoints."""
    T = 6
    beta = np.linspace(0, 1, T + 1)
    bn, lam, st = orc.optimise_schedule(beta, np.zeros((3, T)), 5)
    assert st == 0 and np.allclose(bn, np.linspace(0, 1, 6)) and lam[-1] == 0
    lg = np.zeros((3, T))
    lg[2, 2] = np.nan
    bn, _, st = orc.optimise_schedule(beta, lg, 4)
    assert st == -4 and np.allclose(bn, np.linspace(0, 1, 5))
    lg = np.zeros((3, T))
    lg[2, [0, 4]] = [0.5, 0.2]  # D = 0 at t = 2, 3, 4, 6: repeated knots
    bn, lam, st = orc.optimise_schedule(beta, lg, 50)
    assert st == 0 and bn[0] == 0.0 and bn[-1] == 1.0 and np.all(np.diff(bn) > 0)


# --------------------------------------------------------------------------- resampling
def test_systematic_matches_searchsorted_reference(orc):
    """Ancestors equal the textbook systematic rule a_n = #{m : C_m <= (n+U)/N}
    computed with numpy searchsorted on the float CDF (ties have probability 0)."""
    rng = np.random.default_rng(1)
    for N in (1, 2, 3, 7, 8, 100, 1000):
        for _ in range(20):
            lw = rng.normal(scale=3.0, size=N)
            u = int(rng.integers(0, 2 ** 32))
            a = orc.systematic(lw, u)
            W = np.exp(lw - lw.max())
            cdf = np.cumsum(W) / W.sum()
            U = (u + 0.5) / 2 ** 32
            ref = np.searchsorted(cdf, (np.arange(N) + U) / N, side="right")
            np.testing.assert_array_equal(a, np.minimum(ref, N - 1))


def test_systematic_expected_offspring(orc):
    """Integrating the offspring count over U gives exactly N W_m (systematic
    resampling is unbiased), and every count is floor or ceil of N W_m."""
    rng = np.random.default_rng(2)
    N = 7
    lw = rng.normal(scale=1.5, size=N)
    W = np.exp(lw - lw.max())
    W /= W.sum()
    grid = 4096
    counts = np.zeros(N)
    for j in range(grid):
        u = int((j * 2 ** 32) // grid)
        c = np.bincount(orc.systematic(lw, u), minlength=N)
        assert np.all((c == np.floor(N * W)) | (c == np.ceil(N * W)))
        counts += c
    np.testing.assert_allclose(counts / grid, N * W, atol=2.0 * N / grid)


def test_systematic_degenerate(orc):
    """One finite weight takes every slot; -inf weights are never chosen."""
    lw = np.full(9, -np.inf)
    lw[4] = -3.0
    np.testing.assert_array_equal(orc.systematic(lw, 12345), np.full(9, 4))
    lw = np.array([0.0, -np.inf, 0.0, -np.inf])
    a = orc.systematic(lw, 0)
    assert set(a.tolist()) <= {0, 2}


# --------------------------------------------------------------------------- Alg. 2
def test_run_budget_and_rounds(orc):
    """Round loop: N doubles per round with T fixed (the d=10 Gaussian
    configuration), the first schedule is uniform, every round's schedule is a
    valid partition and is the Alg. 3 update of the previous round."""
    d = 10
    P = _gauss_problem(orc, d, 2.0, 0.25)
    ro = orc.RunOpts(budget=1, T1=64, eps_adapt=0, eps0=0.5 / np.sqrt(d))
    r = orc.run(P, orc.Opts(move=orc.MOVE_RWMH), ro, 128, 4, seed=9)
    assert r["status"] == 0
    assert list(r["N"]) == [128, 256, 512, 1024] and list(r["T"]) == [64] * 4
    np.testing.assert_allclose(r["beta"][0], np.linspace(0, 1, 65), atol=1e-15)
    for k in range(3):
        bn, lam, _ = orc.optimise_schedule(r["beta"][k], r["log_g"][k], 64)
        np.testing.assert_array_equal(r["beta"][k + 1], bn)
        np.testing.assert_array_equal(r["Lambda"][k], lam)
    assert np.all(np.isfinite(r["logZ"]))


def test_run_budget_rules(orc):
    """Budget: doubling T up to Tmax with N fixed, and the sqrt(2) rule."""
    d = 2
    P = _gauss_problem(orc, d, 1.0, 0.5)
    ro = orc.RunOpts(budget=2, T1=1, Tmax=12, eps_adapt=1, eps0=0.5, eps_kappa=1.0,
                     accept_target=0.65)
    r = orc.run(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=2), ro, 64, 6, seed=1)
    assert list(r["T"]) == [1, 2, 4, 8, 12, 12] and list(r["N"]) == [64] * 6
    ro = orc.RunOpts(budget=3, T1=4, Tmax=100, Nmax=300, eps0=0.5)
    r = orc.run(P, orc.Opts(move=orc.MOVE_RWMH), ro, 100, 6, seed=1)
    assert list(r["N"]) == [100, 141, 199, 281, 281, 281]
    assert list(r["T"]) == [4, 6, 8, 11, 22, 44]


# --------------------------------------------------------------------------- trigger statistics
def _lse(a, axis=0):
    m = np.max(a, axis=axis, keepdims=True)
    return np.squeeze(m, axis=axis) + np.log(np.sum(np.exp(a - m), axis=axis))


@pytest.mark.parametrize("trigger", [0, 1])
def test_ess_cess_and_events_recomputed(orc, trigger):
    """The relative ESS of w_{t^-} (AR strategy), CESS_t / N = exp(-D_hat_t)
    (eq. CESS), the moments log g_hat_{t,i}, the trigger decisions and the AR
    estimator of log Z (eq. estimator_Z) recomputed in numpy from the oracle's
    per-particle log w_{t^-} trace.  The weights before the reweight are
    w_{t-1} = w_{(t-1)^-}, or 1 after an event at t-1, so the trace fixes
    every statistic.  A wrong variant (the ESS of w_{t-1} instead of w_{t^-})
    is computed here too and must disagree, so the pin has power."""
    d, N, T = 4, 300, 8
    mu = np.array([2.0, -1.0, 1.5, 0.5])
    P = _gauss_problem(orc, d, mu, 0.02, s2_ref=1.5)
    beta = np.linspace(0, 1, T + 1) ** 2
    o = orc.asmc(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=3, resample=1, trigger=trigger, nu=0.5,
                             state_f32=1), N, beta, 0.25, seed=5, traces=True)
    assert o["status"] == 0
    lwm = o["lw_minus"]                      # [N, T]: log w_{t^-}
    res = o["resampled"]
    assert 2 <= o["n_resample"] <= T - 2     # several events, not every step
    prev = np.zeros((N, T))                  # log w_{t-1}
    for t in range(1, T):
        prev[:, t] = 0.0 if res[t - 1] else lwm[:, t - 1]
    lg = lwm - prev
    # moments
    for i in range(3):
        np.testing.assert_allclose(o["log_g"][i], _lse(prev + i * lg), rtol=0, atol=1e-10)
    # relative ESS of w_{t^-}: (sum w)^2 / (N sum w^2)
    ess = np.exp(2 * _lse(lwm) - _lse(2 * lwm) - np.log(N))
    np.testing.assert_allclose(o["ess"], ess, rtol=1e-11, atol=0)
    wrong = np.exp(2 * _lse(prev) - _lse(2 * prev) - np.log(N))
    assert np.max(np.abs(wrong - o["ess"])) > 1e-2
    # trigger decisions (none at T: the final event only closes the estimate)
    D = _lse(prev + 2 * lg) - 2 * _lse(prev + lg) + _lse(prev)
    stat = ess if trigger == 0 else np.exp(-D)
    np.testing.assert_array_equal(res[:-1], (stat[:-1] < 0.5).astype(np.int32))
    assert res[-1] == 0
    # AR estimator: sum over events (and T) of logmeanexp(log w_{tau^-})
    ev = [t for t in range(T - 1) if res[t]] + [T - 1]
    lz = sum(_lse(lwm[:, t]) - np.log(N) for t in ev)
    assert abs(lz - o["logZ"]) < 1e-10
    np.testing.assert_allclose(o["lw"], lwm[:, -1], rtol=0, atol=0)


def test_step_size_rule_recomputed(orc):
    """Step sizes across rounds (kernel adaptation between rounds): round 1 uses
    eps0 (1 + beta_t kappa)^(-1/2); round k+1 uses
    exp(L(beta)) with L the piecewise-linear function through the knots
    (beta_t^{(k)}, log eps_t^{(k)} + acc_t^{(k)} - a*), t >= 1, constant beyond
    its ends, evaluated at the new schedule.  Recomputed with numpy.interp from
    the oracle's own round outputs.  Wrong variants (knots at t/T instead of
    beta_t, the new round's acceptance instead of the old one's) must
    disagree."""
    d = 3
    P = _gauss_problem(orc, d, 1.0, 0.3, s2_ref=2.0)
    a_star, eps0, kappa = 0.65, 0.6, 3.0
    ro = orc.RunOpts(budget=2, T1=4, Tmax=32, eps_adapt=1, eps0=eps0, eps_kappa=kappa,
                     accept_target=a_star)
    r = orc.run(P, orc.Opts(move=orc.MOVE_HMC, leapfrog=3), ro, 200, 4, seed=3)
    assert r["status"] == 0 and list(r["T"]) == [4, 8, 16, 32]
    T0 = r["T"][0]
    b0 = r["beta"][0][:T0 + 1]
    np.testing.assert_allclose(r["eps"][0][:T0], eps0 / np.sqrt(1 + b0[1:] * kappa),
                               rtol=1e-15)
    far = []
    for k in range(3):
        T, Tn = r["T"][k], r["T"][k + 1]
        b, bn = r["beta"][k][:T + 1], r["beta"][k + 1][:Tn + 1]
        ky = np.log(r["eps"][k][:T]) + r["acc"][k][:T] - a_star
        want = np.exp(np.interp(bn[1:], b[1:], ky))
        np.testing.assert_allclose(r["eps"][k + 1][:Tn], want, rtol=1e-13)
        # wrong variants
        w1 = np.exp(np.interp(np.arange(1, Tn + 1) / Tn, np.arange(1, T + 1) / T, ky))
        acc_new = np.interp(bn[1:], bn[1:], r["acc"][k + 1][:Tn])
        w2 = np.exp(np.interp(bn[1:], b[1:], np.log(r["eps"][k][:T])) + acc_new - a_star)
        far.append((np.max(np.abs(w1 / want - 1)), np.max(np.abs(w2 / want - 1))))
    assert max(f[0] for f in far) > 1e-3 and max(f[1] for f in far) > 1e-3
