"""Pins of the oracle's pathwise gradient of log Z_hat (mixture target, MALA,
accept decisions held fixed) against finite differences and a closed form."""
import numpy as np
import pytest


def _gmm(orc, th, K, d, ref_s2):
    return orc.Problem(family=orc.FAM_GMM, d=d, means=th[:K * d].reshape(K, d),
                       log_scales=th[K * d:], ref_sigma2=ref_s2)


def test_mixture_derivatives_match_finite_differences(orc):
    """Hessian of ell in x, d grad ell / d theta and d ell / d theta against
    central differences of the oracle's own ell and gradient (a wrong sign or a
    dropped responsibility term fails)."""
    rng = np.random.default_rng(0)
    d, K = 4, 3
    th = np.concatenate([rng.normal(size=K * d), rng.uniform(-0.4, 0.3, size=K)])
    P = _gmm(orc, th, K, d, 4.0)
    x = rng.normal(size=d)
    H, M, dl = orc.gmm_derivs(P, x)
    h = 1e-6
    Hfd = np.array([(orc.ell(P, x + h * e)[1] - orc.ell(P, x - h * e)[1]) / (2 * h)
                    for e in np.eye(d)]).T
    np.testing.assert_allclose(H, Hfd, atol=1e-8)
    np.testing.assert_allclose(H, H.T, atol=1e-12)
    for c in range(th.size):
        e = np.zeros_like(th)
        e[c] = h
        vp, gp = orc.ell(_gmm(orc, th + e, K, d, 4.0), x)
        vm, gm = orc.ell(_gmm(orc, th - e, K, d, 4.0), x)
        np.testing.assert_allclose(M[:, c], (gp - gm) / (2 * h), atol=1e-8)
        assert abs(dl[c] - (vp - vm) / (2 * h)) < 1e-8


def test_logZ_gradient_matches_replayed_mask_differences(orc):
    """The forward-mode gradient equals central differences of log Z_hat at
    theta +- h with the same random numbers and the same accept decisions
    replayed (the exact derivative of the piecewise-smooth estimator)."""
    rng = np.random.default_rng(1)
    d, K, N, T = 3, 2, 40, 10
    th = np.concatenate([rng.normal(size=K * d), np.array([0.1, -0.3])])
    P = _gmm(orc, th, K, d, 4.0)
    beta = np.linspace(0, 1, T + 1) ** 2
    eps = 1.3
    O = orc.Opts(move=orc.MOVE_MALA, state_f32=0)
    lz, g, acc = orc.logZ_grad(P, O, N, beta, eps, seed=3, want_accept=True)
    assert 0.2 < acc.mean() < 0.95  # both branches of the mask occur
    r = orc.asmc(P, O, N, beta, eps, seed=3)
    assert abs(r["logZ"] - lz) < 1e-12
    O2 = orc.Opts(move=orc.MOVE_MALA, state_f32=0, force_accept=acc)
    hh = 1e-5
    for c in range(th.size):
        e = np.zeros_like(th)
        e[c] = hh
        lp = orc.asmc(_gmm(orc, th + e, K, d, 4.0), O2, N, beta, eps, seed=3)["logZ"]
        lm = orc.asmc(_gmm(orc, th - e, K, d, 4.0), O2, N, beta, eps, seed=3)["logZ"]
        assert abs((lp - lm) / (2 * hh) - g[c]) < 1e-7 * max(1.0, abs(g[c]))


def test_logZ_gradient_single_component_closed_form(orc):
    """K = 1, s = 0: log Z = (d/2) log(2 pi e^{2s}), so d/ds = d and d/dmu = 0.
    The pathwise estimator is biased at finite N and T; its mean over seeds
    must approach the closed form (statistical check)."""
    d = 2
    P = orc.Problem(family=orc.FAM_GMM, d=d, means=np.array([[1.0, -1.0]]),
                    log_scales=np.array([0.0]), ref_sigma2=9.0)
    T = 64
    beta = np.linspace(0, 1, T + 1) ** 3
    eps = 0.5 / np.sqrt(1 + 8 * beta[1:])
    gs = np.array([orc.logZ_grad(P, orc.Opts(move=orc.MOVE_MALA), 2000, beta, eps, seed=s)[1]
                   for s in range(6)])
    m = gs.mean(0)
    assert abs(m[2] - d) < 0.05
    assert np.all(np.abs(m[:2]) < 0.05)
