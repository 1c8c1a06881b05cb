"""Closed forms used to pin the oracle (test helper, independent of the oracle's code).

For the linear path pi_beta ∝ eta^{1-beta} gamma^beta with Gaussian eta and
Gaussian-shaped gamma, A(beta) = log Z_beta is a Gaussian integral.  The
incremental discrepancy of an MCMC (or exact) forward kernel is the discrete
second difference of A (appendix example "MCMC kernels with Linear path"),
the local barrier is delta = A'' and the global barrier is the integral of
sqrt(delta) (dense-schedule limit).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, optimize


def log_Z_beta(beta, m_ref, s2_ref, mu, s2_tgt):
    """A(beta) for eta = N(m_ref, s2_ref I) (normalised) and
    gamma(x) = exp(-|x - mu|^2 / (2 s2_tgt)) (unnormalised), per-coordinate sums."""
    beta = np.asarray(beta, dtype=np.float64)
    m_ref = np.atleast_1d(np.asarray(m_ref, dtype=np.float64))
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    a = (1.0 - beta) / s2_ref
    b = beta / s2_tgt
    lam = a + b
    d = max(m_ref.shape[0], mu.shape[0])
    diff2 = np.sum((np.broadcast_to(m_ref, (d,)) - np.broadcast_to(mu, (d,))) ** 2)
    # integral of exp(-a (x-m)^2/2 - b (x-mu)^2/2) = sqrt(2 pi / lam) exp(-ab/(2 lam) (m-mu)^2)
    out = d * (0.5 * np.log(2 * np.pi / lam) - 0.5 * (1.0 - beta) * np.log(2 * np.pi * s2_ref))
    out = out - 0.5 * a * b / lam * diff2
    return out


def discrepancy(beta_prev, beta_next, A):
    """D(beta, beta') = A(beta' + Delta) + A(beta' - Delta) - 2 A(beta')."""
    dl = beta_next - beta_prev
    return A(beta_next + dl) + A(beta_prev) - 2.0 * A(beta_next)


def local_barrier(beta, A, h=1e-4):
    """delta(beta) = A''(beta) by a central difference of the closed form."""
    return (A(beta + h) - 2 * A(beta) + A(beta - h)) / (h * h)


def delta_gauss(beta, m_ref, s2_ref, mu, s2_tgt):
    """Exact A''(beta): Var_beta[V] with V = log gamma - log eta, for the Gaussian case."""
    m_ref = np.atleast_1d(np.asarray(m_ref, dtype=np.float64))
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    d = max(m_ref.shape[0], mu.shape[0])
    m_ref = np.broadcast_to(m_ref, (d,))
    mu = np.broadcast_to(mu, (d,))
    # V(x) = -(x-mu)^2/(2 s2t) + (x-m)^2/(2 s2r) + c  = q x^2 + l x + c per coordinate
    q = -0.5 / s2_tgt + 0.5 / s2_ref
    lin = mu / s2_tgt - m_ref / s2_ref
    lam = (1 - beta) / s2_ref + beta / s2_tgt
    mean = ((1 - beta) * m_ref / s2_ref + beta * mu / s2_tgt) / lam
    var = 1.0 / lam
    # Var[q x^2 + l x] for x ~ N(mean, var): 2 q^2 var^2 + (2 q mean + l)^2 var
    return float(np.sum(2 * q * q * var * var + (2 * q * mean + lin) ** 2 * var))


def global_barrier(delta):
    val, _ = integrate.quad(lambda b: np.sqrt(delta(b)), 0.0, 1.0, limit=200, epsabs=1e-12,
                            epsrel=1e-12)
    return val


def phi_star(u, delta):
    """Optimal schedule generator Lambda^{-1}(Lambda u)."""
    Lam = global_barrier(delta)

    def cum(b):
        return integrate.quad(lambda s: np.sqrt(delta(s)), 0.0, b, limit=200, epsabs=1e-13,
                              epsrel=1e-13)[0]

    return optimize.brentq(lambda b: cum(b) - Lam * u, 0.0, 1.0, xtol=1e-14)
