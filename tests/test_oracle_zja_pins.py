"""Pins of the oracle's pieces for the paper's GPU comparison (Sec.
"High-performance GPU implementation of adaptive schemes"): the Unid target
(unidentifiable product parameterisation), the alternating three-scale RWMH
kernel, and the online CESS-adaptive AIS of Zhou, Johansen and Aston (ZJA).

What pins them: the binomial log-likelihood from scipy and in extended
precision; the evidence of the Unid model reduced to a one-dimensional
integral (checked against a two-dimensional grid) and its large-n Laplace
form; unbiasedness of Z_hat (Prop. 1) with the three-scale kernel; chains of
that kernel at beta = 1 reproducing a Gaussian target; for ZJA the defining
property (CESS_t = rho N at every step but the last) recomputed from its
moments, and, under the exact kernel, its schedule converging to the optimal
one phi* of the dense-schedule analysis (Sec. "Connection to online
conditional ESS optimisation").
"""
import numpy as np
import pytest
from scipy import integrate, stats

import closed_forms as cf

PHI_STAR = {0.25: 0.1054253, 0.5: 0.2674865, 0.75: 0.5323976}  # c1 target, closed form


def _unid(orc, n, k, box=10.0):
    return orc.Problem(family=orc.FAM_UNID, d=2, binom_n=float(n), binom_k=float(k), box=box)


def _log_z_unid(n, k, box=10.0):
    """log Z for the Unid model with the likelihood divided by its maximum:
    Z = box^-2 int_0^1 f(u) log(box^2 / u) du, f(u) = (u/p)^k ((1-u)/(1-p))^(n-k),
    after integrating x out along u = x y (|dy| = du / x, x from u/box to box)."""
    p = k / n
    sd = np.sqrt(p * (1 - p) / n)
    lo, hi = max(1e-300, p - 60 * sd), min(1.0, p + 60 * sd)

    def f(u):
        return np.exp(k * np.log(u / p) + (n - k) * np.log1p(-u) - (n - k) * np.log1p(-p))

    val, _ = integrate.quad(lambda u: f(u) * np.log(box * box / u), lo, hi, points=[p],
                            limit=400, epsabs=0, epsrel=1e-10)
    return np.log(val) - 2 * np.log(box)


# --------------------------------------------------------------------------- Unid target
def test_unid_ell_matches_binomial_and_extended_precision(orc):
    rng = np.random.default_rng(1)
    P = _unid(orc, 1e4, 5e3)
    for _ in range(50):
        x = rng.uniform(0.05, 10, 2)
        u = x[0] * x[1]
        v = orc.ell(P, x)[0]
        if u >= 1:
            assert v == -np.inf
            continue
        ref = stats.binom.logpmf(5000, 10000, u) - stats.binom.logpmf(5000, 10000, 0.5)
        assert abs(v - ref) < 1e-8 * max(1.0, abs(ref))
    # the paper's GPU parameters: n = 1e11, k = 1e10, near the ridge x y = 0.1
    n, k = 1e11, 1e10
    P = _unid(orc, n, k)
    L = np.longdouble
    for _ in range(50):
        x0 = rng.uniform(0.02, 10)
        x = np.array([x0, (0.1 + rng.normal() * 3e-6) / x0])
        u = x[0] * x[1]
        pl = L(k) / L(n)
        ref = L(k) * np.log(L(u) / pl) + (L(n) - L(k)) * np.log((1 - L(u)) / (1 - pl))
        assert abs(orc.ell(P, x)[0] - float(ref)) < 1e-6
    assert orc.ell(P, np.array([11.0, 0.01]))[0] == -np.inf  # outside the reference's support


def test_unid_evidence_reduction_and_laplace_form():
    """The one-dimensional form of log Z against a brute-force two-dimensional
    grid (small n), and against its Laplace form at the paper's n = 1e11."""
    n, k, box = 40, 20, 10.0
    g = np.linspace(0, box, 4001)[1:]
    xx, yy = np.meshgrid(g, g)
    u = xx * yy
    f = np.where(u < 1, (u / 0.5) ** k * ((1 - np.minimum(u, 1)) / 0.5) ** (n - k), 0.0)
    z2 = f.sum() * (g[1] - g[0]) ** 2 / box ** 2
    assert abs(np.log(z2) - _log_z_unid(n, k, box)) < 5e-3
    n, k = 1e11, 1e10
    p = k / n
    lap = np.log(np.log(box * box / p)) - 2 * np.log(box) + 0.5 * np.log(2 * np.pi * p * (1 - p) / n)
    assert abs(_log_z_unid(n, k, box) - lap) < 1e-6


def test_unid_init_is_uniform_on_the_box(orc):
    """X_0 ~ Uniform(0, 10)^2: with the identity kernel the final states are the
    initial draws; moments and a KS test of each coordinate."""
    P = _unid(orc, 1e4, 5e3)
    r = orc.asmc(P, orc.Opts(move=orc.MOVE_IDENTITY, state_f32=1), 20000, np.array([0.0, 1.0]),
                 0.1, seed=3)
    for i in range(2):
        assert stats.kstest(r["x"][:, i] / 10.0, "uniform").pvalue > 1e-3


def test_unid_oais_unbiased_with_three_scale_kernel(orc):
    """Prop. 1 on the Unid model (n = 1000, k = 500): E[Z_hat] matches the
    quadrature of the evidence, with the alternating three-scale RWMH kernel."""
    n, k = 1000, 500
    P = _unid(orc, n, k)
    logZ = _log_z_unid(n, k)
    T, N, S = 32, 256, 200
    beta = np.linspace(0, 1, T + 1) ** 3
    lz = np.array([orc.asmc(P, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), N, beta, 0.2,
                            seed=s)["logZ"] for s in range(S)])
    ratio = np.exp(lz - logZ)
    assert abs(ratio.mean() - 1) < 4.5 * ratio.std() / np.sqrt(S)


# --------------------------------------------------------------------------- three-scale kernel
def test_three_scale_kernel_is_target_invariant(orc):
    """Chains of the three-scale kernel at beta = 1 reproduce the moments of the
    d = 10 Gaussian target (mean 2, variance 0.25)."""
    d = 10
    P = orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.full(d, 2.0), sigma2=0.25)
    beta = np.linspace(0, 1, 129) ** 2
    fin = orc.asmc(P, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), 256, beta, 0.3, 4)
    r = orc.rejuvenate(P, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1), fin["lw"], fin["x"], 400,
                       0.3, 4)
    np.testing.assert_allclose(r["mean"], 2.0, atol=0.04)
    np.testing.assert_allclose(r["second"] - r["mean"] ** 2, 0.25, atol=0.04)


# --------------------------------------------------------------------------- ZJA
def test_zja_holds_cess_at_rho(orc):
    """Every step but the last has CESS_t / N = rho (to the bisection's
    resolution) and the last has CESS_T >= rho N, recomputed from the returned
    moments; beta increases strictly to 1."""
    d = 10
    P = orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.full(d, 2.0), sigma2=0.25)
    rho = 0.97
    r = orc.zja(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1), 2048, rho, 400, 0.15, seed=1)
    assert r["status"] == 0
    T, lg = r["T"], r["log_g"]
    assert 10 < T < 400 and r["beta"][T] == 1.0 and np.all(np.diff(r["beta"]) > 0)
    log_cess = 2 * lg[1] - lg[2] - lg[0]
    np.testing.assert_allclose(log_cess[:-1], np.log(rho), atol=1e-7)
    assert log_cess[-1] >= np.log(rho) - 1e-12


def test_zja_schedule_converges_to_optimal_under_exact_kernel(orc):
    """With the exact kernel and N = 2^14 the ZJA schedule approaches the
    optimal schedule phi* (both equalise the step discrepancy), and its length
    approaches Lambda / sqrt(-log rho) with Lambda = 9.0034 (c1 target)."""
    d = 10
    P = orc.Problem(family=orc.FAM_GAUSS, d=d, mu=np.full(d, 2.0), sigma2=0.25)
    Lam = 9.0033663
    rho = np.exp(-(Lam / 64) ** 2)
    r = orc.zja(P, orc.Opts(move=orc.MOVE_EXACT, state_f32=0), 1 << 14, rho, 200, 0.0, seed=7)
    T = r["T"]
    assert abs(T - 64) <= 3
    for u, b in PHI_STAR.items():
        assert abs(np.interp(u * T, np.arange(T + 1), r["beta"]) - b) < 0.02


def test_zja_stops_at_tmax(orc):
    P = orc.Problem(family=orc.FAM_GAUSS, d=10, mu=np.full(10, 2.0), sigma2=0.25)
    r = orc.zja(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1), 256, 0.999, 12, 0.15, seed=2)
    assert r["T"] == 12 and r["beta"][12] == 1.0 and r["beta"][11] < 0.5
