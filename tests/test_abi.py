"""The C-ABI library: it loads, exports every entry point include/oasmc.h
declares, and its host-side schedule optimiser (Alg. 3) agrees with the oracle.
No device work runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import closed_forms as cf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oasmc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oasmc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2408_12057_amd as oa
    path = oa.library_path()
    if not os.path.exists(path):
        from paper_2408_12057_amd import build
        build.build()
    return ctypes.CDLL(path)


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert {"oasmc_asmc", "oasmc_run", "oasmc_adapt_schedule", "oasmc_resample"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_last_error_initially_empty(lib):
    lib.oasmc_last_error.restype = ctypes.c_char_p
    assert lib.oasmc_last_error() is not None


@pytest.mark.parametrize("T,T_new,interp", [(1, 1, 0), (1, 9, 0), (7, 16, 0), (40, 13, 0),
                                           (40, 64, 1), (300, 1000, 0)])
def test_adapt_schedule_matches_oracle(orc, T, T_new, interp):
    """Alg. 3 on the host (product) against the oracle's independent code on
    random moments, including repeated knots (D = 0 steps)."""
    import paper_2408_12057_amd as oa
    rng = np.random.default_rng(T * 131 + T_new)
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)), [1.0]]) if T > 1 else np.array([0, 1.0])
    D = rng.gamma(0.5, 0.2, size=T)
    D[rng.random(T) < 0.1] = 0.0
    lg0 = rng.normal(size=T)
    lg1 = rng.normal(size=T)
    lg = np.stack([lg0, lg1, D + 2 * lg1 - lg0])
    bn, lam = oa.adapt_schedule(beta, lg, T_new, interp)
    ob, olam, st = orc.optimise_schedule(beta, lg, T_new, interp)
    np.testing.assert_allclose(lam, olam, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(bn, ob, rtol=1e-12, atol=1e-13)
    assert bn[0] == 0.0 and bn[-1] == 1.0 and np.all(np.diff(bn) > 0)


def test_adapt_schedule_optimal_generator(orc):
    """The product's Alg. 3 fed exact D reproduces phi*(u) of the d=10 Gaussian
    target to the O(1/T) accuracy of the cumulative barrier."""
    import paper_2408_12057_amd as oa
    d, T = 10, 4000
    A = lambda b: cf.log_Z_beta(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    dl = lambda b: cf.delta_gauss(b, np.zeros(d), 1.0, np.full(d, 2.0), 0.25)
    beta = np.linspace(0, 1, T + 1)
    D = np.array([cf.discrepancy(beta[t - 1], beta[t], A) for t in range(1, T + 1)])
    bn, lam = oa.adapt_schedule(beta, np.stack([np.zeros(T), np.zeros(T), D]), 4)
    ref = [cf.phi_star(k / 4, dl) for k in range(5)]
    np.testing.assert_allclose(bn, ref, atol=1e-4)
    # Lambda_hat is a right Riemann sum of sqrt(delta): bias (sqrt(delta(0)) - sqrt(delta(1)))/(2T)
    assert abs(lam[-1] - 9.0033663) < 12.0 / T


def test_adapt_schedule_rejects_bad_input():
    import paper_2408_12057_amd as oa
    with pytest.raises(oa.OasmcError):
        oa.adapt_schedule(np.array([0.0, 0.7, 0.5, 1.0]), np.zeros((3, 3)), 4)
    with pytest.raises(oa.OasmcError):
        oa.adapt_schedule(np.array([0.1, 1.0]), np.zeros((3, 1)), 4)


@pytest.mark.parametrize("T,T_new,interp,nu", [(1, 8, 0, 0.5), (7, 16, 0, 0.5), (40, 64, 1, 0.7),
                                              (40, 80, 0, 0.3), (300, 1000, 0, 0.5)])
def test_dar_times_match_oracle(orc, T, T_new, interp, nu):
    """DAR resampling times (eq. (DAR-times)) on the host, product against the
    oracle's independent code: predicted discrepancies to rounding, identical
    event flags, on random moments and random new schedules."""
    import paper_2408_12057_amd as oa
    rng = np.random.default_rng(T * 7 + T_new)
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)), [1.0]]) if T > 1 else np.array([0, 1.0])
    bn = np.concatenate([[0.0], np.sort(rng.random(T_new - 1)), [1.0]])
    D = rng.gamma(0.5, 2.0 * T_new / T / T_new, size=T) * 10
    D[rng.random(T) < 0.1] = 0.0
    lg0, lg1 = rng.normal(size=T), rng.normal(size=T)
    lg = np.stack([lg0, lg1, D + 2 * lg1 - lg0])
    f, Dp = oa.dar_times(beta, lg, bn, nu, interp)
    of, oDp, st = orc.dar_times(beta, lg, bn, nu, interp)
    assert st == 0
    np.testing.assert_allclose(Dp, oDp, rtol=1e-11, atol=1e-14)
    np.testing.assert_array_equal(f, of.astype(np.int32))
    assert f[-1] == 0
