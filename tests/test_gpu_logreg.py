"""GPU parity of the logistic-regression path: the FP32-MFMA log-likelihood
contraction against binary64 numpy, and the MALA sweep against the oracle.

Tolerances come from the arithmetic.  The device forms z = X theta with fp32
products accumulated in fp32 (a d-term dot product), the epilogue in fp32
(exp, log, reciprocal), per-lane sums of 16 terms in fp32 and everything after
that in binary64 (log-likelihood) or fp32 (gradient, 32-row MFMA chunks plus an
8-way tree).  With u = 2^-24:
  |dz_i|   <= gamma_d sum_k |x_ik theta_k|,            gamma_d = d u / (1 - d u)
  |d ell|  <= sum_i [ |y_i - s(z_i)| |dz_i| + 4u (|term_i| + 1) ] + 16 u sum_i |term_i|
  |d g_k|  <= sum_i |x_ik| (|dz_i|/4 + 4u) + (n/8 + 40) u sum_i |r_i x_ik|
(s' <= 1/4; the last term is the fp32 accumulation over a wave's rows).
An MH decision can differ from the oracle's only when the oracle's margin
|log alpha - log u| is within a few of these errors; such particles are
excused from trajectory comparison (first_flips)."""
import numpy as np
import pytest
import torch

import oracle as orc
from parity_util import first_flips, unpack_bits
from paper_2408_12057_amd import workloads as wl

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def oa():
    import paper_2408_12057_amd as m
    assert torch.cuda.is_available()
    return m


def _bounds(X, y, theta):
    X64 = X.astype(np.float64)
    th = theta.astype(np.float64)
    n, d = X64.shape
    z = th @ X64.T                                   # [N, n]
    S = np.abs(th) @ np.abs(X64).T                   # sum_k |x_ik theta_k|
    gd = d * U32 / (1 - d * U32)
    dz = gd * S
    sig = 1 / (1 + np.exp(-z))
    term = y * z - np.logaddexp(0, z)
    r = y - sig
    b_ell = np.sum(np.abs(r) * dz + 4 * U32 * (np.abs(term) + 1), 1) + 16 * U32 * np.sum(np.abs(term), 1)
    b_g = (dz / 4 + 4 * U32) @ np.abs(X64) + (n / 8 + 40) * U32 * (np.abs(r) @ np.abs(X64))
    ell = np.sum(term, 1)
    g = r @ X64
    return ell, g, b_ell, b_g


@pytest.mark.parametrize("n,d,N", [(1000, 50, 200), (777, 7, 64), (300, 64, 65), (5000, 33, 130),
                                   (1, 1, 1),
                                   (512, 50, 100),    # no padding rows
                                   (257, 20, 70),     # one data row in the last chunk
                                   (2048, 64, 64),    # widest 64-column layout
                                   # one gradient tile (d <= 32): half-widths 16 and 12,
                                   # and the one-panel layout's (N >= 4096: tiles of 32)
                                   (700, 32, 90), (300, 29, 64), (600, 24, 4500),
                                   # panel layouts above 64 features: 2, 3 and 4 panels,
                                   # ragged panels and tiles, one data row past a chunk
                                   (1000, 80, 70), (777, 130, 33), (2000, 200, 100),
                                   (257, 65, 31), (300, 256, 40), (4096, 199, 32)])
def test_contraction_within_fp32_bound(oa, n, d, N):
    X, y, th_star = wl.logreg_data(n, d, 1000 + n + d)
    rng = np.random.default_rng(n)
    theta = (th_star[None, :] + 0.3 * rng.normal(size=(N, d))).astype(np.float32)
    prob = oa.Problem.logreg(X, y)
    ell, grad = oa.logreg_eval(prob, torch.tensor(theta, device="cuda"))
    ell = ell.cpu().numpy()
    grad = grad.cpu().numpy().astype(np.float64)
    e_ref, g_ref, b_ell, b_g = _bounds(X, y, theta)
    assert np.all(np.abs(ell - e_ref) <= b_ell), np.max(np.abs(ell - e_ref) / b_ell)
    assert np.all(np.abs(grad - g_ref) <= b_g), np.max(np.abs(grad - g_ref) / b_g)
    # and the oracle's own evaluation agrees with numpy at binary64 level
    P = orc.Problem(family=orc.FAM_LOGREG, d=d, X=X, y=y)
    v, gg = orc.ell(P, theta[0])
    assert abs(v - e_ref[0]) < 1e-9 * (1 + abs(v))
    np.testing.assert_allclose(gg, g_ref[0], rtol=1e-9, atol=1e-9)


def _eps(beta, n, d):
    return 0.5 * d ** (-1 / 6) / np.sqrt(1 + beta[1:] * n / 4)


def _round(oa, n, d, N, T, seed, subset=None, ref_mean=None, slots=0):
    X, y, _ = wl.logreg_data(n, d, 7 * n + d)
    rng = np.random.default_rng(seed)
    beta = np.concatenate([[0.0], np.sort(rng.random(T - 1)) ** 2, [1.0]])
    eps = _eps(beta, n, d)
    prob = oa.Problem.logreg(X, y, ref_mean=ref_mean)
    g = oa.asmc(prob, N, beta, eps, seed, round_k=2, move="mala", accept_bits=True, slots=slots)
    P = orc.Problem(family=orc.FAM_LOGREG, d=d, X=X, y=y, ref_mean=ref_mean)
    o = orc.asmc(P, orc.Opts(move=orc.MOVE_MALA, state_f32=1), N, beta, eps, seed, round_k=2,
                 traces=True, subset=subset)
    assert o["status"] == 0
    return X, y, beta, g, o


def _measured_errors(oa, X, y, states):
    """Observed |ell_gpu - ell| and max |grad_gpu - grad| of the FP32-MFMA
    contraction at the given binary32 states (binary64 numpy reference)."""
    prob = oa.Problem.logreg(X, y)
    st = np.ascontiguousarray(states, dtype=np.float32)
    ell, grad = oa.logreg_eval(prob, torch.tensor(st, device="cuda"))
    e_ref, g_ref, _, _ = _bounds(X, y, st)
    de = np.abs(ell.cpu().numpy() - e_ref)
    dg = np.abs(grad.cpu().numpy().astype(np.float64) - g_ref).max(1)
    return de, dg


def _check(oa, X, y, g, o, T, rows, eps):
    """rows: the particle indices the oracle ran (all, or a sample).

    Decision tolerance, measured: log alpha = beta (ell(x') - ell(x)) + the
    MALA proposal terms; at states of this run (and at reference draws) the
    contraction errs by at most
    de in ell and dg per gradient coordinate, and the proposal terms move by at
    most about eps sqrt(d) dg (the displacement is eps sqrt(d) in size), so an
    MH decision may differ from the oracle's only within
    tau = 4 (2 de + eps_max sqrt(d) dg) of its threshold.  The a-priori fp32
    bound (4 x the worst-case ell error) is reported beside it."""
    d = X.shape[1]
    xg = g["x"].cpu().numpy()[rows]
    acc_g = unpack_bits(g["accept_bits"].cpu().numpy(), T)[rows]
    # the run's end states and 64 draws from the reference, where the terms of
    # ell (and so its rounding error) are largest
    prior = np.random.default_rng(d).standard_normal((64, d))
    states = np.concatenate([xg, o["x"].astype(np.float32), prior.astype(np.float32)])
    de, dg = _measured_errors(oa, X, y, states)
    _, _, b_ell, _ = _bounds(X, y, states)
    tau = 4.0 * (2.0 * de.max() + float(np.max(eps)) * np.sqrt(d) * dg.max())
    tau_apriori = 4.0 * b_ell.max()
    excused, bad = first_flips(acc_g, o["accept"], o["margin"], tau)
    print(f"n={X.shape[0]} d={d} particles={len(rows)}: measured max|d ell|={de.max():.3e} "
          f"max|d grad|={dg.max():.3e} tau={tau:.3e} (a-priori {tau_apriori:.3e}); "
          f"excused {len(excused)} (margins {[round(m, 9) for _, _, m in excused][:6]})",
          flush=True)
    assert not bad, f"unexcused MH disagreements (particle, step, margin) tau={tau}: {bad[:5]}"
    keep = np.ones(len(rows), dtype=bool)
    for k, _, _ in excused:
        keep[k] = False
    assert len(excused) <= max(1, len(rows) // 20)
    np.testing.assert_allclose(xg[keep], o["x"][keep], rtol=1e-5, atol=1e-5)
    lwg = g["lw"].cpu().numpy()[rows]
    # log w_T = sum_t Delta beta_t ell(x_{t-1}), sum of Delta beta = 1: within
    # twice the measured ell error (states differ in the last bits)
    np.testing.assert_allclose(lwg[keep], o["lw"][keep], rtol=0, atol=4 * de.max() + 1e-9)
    # log Z_hat over the particles that followed the oracle, on both sides
    lz_g = np.logaddexp.reduce(lwg[keep]) - np.log(keep.sum())
    lz_o = np.logaddexp.reduce(o["lw"][keep]) - np.log(keep.sum())
    assert abs(lz_g - lz_o) < 4 * de.max() + 1e-9, (lz_g, lz_o)
    return excused, tau


@pytest.mark.parametrize("n,d,N,T", [(777, 50, 130, 6), (400, 7, 64, 9), (1500, 64, 70, 4),
                                     (256, 25, 1, 3),
                                     # panel layouts (tiles of 32 particles, gradients in HBM)
                                     (800, 100, 70, 5), (600, 200, 40, 4), (300, 129, 33, 3),
                                     (500, 65, 1, 3)])
def test_mala_round_matches_oracle(oa, n, d, N, T):
    X, y, beta, g, o = _round(oa, n, d, N, T, seed=n + d)
    excused, tau = _check(oa, X, y, g, o, T, np.arange(N), _eps(beta, n, d))
    if not excused:
        np.testing.assert_allclose(g["accept"], o["acc"], atol=1e-15)
        # log g_hat_{t,i} are log-sum-exps of weights within the ell bound
        np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=0, atol=2 * tau)
        assert abs(g["logZ"] - o["logZ"]) < 2 * tau


@pytest.mark.parametrize("N,d", [(4096, 50), (8000, 20), (5000, 7), (20000, 64)])
def test_one_panel_layout_when_tiles_are_few(oa, N, d):
    """Up to 64 features with 4096 <= N particles whose 64-particle tiles would
    leave CUs idle, the sweep runs the one-panel layout (tiles of 32; one
    gradient tile up to 32 features): a round against the oracle on a sample
    of particles spread over the tiles."""
    n, T = 200, 3
    rows = np.unique(np.linspace(0, N - 1, 40).astype(int))
    X, y, beta, g, o = _round(oa, n, d, N, T, seed=N + d, subset=rows)
    _check(oa, X, y, g, o, T, rows, _eps(beta, n, d))


@pytest.mark.parametrize("slots,d", [(1, 20), (3, 20), (2, 150)])
def test_mala_round_several_tiles_per_slot(oa, slots, d):
    """Tiles folded several to a moment slot (the accumulation branch the
    default slot count reaches only above 2048 tiles): 5 tiles of 64
    particles at d = 20, 10 tiles of 32 at d = 150, the last one ragged."""
    n, N, T = 600, 300, 5
    X, y, beta, g, o = _round(oa, n, d, N, T, seed=41, slots=slots)
    excused, tau = _check(oa, X, y, g, o, T, np.arange(N), _eps(beta, n, d))
    if not excused:
        np.testing.assert_allclose(g["accept"], o["acc"], atol=1e-15)
        np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=0, atol=2 * tau)
        assert abs(g["logZ"] - o["logZ"]) < 2 * tau


@pytest.mark.parametrize("d", [10, 90])
def test_mala_round_with_reference_mean(oa, d):
    rm = np.linspace(-0.5, 0.5, d).astype(np.float32)
    X, y, beta, g, o = _round(oa, 600, d, 100, 5, seed=3, ref_mean=rm)
    _check(oa, X, y, g, o, 5, np.arange(100), _eps(beta, 600, d))


def test_full_size_sampled_particles(oa):
    """The benchmark's launch configuration (N = 16384, n = 10000, d = 50) for
    one T = 32 round: sampled particles (first/last of tiles, the last
    particle) follow the oracle's trajectories; whole-population properties:
    D_hat >= 0, finite moments, acceptance in (0, 1)."""
    w = wl.logreg_n10000_d50()
    T = 32
    beta = np.linspace(0, 1, T + 1) ** 3
    eps = w.eps0 / np.sqrt(1 + beta[1:] * 10000 / 4)
    prob = oa.Problem.logreg(w.params["X"], w.params["y"])
    g = oa.asmc(prob, w.N, beta, eps, 11, round_k=1, move="mala", accept_bits=True)
    rows = np.array([0, 1, 63, 64, 5000, 8191, 12345, 16383])
    P = orc.Problem(family=orc.FAM_LOGREG, d=50, X=w.params["X"], y=w.params["y"])
    o = orc.asmc(P, orc.Opts(move=orc.MOVE_MALA, state_f32=1), w.N, beta, eps, 11, round_k=1,
                 traces=True, subset=rows)
    _check(oa, w.params["X"], w.params["y"], g, o, T, rows, eps)
    lg = g["log_g"]
    assert np.all(np.isfinite(lg))
    assert np.all(lg[2] - 2 * lg[1] + lg[0] >= -1e-9)
    assert np.all((g["accept"] > 0) & (g["accept"] <= 1))
    assert np.isfinite(g["logZ"])


def test_full_size_logZ_over_seeds(oa):
    """The benchmark's data and particle count (n = 10000, d = 50, N = 16384)
    over 8 seeds: on 16 sampled particles per seed (spread over the tiles),
    trajectories follow the oracle's within the measured decision tolerance,
    and log Z_hat over the sampled particles agrees per seed; over the seeds
    the mean difference lies within three standard errors of zero plus the
    measured contraction error.  Excused flips and the measured errors are
    printed per seed."""
    w = wl.logreg_n10000_d50()
    T = 16
    beta = np.linspace(0, 1, T + 1) ** 4
    eps = w.eps0 / np.sqrt(1 + beta[1:] * 10000 / 4)
    prob = oa.Problem.logreg(w.params["X"], w.params["y"])
    P = orc.Problem(family=orc.FAM_LOGREG, d=50, X=w.params["X"], y=w.params["y"])
    rows = np.array([0, 63, 64, 1000, 2047, 4096, 5000, 7777, 8191, 9000, 10240, 12345, 13000,
                     15000, 16320, 16383])
    diffs, tot_excused = [], 0
    for seed in range(8):
        g = oa.asmc(prob, w.N, beta, eps, 100 + seed, round_k=3, move="mala", accept_bits=True)
        o = orc.asmc(P, orc.Opts(move=orc.MOVE_MALA, state_f32=1), w.N, beta, eps, 100 + seed,
                     round_k=3, traces=True, subset=rows)
        excused, tau = _check(oa, w.params["X"], w.params["y"], g, o, T, rows, eps)
        tot_excused += len(excused)
        lwg = g["lw"].cpu().numpy()[rows]
        diffs.append((np.logaddexp.reduce(lwg) - np.log(len(rows)))
                     - (np.logaddexp.reduce(o["lw"]) - np.log(len(rows))))
        assert np.isfinite(g["logZ"])
    diffs = np.array(diffs)
    print(f"full size over 8 seeds: log Z_hat(subset) differences {diffs}; excused flips "
          f"{tot_excused} of {8 * len(rows)} particles", flush=True)
    se = diffs.std(ddof=1) / np.sqrt(len(diffs))
    assert abs(diffs.mean()) <= 3 * se + 1e-6
