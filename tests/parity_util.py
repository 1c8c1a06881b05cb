"""Helpers for GPU-vs-oracle comparisons (no method arithmetic here)."""
import numpy as np

import oracle as orc
from paper_2408_12057_amd import workloads as wl


def unpack_bits(bits: np.ndarray, T: int) -> np.ndarray:
    """accept_bits [N, ceil(T/32)] int32 -> bool [N, T]."""
    b = bits.astype(np.uint32)
    out = np.zeros((b.shape[0], T), dtype=bool)
    for t in range(T):
        out[:, t] = (b[:, t // 32] >> np.uint32(t % 32)) & np.uint32(1)
    return out


def first_flips(gpu_acc: np.ndarray, orc_acc: np.ndarray, margin: np.ndarray, tol: float):
    """Particles whose accept sequences differ; each difference must sit at a
    decision whose oracle margin |log alpha - log u| is below tol (excused)."""
    diff = gpu_acc != orc_acc.astype(bool)
    bad = []
    excused = []
    for n in np.nonzero(diff.any(1))[0]:
        t = int(np.argmax(diff[n]))
        (excused if abs(margin[n, t]) < tol else bad).append((int(n), t, float(margin[n, t])))
    return excused, bad


def oracle_problem(family: str, d: int, params: dict, ref_sigma2: float, ref_mean=None):
    if family == "gauss":
        return orc.Problem(family=orc.FAM_GAUSS, d=d, mu=params["mu"], sigma2=params["sigma2"],
                           ref_mean=ref_mean, ref_sigma2=ref_sigma2)
    if family == "gmm":
        return orc.Problem(family=orc.FAM_GMM, d=d, means=params["means"],
                           log_scales=params["log_scales"], ref_mean=ref_mean,
                           ref_sigma2=ref_sigma2)
    return orc.Problem(family=orc.FAM_LOGREG, d=d, X=params["X"], y=params["y"],
                       ref_mean=ref_mean, ref_sigma2=ref_sigma2)


def gpu_problem(oa, family: str, params: dict, ref_sigma2: float, ref_mean=None):
    if family == "gauss":
        return oa.Problem.gauss(params["mu"], params["sigma2"], ref_sigma2, ref_mean)
    if family == "gmm":
        return oa.Problem.gmm(params["means"], params["log_scales"], ref_sigma2, ref_mean)
    return oa.Problem.logreg(params["X"], params["y"], ref_sigma2, ref_mean)


ORC_MOVE = {"rwmh": orc.MOVE_RWMH, "mala": orc.MOVE_MALA, "hmc": orc.MOVE_HMC}


def compare_round(g, o, T, N, flip_tol=1e-9, rtol_lw=1e-12, exact=True):
    """GPU pass ``g`` against the oracle pass ``o`` (traces on): MH decisions
    equal except excused flips; states (bitwise, or within 1e-5 relative) and
    final log-weights of the particles that followed the oracle; moments,
    acceptance and log Z_hat when nothing was excused.  Returns the number of
    excused particles."""
    acc_g = unpack_bits(g["accept_bits"].cpu().numpy(), T)
    excused, bad = first_flips(acc_g, o["accept"], o["margin"], flip_tol)
    assert not bad, f"unexcused MH disagreements (particle, step, margin): {bad[:5]}"
    keep = np.ones(N, dtype=bool)
    for n, _, _ in excused:
        keep[n] = False
    xg = g["x"].cpu().numpy().astype(np.float64)
    lwg = g["lw"].cpu().numpy()
    if exact:
        np.testing.assert_array_equal(xg[keep], o["x"][keep])
    else:
        np.testing.assert_allclose(xg[keep], o["x"][keep], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(lwg[keep], o["lw"][keep], rtol=rtol_lw, atol=rtol_lw)
    if not excused:
        np.testing.assert_allclose(g["log_g"], o["log_g"], rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(g["accept"], o["acc"], rtol=0, atol=1e-15)
        # relative to the size of log Z_hat: binary64 sums of log-weights of
        # magnitude |log Z_hat| carry rounding of that relative size
        assert abs(g["logZ"] - o["logZ"]) < 1e-10 * max(1.0, abs(o["logZ"]))
    return len(excused)
