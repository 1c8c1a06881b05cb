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
