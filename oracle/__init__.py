"""Plain fp64 CPU oracle for Optimised Annealed SMC / OAIS (arXiv 2408.12057).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2408_12057_amd``) never imports it, and it imports nothing
from the product.

The numerical work lives in ``oasmc_oracle.c`` (plain C, binary64, OpenMP over
independent particles).  This module only marshals numpy arrays through
``ctypes``.  Which section of the paper each C function follows is stated in
that file's header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oasmc_oracle.c")
_LIB = os.path.join(_HERE, "liboasmc_oracle.so")

FAM_GAUSS, FAM_LOGREG, FAM_GMM, FAM_UNID = 1, 2, 3, 4
MOVE_RWMH, MOVE_MALA, MOVE_HMC, MOVE_EXACT, MOVE_IDENTITY, MOVE_RWMH3 = 1, 2, 3, 4, 5, 6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


class _Problem(C.Structure):
    _fields_ = [
        ("family", C.c_int), ("d", C.c_int),
        ("mu", C.c_void_p), ("sigma2", C.c_double),
        ("X", C.c_void_p), ("y", C.c_void_p), ("n", C.c_int),
        ("K", C.c_int), ("means", C.c_void_p), ("log_scales", C.c_void_p),
        ("ref_mean", C.c_void_p), ("ref_sigma2", C.c_double),
        ("binom_n", C.c_double), ("binom_k", C.c_double), ("box", C.c_double),
    ]


class _Opts(C.Structure):
    _fields_ = [
        ("move", C.c_int), ("leapfrog", C.c_int), ("resample", C.c_int),
        ("trigger", C.c_int), ("nu", C.c_double), ("state_f32", C.c_int),
        ("nthreads", C.c_int), ("force_accept", C.c_void_p), ("resample_at", C.c_void_p),
    ]


class _RunOpts(C.Structure):
    _fields_ = [
        ("budget", C.c_int), ("T1", C.c_int), ("Tmax", C.c_int), ("Nmax", C.c_int64),
        ("eps_adapt", C.c_int), ("eps0", C.c_double), ("eps_kappa", C.c_double),
        ("accept_target", C.c_double), ("interp", C.c_int), ("dar", C.c_int),
    ]


_dp = C.POINTER(C.c_double)


def _declare(L):
    L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                    C.POINTER(C.c_uint32)]
    L.orc_philox4x32_10.restype = None
    L.orc_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_uint32, C.c_uint32, C.c_int, _dp]
    L.orc_normals.restype = None
    L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_uint32, C.c_uint32]
    L.orc_uniform.restype = C.c_double
    L.orc_systematic.argtypes = [C.c_int64, _dp, C.c_uint32, C.POINTER(C.c_int32)]
    L.orc_systematic.restype = C.c_int
    L.orc_pchip_eval.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, _dp]
    L.orc_pchip_eval.restype = None
    L.orc_optimise_schedule.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_int, _dp, _dp]
    L.orc_optimise_schedule.restype = C.c_int
    L.orc_asmc.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_int64, C.c_int, _dp, _dp,
                           C.c_uint64, C.c_uint32, C.c_uint32, _dp, _dp, _dp, _dp, _dp,
                           C.POINTER(C.c_int), C.POINTER(C.c_ubyte), _dp, C.POINTER(C.c_int),
                           _dp, C.POINTER(C.c_int64), C.c_int64, _dp]
    L.orc_asmc.restype = C.c_int
    L.orc_run.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.POINTER(_RunOpts), C.c_int64,
                          C.c_int, C.c_uint64, C.c_uint32, C.c_int, _dp,
                          C.POINTER(C.c_int64), C.POINTER(C.c_int), _dp, _dp, _dp, _dp, _dp,
                          C.POINTER(C.c_int)]
    L.orc_run.restype = C.c_int
    L.orc_ell.argtypes = [C.POINTER(_Problem), _dp, _dp]
    L.orc_ell.restype = C.c_double
    L.orc_gmm_derivs.argtypes = [C.POINTER(_Problem), _dp, _dp, _dp, _dp]
    L.orc_gmm_derivs.restype = None
    L.orc_logZ_grad.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_int64, C.c_int, _dp,
                                _dp, C.c_uint64, C.c_uint32, C.c_uint32, _dp,
                                C.POINTER(C.c_double), C.POINTER(C.c_ubyte)]
    L.orc_logZ_grad.restype = C.c_int
    L.orc_dar_times.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, C.c_int, C.c_double,
                                C.POINTER(C.c_ubyte), _dp]
    L.orc_dar_times.restype = C.c_int
    L.orc_rejuvenate.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_int64, C.c_int,
                                 C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, _dp, _dp, _dp,
                                 _dp, _dp, _dp]
    L.orc_rejuvenate.restype = C.c_int
    L.orc_zja.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_int64, C.c_double, C.c_int,
                          C.c_int, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, _dp,
                          C.POINTER(C.c_int), _dp, _dp, _dp, _dp]
    L.orc_zja.restype = C.c_int
    L.orc_pt.argtypes = [C.POINTER(_Problem), C.POINTER(_Opts), C.c_int, C.c_int, C.c_int, _dp,
                         _dp, C.c_uint64, C.c_uint32, C.c_uint32, _dp, _dp, _dp,
                         C.POINTER(C.c_int64), _dp, _dp]
    L.orc_pt.restype = C.c_int


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray], t=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(t)


@dataclass
class Problem:
    """A target family plus the Gaussian reference eta = N(ref_mean, ref_sigma2 I).

    Arrays are converted to float64 (fp32 inputs convert exactly)."""
    family: int
    d: int
    mu: Optional[np.ndarray] = None
    sigma2: float = 1.0
    X: Optional[np.ndarray] = None
    y: Optional[np.ndarray] = None
    means: Optional[np.ndarray] = None
    log_scales: Optional[np.ndarray] = None
    ref_mean: Optional[np.ndarray] = None
    ref_sigma2: float = 1.0
    binom_n: float = 0.0   # FAM_UNID: Binomial(k | n, x y) likelihood, uniform (0, box)^2 reference
    binom_k: float = 0.0
    box: float = 10.0
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Problem:
        P = _Problem()
        P.family = self.family
        P.d = self.d
        keep = []

        def arr(a):
            if a is None:
                return None
            b = _f64(a)
            keep.append(b)
            return b.ctypes.data

        P.mu = arr(self.mu)
        P.sigma2 = float(self.sigma2)
        P.X = arr(self.X)
        P.y = arr(self.y)
        P.n = 0 if self.X is None else int(np.asarray(self.X).shape[0])
        P.K = 0 if self.means is None else int(np.asarray(self.means).shape[0])
        P.means = arr(self.means)
        P.log_scales = arr(self.log_scales)
        P.ref_mean = arr(self.ref_mean)
        P.ref_sigma2 = float(self.ref_sigma2)
        P.binom_n, P.binom_k, P.box = float(self.binom_n), float(self.binom_k), float(self.box)
        self._keep = keep
        return P


@dataclass
class Opts:
    move: int = MOVE_RWMH
    leapfrog: int = 5
    resample: int = 0
    trigger: int = 0
    nu: float = 0.5
    state_f32: int = 1
    nthreads: int = 0
    force_accept: Optional[np.ndarray] = None  # uint8 [N, T]: replayed MH decisions (AIS)
    resample_at: Optional[np.ndarray] = None   # trigger 3: [T], 1 = resample after step t

    def c(self) -> _Opts:
        fa = ra = None
        if self.force_accept is not None:
            self._fa = np.ascontiguousarray(self.force_accept, dtype=np.uint8)
            fa = self._fa.ctypes.data
        if self.resample_at is not None:
            self._ra = np.ascontiguousarray(self.resample_at, dtype=np.uint8)
            ra = self._ra.ctypes.data
        return _Opts(self.move, self.leapfrog, self.resample, self.trigger, self.nu,
                     self.state_f32, self.nthreads, fa, ra)


@dataclass
class RunOpts:
    budget: int = 1
    T1: int = 64
    Tmax: int = 0
    Nmax: int = 1 << 40
    eps_adapt: int = 0
    eps0: float = 0.1
    eps_kappa: float = 0.0
    accept_target: float = 0.574
    interp: int = 0
    dar: int = 0

    def c(self) -> _RunOpts:
        return _RunOpts(self.budget, self.T1, self.Tmax, self.Nmax, self.eps_adapt, self.eps0,
                        self.eps_kappa, self.accept_target, self.interp, self.dar)


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals(seed, round_k, problem, n, t, stream, substep, count) -> np.ndarray:
    z = np.zeros(count)
    lib().orc_normals(seed, round_k, problem, n, t, stream, substep, count, _ptr(z))
    return z


def uniform(seed, round_k, problem, n, t, stream, substep) -> float:
    return lib().orc_uniform(seed, round_k, problem, n, t, stream, substep)


def systematic(lw, u: int) -> np.ndarray:
    lw = _f64(lw)
    a = np.zeros(lw.shape[0], dtype=np.int32)
    st = lib().orc_systematic(lw.shape[0], _ptr(lw), int(u) & 0xFFFFFFFF,
                              a.ctypes.data_as(C.POINTER(C.c_int32)))
    if st != 0:
        raise RuntimeError(f"orc_systematic status {st}")
    return a


def pchip(xs, ys, xq) -> np.ndarray:
    xs, ys, xq = _f64(xs), _f64(ys), _f64(xq)
    yq = np.zeros_like(xq)
    lib().orc_pchip_eval(xs.shape[0], _ptr(xs), _ptr(ys), xq.shape[0], _ptr(xq), _ptr(yq))
    return yq


def optimise_schedule(beta, log_g, T_new: int, interp: int = 0):
    """Alg. 3.  log_g is [3, T] (row i = log g_hat_{., i}).  Returns (beta_new, Lambda_hat, status)."""
    beta = _f64(beta)
    T = beta.shape[0] - 1
    lg = _f64(np.asarray(log_g).reshape(3, T))
    bn = np.zeros(T_new + 1)
    lam = np.zeros(T + 1)
    st = lib().orc_optimise_schedule(T, _ptr(beta), _ptr(lg), T_new, interp, _ptr(bn), _ptr(lam))
    return bn, lam, st


def dar_times(beta, log_g, beta_new, nu: float, interp: int = 0):
    """DAR resampling times on schedule beta_new predicted from a previous
    round (beta, log_g [3, T]).  Returns (flags uint8 [T_new], D_pred [T_new], status)."""
    beta, beta_new = _f64(beta), _f64(beta_new)
    T, Tn = beta.shape[0] - 1, beta_new.shape[0] - 1
    lg = _f64(np.asarray(log_g).reshape(3, T))
    flags = np.zeros(Tn, dtype=np.uint8)
    Dp = np.zeros(Tn)
    st = lib().orc_dar_times(T, _ptr(beta), _ptr(lg), Tn, _ptr(beta_new), interp, float(nu),
                             flags.ctypes.data_as(C.POINTER(C.c_ubyte)), _ptr(Dp))
    return flags, Dp, st


def rejuvenate(problem: Problem, opts: Opts, lw, x, T: int, eps_T: float, seed: int,
               round_k: int = 1, problem_id: int = 0, want_states: bool = False) -> dict:
    """Final-iteration rejuvenation: resample (lw [N], x [N, d]) and run N chains
    for T steps at beta = 1.  Returns mean [d], second [d], accept (and x [N, d])."""
    lw = _f64(lw)
    x = _f64(x)
    N, d = x.shape
    mean, second = np.zeros(d), np.zeros(d)
    acc = C.c_double(0.0)
    xo = np.zeros((N, d)) if want_states else None
    P = problem.c()
    O = opts.c()
    st = lib().orc_rejuvenate(C.byref(P), C.byref(O), N, T, float(eps_T), seed, round_k,
                              problem_id, _ptr(lw), _ptr(x), _ptr(mean), _ptr(second),
                              C.cast(C.byref(acc), _dp), _ptr(xo))
    out = dict(status=st, mean=mean, second=second, accept=acc.value)
    if want_states:
        out["x"] = xo
    return out


def zja(problem: Problem, opts: Opts, N: int, rho: float, Tmax: int, eps: float, seed: int,
        iters: int = 40, round_k: int = 1, problem_id: int = 0) -> dict:
    """ZJA online CESS-adaptive AIS: beta [T+1], T, log_g [3, T], logZ, lw [N], x [N, d]."""
    d = problem.d
    beta = np.zeros(Tmax + 1)
    lg = np.zeros(3 * Tmax)
    lw = np.zeros(N)
    x = np.zeros(N * d)
    T = C.c_int(0)
    lz = C.c_double(0.0)
    P = problem.c()
    O = opts.c()
    st = lib().orc_zja(C.byref(P), C.byref(O), N, float(rho), Tmax, iters, float(eps), seed,
                       round_k, problem_id, _ptr(beta), C.byref(T), _ptr(lg), C.cast(C.byref(lz), _dp),
                       _ptr(lw), _ptr(x))
    Tv = T.value
    return dict(status=st, T=Tv, beta=beta[:Tv + 1], log_g=lg.reshape(3, Tmax)[:, :Tv],
                logZ=lz.value, lw=lw, x=x.reshape(N, d))


def pt(problem: Problem, opts: Opts, K: int, beta, eps, Tp: int, seed: int, round_k: int = 1,
       problem_id: int = 0) -> dict:
    """Parallel tempering (K copies of N'+1 chains, T' iterations, even/odd swaps):
    logZ (stepping stone), ss [N'], rej [N'] (swap rejection per pair), Lambda_PT,
    round trips, tmean / tsecond [d] (target chain)."""
    beta = _f64(beta)
    Np = beta.shape[0] - 1
    eps = _f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (Np + 1,)))
    d = problem.d
    ss, rej = np.zeros(Np), np.zeros(Np)
    tm, ts = np.zeros(d), np.zeros(d)
    lz = C.c_double(0.0)
    trips = C.c_int64(0)
    P = problem.c()
    O = opts.c()
    st = lib().orc_pt(C.byref(P), C.byref(O), K, Np, Tp, _ptr(beta), _ptr(eps), seed, round_k,
                      problem_id, C.cast(C.byref(lz), _dp), _ptr(ss), _ptr(rej), C.byref(trips),
                      _ptr(tm), _ptr(ts))
    return dict(status=st, logZ=lz.value, ss=ss, rej=rej, Lambda_PT=float(np.sum(rej)),
                trips=trips.value, tmean=tm, tsecond=ts)


def ell(problem: Problem, x) -> tuple:
    x = _f64(x)
    g = np.zeros(problem.d)
    P = problem.c()
    v = lib().orc_ell(C.byref(P), _ptr(x), _ptr(g))
    return v, g


def asmc(problem: Problem, opts: Opts, N: int, beta, eps, seed: int, round_k: int = 1,
         problem_id: int = 0, traces: bool = False, subset=None) -> dict:
    """Alg. 1 for one schedule.  Returns a dict of numpy arrays (see oasmc_oracle.c)."""
    beta = _f64(beta)
    eps = _f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (beta.shape[0] - 1,)))
    T = beta.shape[0] - 1
    d = problem.d
    M = N if subset is None else len(subset)
    out = dict(log_g=np.zeros(3 * T), acc=np.zeros(T), lw=np.zeros(M), x=np.zeros(M * d),
               resampled=np.zeros(T, dtype=np.int32), ess=np.zeros(T))
    logZ = C.c_double(0.0)
    nres = C.c_int(0)
    acc_tr = np.zeros(M * T, dtype=np.uint8) if traces else None
    mar_tr = np.zeros(M * T) if traces else None
    lw_tr = np.zeros(M * T) if traces else None
    sub = None if subset is None else np.ascontiguousarray(np.asarray(subset, dtype=np.int64))
    P = problem.c()
    O = opts.c()
    st = lib().orc_asmc(
        C.byref(P), C.byref(O), N, T, _ptr(beta), _ptr(eps), seed, round_k, problem_id,
        _ptr(out["log_g"]), _ptr(out["acc"]), C.byref(logZ), _ptr(out["lw"]), _ptr(out["x"]),
        C.byref(nres), None if acc_tr is None else acc_tr.ctypes.data_as(C.POINTER(C.c_ubyte)),
        _ptr(mar_tr), out["resampled"].ctypes.data_as(C.POINTER(C.c_int)), _ptr(out["ess"]),
        None if sub is None else sub.ctypes.data_as(C.POINTER(C.c_int64)),
        0 if sub is None else sub.shape[0], _ptr(lw_tr))
    out["status"] = st
    out["logZ"] = logZ.value
    out["n_resample"] = nres.value
    out["log_g"] = out["log_g"].reshape(3, T)
    out["x"] = out["x"].reshape(M, d)
    if traces:
        out["accept"] = acc_tr.reshape(M, T)
        out["margin"] = mar_tr.reshape(M, T)
        out["lw_minus"] = lw_tr.reshape(M, T)  # log w_{t^-} after the reweight of step t
    return out


def run(problem: Problem, opts: Opts, ropts: RunOpts, N1: int, rounds: int, seed: int,
        problem_id: int = 0, Tcap: Optional[int] = None) -> dict:
    """Alg. 2: `rounds` rounds of ASMC with schedule optimisation between them."""
    if Tcap is None:
        Tcap = ropts.T1 if ropts.budget in (0, 1) else max(ropts.T1, ropts.Tmax)
    R = rounds
    logZ = np.full(R, np.nan)
    Ns = np.zeros(R, dtype=np.int64)
    Ts = np.zeros(R, dtype=np.int32)
    beta = np.zeros((R, Tcap + 1))
    lam = np.zeros((R, Tcap + 1))
    lg = np.zeros((R, 3, Tcap))
    acc = np.zeros((R, Tcap))
    eps = np.zeros((R, Tcap))
    nres = np.zeros(R, dtype=np.int32)
    P = problem.c()
    O = opts.c()
    RO = ropts.c()
    st = lib().orc_run(C.byref(P), C.byref(O), C.byref(RO), N1, R, seed, problem_id, Tcap,
                       _ptr(logZ), Ns.ctypes.data_as(C.POINTER(C.c_int64)),
                       Ts.ctypes.data_as(C.POINTER(C.c_int)), _ptr(beta), _ptr(lam), _ptr(lg),
                       _ptr(acc), _ptr(eps), nres.ctypes.data_as(C.POINTER(C.c_int)))
    return dict(status=st, logZ=logZ, N=Ns, T=Ts, beta=beta, Lambda=lam, log_g=lg, acc=acc,
                eps=eps, n_resample=nres)


def gmm_derivs(problem: Problem, x):
    """(H [d,d] hessian of ell, M [d, np] d grad ell / d theta, dl [np] d ell / d theta)."""
    x = _f64(x)
    d, K = problem.d, int(np.asarray(problem.means).shape[0])
    npar = K * d + K
    H = np.zeros((d, d))
    M = np.zeros((d, npar))
    dl = np.zeros(npar)
    P = problem.c()
    lib().orc_gmm_derivs(C.byref(P), _ptr(x), _ptr(H), _ptr(M), _ptr(dl))
    return H, M, dl


def logZ_grad(problem: Problem, opts: Opts, N: int, beta, eps, seed: int, round_k: int = 1,
              problem_id: int = 0, want_accept: bool = False):
    """Pathwise gradient of log Z_hat w.r.t. (means, log_scales) with fixed accept decisions."""
    beta = _f64(beta)
    T = beta.shape[0] - 1
    eps = _f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (T,)))
    K = int(np.asarray(problem.means).shape[0])
    g = np.zeros(K * problem.d + K)
    lz = C.c_double(0.0)
    acc = np.zeros((N, T), dtype=np.uint8) if want_accept else None
    P = problem.c()
    O = opts.c()
    st = lib().orc_logZ_grad(C.byref(P), C.byref(O), N, T, _ptr(beta), _ptr(eps), seed, round_k,
                             problem_id, _ptr(g), C.byref(lz),
                             None if acc is None else acc.ctypes.data_as(C.POINTER(C.c_ubyte)))
    if st != 0:
        raise RuntimeError(f"orc_logZ_grad status {st}")
    return (lz.value, g, acc) if want_accept else (lz.value, g)
