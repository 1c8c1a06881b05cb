"""Python binding of include/oasmc.h (ctypes).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboasmc.so")

OK, EINVAL, EHIP, ENOMEM, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GAUSS, LOGREG, GMM, UNID = 1, 2, 3, 4
MOVES = {"rwmh": 1, "mala": 2, "hmc": 3, "rwmh3": 4}
TRIGGERS = {"ess": 0, "cess": 1, "sir": 2, "fixed": 3}
BUDGETS = {"fixed": 0, "double_n": 1, "double_t": 2, "sqrt2": 3}


class OasmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oasmc status {code}: {msg}")
        self.code = code


class _Problem(C.Structure):
    _fields_ = [
        ("family", C.c_int32), ("d", C.c_int32), ("mu", C.c_void_p), ("sigma2", C.c_double),
        ("X", C.c_void_p), ("y", C.c_void_p), ("n", C.c_int32), ("K", C.c_int32),
        ("means", C.c_void_p), ("log_scales", C.c_void_p), ("ref_mean", C.c_void_p),
        ("ref_sigma2", C.c_double), ("binom_n", C.c_double), ("binom_k", C.c_double),
        ("box", C.c_double),
    ]


class _Kernel(C.Structure):
    _fields_ = [("move", C.c_int32), ("leapfrog", C.c_int32), ("resample", C.c_int32),
                ("trigger", C.c_int32), ("nu", C.c_double), ("slots", C.c_int32),
                ("resample_at", C.c_void_p)]


class _RoundOut(C.Structure):
    _fields_ = [
        ("log_g", C.c_void_p), ("accept", C.c_void_p), ("ess", C.c_void_p),
        ("resampled", C.c_void_p), ("logZ", C.c_double), ("n_resample", C.c_int32),
        ("lw", C.c_void_p), ("x", C.c_void_p), ("accept_bits", C.c_void_p),
    ]


class _RunOpts(C.Structure):
    _fields_ = [
        ("budget", C.c_int32), ("T1", C.c_int32), ("T_max", C.c_int32), ("N_max", C.c_int64),
        ("eps_adapt", C.c_int32), ("eps0", C.c_double), ("eps_kappa", C.c_double),
        ("accept_target", C.c_double), ("interp", C.c_int32), ("dar", C.c_int32),
    ]


class _BatchProblem(C.Structure):
    _fields_ = [("problem", _Problem), ("kernel", _Kernel), ("N", C.c_int64), ("T", C.c_int32),
                ("eps_adapt", C.c_int32), ("eps0", C.c_double), ("eps_kappa", C.c_double),
                ("accept_target", C.c_double), ("seed", C.c_uint64), ("problem_id", C.c_uint32)]


class _BatchOut(C.Structure):
    _fields_ = [("logZ", C.c_void_p), ("Lambda_T", C.c_void_p), ("status", C.c_void_p)]


class _RunOut(C.Structure):
    _fields_ = [
        ("rounds", C.c_int32), ("Tcap", C.c_int32), ("logZ", C.c_void_p), ("N", C.c_void_p),
        ("T", C.c_void_p), ("beta", C.c_void_p), ("Lambda_hat", C.c_void_p),
        ("log_g", C.c_void_p), ("accept", C.c_void_p), ("eps", C.c_void_p),
        ("n_resample", C.c_void_p), ("rounds_done", C.c_int32),
        ("rejuv_mean", C.c_void_p), ("rejuv_second", C.c_void_p),
    ]


_lib = None
_handles = {}


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise OasmcError(EINVAL, f"HIP library not built: {_LIB_PATH} is missing "
                                 "(run paper_2408_12057_amd/build.py)")
    L = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    L.oasmc_last_error.restype = C.c_char_p
    L.oasmc_handle_create.argtypes = [C.POINTER(vp), C.c_int]
    L.oasmc_handle_destroy.argtypes = [vp]
    L.oasmc_asmc.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int64, C.c_int32,
                             vp, vp, C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(_RoundOut), vp]
    L.oasmc_adapt_schedule.argtypes = [C.c_int32, vp, vp, C.c_int32, C.c_int32, vp, vp]
    L.oasmc_dar_times.argtypes = [C.c_int32, vp, vp, C.c_int32, vp, C.c_int32, C.c_double, vp,
                                  vp]
    L.oasmc_run.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.POINTER(_RunOpts),
                            C.c_int64, C.c_uint64, C.c_uint32, C.POINTER(_RunOut), vp]
    L.oasmc_resample.argtypes = [vp, C.c_int64, vp, C.c_uint32, vp, vp]
    L.oasmc_resample_noalloc.argtypes = [C.c_int64, vp, C.c_uint32, vp, vp]
    L.oasmc_philox.argtypes = [vp, C.c_uint64, vp, vp, C.c_int64, vp]
    L.oasmc_logZ_backward.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int64,
                                      C.c_int32, vp, vp, C.c_uint64, C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_double), vp, vp]
    L.oasmc_run_batch.argtypes = [vp, C.POINTER(_BatchProblem), C.c_int32, C.c_int32, C.c_int32,
                                  C.POINTER(_BatchOut), vp]
    L.oasmc_logreg_eval.argtypes = [vp, C.POINTER(_Problem), C.c_int64, vp, vp, vp, vp]
    L.oasmc_target_eval.argtypes = [vp, C.POINTER(_Problem), C.c_int64, vp, C.c_int32, C.c_int32,
                                    vp, vp, vp]
    L.oasmc_pt.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int32, C.c_int32,
                           C.c_int32, vp, vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, vp, vp, vp,
                           vp, vp, vp]
    L.oasmc_autotune.argtypes = [vp, C.c_int32, vp]
    L.oasmc_shape.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int64, vp, vp, vp]
    L.oasmc_zja.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int64, C.c_double,
                            C.c_int32, C.c_int32, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32,
                            vp, vp, vp, vp, vp, vp, vp]
    L.oasmc_rejuvenate.argtypes = [vp, C.POINTER(_Problem), C.POINTER(_Kernel), C.c_int64,
                                   C.c_int32, C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, vp,
                                   vp, vp, vp, vp, vp, vp]
    L.oasmc_profile.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
    for f in ("oasmc_handle_create", "oasmc_handle_destroy", "oasmc_asmc", "oasmc_adapt_schedule",
              "oasmc_dar_times",
              "oasmc_run", "oasmc_resample", "oasmc_resample_noalloc", "oasmc_philox", "oasmc_logreg_eval",
              "oasmc_profile", "oasmc_logZ_backward", "oasmc_run_batch", "oasmc_rejuvenate",
              "oasmc_zja", "oasmc_autotune", "oasmc_shape", "oasmc_pt", "oasmc_target_eval"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(code: int):
    if code != OK:
        raise OasmcError(code, _load().oasmc_last_error().decode())


def _handle(device: int):
    if device not in _handles:
        h = C.c_void_p()
        _check(_load().oasmc_handle_create(C.byref(h), device))
        _handles[device] = h
    return _handles[device]


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f32(t, device) -> Optional[torch.Tensor]:
    if t is None:
        return None
    return torch.as_tensor(t, dtype=torch.float32).to(device).contiguous()


def _host_f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


@dataclass
class Problem:
    """Target gamma and Gaussian reference eta = N(ref_mean, ref_sigma2 I) on a device.

    Build with ``Problem.gauss``, ``Problem.logreg`` or ``Problem.gmm``; array
    fields are fp32 device tensors (kept alive by this object)."""
    family: int
    d: int
    device: torch.device
    mu: Optional[torch.Tensor] = None
    sigma2: float = 1.0
    X: Optional[torch.Tensor] = None
    y: Optional[torch.Tensor] = None
    means: Optional[torch.Tensor] = None
    log_scales: Optional[torch.Tensor] = None
    ref_mean: Optional[torch.Tensor] = None
    ref_sigma2: float = 1.0
    binom_n: float = 0.0
    binom_k: float = 0.0
    box: float = 10.0

    @staticmethod
    def unid(n: float, k: float, box: float = 10.0, device="cuda"):
        """The unidentifiable product parameterisation: Uniform(0, box)^2 reference,
        Binomial(k | n, x y) likelihood divided by its maximum."""
        return Problem(UNID, 2, torch.device(device), binom_n=float(n), binom_k=float(k),
                       box=float(box))

    @staticmethod
    def gauss(mu, sigma2: float, ref_sigma2: float = 1.0, ref_mean=None, device="cuda"):
        dev = torch.device(device)
        mu = _dev_f32(mu, dev)
        return Problem(GAUSS, int(mu.numel()), dev, mu=mu, sigma2=float(sigma2),
                       ref_mean=_dev_f32(ref_mean, dev), ref_sigma2=float(ref_sigma2))

    @staticmethod
    def logreg(X, y, ref_sigma2: float = 1.0, ref_mean=None, device="cuda"):
        dev = torch.device(device)
        X = _dev_f32(X, dev)
        return Problem(LOGREG, int(X.shape[1]), dev, X=X, y=_dev_f32(y, dev),
                       ref_mean=_dev_f32(ref_mean, dev), ref_sigma2=float(ref_sigma2))

    @staticmethod
    def gmm(means, log_scales, ref_sigma2: float = 1.0, ref_mean=None, device="cuda"):
        dev = torch.device(device)
        means = _dev_f32(means, dev)
        return Problem(GMM, int(means.shape[1]), dev, means=means,
                       log_scales=_dev_f32(log_scales, dev), ref_mean=_dev_f32(ref_mean, dev),
                       ref_sigma2=float(ref_sigma2))

    def c(self) -> _Problem:
        def p(t):
            return None if t is None else C.c_void_p(t.data_ptr())
        return _Problem(self.family, self.d, p(self.mu), self.sigma2, p(self.X), p(self.y),
                        0 if self.X is None else int(self.X.shape[0]),
                        0 if self.means is None else int(self.means.shape[0]),
                        p(self.means), p(self.log_scales), p(self.ref_mean), self.ref_sigma2,
                        self.binom_n, self.binom_k, self.box)


def _kernel(move, leapfrog, resample_, trigger, nu, slots=0, resample_at=None) -> _Kernel:
    """resample_at: host int32 array (trigger "fixed"), kept alive by the caller."""
    return _Kernel(MOVES[move] if isinstance(move, str) else int(move), int(leapfrog),
                   int(bool(resample_)), TRIGGERS[trigger] if isinstance(trigger, str)
                   else int(trigger), float(nu), int(slots),
                   None if resample_at is None else C.c_void_p(resample_at.ctypes.data))


def asmc(problem: Problem, N: int, beta, eps, seed: int, round_k: int = 1, problem_id: int = 0,
         move="rwmh", leapfrog: int = 5, resample_: bool = False, trigger="ess",
         nu: float = 0.5, return_state: bool = True, accept_bits: bool = False,
         slots: int = 0, resample_at=None) -> dict:
    """Alg. 1, ASMC(N, B_T): one pass with schedule ``beta`` (T+1) and step sizes ``eps`` (T).
    ``trigger``: "ess", "cess" (adaptive), "sir" (every step) or "fixed" (after the
    steps t with ``resample_at[t-1]`` nonzero)."""
    dev = problem.device
    beta = _host_f64(beta)
    T = beta.shape[0] - 1
    eps = _host_f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (T,)))
    log_g = np.zeros(3 * T)
    acc = np.zeros(T)
    ess = np.zeros(T)
    res = np.zeros(T, dtype=np.int32)
    out = _RoundOut()
    out.log_g, out.accept, out.ess, out.resampled = (_np_ptr(log_g), _np_ptr(acc), _np_ptr(ess),
                                                     _np_ptr(res))
    lw = x = bits = None
    if return_state:
        lw = torch.empty(N, dtype=torch.float64, device=dev)
        x = torch.empty((N, problem.d), dtype=torch.float32, device=dev)
        out.lw, out.x = lw.data_ptr(), x.data_ptr()
    if accept_bits:
        bits = torch.zeros((N, (T + 31) // 32), dtype=torch.int32, device=dev)
        out.accept_bits = bits.data_ptr()
    P = problem.c()
    ra = None
    if resample_at is not None:
        ra = np.ascontiguousarray(np.asarray(resample_at, dtype=np.int32))
        assert ra.shape == (T,)
    K = _kernel(move, leapfrog, resample_, trigger, nu, slots, ra)
    code = _load().oasmc_asmc(_handle(dev.index or 0), C.byref(P), C.byref(K), int(N), int(T),
                              _np_ptr(beta), _np_ptr(eps), int(seed) & (2 ** 64 - 1),
                              int(round_k), int(problem_id), C.byref(out), _stream(dev))
    _check(code)
    r = dict(log_g=log_g.reshape(3, T), accept=acc, ess=ess, resampled=res, logZ=out.logZ,
             n_resample=out.n_resample)
    if return_state:
        r["lw"], r["x"] = lw, x
    if accept_bits:
        r["accept_bits"] = bits
    return r


def adapt_schedule(beta, log_g, T_new: int, interp: int = 0):
    """Alg. 3 (host): returns (beta_new[T_new+1], Lambda_hat[T+1])."""
    beta = _host_f64(beta)
    T = beta.shape[0] - 1
    lg = _host_f64(np.asarray(log_g).reshape(3 * T))
    bn = np.zeros(T_new + 1)
    lam = np.zeros(T + 1)
    code = _load().oasmc_adapt_schedule(T, _np_ptr(beta), _np_ptr(lg), int(T_new), int(interp),
                                        _np_ptr(bn), _np_ptr(lam))
    if code not in (OK, ENONFINITE):
        _check(code)
    return bn, lam


def run(problem: Problem, N1: int, rounds: int, seed: int, problem_id: int = 0, move="rwmh",
        leapfrog: int = 5, resample_: bool = False, trigger="ess", nu: float = 0.5,
        budget="double_n", T1: int = 64, T_max: int = 0, N_max: int = 1 << 40,
        eps0: float = 0.1, eps_adapt: bool = False, eps_kappa: float = 0.0,
        accept_target: float = 0.574, interp: int = 0, Tcap: Optional[int] = None,
        slots: int = 0, dar: bool = False, rejuvenate: bool = False) -> dict:
    """Alg. 2, OASMC: `rounds` rounds with Budget and OptimiseSchedule between them.
    ``dar`` (with ``resample_``): rounds after the first resample at the DAR times
    predicted from the previous round.  ``rejuvenate``: final-iteration rejuvenation
    after every round (``rejuv_mean``, ``rejuv_second`` [rounds, d])."""
    dev = problem.device
    b = BUDGETS[budget] if isinstance(budget, str) else int(budget)
    if Tcap is None:
        Tcap = T1 if b in (0, 1) else max(T1, T_max)
    R = int(rounds)
    logZ = np.full(R, np.nan)
    Ns = np.zeros(R, dtype=np.int64)
    Ts = np.zeros(R, dtype=np.int32)
    beta = np.zeros((R, Tcap + 1))
    lam = np.zeros((R, Tcap + 1))
    lg = np.zeros((R, 3, Tcap))
    acc = np.zeros((R, Tcap))
    eps = np.zeros((R, Tcap))
    nres = np.zeros(R, dtype=np.int32)
    rj_m = np.zeros((R, problem.d)) if rejuvenate else None
    rj_s = np.zeros((R, problem.d)) if rejuvenate else None
    out = _RunOut(R, Tcap, _np_ptr(logZ), _np_ptr(Ns), _np_ptr(Ts), _np_ptr(beta), _np_ptr(lam),
                  _np_ptr(lg), _np_ptr(acc), _np_ptr(eps), _np_ptr(nres), 0, _np_ptr(rj_m),
                  _np_ptr(rj_s))
    ro = _RunOpts(b, int(T1), int(T_max), int(N_max), int(bool(eps_adapt)), float(eps0),
                  float(eps_kappa), float(accept_target), int(interp), int(bool(dar)))
    P = problem.c()
    K = _kernel(move, leapfrog, resample_, trigger, nu, slots)
    code = _load().oasmc_run(_handle(dev.index or 0), C.byref(P), C.byref(K), C.byref(ro),
                             int(N1), int(seed) & (2 ** 64 - 1), int(problem_id), C.byref(out),
                             _stream(dev))
    _check(code)
    r = dict(logZ=logZ, N=Ns, T=Ts, beta=beta, Lambda=lam, log_g=lg, acc=acc, eps=eps,
             n_resample=nres, rounds_done=out.rounds_done)
    if rejuvenate:
        r["rejuv_mean"], r["rejuv_second"] = rj_m, rj_s
    return r


def pt(problem: Problem, K: int, beta, eps, Tp: int, seed: int, move="rwmh", leapfrog: int = 5,
       round_k: int = 1, problem_id: int = 0) -> dict:
    """Parallel tempering: K copies of len(beta) chains, Tp iterations, even/odd swaps.
    Returns logZ (stepping stone), ss [N'], rej [N'], Lambda_PT, trips, tmean, tsecond."""
    dev = problem.device
    beta = _host_f64(beta)
    Np = beta.shape[0] - 1
    eps = _host_f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (Np + 1,)))
    ss, rej = np.zeros(Np), np.zeros(Np)
    tm, ts = np.zeros(problem.d), np.zeros(problem.d)
    lz = C.c_double(0.0)
    trips = C.c_int64(0)
    P = problem.c()
    Kn = _kernel(move, leapfrog, False, "ess", 0.5)
    _check(_load().oasmc_pt(_handle(dev.index or 0), C.byref(P), C.byref(Kn), int(K), Np, int(Tp),
                            _np_ptr(beta), _np_ptr(eps), int(seed) & (2 ** 64 - 1), int(round_k),
                            int(problem_id), C.c_void_p(C.addressof(lz)), _np_ptr(ss), _np_ptr(rej),
                            C.c_void_p(C.addressof(trips)), _np_ptr(tm), _np_ptr(ts),
                            _stream(dev)))
    return dict(logZ=lz.value, ss=ss, rej=rej, Lambda_PT=float(np.sum(rej)), trips=trips.value,
                tmean=tm, tsecond=ts)


def autotune(enable: int, device: int = 0) -> int:
    """Launch-shape autotuning of the VALU sweeps on (1) or off (0); -1 also
    forgets the measured shapes.  Returns the number of classes measured."""
    n = C.c_int32(0)
    _check(_load().oasmc_autotune(_handle(device), int(enable), C.c_void_p(C.addressof(n))))
    return n.value


def shape(problem: Problem, N: int, move="rwmh", leapfrog: int = 5) -> tuple:
    """(lanes per particle, coordinates per lane) of the next AIS pass of ``problem``."""
    dev = problem.device
    lpp, dpl = C.c_int32(0), C.c_int32(0)
    P = problem.c()
    K = _kernel(move, leapfrog, False, "ess", 0.5)
    _check(_load().oasmc_shape(_handle(dev.index or 0), C.byref(P), C.byref(K), int(N),
                               C.c_void_p(C.addressof(lpp)), C.c_void_p(C.addressof(dpl)),
                               _stream(dev)))
    return lpp.value, dpl.value


def zja(problem: Problem, N: int, rho: float, Tmax: int, eps: float, seed: int, move="rwmh3",
        leapfrog: int = 5, iters: int = 40, round_k: int = 1, problem_id: int = 0,
        return_state: bool = True) -> dict:
    """ZJA online CESS-adaptive AIS: beta [T+1], T, log_g [3, T], logZ (and final lw, x)."""
    dev = problem.device
    beta = np.zeros(Tmax + 1)
    lg = np.zeros(3 * Tmax)
    T = C.c_int32(0)
    lz = C.c_double(0.0)
    lw = x = None
    if return_state:
        lw = torch.empty(N, dtype=torch.float64, device=dev)
        x = torch.empty((N, problem.d), dtype=torch.float32, device=dev)
    P = problem.c()
    K = _kernel(move, leapfrog, False, "ess", 0.5)
    _check(_load().oasmc_zja(_handle(dev.index or 0), C.byref(P), C.byref(K), int(N), float(rho),
                             int(Tmax), int(iters), float(eps), int(seed) & (2 ** 64 - 1),
                             int(round_k), int(problem_id), _np_ptr(beta),
                             C.c_void_p(C.addressof(T)), _np_ptr(lg), C.c_void_p(C.addressof(lz)),
                             None if lw is None else C.c_void_p(lw.data_ptr()),
                             None if x is None else C.c_void_p(x.data_ptr()), _stream(dev)))
    Tv = T.value
    r = dict(T=Tv, beta=beta[:Tv + 1], log_g=lg.reshape(3, Tmax)[:, :Tv], logZ=lz.value)
    if return_state:
        r["lw"], r["x"] = lw, x
    return r


def rejuvenate(problem: Problem, lw: torch.Tensor, x: torch.Tensor, T: int, eps_T: float,
               seed: int, round_k: int = 1, problem_id: int = 0, move="rwmh", leapfrog: int = 5,
               return_states: bool = False) -> dict:
    """Final-iteration rejuvenation of a pass's final population (device lw [N],
    x [N, d]): N chains of T steps at beta = 1; returns the averages of x and x^2
    over the TN chain states and the accepted fraction (and the end states)."""
    dev = problem.device
    lw = lw.to(device=dev, dtype=torch.float64).contiguous()
    x = x.to(device=dev, dtype=torch.float32).contiguous()
    N = int(x.shape[0])
    mean, second = np.zeros(problem.d), np.zeros(problem.d)
    acc = C.c_double(0.0)
    xo = torch.empty_like(x) if return_states else None
    P = problem.c()
    K = _kernel(move, leapfrog, False, "ess", 0.5)
    _check(_load().oasmc_rejuvenate(_handle(dev.index or 0), C.byref(P), C.byref(K), N, int(T),
                                    float(eps_T), int(seed) & (2 ** 64 - 1), int(round_k),
                                    int(problem_id), C.c_void_p(lw.data_ptr()),
                                    C.c_void_p(x.data_ptr()), _np_ptr(mean), _np_ptr(second),
                                    C.c_void_p(C.addressof(acc)),
                                    None if xo is None else C.c_void_p(xo.data_ptr()),
                                    _stream(dev)))
    out = dict(mean=mean, second=second, accept=acc.value)
    if return_states:
        out["x"] = xo
    return out


def dar_times(beta, log_g, beta_new, nu: float, interp: int = 0):
    """DAR resampling times for schedule ``beta_new`` predicted from a previous round
    (``beta``, ``log_g`` [3, T]): (flags int32 [T_new], D_pred [T_new])."""
    beta, bn = _host_f64(beta), _host_f64(beta_new)
    T, Tn = beta.shape[0] - 1, bn.shape[0] - 1
    lg = _host_f64(np.asarray(log_g).reshape(3 * T))
    flags = np.zeros(Tn, dtype=np.int32)
    Dp = np.zeros(Tn)
    code = _load().oasmc_dar_times(T, _np_ptr(beta), _np_ptr(lg), Tn, _np_ptr(bn), int(interp),
                                   float(nu), _np_ptr(flags), _np_ptr(Dp))
    _check(code)
    return flags, Dp


def resample(lw: torch.Tensor, u: int) -> torch.Tensor:
    """Systematic resampling of device log-weights (float64) with 32-bit uniform word u."""
    lw = lw.to(torch.float64).contiguous()
    anc = torch.empty(lw.numel(), dtype=torch.int32, device=lw.device)
    _check(_load().oasmc_resample(_handle(lw.device.index or 0), int(lw.numel()),
                                  C.c_void_p(lw.data_ptr()), int(u) & 0xFFFFFFFF,
                                  C.c_void_p(anc.data_ptr()), _stream(lw.device)))
    return anc


NOALLOC_MAX_N = 1 << 20


def resample_noalloc(lw: torch.Tensor, u: int, anc: torch.Tensor) -> torch.Tensor:
    """oasmc_resample_noalloc: the same resampling into the caller's int32
    buffer anc[N], with the library's static scratch (nothing allocated;
    asynchronous on the current stream).  lw must already be float64 and
    contiguous on the same device."""
    assert lw.dtype == torch.float64 and lw.is_contiguous()
    assert anc.dtype == torch.int32 and anc.is_contiguous() and anc.numel() == lw.numel()
    with torch.cuda.device(lw.device):
        _check(_load().oasmc_resample_noalloc(int(lw.numel()), C.c_void_p(lw.data_ptr()),
                                              int(u) & 0xFFFFFFFF, C.c_void_p(anc.data_ptr()),
                                              _stream(lw.device)))
    return anc


def philox(seed: int, ctr: torch.Tensor) -> torch.Tensor:
    """Raw Philox4x32-10 blocks for device counters ctr [count, 4] (int32 bit patterns)."""
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    _check(_load().oasmc_philox(_handle(ctr.device.index or 0), int(seed) & (2 ** 64 - 1),
                                C.c_void_p(ctr.data_ptr()), C.c_void_p(out.data_ptr()),
                                int(ctr.shape[0]), _stream(ctr.device)))
    return out


def logreg_eval(problem: Problem, theta: torch.Tensor):
    """Log-likelihood (float64) and its gradient (float32) at states theta [N, d]
    with the sweep's FP32-MFMA contraction."""
    theta = theta.to(device=problem.device, dtype=torch.float32).contiguous()
    N = int(theta.shape[0])
    ell = torch.empty(N, dtype=torch.float64, device=problem.device)
    grad = torch.empty((N, problem.d), dtype=torch.float32, device=problem.device)
    P = problem.c()
    _check(_load().oasmc_logreg_eval(_handle(problem.device.index or 0), C.byref(P), N,
                                     C.c_void_p(theta.data_ptr()), C.c_void_p(ell.data_ptr()),
                                     C.c_void_p(grad.data_ptr()), _stream(problem.device)))
    return ell, grad


def target_eval(problem: Problem, x: torch.Tensor, lpp: int = 0, dpl: int = 0):
    """ell (float64) and its gradient (float64) of a closed-form target at
    states x [N, d], by the sweeps' particle arithmetic in the lane layout
    lpp x dpl (0, 0: the default shape)."""
    x = x.to(device=problem.device, dtype=torch.float32).contiguous()
    N = int(x.shape[0])
    ell = torch.empty(N, dtype=torch.float64, device=problem.device)
    grad = torch.empty((N, problem.d), dtype=torch.float64, device=problem.device)
    P = problem.c()
    _check(_load().oasmc_target_eval(_handle(problem.device.index or 0), C.byref(P), N,
                                     C.c_void_p(x.data_ptr()), int(lpp), int(dpl),
                                     C.c_void_p(ell.data_ptr()), C.c_void_p(grad.data_ptr()),
                                     _stream(problem.device)))
    return ell, grad


def profile(enable: bool, device: int = 0) -> dict:
    """Start (enable=True, clears totals) or stop live timing of the sweep kernels;
    returns the totals recorded so far."""
    ms, n = C.c_double(), C.c_int64()
    steps, flops = C.c_double(), C.c_double()
    _check(_load().oasmc_profile(_handle(device), int(bool(enable)), C.byref(ms), C.byref(n),
                                 C.byref(steps), C.byref(flops)))
    return dict(kernel_ms=ms.value, launches=n.value, particle_steps=steps.value, flops=flops.value)


def logZ_backward(problem: Problem, N: int, beta, eps, seed: int, round_k: int = 1,
                  problem_id: int = 0, slots: int = 0):
    """(log Z_hat, grad of log Z_hat w.r.t. (means.ravel(), log_scales)) for the mixture
    target with MALA, accept decisions held fixed."""
    dev = problem.device
    beta = _host_f64(beta)
    T = beta.shape[0] - 1
    eps = _host_f64(np.broadcast_to(np.asarray(eps, dtype=np.float64), (T,)))
    K = int(problem.means.shape[0])
    grad = np.zeros(K * problem.d + K)
    lz = C.c_double(0.0)
    P = problem.c()
    Kn = _kernel("mala", 1, False, "ess", 0.5, slots)
    _check(_load().oasmc_logZ_backward(_handle(dev.index or 0), C.byref(P), C.byref(Kn), int(N),
                                       int(T), _np_ptr(beta), _np_ptr(eps),
                                       int(seed) & (2 ** 64 - 1), int(round_k), int(problem_id),
                                       C.byref(lz), _np_ptr(grad), _stream(dev)))
    return lz.value, grad


class LogZ(torch.autograd.Function):
    """log Z_hat(means, log_scales) of the mixture target as a differentiable
    torch function: forward and backward both run the HIP path (forward pass
    with checkpoints, then the reverse pass).  Use ``LogZ.apply(means,
    log_scales, ref_sigma2, N, beta, eps, seed)``."""

    @staticmethod
    def forward(ctx, means, log_scales, ref_sigma2, N, beta, eps, seed):
        prob = Problem.gmm(means.detach(), log_scales.detach(), ref_sigma2, device=means.device)
        lz, g = logZ_backward(prob, N, beta, eps, seed)
        K, d = means.shape
        ctx.save_for_backward(torch.tensor(g[:K * d].reshape(K, d), dtype=means.dtype,
                                           device=means.device),
                              torch.tensor(g[K * d:], dtype=log_scales.dtype,
                                           device=log_scales.device))
        return torch.tensor(lz, dtype=torch.float64, device=means.device)

    @staticmethod
    def backward(ctx, grad_out):
        gm, gs = ctx.saved_tensors
        go = grad_out.to(gm.dtype)
        return go * gm, go * gs, None, None, None, None, None


@dataclass
class BatchItem:
    """One problem of a batch (see oasmc_batch_problem)."""
    problem: Problem
    N: int
    T: int
    move: str = "rwmh"
    leapfrog: int = 5
    eps0: float = 0.1
    eps_adapt: bool = False
    eps_kappa: float = 0.0
    accept_target: float = 0.574
    seed: int = 0
    problem_id: int = 0
    slots: int = 0


def run_batch(items, rounds: int, use_graph: bool = True) -> dict:
    """Alg. 2 for many independent problems in one enqueue (optionally one hipGraph)."""
    items = list(items)
    P = len(items)
    dev = items[0].problem.device
    arr = (_BatchProblem * P)()
    for i, it in enumerate(items):
        arr[i].problem = it.problem.c()
        arr[i].kernel = _kernel(it.move, it.leapfrog, False, "ess", 0.5, it.slots)
        arr[i].N = int(it.N)
        arr[i].T = int(it.T)
        arr[i].eps_adapt = int(bool(it.eps_adapt))
        arr[i].eps0 = float(it.eps0)
        arr[i].eps_kappa = float(it.eps_kappa)
        arr[i].accept_target = float(it.accept_target)
        arr[i].seed = int(it.seed) & (2 ** 64 - 1)
        arr[i].problem_id = int(it.problem_id)
    logZ = np.zeros((P, rounds))
    lam = np.zeros((P, rounds))
    status = np.zeros((P, rounds), dtype=np.int32)
    out = _BatchOut(_np_ptr(logZ), _np_ptr(lam), _np_ptr(status))
    _check(_load().oasmc_run_batch(_handle(dev.index or 0), arr, P, int(rounds), int(bool(use_graph)),
                                   C.byref(out), _stream(dev)))
    return dict(logZ=logZ, Lambda_T=lam, status=status)
