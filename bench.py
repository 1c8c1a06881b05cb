"""Benchmark: particle-steps/s of the OAIS hot path on one MI355X.

One step = one full Alg. 2 run (all rounds) of the Bayesian logistic
regression workload: synthetic X in R^{10000 x 50} (fp32, iid N(0,1)),
theta* ~ N(0, I), y ~ Bernoulli(sigmoid(X theta*)), prior eta = N(0, I_50),
N = 16384 particles, T = 1, 2, 4, ..., 512, 1000 (11 rounds), MALA with
adapted per-temperature step sizes, schedules rebuilt by Alg. 3 between rounds.
Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  Besides the throughput it reports, outside the timed
region, the error of the last round's log Z_hat over independent seeds
against a reference value (closed form where the target has one, otherwise a
long run of the same estimator), so that throughputs are quoted at a stated
log Z error.  --workload selects the other synthetic workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
# plain-ALU issue budget: 256 CUs x 64 lanes x 2.4 GHz lane-cycles per second
PEAK_LANE_CYCLES = 256 * 64 * 2.4e9
# algorithmic ALU work per particle-step in lane-cycles (Philox blocks, binary64
# Box-Muller, target and gradient arithmetic, moment statistics; the model is
# derived per workload alongside the kernel descriptions)
ALU_WORK = {"gauss": 700.0, "gauss_sat": 700.0, "asmc": 1.0e4, "asmc_ess": 1.0e4,
            "asmc_dar": 1.0e4}
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by the copy-kernel calibration), with the sha256 prefix of
# the kernel source they were measured on and the summary that records them;
# reported only while the source is unchanged.
TRAFFIC = {
    "logreg": dict(bytes=3.369e9, source="paper_2408_12057_amd/csrc/sweep_logreg.hip",
                   sha256="ba129d35b9f0f6a0",
                   profile="profiles/k_oais_logreg_batch__logreg_n10000_d50.md"),
    "logreg_d200": dict(bytes=10.39e9, source="paper_2408_12057_amd/csrc/sweep_logreg.hip",
                        sha256="ba129d35b9f0f6a0",
                        profile="profiles/k_oais_logreg_wide_batch__logreg_n5000_d200.md"),
}


def measured_traffic(workload: str):
    """(bytes, profile) of the workload's dominant kernel if its source still
    has the hash the counters were taken on, else (None, None)."""
    import hashlib
    t = TRAFFIC.get(workload)
    if not t:
        return None, None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return (t["bytes"], t["profile"]) if h == t["sha256"] else (None, None)
METRIC = "particle-steps/sec and fraction of roofline at matched log Z error"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


class Spec:
    """A workload: problem, run options, rounds, the first round's N, the
    reference log Z and the default number of seeds for the error estimate."""

    def __init__(self, w, prob, kw, rounds, N1, ref, ref_kind, seeds):
        self.w, self.prob, self.kw, self.rounds, self.N1 = w, prob, kw, rounds, N1
        self.ref, self.ref_kind, self.seeds = ref, ref_kind, seeds


def logreg_spec(oa, wl):
    w = wl.logreg_n10000_d50()
    prob = oa.Problem.logreg(w.params["X"], w.params["y"], w.ref_sigma2)
    kw = dict(move="mala", budget="double_t", T1=1, T_max=1000, eps0=w.eps0, eps_adapt=True,
              eps_kappa=w.params["X"].shape[0] / 4.0, accept_target=0.574, interp=0)
    return Spec(w, prob, kw, 11, w.N, None, "long run", 16)


def logreg_d200_spec(oa, wl):
    """The panel layout: n = 5000, d = 200, N = 8192, T = 1, 2, ..., 512
    (10 rounds); no log Z error by default (its long-run reference costs
    minutes at this d)."""
    w = wl.logreg_n5000_d200()
    prob = oa.Problem.logreg(w.params["X"], w.params["y"], w.ref_sigma2)
    kw = dict(move="mala", budget="double_t", T1=1, T_max=512, eps0=w.eps0, eps_adapt=True,
              eps_kappa=w.params["X"].shape[0] / 4.0, accept_target=0.574, interp=0)
    return Spec(w, prob, kw, 10, w.N, None, "long run", 0)


def gauss_spec(oa, wl):
    """The d = 10 Gaussian workload as stated: N = 128, 256, 512, 1024 over 4
    rounds, T = 64 (log Z = 5 ln(pi/2))."""
    w = wl.gaussian_d10(N=1024)
    prob = oa.Problem.gauss(w.params["mu"], w.params["sigma2"], w.ref_sigma2)
    kw = dict(move="rwmh", budget="double_n", T1=64, eps0=w.eps0)
    return Spec(w, prob, kw, 4, 128, 5 * np.log(np.pi / 2), "closed form", 32)


def gauss_sat_spec(oa, wl):
    """The same target at a particle count that fills the GPU (2^22, fixed), T = 64."""
    w = wl.gaussian_d10(N=1 << 22)
    prob = oa.Problem.gauss(w.params["mu"], w.params["sigma2"], w.ref_sigma2)
    kw = dict(move="rwmh", budget="fixed", T1=64, eps0=w.eps0)
    return Spec(w, prob, kw, 2, w.N, 5 * np.log(np.pi / 2), "closed form", 8)


def asmc_spec(oa, wl, trigger):
    """8-component mixture in d = 100, HMC (5 leapfrogs), resampling when the
    trigger (CESS_t / N or the relative ESS) drops below 0.5, or at the DAR
    times predicted from the previous round (trigger "dar"), N = 65536,
    T = 1, 2, ..., 1024, 2000 (log Z = 50 ln(0.2 pi))."""
    w = wl.gmm8_d100()
    prob = oa.Problem.gmm(w.params["means"], w.params["log_scales"], w.ref_sigma2)
    dar = trigger == "dar"
    kw = dict(move="hmc", leapfrog=5, resample_=True, trigger="ess" if dar else trigger, nu=0.5,
              budget="double_t", T1=1, T_max=2000, eps0=w.eps0, eps_adapt=True,
              eps_kappa=25.0 / 0.1 - 1.0, accept_target=0.65, dar=dar)
    return Spec(w, prob, kw, 12, w.N, 50 * np.log(0.2 * np.pi), "closed form", 4)


WORKLOADS = {"logreg": logreg_spec, "logreg_d200": logreg_d200_spec, "gauss": gauss_spec,
             "gauss_sat": gauss_sat_spec,
             "asmc": lambda oa, wl: asmc_spec(oa, wl, "cess"),
             "asmc_ess": lambda oa, wl: asmc_spec(oa, wl, "ess"),
             "asmc_dar": lambda oa, wl: asmc_spec(oa, wl, "dar")}


def cpu_baseline(w, res, spec, budget_s: float = 15.0) -> dict:
    """The CPU oracle on a bounded sample of the same workload: a particle
    subset of the last round (same schedule, step sizes and seed); for the
    resampling variant, whose particles interact, the last round at a smaller N."""
    import oracle as orc

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    k = int(np.max(np.nonzero(res["T"])[0]))
    T = int(res["T"][k])
    beta = res["beta"][k][: T + 1]
    eps = res["eps"][k][:T]
    resample = bool(spec.kw.get("resample_"))
    if w.family == "logreg":
        P = orc.Problem(family=orc.FAM_LOGREG, d=w.d, X=w.params["X"], y=w.params["y"],
                        ref_sigma2=w.ref_sigma2)
        move = orc.MOVE_MALA
    elif w.family == "gmm":
        P = orc.Problem(family=orc.FAM_GMM, d=w.d, means=w.params["means"],
                        log_scales=w.params["log_scales"], ref_sigma2=w.ref_sigma2)
        move = orc.MOVE_HMC
    else:
        P = orc.Problem(family=orc.FAM_GAUSS, d=w.d, mu=w.params["mu"], sigma2=w.params["sigma2"],
                        ref_sigma2=w.ref_sigma2)
        move = orc.MOVE_RWMH
    trig = {"ess": 0, "cess": 1}.get(spec.kw.get("trigger"), 0)
    opts = orc.Opts(move=move, leapfrog=spec.kw.get("leapfrog", 5), state_f32=1, nthreads=cores,
                    resample=int(resample), trigger=trig, nu=spec.kw.get("nu", 0.5))

    def go(n):
        if resample:
            orc.asmc(P, opts, n, beta, eps, 1234, round_k=k + 1)
        else:
            orc.asmc(P, opts, int(res["N"][k]), beta, eps, 1234, round_k=k + 1,
                     subset=np.arange(n), traces=False)

    # calibrate on a small sample, then size the timed sample to the budget
    n0 = cores
    t0 = time.perf_counter()
    go(n0)
    dt0 = time.perf_counter() - t0
    n1 = max(cores, int(n0 * budget_s / max(dt0, 1e-3)) // cores * cores)
    n1 = min(n1, int(res["N"][k]))
    t0 = time.perf_counter()
    go(n1)
    dt = time.perf_counter() - t0
    what = (f"the last round (schedule, step sizes, trigger) at N={n1}" if resample else
            f"{n1} particles x T={T} (last round's schedule) of the same workload")
    return {"value": n1 * T / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}, {dt:.1f} s"}


def long_run_reference(oa, spec, res, N: int = 1 << 17, T: int = 4000) -> float:
    """log Z_hat of one long run (N = 2^17, T = 4000) on a schedule rebuilt by
    Alg. 3 from the last round of `res`, with step sizes interpolated in beta."""
    k = int(np.max(np.nonzero(res["T"])[0]))
    Tk = int(res["T"][k])
    beta_k = res["beta"][k][: Tk + 1]
    beta, _ = oa.adapt_schedule(beta_k, res["log_g"][k][:, :Tk], T)
    eps = np.interp(beta[1:], beta_k[1:], res["eps"][k][:Tk])
    out = oa.asmc(spec.prob, N, beta, eps, 7777, round_k=99, move=spec.kw["move"],
                  return_state=False)
    return float(out["logZ"])


def logz_error(oa, spec, args, last_logz, res) -> dict:
    """Error of the last round's log Z_hat over independent seeds (the timed
    runs plus untimed ones), against the reference value."""
    S = args.rmse_seeds if args.rmse_seeds > 0 else spec.seeds
    vals = list(last_logz)
    i = 0
    while len(vals) < S:
        r = oa.run(spec.prob, spec.N1, spec.rounds, seed=args.seed + 5000 + i, **spec.kw)
        vals.append(float(r["logZ"][-1]))
        i += 1
    vals = np.array(vals[:S])
    ref = spec.ref
    if ref is None:
        ref = long_run_reference(oa, spec, res)
    err = vals - ref
    return {"seeds": int(len(vals)), "reference": float(ref), "reference_kind": spec.ref_kind,
            "rmse": float(np.sqrt(np.mean(err ** 2))), "mean_error": float(np.mean(err)),
            "sd": float(np.std(vals, ddof=1)) if len(vals) > 1 else None}


# ALU work models (lane-cycles per particle-step) of the extra workloads:
#  * gradient (mixture d = 20, K = 4, MALA): forward about 1.1e3 (5 Philox
#    blocks, 10 Box-Muller pairs, the mixture gradient) plus reverse about
#    2.8e3 (recomputation and the Hessian-vector adjoint);
#  * rejuvenation chains (Gaussian d = 10, RWMH): the sweep's 700 without the
#    moment statistics (100) plus the test-function sums (20): 620;
#  * a d-dimensional Gaussian RWMH problem of the batch: 140 per Philox block of
#    normals (ceil(d/4)), 22 per Box-Muller pair (ceil(d/2)), 3 per coordinate
#    for proposal and Delta log pi, 140 for the accept block, statistics and MH
#    (700 at d = 10, the sweep's model).
GRAD_WORK = 3.9e3
REJUV_WORK = 620.0
# Unid (d = 2) with the three-scale RWMH kernel: per substep one Philox block of
# normals (140), one Box-Muller pair (22), one accept block (140), the binomial
# log-likelihood ratio (two log1p, about 10) and the proposal/MH arithmetic
# (about 20); three substeps plus the moment statistics (100)
UNID_WORK = 3 * (140 + 22 + 140 + 10 + 20) + 100.0


def gauss_work(d: int) -> float:
    return 140.0 * -(-d // 4) + 22.0 * -(-d // 2) + 3.0 * d + 140.0


def oracle_rate(fn, n_lo: int, cap: int, budget_s: float = 12.0):
    """Times fn(n) for a calibrated n (particles) so that it takes about budget_s;
    returns (n, seconds)."""
    n0 = n_lo
    t0 = time.perf_counter()
    fn(n0)
    dt0 = time.perf_counter() - t0
    n1 = max(n_lo, min(cap, int(n0 * budget_s / max(dt0, 1e-3))))
    t0 = time.perf_counter()
    fn(n1)
    return n1, time.perf_counter() - t0


def zja_workload(args, oa, torch) -> int:
    """The paper's GPU comparison (Sec. "High-performance GPU implementation of
    adaptive schemes") on the Unid model with its GPU parameters (n = 1e11,
    k = 1e10, Uniform(0, 10)^2 reference), N = 2^14 particles, the three-scale
    RWMH kernel (0.1, 1, 10): one step = one OAIS run (T = 1, 2, ..., doubling
    over the rounds); ZJA runs beside it with the CESS threshold matched through
    D ~ Lambda^2 / T^2 (Lambda_hat and T of OAIS's last round).  Both are timed
    over the same seeds, with the relative variance of Z_hat against the Laplace
    form of the evidence, so the line reports OAIS's speed-up over ZJA at equal
    variance (time x variance, since the variance falls as 1/cost).  The
    relative variance is the sample variance of Z_hat over the seeds divided by
    the square of its sample mean; the log Z error against the Laplace form is
    reported beside it (at n = 1e11 the posterior sits on a ridge about 1e-7
    wide, which the three random-walk scales rarely move along, so both methods'
    estimates fall far below Z at these budgets)."""
    n, k, box, N, R = 1e11, 1e10, 10.0, 1 << 14, args.zja_rounds
    p = k / n
    logZ_ref = (np.log(np.log(box * box / p)) - 2 * np.log(box) +
                0.5 * np.log(2 * np.pi * p * (1 - p) / n))
    prob = oa.Problem.unid(n, k, box)
    kw = dict(move="rwmh3", budget="double_t", T1=1, T_max=1 << (R - 1), eps0=1.0)
    S = max(args.steps, 2)
    for i in range(args.warmup):
        oa.run(prob, N, R, seed=args.seed + i, **kw)
    torch.cuda.synchronize()
    oa.profile(True)
    t0 = time.perf_counter()
    runs = [oa.run(prob, N, R, seed=args.seed + 1000 + i, **kw) for i in range(S)]
    torch.cuda.synchronize()
    t_oais = (time.perf_counter() - t0) / S
    prof = oa.profile(False)
    TR = int(runs[0]["T"][-1])
    lam = float(np.mean([r["Lambda"][-1][TR] for r in runs]))
    rho = float(np.exp(-(lam / TR) ** 2))
    for i in range(args.warmup):
        oa.zja(prob, N, rho, 1 << 16, 1.0, args.seed + i, return_state=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zr = [oa.zja(prob, N, rho, 1 << 16, 1.0, args.seed + 1000 + i, return_state=False)
          for i in range(S)]
    torch.cuda.synchronize()
    t_zja = (time.perf_counter() - t0) / S
    lz_o = np.array([r["logZ"][-1] for r in runs])
    lz_z = np.array([r["logZ"] for r in zr])

    def rel_var(lz):
        # sample variance of Z_hat over the seeds relative to its mean (the
        # estimator is unbiased, so the mean stands in for Z); on log values
        w = np.exp(lz - lz.max())
        return float(np.var(w, ddof=1) / np.mean(w) ** 2)
    v_o, v_z = rel_var(lz_o), rel_var(lz_z)
    steps_run = float(np.sum(runs[0]["N"].astype(np.float64) * runs[0]["T"]))
    rate = prof["particle_steps"] / (prof["kernel_ms"] * 1e-3) if prof["kernel_ms"] else None
    peak = PEAK_LANE_CYCLES / UNID_WORK
    line = {"metric": METRIC, "value": steps_run / t_oais, "unit": "particle-steps/s",
            "n_gpus": 1, "steps": S, "warmup": args.warmup, "ms_per_step": t_oais * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 state / f64 arithmetic and weights", "data": "synthetic",
            "config": {"workload": "unid_n1e11_k1e10_rwmh3_oais_vs_zja", "N": N, "rounds": R,
                       "T_last": TR},
            "logZ_error": {"seeds": S, "reference": float(logZ_ref),
                           "reference_kind": "Laplace form of the evidence",
                           "rmse": float(np.sqrt(np.mean((lz_o - logZ_ref) ** 2))),
                           "mean_error": float(np.mean(lz_o - logZ_ref)),
                           "mean_error_zja": float(np.mean(lz_z - logZ_ref)),
                           "rel_var_Z_oais": v_o, "rel_var_Z_zja": v_z},
            "comparison": {"zja_rho": rho, "zja_T_mean": float(np.mean([r["T"] for r in zr])),
                           "oais_ms_per_run": t_oais * 1e3, "zja_ms_per_run": t_zja * 1e3,
                           "zja_over_oais_time": t_zja / t_oais,
                           "zja_over_oais_time_x_variance": (t_zja * v_z) / (t_oais * v_o)
                           if v_o > 0 else None},
            "roofline": {"bound": "alu", "achieved": rate, "peak": peak,
                         "unit": "particle-steps/s", "frac": rate / peak if rate else None,
                         "traffic": None, "kernel": "k_oais_valu (OAIS sweeps)",
                         "work_lane_cycles_per_particle_step": UNID_WORK,
                         "avg_launch_ms": prof["kernel_ms"] / max(prof["launches"], 1),
                         "launches": prof["launches"]},
            "cpu_baseline": None}
    if not args.no_cpu_baseline:
        import oracle as orc
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        P = orc.Problem(family=orc.FAM_UNID, d=2, binom_n=n, binom_k=k, box=box)
        bt = runs[0]["beta"][R - 1][:TR + 1]
        ep = runs[0]["eps"][R - 1][:TR]

        def go(m):
            orc.asmc(P, orc.Opts(move=orc.MOVE_RWMH3, state_f32=1, nthreads=cores), N, bt, ep,
                     args.seed, round_k=R, subset=np.arange(m))
        m, dt = oracle_rate(go, cores, N)
        line["cpu_baseline"] = {"value": m * TR / dt, "unit": "particle-steps/s", "cores": cores,
                                "kind": "oracle",
                                "sample": f"{m} particles x T={TR} (last OAIS round), {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    return 0


def pt_workload(args, oa, wl, torch) -> int:
    """Parallel tempering through the duality (Sec. "Computational duality with
    parallel tempering") on the d = 10 Gaussian target: K = 2048 copies of
    N' + 1 = 64 chains (one wave per copy) on the schedule Alg. 3 builds from an
    OAIS round, T' = 16384 iterations of RWMH plus even/odd swaps, RWMH scale
    2.38 / sqrt(d) times the standard deviation of pi_beta along the path
    (1 / sqrt(1 + 3 beta) here).  One step = one PT run; value = chain-steps/s;
    the stepping-stone log Z error over seeds against the closed form,
    Lambda_PT and the round-trip rate beside it.  Every chain starts from eta,
    so the stepping-stone estimate carries a burn-in bias of order 1 / T'
    (about -4.4, -1.1, -0.29 at T' = 256, 1024, 4096 in the oracle), and the
    round-trip rate approaches the non-reversible PT value from below."""
    import oracle as orc

    w = wl.gaussian_d10()
    prob = oa.Problem.gauss(w.params["mu"], w.params["sigma2"], w.ref_sigma2)
    K, Np, Tp = 2048, 63, 16384
    if args.autotune:
        oa.autotune(1)
    r0 = oa.run(prob, 1024, 2, seed=args.seed, move="rwmh", budget="fixed", T1=64, eps0=w.eps0)
    beta, _ = oa.adapt_schedule(r0["beta"][1], r0["log_g"][1], Np)
    eps = 2.38 / np.sqrt(w.d) / np.sqrt(1.0 + 3.0 * np.asarray(beta))
    for i in range(args.warmup):
        oa.pt(prob, K, beta, eps, Tp, args.seed + i)
    torch.cuda.synchronize()
    oa.profile(True)
    t0 = time.perf_counter()
    outs = [oa.pt(prob, K, beta, eps, Tp, args.seed + 100 + i) for i in range(args.steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = oa.profile(False)
    steps = float(K * (Np + 1) * Tp)
    ref = 5 * np.log(np.pi / 2)
    lz = np.array([o["logZ"] for o in outs])
    rej = outs[0]["rej"]
    rate = prof["particle_steps"] / (prof["kernel_ms"] * 1e-3)
    peak = PEAK_LANE_CYCLES / ALU_WORK["gauss"]
    line = {"metric": METRIC, "value": steps * args.steps / el, "unit": "particle-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 state / f64 arithmetic and weights",
            "data": "synthetic",
            "config": {"workload": "gauss_d10_rwmh_parallel_tempering", "copies": K,
                       "chains_per_copy": Np + 1, "iterations": Tp,
                       "shape": list(oa.shape(prob, K * (Np + 1)))},
            "logZ_error": {"seeds": int(len(lz)), "reference": float(ref),
                           "reference_kind": "closed form",
                           "rmse": float(np.sqrt(np.mean((lz - ref) ** 2))),
                           "mean_error": float(np.mean(lz - ref))},
            "pt": {"Lambda_PT": float(np.sum(rej)),
                   "round_trips_per_copy_iteration": outs[0]["trips"] / (K * Tp),
                   "nrpt_rate_from_rejections": float(1 / (2 + 2 * np.sum(rej / (1 - rej))))},
            "roofline": {"bound": "alu", "achieved": rate, "peak": peak, "unit": "particle-steps/s",
                         "frac": rate / peak, "traffic": None, "kernel": "k_pt",
                         "work_lane_cycles_per_particle_step": ALU_WORK["gauss"],
                         "avg_launch_ms": prof["kernel_ms"] / max(prof["launches"], 1),
                         "launches": prof["launches"]},
            "cpu_baseline": None}
    if not args.no_cpu_baseline:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        P = orc.Problem(family=orc.FAM_GAUSS, d=w.d, mu=w.params["mu"], sigma2=w.params["sigma2"],
                        ref_sigma2=w.ref_sigma2)

        def go(m):
            orc.pt(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1, nthreads=cores), m, beta, eps, Tp,
                   args.seed)
        m, dt = oracle_rate(go, cores, K)
        line["cpu_baseline"] = {"value": m * (Np + 1) * Tp / dt, "unit": "particle-steps/s",
                                "cores": cores, "kind": "oracle",
                                "sample": f"{m} copies x {Np + 1} chains x {Tp} iterations, {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    return 0


def extra_workload(args, oa, wl, torch) -> int:
    """The gradient (mixture d = 20, K = 4, N = 8192, T = 256 MALA, checkpoints
    every 16), final-iteration rejuvenation (N = 2^20 chains of 64 RWMH steps on
    the d = 10 Gaussian target), and the 256-problem batch (4 rounds: one
    hipGraph, or the same problems one plain run after another)."""
    import oracle as orc

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu = roof = None
    err = None
    if args.workload == "grad":
        w = wl.gmm4_d20()
        T = 256
        beta = np.linspace(0, 1, T + 1) ** 2
        eps = w.eps0 / np.sqrt(1 + 8 * beta[1:])
        prob = oa.Problem.gmm(w.params["means"], w.params["log_scales"], w.ref_sigma2)
        run = lambda i: oa.logZ_backward(prob, w.N, beta, eps, args.seed + i)
        steps_per = float(w.N * T)
        name, cfg = w.name + "_gradient", {"N": w.N, "T": T, "d": w.d, "K": 4}
        work, work_note = GRAD_WORK, "forward + reverse lane-cycles per particle-step"
        kern = "k_oais_valu (forward) + k_merge_slots + k_adjoint_gmm + k_adjoint_reduce"

        def cpu_fn(n):
            P = orc.Problem(family=orc.FAM_GMM, d=w.d, means=w.params["means"],
                            log_scales=w.params["log_scales"], ref_sigma2=w.ref_sigma2)
            orc.logZ_grad(P, orc.Opts(move=orc.MOVE_MALA, state_f32=1, nthreads=cores), n, beta,
                          eps, args.seed)
        cpu_what = "forward-mode gradient of log Z_hat over {n} particles x T=256 (same schedule)"
    elif args.workload == "rejuv":
        w = wl.gaussian_d10(N=1 << 20, T=64)
        T = 64
        prob = oa.Problem.gauss(w.params["mu"], w.params["sigma2"], w.ref_sigma2)
        beta = np.linspace(0, 1, T + 1)
        fin = oa.asmc(prob, w.N, beta, w.eps0, args.seed, move="rwmh")
        run = lambda i: oa.rejuvenate(prob, fin["lw"], fin["x"], T, w.eps0, args.seed + i)
        steps_per = float(w.N * T)
        name, cfg = w.name + "_rejuvenation", {"N": w.N, "T": T, "d": w.d}
        work, work_note = REJUV_WORK, "lane-cycles per chain step"
        kern = "k_rejuv"
        lw_h, x_h = fin["lw"].cpu().numpy(), fin["x"].cpu().numpy().astype(np.float64)

        def cpu_fn(n):
            P = orc.Problem(family=orc.FAM_GAUSS, d=w.d, mu=w.params["mu"],
                            sigma2=w.params["sigma2"], ref_sigma2=w.ref_sigma2)
            orc.rejuvenate(P, orc.Opts(move=orc.MOVE_RWMH, state_f32=1, nthreads=cores),
                           lw_h[:n], x_h[:n], T, w.eps0, args.seed)
        cpu_what = "rejuvenation of the first {n} particles of the population, T=64 chain steps"
    else:
        specs = wl.batch_problems()
        probs = []
        for s in specs:
            if s["family"] == "gauss":
                probs.append(oa.Problem.gauss(s["params"]["mu"], s["params"]["sigma2"], 1.0))
            else:
                probs.append(oa.Problem.logreg(s["params"]["X"], s["params"]["y"], 1.0))
        items = [oa.BatchItem(problem=p, N=s["N"], T=s["T"], move=s["move"], eps0=s["eps0"],
                              eps_adapt=s["eps_adapt"], eps_kappa=s["eps_kappa"], seed=args.seed,
                              problem_id=i) for i, (p, s) in enumerate(zip(probs, specs))]
        rounds = 4
        sequential = args.workload == "batch_seq"

        def run(i):
            if not sequential:
                return oa.run_batch(items, rounds, use_graph=True)
            for it in items:
                oa.run_batch([it], rounds, use_graph=False)

        Tks = [[min(max(1, s["T"] >> (rounds - 1)) << k, s["T"]) for k in range(rounds)]
               for s in specs]
        steps_per = float(sum(s["N"] * sum(tk) for s, tk in zip(specs, Tks)))
        # roofline time of one batch: each problem at its own bound (ALU model
        # for the Gaussian problems, FP32 MFMA for the contraction of the
        # logistic-regression problems, T + 1 evaluations per pass)
        roof_time = 0.0
        for s, tk in zip(specs, Tks):
            if s["family"] == "gauss":
                roof_time += s["N"] * sum(tk) * gauss_work(s["d"]) / PEAK_LANE_CYCLES
            else:
                n = s["params"]["X"].shape[0]
                roof_time += (s["N"] * sum(t + 1 for t in tk) * 4.0 * s["d"] * n /
                              (PEAK_FP32_MFMA_TFLOPS * 1e12))
        name = "batch_256_problems" + ("_sequential" if sequential else "_graph")
        cfg = {"problems": len(specs), "rounds": rounds,
               "d_logreg_max": max(s["d"] for s in specs if s["family"] == "logreg")}
        work = None
        kern = "k_oais_valu_batch + k_oais_logreg_batch + k_round_merge + k_round_schedule"
        g0 = next(i for i, s in enumerate(specs) if s["family"] == "gauss")
        l0 = next(i for i, s in enumerate(specs) if s["family"] == "logreg")

        def cpu_fn(n):
            for j in (g0, l0):
                s = specs[j]
                if s["family"] == "gauss":
                    P = orc.Problem(family=orc.FAM_GAUSS, d=s["d"], mu=s["params"]["mu"],
                                    sigma2=s["params"]["sigma2"])
                    mv = orc.MOVE_RWMH
                else:
                    P = orc.Problem(family=orc.FAM_LOGREG, d=s["d"], X=s["params"]["X"],
                                    y=s["params"]["y"])
                    mv = orc.MOVE_MALA
                T = s["T"]
                orc.asmc(P, orc.Opts(move=mv, state_f32=1, nthreads=cores), s["N"],
                         np.linspace(0, 1, T + 1), s["eps0"], args.seed, subset=np.arange(n))
        cpu_what = ("the last round of problems {g0} (Gaussian) and {l0} (logistic regression) "
                    "on the first {n} particles each")
        cpu_steps = lambda n: n * (specs[g0]["T"] + specs[l0]["T"])
    if args.autotune:
        oa.autotune(1)
        cfg["autotune"] = True
    oa.profile(True)
    for i in range(args.warmup):
        run(i)
    torch.cuda.synchronize()
    if args.autotune:
        cfg["autotuned_classes"] = oa.autotune(1)
    oa.profile(True)  # totals cleared: the timed region only
    t0 = time.perf_counter()
    for i in range(args.steps):
        run(i)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = oa.profile(False)
    if work is not None and prof["kernel_ms"] > 0:
        rate = prof["particle_steps"] / (prof["kernel_ms"] * 1e-3)
        peak = PEAK_LANE_CYCLES / work
        roof = {"bound": "alu", "achieved": rate, "peak": peak, "unit": "particle-steps/s",
                "frac": rate / peak, "traffic": None, "kernel": kern,
                "work_lane_cycles_per_particle_step": work, "work_note": work_note,
                "avg_launch_ms": prof["kernel_ms"] / max(prof["launches"], 1),
                "launches": prof["launches"]}
    elif work is None:
        t_batch = el / args.steps
        roof = {"bound": "mixed (alu per Gaussian problem, mfma per logistic-regression problem)",
                "achieved": steps_per / t_batch, "peak": steps_per / roof_time,
                "unit": "particle-steps/s", "frac": roof_time / t_batch, "traffic": None,
                "kernel": kern, "roofline_time_s": roof_time, "measured_time_s": t_batch}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        cap = {"grad": 8192, "rejuv": 1 << 20}.get(args.workload, 4096)
        n, dt = oracle_rate(cpu_fn, cores, cap)
        steps = cpu_steps(n) if args.workload in ("batch", "batch_seq") else n * T
        cpu = {"value": steps / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
               "sample": cpu_what.format(n=n, g0=locals().get("g0"), l0=locals().get("l0")) +
               f", {dt:.1f} s"}
    line = {"metric": METRIC, "value": steps_per * args.steps / el, "unit": "particle-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32 state / f64 arithmetic and weights",
            "data": "synthetic", "config": dict(workload=name, **cfg), "logZ_error": err,
            "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="logreg",
                    choices=sorted(WORKLOADS) + ["grad", "rejuv", "batch", "batch_seq", "zja",
                                                 "pt"])
    ap.add_argument("--autotune", action="store_true",
                    help="measure the VALU sweeps' launch shapes per problem class first")
    ap.add_argument("--zja-rounds", type=int, default=10,
                    help="OAIS rounds of the zja workload (T doubles from 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rmse-seeds", type=int, default=-1,
                    help="seeds for the log Z error (default per workload; 0 skips it)")
    ap.add_argument("--seed", type=int, default=20240812)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (3 times) and exit: "
                         "the reference for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import paper_2408_12057_amd as oa
    from paper_2408_12057_amd import workloads as wl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.calibrate_copy_mib:
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "repeats": 3}), flush=True)
        return 0
    if args.workload == "zja":
        return zja_workload(args, oa, torch)
    if args.workload == "pt":
        return pt_workload(args, oa, wl, torch)
    if args.workload in ("grad", "rejuv", "batch", "batch_seq"):
        return extra_workload(args, oa, wl, torch)
    spec = WORKLOADS[args.workload](oa, wl)
    w = spec.w
    log(f"workload {w.name}: N1={spec.N1} d={w.d} rounds={spec.rounds}")
    # the resampling path always takes the rule's shape; the autotuner serves
    # the AIS passes
    mv, lf = spec.kw.get("move", "rwmh"), spec.kw.get("leapfrog", 5)
    rule_shape = (oa.shape(spec.prob, spec.N1, move=mv, leapfrog=lf)
                  if w.family != "logreg" else None)
    if args.autotune:
        oa.autotune(1)
    res = None
    for i in range(args.warmup):
        res = oa.run(spec.prob, spec.N1, spec.rounds, seed=args.seed + i, **spec.kw)
    torch.cuda.synchronize()
    oa.profile(True)
    t0 = time.perf_counter()
    steps_done = 0.0
    last_logz = []
    for i in range(args.steps):
        res = oa.run(spec.prob, spec.N1, spec.rounds, seed=args.seed + 1000 + i, **spec.kw)
        steps_done += float(np.sum(res["N"].astype(np.float64) * res["T"]))
        last_logz.append(float(res["logZ"][-1]))
        log(f"step {i}: logZ per round {np.round(res['logZ'], 3).tolist()}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = oa.profile(False)
    value = steps_done / elapsed
    avg_ms = prof["kernel_ms"] / prof["launches"] if prof["launches"] else None
    if w.family == "logreg":
        traffic, traffic_profile = measured_traffic(args.workload)
        achieved = prof["flops"] / (prof["kernel_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                "traffic": traffic, "traffic_profile": traffic_profile,
                "kernel": ("k_oais_logreg_wide_batch<4, false>" if w.d > 64 else
                           "k_oais_logreg_batch<25, false>"), "avg_launch_ms": avg_ms,
                "launches": prof["launches"]}
    else:
        rate = prof["particle_steps"] / (prof["kernel_ms"] * 1e-3) if prof["kernel_ms"] else None
        peak = PEAK_LANE_CYCLES / ALU_WORK[args.workload]
        if spec.kw.get("dar"):
            kern = "k_oais_valu segments + k_seg_merge + resampler, per step"
        elif spec.kw.get("resample_"):
            kern = "k_asmc_step + k_asmc_merge + resampler, per step"
        else:
            kern = "k_oais_valu_batch"
        roof = {"bound": "alu", "achieved": rate, "peak": peak, "unit": "particle-steps/s",
                "frac": rate / peak if rate else None, "traffic": None, "kernel": kern,
                "work_lane_cycles_per_particle_step": ALU_WORK[args.workload],
                "avg_launch_ms": avg_ms, "launches": prof["launches"]}
    err = None
    if args.rmse_seeds > 0 or (args.rmse_seeds < 0 and spec.seeds > 0):
        log("log Z error over seeds (untimed) ...")
        err = logz_error(oa, spec, args, last_logz, res)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        cpu = cpu_baseline(w, res, spec)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state / f32 MFMA contraction / f64 weights",
        "data": "synthetic",
        "config": {"workload": w.name, "N_per_round": res["N"].tolist(), "d": w.d,
                   "rounds": spec.rounds, "T_per_round": res["T"].tolist(),
                   "n": int(w.params["X"].shape[0]) if w.family == "logreg" else None,
                   "trigger": (("dar" if spec.kw.get("dar") else spec.kw.get("trigger"))
                               if spec.kw.get("resample_") else None),
                   "n_resample_per_round": res["n_resample"].tolist(),
                   "Lambda_hat_last_round": float(res["Lambda"][-1][res["T"][-1]]),
                   "parallelism": "single GPU"},
        "logZ_error": err,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if w.family != "logreg":
        tuned = args.autotune and not spec.kw.get("resample_")
        shp = oa.shape(spec.prob, int(res["N"][-1]), move=mv, leapfrog=lf) if tuned else rule_shape
        line["config"]["shape"] = list(shp)
        line["config"]["autotune"] = bool(tuned)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
