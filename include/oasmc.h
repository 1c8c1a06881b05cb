/*
 * oasmc.h -- C ABI of the MI355X (gfx950) implementation of Optimised Annealed
 * SMC (OASMC) and Optimised Annealed Importance Sampling (OAIS), from
 * "Optimised Annealed Sequential Monte Carlo Samplers" (Syed, Bouchard-Cote,
 * Chern, Doucet, arXiv 2408.12057).
 *
 * Conventions for every entry point:
 *   - Plain C types only.  "device" pointers are HIP device memory owned by the
 *     caller; "host" pointers are host memory owned by the caller.  The library
 *     never returns memory it allocated; the only memory it owns is the
 *     workspace cached inside an oasmc_handle (released by
 *     oasmc_handle_destroy).
 *   - Every call returns an oasmc_status.  On failure nothing is thrown; a
 *     thread-local message is available from oasmc_last_error().  Arguments are
 *     validated before any device work (0 = beta_0 < ... < beta_T = 1, N >= 1,
 *     supported (family, move, d), finite scalars).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it.  Calls that return host results
 *     (oasmc_asmc, oasmc_run) synchronise that stream before returning.
 *   - Annealing path: the linear (geometric) path
 *       log gamma_beta(x) = log eta(x) + beta * ell(x),  ell = log gamma - log eta
 *     (Sec. 2; the linear-path example of the appendix on forward/backward
 *     kernels).  eta is the normalised Gaussian reference N(ref_mean, ref_sigma2 I).
 *   - Randomness: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed,
 *     counter (particle n, step t, round k | problem << 16,
 *     stream << 24 | substep << 16 | block); normals by Box-Muller in binary64
 *     from the words of each block.  Equal inputs give bitwise equal outputs.
 */
#ifndef OASMC_H
#define OASMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OASMC_OK = 0,
    OASMC_EINVAL = -1,       /* invalid argument (message says which) */
    OASMC_EHIP = -2,         /* a HIP runtime call failed */
    OASMC_ENOMEM = -3,       /* workspace allocation failed */
    OASMC_ENONFINITE = -4,   /* log Z_hat or the moments are not finite */
    OASMC_EUNSUPPORTED = -5  /* (family, move, d) combination not built */
} oasmc_status;

typedef enum { OASMC_GAUSS = 1, OASMC_LOGREG = 2, OASMC_GMM = 3, OASMC_UNID = 4 } oasmc_family;
/* OASMC_RWMH3: the alternation of three random-walk MH steps with proposal
 * standard deviations eps (0.1, 1, 10), one kernel per annealing step, used by
 * the paper's GPU experiments (appendix "GPU implementation"); the step's
 * accept bit is set when any of the three was accepted. */
typedef enum { OASMC_RWMH = 1, OASMC_MALA = 2, OASMC_HMC = 3, OASMC_RWMH3 = 4 } oasmc_move;

/*
 * Target gamma and reference eta.  All array pointers are DEVICE pointers to
 * fp32 data, read-only during the call.
 *   OASMC_GAUSS : gamma(x) = exp(-|x - mu|^2 / (2 sigma2))             mu[d]
 *   OASMC_LOGREG: gamma(x) = eta(x) prod_i s(z_i)^y_i (1 - s(z_i))^(1-y_i),
 *                 z_i = X[i,:] . x, s the logistic function;  X[n][d]
 *                 row-major, y[n] in {0, 1} (a label other than 0 is read
 *                 as 1), 1 <= d <= 256 (OASMC_EUNSUPPORTED above).  ell is
 *                 the log-likelihood.
 *   OASMC_GMM   : gamma(x) = (1/K) sum_k exp(-|x - means[k]|^2 / (2 exp(2 log_scales[k])))
 *                 means[K][d], log_scales[K].
 *   OASMC_UNID  : the unidentifiable product parameterisation (appendix on the
 *                 models): d = 2, eta = Uniform(0, box)^2, gamma = eta times the
 *                 likelihood Binomial(binom_k | binom_n, x y) divided by its
 *                 maximum (at x y = k / n), zero unless 0 < x y < 1; so
 *                 log Z_hat estimates log Z - log Binomial(k | n, k / n).
 *                 Moves RWMH and RWMH3 only.
 *   eta         : N(ref_mean, ref_sigma2 I) (all families but OASMC_UNID);
 *                 ref_mean may be NULL (zero mean).
 */
typedef struct {
    int32_t family;
    int32_t d;
    const float* mu;
    double sigma2;
    const float* X;
    const float* y;
    int32_t n;
    int32_t K;
    const float* means;
    const float* log_scales;
    const float* ref_mean;
    double ref_sigma2;
    double binom_n, binom_k, box; /* OASMC_UNID */
} oasmc_problem;

/*
 * Forward kernel and resampling (Alg. 1).
 *   move     : pi_beta-invariant MH kernel K_{beta_t} (one step per t).
 *   leapfrog : HMC leapfrog steps per trajectory (>= 1).
 *   resample : 0 = AIS (no intermediate resampling; particle and time loops
 *              swapped, Sec. "Optimised AIS"), 1 = resampling at the times
 *              `trigger` selects (Sec. "Resample step", resampling strategies).
 *   trigger  : 0 = relative ESS of w_{t^-} < nu (adaptive, AR),
 *              1 = CESS_t / N < nu (CESS of the section connecting to online
 *                  CESS optimisation),
 *              2 = after every step t < T (SIR),
 *              3 = after the steps t < T with resample_at[t-1] != 0 (times fixed
 *                  in advance, e.g. the DAR times of oasmc_dar_times).  Between
 *                  two such times the particles run loop-swapped as in an AIS
 *                  pass (state in registers, no per-step synchronisation); the
 *                  per-step relative ESS is then not streamed (NaN).
 *   nu       : threshold in (0, 1) (triggers 0 and 1; also the DAR threshold of
 *              oasmc_run_opts.dar).
 *   slots    : AIS passes only: number S of O(T) moment accumulators the
 *              particle tiles are folded into (tile i into slot i mod S, in
 *              tile order).  0 = min(#tiles, 2048), the default; otherwise
 *              min(#tiles, slots).  Trajectories do not depend on S; the
 *              moments and log Z_hat change only by rounding (a smaller S
 *              folds several tiles into each accumulator).
 */
typedef struct {
    int32_t move;
    int32_t leapfrog;
    int32_t resample;
    int32_t trigger;
    double nu;
    int32_t slots;
    const int32_t* resample_at; /* host [T] (trigger 3), read during the call; else unused */
} oasmc_kernel;

/* Outputs of one ASMC pass.  Host arrays sized by the caller; NULL skips. */
typedef struct {
    double* log_g;        /* host [3*T]: log g_hat_{t,i} at [i*T + t-1]  (eq. CESS) */
    double* accept;       /* host [T]: fraction of moves accepted at step t */
    double* ess;          /* host [T] or NULL: relative ESS of w_{t^-} */
    int32_t* resampled;   /* host [T] or NULL: 1 where step t resampled */
    double logZ;          /* out: log Z_hat (estimator_Z) */
    int32_t n_resample;   /* out: resampling events before T */
    double* lw;           /* device [N] or NULL: final log-weights */
    float* x;             /* device [N*d] or NULL: final states, row-major */
    uint32_t* accept_bits;/* device [N * ceil(T/32)] or NULL: bit (t-1)%32 of word
                             n*ceil(T/32) + (t-1)/32 is set when particle n's
                             move at step t was accepted */
} oasmc_round_out;

typedef struct oasmc_handle_s oasmc_handle;

/* Create a handle bound to HIP device `device`; owns the workspace. */
int oasmc_handle_create(oasmc_handle** h, int device);
/* Free the workspace and the handle.  NULL is accepted. */
int oasmc_handle_destroy(oasmc_handle* h);
/* Message for the last failure on the calling thread ("" if none). */
const char* oasmc_last_error(void);

/*
 * Alg. 1, ASMC(N, B_T): one pass with schedule beta[0..T] (host, strictly
 * increasing, beta[0] = 0, beta[T] = 1) and per-step step sizes eps[0..T-1]
 * (host; RWMH proposal standard deviation, MALA Langevin step, HMC leapfrog
 * step).  Particles start iid from eta, carry binary32 states and binary64
 * log-weights; the incremental weight is evaluated at the pre-move state,
 *   log g_t = (beta_t - beta_{t-1}) ell(X_{t-1}),
 * then one MH move targeting pi_{beta_t} is applied.  round_k and problem_id
 * only select random-number streams.
 */
int oasmc_asmc(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
               int64_t N, int32_t T, const double* beta, const double* eps, uint64_t seed,
               uint32_t round_k, uint32_t problem_id, oasmc_round_out* out, void* stream);

/*
 * The online CESS-adaptive AIS of Zhou, Johansen and Aston (ZJA), the
 * comparison method of Sec. "Connection to online conditional ESS
 * optimisation" and of the GPU comparison: after each step the next annealing
 * parameter is chosen from the current weighted particles so that
 * CESS_t / N = g_1^2 / (g_0 g_2) (eq. CESS) equals rho: beta_t = 1 when CESS at
 * 1 is already >= rho N, else `iters` bisection halvings of (beta_{t-1}, 1]
 * keeping the upper part while CESS >= rho N; at t = Tmax beta_t is set to 1.
 * The selection runs on the device (one workgroup over all particles), then the
 * step reweights and moves every particle as oasmc_asmc does (AIS: kernel's
 * resample must be 0; constant step size eps).  Random streams as oasmc_asmc.
 * Outputs: beta[0..T] (host, capacity Tmax + 1), *T_out, log_g (host [3*Tmax],
 * layout i * Tmax + t - 1, may be NULL), *logZ, final lw[N] and x[N*d]
 * (device, may be NULL).  Gaussian, mixture and Unid families.  Synchronises
 * `stream` once per 32 steps.
 */
int oasmc_zja(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel, int64_t N,
              double rho, int32_t Tmax, int32_t iters, double eps, uint64_t seed, uint32_t round_k,
              uint32_t problem_id, double* beta, int32_t* T_out, double* log_g, double* logZ,
              double* lw, float* x, void* stream);

/*
 * Parallel tempering (Sec. "Computational duality with parallel tempering"):
 * K independent copies of Np + 1 chains at the temperatures beta[0..Np] (host,
 * 0 = beta_0 < ... < beta_Np = 1) with step sizes eps[0..Np] (host), run for
 * Tp iterations.  Every chain starts from eta; iteration t applies the kernel's
 * move at each chain's temperature (counters (copy (Np + 1) + replica, t)) and
 * then proposes the swaps of temperatures (n, n + 1) for the n of the parity of
 * t (non-reversible, deterministic even/odd), accepted iff
 * log u < (beta_{n+1} - beta_n)(ell(y at n) - ell(y at n + 1)) with u from stream
 * 4, counter (copy (Np + 1) + n, t).  One workgroup per copy; a copy holds at
 * most 8 waves of chains (OASMC_EUNSUPPORTED above).  Outputs (host; each but
 * logZ may be NULL):
 * *logZ = sum_n ss[n], ss[n] the log of the mean of
 * exp((beta_{n+1} - beta_n) ell) over the K Tp states at temperature n (the
 * stepping-stone estimator eq. (Z_PT), pooled over copies); rej[n] the mean
 * swap rejection 1 - min(1, alpha) of pair (n, n + 1), whose sum estimates the
 * communication barrier Lambda_PT; *trips the round trips (temperature 0 to Np
 * and back) of all replicas; tmean[d], tsecond[d] the averages of x_i and x_i^2
 * over the K Tp states at temperature Np.  Gaussian, mixture and Unid families.
 * Synchronises `stream`.
 */
int oasmc_pt(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel, int32_t K,
             int32_t Np, int32_t Tp, const double* beta, const double* eps, uint64_t seed,
             uint32_t round_k, uint32_t problem_id, double* logZ, double* ss, double* rej,
             int64_t* trips, double* tmean, double* tsecond, void* stream);

/*
 * Final-iteration rejuvenation (Sec. "Computing expectations"): after a pass,
 * resample its final population (log-weights lw[N], states x[N*d], both
 * device, e.g. oasmc_round_out.lw / .x) with the systematic resampler and the
 * event word of step T (stream 3, particle word 0xFFFFFFFF), then run N chains
 * of T steps of the kernel's move at beta = 1 with step size eps_T, chain n
 * from its resampled particle and drawing with counters (n, T + s), s = 1..T.
 * The TN chain states estimate expectations under the target: host outputs
 * mean[d] and second[d] (averages of x_i and x_i^2), *accept (fraction of
 * accepted chain moves, may be NULL), and the chain end states x_out[N*d]
 * (device, may be NULL).  Gaussian and mixture families; seed, round_k and
 * problem_id those of the pass.  OASMC_ENONFINITE when no weight is finite.
 * Synchronises `stream`.
 */
int oasmc_rejuvenate(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                     int64_t N, int32_t T, double eps_T, uint64_t seed, uint32_t round_k,
                     uint32_t problem_id, const double* lw, const float* x, double* mean,
                     double* second, double* accept, float* x_out, void* stream);

/*
 * Alg. 3, OptimiseSchedule(T_new, B_T, g_hat) on the host:
 *   D_hat_t = log g_hat_{t,2} - 2 log g_hat_{t,1} + log g_hat_{t,0} (negative
 *   roundoff clamped to 0), Lambda_hat_t = sum_{s<=t} sqrt(D_hat_s), a monotone
 *   interpolant of the knots (Lambda_hat_t, beta_t), beta*_{t'} =
 *   Lambda_hat^{-1}(Lambda_hat_T t'/T_new).
 * beta[T+1], log_g[3*T] (layout of oasmc_round_out.log_g) in; beta_new[T_new+1]
 * and Lambda_hat[T+1] (may be NULL) out, all host.  interp: 0 = monotone
 * piecewise cubic (Fritsch-Carlson), 1 = piecewise linear.  A zero or
 * non-finite Lambda_hat_T yields the uniform schedule (status OASMC_ENONFINITE
 * when non-finite).
 */
int oasmc_adapt_schedule(int32_t T, const double* beta, const double* log_g, int32_t T_new,
                         int32_t interp, double* beta_new, double* Lambda_hat);

/*
 * Launch-shape autotuning of the loop-swapped sweeps of the Gaussian and
 * mixture families (AIS passes of oasmc_asmc, oasmc_run and oasmc_run_batch):
 * a particle spans LPP lanes of DPL coordinates.  enable = 1: the first pass of
 * a problem class (family, move, d, N rounded up to a power of two, HMC's
 * leapfrog steps, K) times every built shape that holds d on a 4-step pass of the problem
 * itself (two runs each, HIP events) and keeps the fastest (the fixed rule's
 * shape unless another is 2% faster) in the handle; later passes of the class
 * reuse it.  enable = 0: the fixed rule.  enable = -1: the fixed rule and the
 * measured shapes are forgotten.  *n_classes (may be NULL) gets the number of
 * classes measured.  Results depend on the shape only through the binary64
 * summation order of a particle's lanes.  Not for use under graph capture (the
 * measurement synchronises its stream).
 */
int oasmc_autotune(oasmc_handle* h, int32_t enable, int32_t* n_classes);

/* The shape (lanes per particle, coordinates per lane) the next AIS pass of
 * this problem would use, measuring it first when autotuning is on. */
int oasmc_shape(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                int64_t N, int32_t* lpp, int32_t* dpl, void* stream);

/*
 * Deterministic adaptive resampling (DAR) times for a new schedule, predicted
 * from a previous round (Sec. "Effective resample size for deterministic
 * adaptive resampling", eq. (DAR-times); AR converges to DAR as N grows, by the
 * appendix on adaptive resampling in the large particle limit).  Host only:
 *   - D_hat_t, Lambda_hat_t = sum_{s<=t} sqrt(D_hat_s) on the previous schedule
 *     beta[T+1] from its moments log_g[3*T] (layout of oasmc_round_out.log_g;
 *     negative D_hat clamped to 0, as in Alg. 3);
 *   - Lambda(b): the monotone interpolant through (beta_t, Lambda_hat_t)
 *     (interp 0: Fritsch-Carlson cubic, 1: linear);
 *   - predicted D_pred_t = (Lambda(beta_new_t) - Lambda(beta_new_{t-1}))^2 from
 *     sqrt D(b, b') ~ integral of the local barrier over [b, b'];
 *   - an event at the first t after the previous one whose summed D_pred
 *     exceeds -log nu; flags[t-1] = 1 for each event t < T_new.
 * Outputs flags[T_new] (int32) and D_pred[T_new] (may be NULL), host.  nu in
 * (0, 1).  Non-finite moments: no events and OASMC_ENONFINITE.
 */
int oasmc_dar_times(int32_t T, const double* beta, const double* log_g, int32_t T_new,
                    const double* beta_new, int32_t interp, double nu, int32_t* flags,
                    double* D_pred);

/*
 * Budget rule between rounds (Alg. 2, Sec. on increasing N and T):
 *   OASMC_BUDGET_FIXED   : N, T unchanged
 *   OASMC_BUDGET_DOUBLE_N: N doubles, T unchanged
 *   OASMC_BUDGET_DOUBLE_T: N unchanged, T doubles
 *   OASMC_BUDGET_SQRT2   : N and T grow by sqrt(2) until N would exceed
 *                          N_max, then N stays and T doubles
 * T is capped at T_max when T_max > 0.
 */
typedef enum {
    OASMC_BUDGET_FIXED = 0,
    OASMC_BUDGET_DOUBLE_N = 1,
    OASMC_BUDGET_DOUBLE_T = 2,
    OASMC_BUDGET_SQRT2 = 3
} oasmc_budget;

/*
 * Round-loop options.  Round 1 uses the uniform schedule with T1 steps.
 * Step sizes: eps_adapt = 0 keeps eps_t = eps0; eps_adapt = 1 starts from
 * eps0 (1 + beta_t eps_kappa)^(-1/2) and between rounds moves
 * log eps(beta) by (acceptance(beta) - accept_target), piecewise linear in beta
 * (kernel adaptation across rounds, appendix on exploration kernels).
 */
typedef struct {
    int32_t budget;
    int32_t T1;
    int32_t T_max;
    int64_t N_max;
    int32_t eps_adapt;
    double eps0;
    double eps_kappa;
    double accept_target;
    int32_t interp;
    int32_t dar;   /* with resample = 1: rounds k >= 2 resample at the DAR times that
                      oasmc_dar_times predicts from round k-1 for round k's schedule
                      (threshold kernel->nu; trigger and resample_at are ignored);
                      round 1, with no previous round, resamples at no step before T */
} oasmc_run_opts;

/* Per-round outputs (host arrays sized by the caller, row capacity Tcap). */
typedef struct {
    int32_t rounds;       /* in: number of rounds */
    int32_t Tcap;         /* in: row capacity, >= every T_k */
    double* logZ;         /* [rounds] */
    int64_t* N;           /* [rounds] */
    int32_t* T;           /* [rounds] */
    double* beta;         /* [rounds][Tcap+1] */
    double* Lambda_hat;   /* [rounds][Tcap+1] */
    double* log_g;        /* [rounds][3][Tcap] */
    double* accept;       /* [rounds][Tcap] */
    double* eps;          /* [rounds][Tcap] */
    int32_t* n_resample;  /* [rounds] */
    int32_t rounds_done;  /* out: rounds whose outputs are valid (anytime property) */
    double* rejuv_mean;   /* [rounds][d] or NULL: with rejuv_second, final-iteration */
    double* rejuv_second; /* rejuvenation after every round (oasmc_rejuvenate with the
                             round's last step size; Gaussian and mixture families) */
} oasmc_run_out;

/*
 * Alg. 2, OASMC: rounds k = 1..rounds of oasmc_asmc (random streams keyed by
 * round k), each followed by Budget and OptimiseSchedule.  Each round's log
 * Z_hat is unbiased and available at a predictable time; on error the rounds
 * already completed stay valid (rounds_done).
 */
int oasmc_run(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
              const oasmc_run_opts* opts, int64_t N1, uint64_t seed, uint32_t problem_id,
              oasmc_run_out* out, void* stream);

/*
 * One problem of a batch: its target, kernel (resample must be 0), particle
 * count, the number of steps T of its last round (round k of R uses
 * max(1, T >> (R-1)) doubled each round and capped at T), step-size settings
 * as in oasmc_run_opts, and its random streams (seed, problem_id).
 */
typedef struct {
    oasmc_problem problem;
    oasmc_kernel kernel;
    int64_t N;
    int32_t T;
    int32_t eps_adapt;
    double eps0;
    double eps_kappa;
    double accept_target;
    uint64_t seed;
    uint32_t problem_id;
} oasmc_batch_problem;

/* Outputs of a batch (host arrays [P][rounds]; Lambda_T and status may be NULL). */
typedef struct {
    double* logZ;        /* log Z_hat of every problem and round */
    double* Lambda_T;    /* Lambda_hat_T (estimated global barrier) of every problem and round */
    int32_t* status;     /* 1 where a round's moments were not finite */
} oasmc_batch_out;

/*
 * Alg. 2 for P independent problems at once (AIS passes, N fixed, T doubling
 * per round).  Problems are grouped by kernel class; each round launches one
 * kernel per class over a work list of (problem, slot) items, longest first,
 * claimed by the workgroups from a per-class counter, then merges every
 * problem's moments and runs Alg. 3 and the step-size update on the device,
 * one workgroup per problem — no host round trip between rounds.  With more
 * than one problem the classes of a round run on two streams of the
 * handle, forked from `stream` and joined back into it by events before the
 * round's merge (so all work stays ordered after earlier work on `stream`).
 * use_graph = 1 captures all rounds as one hipGraph (kept in the handle and
 * replayed while the batch is unchanged).  Each problem's results are bitwise
 * those of oasmc_run on it alone (budget DOUBLE_T, T1 = max(1, T >> (R-1)),
 * T_max = T, interp 0).  Synchronises `stream`.
 */
int oasmc_run_batch(oasmc_handle* h, const oasmc_batch_problem* problems, int32_t P,
                    int32_t rounds, int32_t use_graph, oasmc_batch_out* out, void* stream);

/*
 * Systematic resampling (Alg. 1 resample step): given device log-weights
 * lw[N] and a 32-bit uniform word u, writes device ancestors anc[N] with
 * Pr[a = m] = W_m.  Weights are quantised to q_m = floor(exp(lw_m - max) 2^B),
 * B = 62 - ceil(log2 N); the CDF is their exact integer prefix sum and point n
 * is floor(S (2 (n 2^32 + u) + 1) / (N 2^33)); a_n = min{m : C_m > p_n}.
 * Weights below 2^-B of the largest are never chosen.  OASMC_ENONFINITE if no
 * weight is finite.
 */
int oasmc_resample(oasmc_handle* h, int64_t N, const double* lw, uint32_t u, int32_t* anc,
                   void* stream);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * systematic resampling as oasmc_resample, with the same kernels and bitwise
 * the same ancestors, but its scratch (integer CDF, block totals, flag words)
 * is a fixed static device array of about 8.0 MiB (OASMC_NOALLOC_MAX_N
 * uint64 words plus 4 KiB), one copy per GPU, held until the process ends.
 * No handle; runs on the current HIP device, whose scratch address is looked
 * up on the first call on that device.  lw[N] (device, binary64) and anc[N]
 * (device, int32) are the caller's; N must lie in [1, OASMC_NOALLOC_MAX_N]
 * (else OASMC_EINVAL before any device work).  Asynchronous: the call only
 * enqueues kernels on `stream` and synchronises nothing; when no weight is
 * finite every anc[n] is -1.  Every call on one GPU shares that GPU's
 * scratch, so calls that overlap on one GPU (other streams or threads) race
 * and must be ordered by the caller.  Allocates nothing.
 */
#define OASMC_NOALLOC_MAX_N ((int64_t)1 << 20)
int oasmc_resample_noalloc(int64_t N, const double* lw, uint32_t u, int32_t* anc, void* stream);

/*
 * Gradient of log Z_hat with respect to the mixture target's parameters
 * theta = (means[K][d], log_scales[K]) for one AIS pass with MALA moves
 * (same arguments and random streams as oasmc_asmc), differentiating the
 * whole T-step chain pathwise with every MH accept decision held at its
 * forward value (binary32 rounding of the states differentiated as the
 * identity).  The forward pass checkpoints the states every 16 steps; the
 * reverse pass recomputes each segment from its checkpoint and applies the
 * adjoint of every step (Hessian-vector and mixed products of the mixture
 * log-density).  Outputs (host): *logZ, and grad[K*d + K] in binary64 in the
 * order of theta.  Supported: OASMC_GMM, OASMC_MALA, resample = 0, d <= 32,
 * K <= 8 (else OASMC_EUNSUPPORTED).  Synchronises `stream`.
 */
int oasmc_logZ_backward(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                        int64_t N, int32_t T, const double* beta, const double* eps,
                        uint64_t seed, uint32_t round_k, uint32_t problem_id, double* logZ,
                        double* grad, void* stream);

/*
 * The log-likelihood contraction of the logistic-regression family on its
 * own: for N states theta[N][d] (device fp32, row-major) writes
 * ell[n] = sum_i y_i z_ni - log(1 + exp(z_ni)), z = theta X^T (device binary64),
 * and grad[n][:] = sum_i (y_i - s(z_ni)) X_i (device fp32), with the same FP32
 * MFMA kernel the sweep uses.  Device-synchronous on `stream`.
 */
int oasmc_logreg_eval(oasmc_handle* h, const oasmc_problem* problem, int64_t N,
                      const float* theta, double* ell, float* grad, void* stream);

/*
 * ell(x) = log gamma(x) - log eta(x) and its gradient for the closed-form
 * families (OASMC_GAUSS, OASMC_GMM, OASMC_UNID; the target definitions above)
 * at N given states x[N][d] (device fp32, row-major), evaluated by the
 * annealing sweeps' own binary64 particle arithmetic in the lane layout of
 * the shape lpp lanes x dpl coordinates per particle (lpp = dpl = 0: the
 * sweep's default shape for this d and N; otherwise a built shape with
 * lpp dpl >= d, else OASMC_EINVAL).  Writes ell[N] and grad[N][d] (device
 * binary64; the Unid target's gradient is zero).  Device-synchronous on
 * `stream`.  Logistic regression: OASMC_EINVAL (use oasmc_logreg_eval).
 */
int oasmc_target_eval(oasmc_handle* h, const oasmc_problem* problem, int64_t N, const float* x,
                      int32_t lpp, int32_t dpl, double* ell, double* grad, void* stream);

/*
 * Live timing of the annealing-sweep kernels.  enable = 1 starts recording a
 * HIP event pair around every sweep-kernel launch (on the launch stream) and
 * clears the totals; enable = 0 stops.  Outputs (each may be NULL): summed
 * kernel time in ms, number of launches, and the algorithmic work of those
 * launches (particle-steps, and for the logistic-regression family the
 * contraction flops 4 d n per particle and evaluation, evaluations = T + 1 per
 * particle per pass).  The resampling variant, which launches several kernels
 * per step, is timed as a whole and counts one launch per step.  A run
 * captured in a hipGraph (oasmc_run_batch with use_graph) is timed as one
 * launch.
 */
int oasmc_profile(oasmc_handle* h, int32_t enable, double* kernel_ms, int64_t* launches,
                  double* particle_steps, double* flops);

/*
 * Raw Philox4x32-10 blocks on the device (used to check the generator):
 * out[4*i .. 4*i+3] = Philox4x32-10(ctr[4*i .. 4*i+3], key = (seed lo, seed hi)).
 * ctr and out are device arrays of 4*count uint32.
 */
int oasmc_philox(oasmc_handle* h, uint64_t seed, const uint32_t* ctr, uint32_t* out,
                 int64_t count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OASMC_H */
