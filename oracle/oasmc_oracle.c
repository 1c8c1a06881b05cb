/*
 * oasmc_oracle.c -- plain, slow, fp64 CPU oracle for Optimised Annealed SMC
 * (OASMC) and its annealed-importance-sampling special case (OAIS), written
 * from "Optimised Annealed Sequential Monte Carlo Samplers" (Syed,
 * Bouchard-Cote, Chern, Doucet, arXiv 2408.12057).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product (the HIP
 * library under paper_2408_12057_amd/) never includes, links or calls it, and
 * this file includes nothing from the product.
 *
 * Everything is IEEE binary64.  The one concession to the fp32 state that the
 * benchmarked configurations prescribe is the `state_f32` option: when set,
 * every stored particle coordinate is rounded to binary32 right after it is
 * produced (initial draw, proposal), and all arithmetic stays fp64.
 *
 * Sections of the paper each function follows:
 *   asmc()            -- Alg. 1 (ASMC): init from eta, propagate with a
 *                        pi_beta-invariant MCMC kernel, incremental weight of
 *                        the quasi-reversal backward kernel at the PRE-move
 *                        state, moments g_hat_{t,i}, reweight, optional
 *                        resampling, Z_hat = prod_r mean(w_{tau_r^-}).
 *   the AIS branch    -- Sec. "Optimised AIS (OAIS)": particle loop outside
 *                        the time loop (no resampling, particles independent).
 *   moments           -- eq. (CESS): g_hat_{t,i} = sum_n w_{t-1}^n (g_t^n)^i.
 *   optimise_schedule -- Alg. 3 with a monotone (Fritsch-Carlson PCHIP)
 *                        interpolant of the knots (Lambda_hat_t, beta_t).
 *   run()             -- Alg. 2 (OASMC round loop) with the Budget rules of
 *                        Sec. "Increasing the number of particles and ASMC
 *                        iterations" and the across-round kernel adaptation of
 *                        the appendix on exploration kernels.
 *   Philox4x32-10     -- Salmon, Moraes, Dror, Shaw, "Parallel random
 *                        numbers: as easy as 1, 2, 3", SC'11 (its published
 *                        definition), used for common random numbers.
 *
 * Readings of the paper where it is silent are listed in the design notes;
 * the ones that shape this code are restated next to the code they shape.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------------ */
/* Status codes (same meaning as the product's, defined independently).     */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)
#define ORC_ENONFINITE (-4)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                                     */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL0 = 0xD2511F53u;
static const uint32_t PHILOX_MUL1 = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL0 = 0x9E3779B9u;
static const uint32_t PHILOX_WEYL1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: Weyl sequence */
            k0 += PHILOX_WEYL0;
            k1 += PHILOX_WEYL1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_MUL0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_MUL1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Counter layout (the paper only asks for split generators so that CPU and
 * GPU produce the same realisation; this layout is the reading adopted):
 *   key  = (seed low 32 bits, seed high 32 bits)
 *   c0   = particle index n (global), c1 = annealing step t (0 = initial draw)
 *   c2   = (round k & 0xFFFF) | (problem id << 16)
 *   c3   = (stream << 24) | (substep << 16) | block
 * streams: 0 initial normals, 1 move normals, 2 accept uniform,
 *          3 resampling uniform.
 */
enum { STREAM_INIT = 0, STREAM_MOVE = 1, STREAM_ACCEPT = 2, STREAM_RESAMPLE = 3 };

typedef struct {
    uint64_t seed;
    uint32_t round_k;
    uint32_t problem;
} rng_key;

static void draw_block(const rng_key* K, uint32_t n, uint32_t t, uint32_t stream,
                       uint32_t substep, uint32_t block, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = n;
    ctr[1] = t;
    ctr[2] = (K->round_k & 0xFFFFu) | (K->problem << 16);
    ctr[3] = (stream << 24) | ((substep & 0xFFu) << 16) | (block & 0xFFFFu);
    key[0] = (uint32_t)(K->seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(K->seed >> 32);
    orc_philox4x32_10(ctr, key, out);
}

/* A 32-bit word w maps to the open-interval uniform (w + 1/2) 2^-32. */
static double word_to_uniform(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/*
 * Standard normals by the Box-Muller transform: block b supplies normals
 * 4b..4b+3; words (w0,w1) give 4b (cosine) and 4b+1 (sine), words (w2,w3)
 * give 4b+2 and 4b+3.  r = sqrt(-2 log u_a), angle = 2 pi u_b.
 */
static void draw_normals(const rng_key* K, uint32_t n, uint32_t t, uint32_t stream,
                         uint32_t substep, int count, double* z)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < count; j += 4) {
        uint32_t w[4];
        draw_block(K, n, t, stream, substep, (uint32_t)(j / 4), w);
        for (int pair = 0; pair < 2; ++pair) {
            double ua = word_to_uniform(w[2 * pair]);
            double ub = word_to_uniform(w[2 * pair + 1]);
            double r = sqrt(-2.0 * log(ua));
            double ang = two_pi * ub;
            int j0 = j + 2 * pair;
            if (j0 < count) z[j0] = r * cos(ang);
            if (j0 + 1 < count) z[j0 + 1] = r * sin(ang);
        }
    }
}

static double draw_uniform(const rng_key* K, uint32_t n, uint32_t t, uint32_t stream,
                           uint32_t substep)
{
    uint32_t w[4];
    draw_block(K, n, t, stream, substep, 0u, w);
    return word_to_uniform(w[0]);
}

/* Exported for the RNG pins. */
void orc_normals(uint64_t seed, uint32_t round_k, uint32_t problem, uint32_t n, uint32_t t,
                 uint32_t stream, uint32_t substep, int count, double* z)
{
    rng_key K = {seed, round_k, problem};
    draw_normals(&K, n, t, stream, substep, count, z);
}

double orc_uniform(uint64_t seed, uint32_t round_k, uint32_t problem, uint32_t n, uint32_t t,
                   uint32_t stream, uint32_t substep)
{
    rng_key K = {seed, round_k, problem};
    return draw_uniform(&K, n, t, stream, substep);
}

/* ------------------------------------------------------------------------ */
/* Targets, reference, annealing path.                                       */
/* ------------------------------------------------------------------------ */
enum { FAM_GAUSS = 1, FAM_LOGREG = 2, FAM_GMM = 3, FAM_UNID = 4 };
enum { MOVE_RWMH = 1, MOVE_MALA = 2, MOVE_HMC = 3, MOVE_EXACT = 4, MOVE_IDENTITY = 5,
       MOVE_RWMH3 = 6 };
/* MOVE_RWMH3: the alternation of three random-walk MH steps with proposal
 * standard deviations eps * (0.1, 1, 10) that the paper's GPU experiments use
 * (appendix "GPU implementation"), applied as one kernel per annealing step
 * (substeps 0, 1, 2 of the counter layout). */
/* MOVE_EXACT (Gaussian family only) draws X ~ pi_beta exactly, the idealised
 * kernel under which the efficient-local-exploration assumption holds;
 * MOVE_IDENTITY leaves X unchanged (AIS then reduces to importance sampling
 * from eta).  Both exist only to pin the oracle against closed forms. */

typedef struct {
    int family;
    int d;
    /* FAM_GAUSS: gamma(x) = exp(-|x - mu|^2 / (2 sigma2)) */
    const double* mu;
    double sigma2;
    /* FAM_LOGREG: gamma(x) = eta(x) prod_i sigmoid(z_i)^y_i (1-sigmoid(z_i))^(1-y_i),
     * z_i = X_i . x, X row-major n x d, y in {0,1} */
    const double* X;
    const double* y;
    int n;
    /* FAM_GMM: gamma(x) = (1/K) sum_k exp(-|x - m_k|^2 / (2 exp(2 s_k))) */
    int K;
    const double* means;      /* K x d */
    const double* log_scales; /* K */
    /* reference eta = N(ref_mean, ref_sigma2 I), normalised (Z_0 = 1) */
    const double* ref_mean;   /* may be NULL: zero mean */
    double ref_sigma2;
    /* FAM_UNID (unidentifiable product parameterisation, d = 2): eta uniform on
     * (0, box)^2; likelihood Binomial(k | binom_n, x y), zero unless 0 < x y < 1;
     * ell is the log-likelihood ratio against its maximum at x y = k / n:
     *   ell = k log(u / p) + (n - k) log((1 - u) / (1 - p)),  u = x y, p = k / n */
    double binom_n, binom_k, box;
} orc_problem;

static double ref_mean_at(const orc_problem* P, int i)
{
    return P->ref_mean ? P->ref_mean[i] : 0.0;
}

static int in_box(const orc_problem* P, const double* x)
{
    for (int i = 0; i < P->d; ++i)
        if (!(x[i] > 0.0 && x[i] < P->box)) return 0;
    return 1;
}

/* log eta(x), the normalised reference density. */
static double log_eta(const orc_problem* P, const double* x)
{
    const double log_two_pi = 1.8378770664093454835606594728112;
    if (P->family == FAM_UNID) return in_box(P, x) ? -P->d * log(P->box) : -INFINITY;
    double ss = 0.0;
    for (int i = 0; i < P->d; ++i) {
        double r = x[i] - ref_mean_at(P, i);
        ss += r * r;
    }
    return -ss / (2.0 * P->ref_sigma2) - 0.5 * P->d * (log_two_pi + log(P->ref_sigma2));
}

static void grad_log_eta(const orc_problem* P, const double* x, double* g)
{
    for (int i = 0; i < P->d; ++i) g[i] = -(x[i] - ref_mean_at(P, i)) / P->ref_sigma2;
}

static double softplus(double z)
{
    return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
}

static double sigmoid(double z)
{
    if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
    double e = exp(z);
    return e / (1.0 + e);
}

/* log gamma(x) for the Gaussian and mixture families. */
static double log_gamma_closed(const orc_problem* P, const double* x)
{
    if (P->family == FAM_GAUSS) {
        double ss = 0.0;
        for (int i = 0; i < P->d; ++i) {
            double r = x[i] - P->mu[i];
            ss += r * r;
        }
        return -ss / (2.0 * P->sigma2);
    }
    /* FAM_GMM: log of the equal-weight average of unnormalised components */
    double mx = -INFINITY;
    double* e = (double*)malloc(sizeof(double) * P->K);
    for (int k = 0; k < P->K; ++k) {
        double ss = 0.0;
        for (int i = 0; i < P->d; ++i) {
            double r = x[i] - P->means[(size_t)k * P->d + i];
            ss += r * r;
        }
        e[k] = -ss / (2.0 * exp(2.0 * P->log_scales[k]));
        if (e[k] > mx) mx = e[k];
    }
    double s = 0.0;
    for (int k = 0; k < P->K; ++k) s += exp(e[k] - mx);
    free(e);
    return mx + log(s) - log((double)P->K);
}

/*
 * ell(x) = log gamma(x) - log eta(x): the sufficient statistic V of the
 * linear (geometric) path, so that log gamma_beta = log eta + beta * ell.
 * For the logistic-regression family gamma = eta * likelihood, so ell is the
 * log-likelihood itself.
 */
static double ell(const orc_problem* P, const double* x)
{
    if (P->family == FAM_UNID) {
        double u = x[0] * x[1];
        if (!in_box(P, x) || !(u > 0.0 && u < 1.0)) return -INFINITY;
        double n = P->binom_n, k = P->binom_k, p = k / n;
        /* log(u/p) and log((1-u)/(1-p)) as log1p of their small offsets near
         * the maximum, where the two large terms cancel */
        return k * log1p((u - p) / p) + (n - k) * log1p(-(u - p) / (1.0 - p));
    }
    if (P->family == FAM_LOGREG) {
        double ll = 0.0;
        for (int i = 0; i < P->n; ++i) {
            const double* row = P->X + (size_t)i * P->d;
            double z = 0.0;
            for (int j = 0; j < P->d; ++j) z += row[j] * x[j];
            ll += P->y[i] * z - softplus(z);
        }
        return ll;
    }
    return log_gamma_closed(P, x) - log_eta(P, x);
}

/* Gradient of ell. */
static void grad_ell(const orc_problem* P, const double* x, double* g)
{
    int d = P->d;
    if (P->family == FAM_LOGREG) {
        for (int j = 0; j < d; ++j) g[j] = 0.0;
        for (int i = 0; i < P->n; ++i) {
            const double* row = P->X + (size_t)i * d;
            double z = 0.0;
            for (int j = 0; j < d; ++j) z += row[j] * x[j];
            double r = P->y[i] - sigmoid(z);
            for (int j = 0; j < d; ++j) g[j] += r * row[j];
        }
        return;
    }
    double* ge = (double*)malloc(sizeof(double) * d);
    grad_log_eta(P, x, ge);
    if (P->family == FAM_GAUSS) {
        for (int i = 0; i < d; ++i) g[i] = -(x[i] - P->mu[i]) / P->sigma2 - ge[i];
    } else {
        /* mixture: responsibilities r_k = softmax_k(-|x - m_k|^2 / (2 v_k)) */
        double* e = (double*)malloc(sizeof(double) * P->K);
        double mx = -INFINITY;
        for (int k = 0; k < P->K; ++k) {
            double ss = 0.0;
            for (int i = 0; i < d; ++i) {
                double r = x[i] - P->means[(size_t)k * d + i];
                ss += r * r;
            }
            e[k] = -ss / (2.0 * exp(2.0 * P->log_scales[k]));
            if (e[k] > mx) mx = e[k];
        }
        double s = 0.0;
        for (int k = 0; k < P->K; ++k) {
            e[k] = exp(e[k] - mx);
            s += e[k];
        }
        for (int i = 0; i < d; ++i) g[i] = -ge[i];
        for (int k = 0; k < P->K; ++k) {
            double rk = e[k] / s;
            double v = exp(2.0 * P->log_scales[k]);
            for (int i = 0; i < d; ++i) g[i] += rk * (P->means[(size_t)k * d + i] - x[i]) / v;
        }
        free(e);
    }
    free(ge);
}

/* log pi_beta(x) up to the constant -log Z_beta, for the linear path. */
static double log_anneal(const orc_problem* P, double beta, const double* x, double ell_x)
{
    return log_eta(P, x) + beta * ell_x;
}

static void grad_log_anneal(const orc_problem* P, double beta, const double* x,
                            const double* gell, double* g)
{
    grad_log_eta(P, x, g);
    for (int i = 0; i < P->d; ++i) g[i] += beta * gell[i];
}

static double store(double v, int state_f32)
{
    return state_f32 ? (double)(float)v : v;
}

/* ------------------------------------------------------------------------ */
/* pi_beta-invariant Metropolis-Hastings moves (forward kernel K_beta).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int move;         /* MOVE_RWMH / MOVE_MALA / MOVE_HMC */
    int leapfrog;     /* HMC: number of leapfrog steps per trajectory */
    int resample;     /* 0: AIS (no resampling), 1: adaptive resampling */
    int trigger;      /* resampling times (Sec. "Resample step", strategies):
                       * 0: ESS < nu N (AR), 1: CESS < nu N (AR with the
                       * conditional ESS), 2: every step (SIR), 3: at the steps
                       * flagged in resample_at (deterministic times, e.g. DAR) */
    double nu;
    int state_f32;
    int nthreads;     /* 0: OpenMP default */
    const unsigned char* force_accept; /* AIS only, [N*T] or NULL: replay these decisions */
    const unsigned char* resample_at;  /* trigger 3: [T], 1 = resample after step t (t < T) */
} orc_opts;

typedef struct {
    double* x;      /* d */
    double ell;     /* ell(x) */
    double* gell;   /* d: gradient of ell at x (MALA, HMC) */
} particle;

/*
 * One MH step targeting pi_beta from particle p, with step size eps (RWMH:
 * proposal standard deviation; MALA: Langevin step; HMC: leapfrog step).
 * Draws: d normals (stream 1) and one uniform (stream 2), keyed (n, t).
 * Returns 1 when accepted.  *margin receives log alpha - log u.
 */
static int mh_step(const orc_problem* P, const orc_opts* O, const rng_key* K, uint32_t n,
                   uint32_t t, double beta, double eps, particle* p, double* work,
                   double* margin, int forced)
{
    int d = P->d;
    double* xi = work;          /* d */
    double* xp = work + d;      /* d: proposal */
    double* gp = work + 2 * d;  /* d: grad ell at proposal */
    double* ga = work + 3 * d;  /* d: grad log pi_beta */
    double* mom = work + 4 * d; /* d: HMC momentum */
    draw_normals(K, n, t, STREAM_MOVE, 0, d, xi);
    if (O->move == MOVE_IDENTITY || O->move == MOVE_EXACT) {
        if (O->move == MOVE_EXACT) {
            /* pi_beta for Gaussian eta and gamma: precision lam, mean m_beta */
            double lam = (1.0 - beta) / P->ref_sigma2 + beta / P->sigma2;
            for (int i = 0; i < d; ++i) {
                double mb = ((1.0 - beta) * ref_mean_at(P, i) / P->ref_sigma2 +
                             beta * P->mu[i] / P->sigma2) / lam;
                p->x[i] = store(mb + xi[i] / sqrt(lam), O->state_f32);
            }
            p->ell = ell(P, p->x);
        }
        if (margin) *margin = INFINITY;
        return 1;
    }
    double log_alpha;
    double ell_p = 0.0;

    if (O->move == MOVE_RWMH3) {
        static const double scale[3] = {0.1, 1.0, 10.0};
        int any = 0;
        double best = INFINITY;
        for (int j = 0; j < 3; ++j) {
            draw_normals(K, n, t, STREAM_MOVE, (uint32_t)j, d, xi);
            for (int i = 0; i < d; ++i)
                xp[i] = store(p->x[i] + eps * scale[j] * xi[i], O->state_f32);
            double el = ell(P, xp);
            double la = log_anneal(P, beta, xp, el) - log_anneal(P, beta, p->x, p->ell);
            double lu = log(draw_uniform(K, n, t, STREAM_ACCEPT, (uint32_t)j));
            if (fabs(la - lu) < fabs(best)) best = la - lu;
            if (lu < la) {
                for (int i = 0; i < d; ++i) p->x[i] = xp[i];
                p->ell = el;
                any = 1;
            }
        }
        if (margin) *margin = best;
        return any;
    }
    if (O->move == MOVE_RWMH) {
        for (int i = 0; i < d; ++i) xp[i] = store(p->x[i] + eps * xi[i], O->state_f32);
        ell_p = ell(P, xp);
        log_alpha = log_anneal(P, beta, xp, ell_p) - log_anneal(P, beta, p->x, p->ell);
    } else if (O->move == MOVE_MALA) {
        /* x' = x + (eps^2/2) grad log pi_beta(x) + eps xi */
        double h = 0.5 * eps * eps;
        grad_log_anneal(P, beta, p->x, p->gell, ga);
        for (int i = 0; i < d; ++i) xp[i] = store(p->x[i] + h * ga[i] + eps * xi[i], O->state_f32);
        ell_p = ell(P, xp);
        grad_ell(P, xp, gp);
        /* log q(x'|x) with q(y|x) = N(y; x + h grad log pi_beta(x), eps^2 I) */
        double fwd = 0.0, bwd = 0.0;
        for (int i = 0; i < d; ++i) {
            double r = xp[i] - p->x[i] - h * ga[i];
            fwd += r * r;
        }
        grad_log_anneal(P, beta, xp, gp, ga);
        for (int i = 0; i < d; ++i) {
            double r = p->x[i] - xp[i] - h * ga[i];
            bwd += r * r;
        }
        log_alpha = log_anneal(P, beta, xp, ell_p) - log_anneal(P, beta, p->x, p->ell)
                    - bwd / (2.0 * eps * eps) + fwd / (2.0 * eps * eps);
    } else {
        /* HMC: H(x, p) = -log pi_beta(x) + |p|^2 / 2, L leapfrog steps of size eps
         * (half momentum step, full position step, half momentum step).  Each
         * position is a stored state, so it is rounded like one. */
        int L = O->leapfrog;
        double kin0 = 0.0;
        for (int i = 0; i < d; ++i) {
            mom[i] = xi[i];
            kin0 += 0.5 * mom[i] * mom[i];
            xp[i] = p->x[i];
        }
        grad_log_anneal(P, beta, p->x, p->gell, ga);
        for (int i = 0; i < d; ++i) gp[i] = p->gell[i];
        for (int l = 0; l < L; ++l) {
            for (int i = 0; i < d; ++i) mom[i] += 0.5 * eps * ga[i];
            for (int i = 0; i < d; ++i) xp[i] = store(xp[i] + eps * mom[i], O->state_f32);
            grad_ell(P, xp, gp);
            grad_log_anneal(P, beta, xp, gp, ga);
            for (int i = 0; i < d; ++i) mom[i] += 0.5 * eps * ga[i];
        }
        ell_p = ell(P, xp);
        double kin1 = 0.0;
        for (int i = 0; i < d; ++i) kin1 += 0.5 * mom[i] * mom[i];
        log_alpha = (log_anneal(P, beta, xp, ell_p) - kin1)
                    - (log_anneal(P, beta, p->x, p->ell) - kin0);
    }

    double log_u = log(draw_uniform(K, n, t, STREAM_ACCEPT, 0));
    if (margin) *margin = log_alpha - log_u;
    int accept = (log_u < log_alpha); /* NaN log_alpha rejects */
    if (forced >= 0) accept = forced;   /* replayed decision (fixed masks) */
    if (accept) {
        for (int i = 0; i < d; ++i) p->x[i] = xp[i];
        p->ell = ell_p;
        if (O->move != MOVE_RWMH)
            for (int i = 0; i < d; ++i) p->gell[i] = gp[i];
    }
    return accept;
}

/* Particle initialisation X_0 ~ eta (stream 0, t = 0). */
static void init_particle(const orc_problem* P, const orc_opts* O, const rng_key* K,
                          uint32_t n, particle* p, double* work)
{
    int d = P->d;
    if (P->family == FAM_UNID) {
        /* uniform reference: coordinate i from word i of block 0 */
        uint32_t w[4];
        draw_block(K, n, 0u, STREAM_INIT, 0, 0, w);
        for (int i = 0; i < d; ++i) p->x[i] = store(P->box * word_to_uniform(w[i]), O->state_f32);
        p->ell = ell(P, p->x);
        return;
    }
    draw_normals(K, n, 0u, STREAM_INIT, 0, d, work);
    double s = sqrt(P->ref_sigma2);
    for (int i = 0; i < d; ++i) p->x[i] = store(ref_mean_at(P, i) + s * work[i], O->state_f32);
    p->ell = ell(P, p->x);
    if (O->move != MOVE_RWMH) grad_ell(P, p->x, p->gell);
}

/* ------------------------------------------------------------------------ */
/* Plain log-sum-exp helpers (two-pass: max, then shifted sum).              */
/* ------------------------------------------------------------------------ */
static double logsumexp(const double* v, int64_t m, int64_t stride)
{
    double mx = -INFINITY;
    for (int64_t j = 0; j < m; ++j) {
        double a = v[j * stride];
        if (a > mx) mx = a;
    }
    if (mx == -INFINITY) return -INFINITY;
    if (!isfinite(mx)) return mx; /* +inf or NaN propagate */
    double s = 0.0;
    for (int64_t j = 0; j < m; ++j) s += exp(v[j * stride] - mx);
    return mx + log(s);
}

/*
 * Moments of eq. (CESS) in log space from the weights before the reweight
 * (w_{t-1}) and the incremental weights g_t:
 *   log g_hat_{t,i} = logsumexp_n (log w_{t-1}^n + i log g_t^n), i = 0, 1, 2.
 */
static void moments(int64_t N, const double* lw_prev, const double* lg, double* out3, double* tmp)
{
    for (int i = 0; i < 3; ++i) {
        /* (g^n_t)^0 = 1 also where g^n_t = 0 (log g = -inf, a zero likelihood) */
        for (int64_t n = 0; n < N; ++n) tmp[n] = (i == 0) ? lw_prev[n] : lw_prev[n] + (double)i * lg[n];
        out3[i] = logsumexp(tmp, N, 1);
    }
}

/* ------------------------------------------------------------------------ */
/* Systematic resampling with an exact integer CDF.                          */
/* ------------------------------------------------------------------------ */
/*
 * The paper names systematic resampling without defining it; the reading:
 * one uniform U per event, points (n + U)/N, ancestor a_n = min{m : C_m > p_n}
 * where C is the cumulative normalised weight.  To make the ancestors an
 * exact function of the log-weights, weights are quantised to integers
 *   q_m = floor(exp(lw_m - max lw) * 2^B),  B = 62 - ceil(log2 N),
 * the CDF is the exact integer prefix sum, and the points are
 *   p_n = floor(S (2 (n 2^32 + u) + 1) / (N 2^33)),  S = sum q,
 * which is floor(S (n + U)/N) with U = (u + 1/2) 2^-32 taken exactly.
 */
static int quant_bits(int64_t N)
{
    int lg = 0;
    while (((int64_t)1 << lg) < N) ++lg;
    return 62 - lg;
}

int orc_systematic(int64_t N, const double* lw, uint32_t u, int32_t* anc)
{
    if (N <= 0) return ORC_EINVAL;
    double mx = -INFINITY;
    for (int64_t m = 0; m < N; ++m)
        if (lw[m] > mx) mx = lw[m];
    if (!(mx > -INFINITY) || !isfinite(mx)) return ORC_ENONFINITE;
    int B = quant_bits(N);
    uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    if (!C) return ORC_ENOMEM;
    uint64_t run = 0;
    double scale = ldexp(1.0, B);
    for (int64_t m = 0; m < N; ++m) {
        double e = exp(lw[m] - mx);
        uint64_t q = (lw[m] == lw[m]) ? (uint64_t)floor(e * scale) : 0u;
        run += q;
        C[m] = run;
    }
    uint64_t S = run;
    int64_t m = 0;
    for (int64_t n = 0; n < N; ++n) {
        unsigned __int128 num = (unsigned __int128)S *
                                (unsigned __int128)(2u * (((uint64_t)n << 32) | (uint64_t)u) + 1u);
        unsigned __int128 den = (unsigned __int128)N << 33;
        uint64_t pn = (uint64_t)(num / den);
        /* points increase with n, so the search resumes where it stopped */
        while (C[m] <= pn) ++m;
        anc[n] = (int32_t)m;
    }
    free(C);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: ASMC(N, B_T).                                                      */
/* ------------------------------------------------------------------------ */
/*
 * Outputs (all host arrays owned by the caller):
 *   log_g[3*T]   log g_hat_{t,i} at [i*T + t-1]
 *   acc[T]       fraction of particles whose move at t was accepted
 *   logZ         log Z_hat
 *   lw_out[N]    final log-weights, x_out[N*d] final states
 *   n_resample   number of resampling events strictly before T
 * Optional (NULL to skip):
 *   accept[N*T]  per particle and step accept flag, margin[N*T] log alpha - log u
 *   resampled[T] 1 where a resampling event happened at t
 *   ess[T]       relative ESS of w_{t^-}
 *   lw_trace[N*T] log w_{t^-} of every particle after the reweight of step t
 *                (before any resampling at t), at [n*T + t-1]
 * subset/n_subset (AIS only): run only these global particle indices; every
 *   per-particle output is then indexed by position in the subset and every
 *   cross-particle statistic is over the subset.
 */
int orc_asmc(const orc_problem* P, const orc_opts* O, int64_t N, int T, const double* beta,
             const double* eps, uint64_t seed, uint32_t round_k, uint32_t problem_id,
             double* log_g, double* acc, double* logZ, double* lw_out, double* x_out,
             int* n_resample, unsigned char* accept, double* margin, int* resampled,
             double* ess, const int64_t* subset, int64_t n_subset, double* lw_trace)
{
    if (!P || !O || T < 1 || P->d < 1 || !beta || !eps) return ORC_EINVAL;
    if (beta[0] != 0.0 || beta[T] != 1.0) return ORC_EINVAL;
    for (int t = 1; t <= T; ++t)
        if (!(beta[t] > beta[t - 1])) return ORC_EINVAL;
    int64_t M = subset ? n_subset : N;
    if (M < 1) return ORC_EINVAL;
    if (subset && O->resample) return ORC_EINVAL;
    int d = P->d;
    rng_key K = {seed, round_k, problem_id};
    if (O->nthreads > 0) omp_set_num_threads(O->nthreads);

    double* X = (double*)malloc(sizeof(double) * (size_t)M * d);
    double* G = (double*)malloc(sizeof(double) * (size_t)M * d);
    double* L = (double*)malloc(sizeof(double) * (size_t)M);
    double* LW = (double*)calloc((size_t)M * (T + 1), sizeof(double)); /* lw before step t */
    double* LG = (double*)malloc(sizeof(double) * (size_t)M * T);
    unsigned char* A = (unsigned char*)malloc((size_t)M * T);
    if (!X || !G || !L || !LW || !LG || !A) {
        free(X); free(G); free(L); free(LW); free(LG); free(A);
        return ORC_ENOMEM;
    }
    int status = ORC_OK;
    int nres = 0;
    double log_z = 0.0;

    if (!O->resample) {
        /* OAIS: the particle loop is outside the time loop (loop swap). */
#pragma omp parallel
        {
            double* work = (double*)malloc(sizeof(double) * 6 * d);
#pragma omp for schedule(dynamic, 1)
            for (int64_t j = 0; j < M; ++j) {
                uint32_t n = (uint32_t)(subset ? subset[j] : j);
                particle p = {X + (size_t)j * d, 0.0, G + (size_t)j * d};
                init_particle(P, O, &K, n, &p, work);
                double lw = 0.0;
                for (int t = 1; t <= T; ++t) {
                    /* incremental weight at the pre-move state:
                     * log g_t = log gamma_{beta_t}(x) - log gamma_{beta_{t-1}}(x) */
                    double lg = (beta[t] - beta[t - 1]) * p.ell;
                    LG[(size_t)j * T + (t - 1)] = lg;
                    lw += lg;
                    LW[(size_t)j * (T + 1) + t] = lw;
                    if (lw_trace) lw_trace[(size_t)j * T + (t - 1)] = lw;
                    double mg = 0.0;
                    const int forced = O->force_accept ? O->force_accept[(size_t)j * T + (t - 1)] : -1;
                    A[(size_t)j * T + (t - 1)] =
                        (unsigned char)mh_step(P, O, &K, n, (uint32_t)t, beta[t], eps[t - 1], &p,
                                               work, &mg, forced);
                    if (margin) margin[(size_t)j * T + (t - 1)] = mg;
                }
                L[j] = p.ell;
            }
            free(work);
        }
        double* tmp = (double*)malloc(sizeof(double) * (size_t)M * 2);
        double* col = tmp + M;
        for (int t = 1; t <= T; ++t) {
            double* lwp = (double*)malloc(sizeof(double) * (size_t)M);
            double* lgt = (double*)malloc(sizeof(double) * (size_t)M);
            for (int64_t j = 0; j < M; ++j) {
                lwp[j] = LW[(size_t)j * (T + 1) + (t - 1)];
                lgt[j] = LG[(size_t)j * T + (t - 1)];
            }
            double m3[3];
            moments(M, lwp, lgt, m3, tmp);
            for (int i = 0; i < 3; ++i) log_g[i * T + (t - 1)] = m3[i];
            if (ess) {
                for (int64_t j = 0; j < M; ++j) col[j] = 2.0 * (lwp[j] + lgt[j]);
                ess[t - 1] = exp(2.0 * m3[1] - logsumexp(col, M, 1) - log((double)M));
            }
            if (resampled) resampled[t - 1] = 0;
            free(lwp);
            free(lgt);
        }
        for (int64_t j = 0; j < M; ++j) tmp[j] = LW[(size_t)j * (T + 1) + T];
        /* Z_hat = (1/N) sum_n w_T^n (a single final event, R = 1) */
        log_z = logsumexp(tmp, M, 1) - log((double)M);
        free(tmp);
    } else {
        /* ASMC with adaptive resampling: time loop outside. */
        double* lw = (double*)calloc((size_t)M, sizeof(double));
        double* lg = (double*)malloc(sizeof(double) * (size_t)M);
        double* tmp = (double*)malloc(sizeof(double) * (size_t)M);
        int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
        double* X2 = (double*)malloc(sizeof(double) * (size_t)M * d);
        double* G2 = (double*)malloc(sizeof(double) * (size_t)M * d);
        double* L2 = (double*)malloc(sizeof(double) * (size_t)M);
#pragma omp parallel
        {
            double* work = (double*)malloc(sizeof(double) * 6 * d);
#pragma omp for schedule(static)
            for (int64_t j = 0; j < M; ++j) {
                particle p = {X + (size_t)j * d, 0.0, G + (size_t)j * d};
                init_particle(P, O, &K, (uint32_t)j, &p, work);
                L[j] = p.ell;
            }
            free(work);
        }
        for (int t = 1; t <= T && status == ORC_OK; ++t) {
            for (int64_t j = 0; j < M; ++j) lg[j] = (beta[t] - beta[t - 1]) * L[j];
            double m3[3];
            moments(M, lw, lg, m3, tmp);
            for (int i = 0; i < 3; ++i) log_g[i * T + (t - 1)] = m3[i];
            for (int64_t j = 0; j < M; ++j) lw[j] += lg[j];
            if (lw_trace)
                for (int64_t j = 0; j < M; ++j) lw_trace[(size_t)j * T + (t - 1)] = lw[j];
            int na = 0;
#pragma omp parallel reduction(+ : na)
            {
                double* work = (double*)malloc(sizeof(double) * 6 * d);
#pragma omp for schedule(static)
                for (int64_t j = 0; j < M; ++j) {
                    particle p = {X + (size_t)j * d, L[j], G + (size_t)j * d};
                    double mg = 0.0;
                    int a = mh_step(P, O, &K, (uint32_t)j, (uint32_t)t, beta[t], eps[t - 1], &p,
                                    work, &mg, -1);
                    L[j] = p.ell;
                    A[(size_t)j * T + (t - 1)] = (unsigned char)a;
                    if (margin) margin[(size_t)j * T + (t - 1)] = mg;
                    na += a;
                }
                free(work);
            }
            (void)na;
            /* relative ESS of w_{t^-} and the conditional ESS of eq. (CESS) */
            for (int64_t j = 0; j < M; ++j) tmp[j] = 2.0 * lw[j];
            double log_sum_w = m3[1]; /* sum_n w_{t-1} g_t = sum_n w_{t^-} */
            double rel_ess = exp(2.0 * log_sum_w - logsumexp(tmp, M, 1) - log((double)M));
            double rel_cess = exp(-(m3[2] - 2.0 * m3[1] + m3[0]));
            if (ess) ess[t - 1] = rel_ess;
            int fire;
            if (O->trigger == 0) fire = rel_ess < O->nu;
            else if (O->trigger == 1) fire = rel_cess < O->nu;
            else if (O->trigger == 2) fire = 1;
            else fire = O->resample_at ? (O->resample_at[t - 1] != 0) : 0;
            if (resampled) resampled[t - 1] = 0;
            if (t == T) {
                /* the final event at tau_R = T: no resampling needed for Z_hat */
                log_z += logsumexp(lw, M, 1) - log((double)M);
            } else if (fire) {
                log_z += logsumexp(lw, M, 1) - log((double)M);
                uint32_t w[4];
                draw_block(&K, 0xFFFFFFFFu, (uint32_t)t, STREAM_RESAMPLE, 0, 0, w);
                int rs = orc_systematic(M, lw, w[0], anc);
                if (rs != ORC_OK) {
                    status = rs;
                    break;
                }
                for (int64_t j = 0; j < M; ++j) {
                    memcpy(X2 + (size_t)j * d, X + (size_t)anc[j] * d, sizeof(double) * d);
                    memcpy(G2 + (size_t)j * d, G + (size_t)anc[j] * d, sizeof(double) * d);
                    L2[j] = L[anc[j]];
                }
                memcpy(X, X2, sizeof(double) * (size_t)M * d);
                memcpy(G, G2, sizeof(double) * (size_t)M * d);
                memcpy(L, L2, sizeof(double) * (size_t)M);
                for (int64_t j = 0; j < M; ++j) lw[j] = 0.0;
                ++nres;
                if (resampled) resampled[t - 1] = 1;
            }
        }
        for (int64_t j = 0; j < M; ++j) LW[(size_t)j * (T + 1) + T] = lw[j];
        free(lw); free(lg); free(tmp); free(anc); free(X2); free(G2); free(L2);
    }

    if (status == ORC_OK) {
        for (int t = 1; t <= T; ++t) {
            int64_t cnt = 0;
            for (int64_t j = 0; j < M; ++j) cnt += A[(size_t)j * T + (t - 1)];
            acc[t - 1] = (double)cnt / (double)M;
        }
        for (int64_t j = 0; j < M; ++j) {
            lw_out[j] = LW[(size_t)j * (T + 1) + T];
            memcpy(x_out + (size_t)j * d, X + (size_t)j * d, sizeof(double) * d);
        }
        if (accept) memcpy(accept, A, (size_t)M * T);
        *logZ = log_z;
        if (n_resample) *n_resample = nres;
        if (!isfinite(log_z)) status = ORC_ENONFINITE;
    }
    free(X); free(G); free(L); free(LW); free(LG); free(A);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Online CESS-adaptive AIS of Zhou, Johansen and Aston (ZJA).               */
/* ------------------------------------------------------------------------ */
/*
 * The comparison method of Sec. "Connection to online conditional ESS
 * optimisation" and Sec. "High-performance GPU implementation of adaptive
 * schemes", applied to AIS (no resampling): with w_{t-1} and ell(X_{t-1}) in
 * hand, beta_t is chosen so that the conditional ESS of the step,
 *   CESS_t / N = g_1^2 / (g_0 g_2),  g_i = sum_n w_{t-1}^n exp(i (b - beta_{t-1}) ell_n)
 * (eq. CESS), equals rho: beta_t = 1 when CESS(1) >= rho N, otherwise
 * `iters` halvings of (beta_{t-1}, 1] on log CESS in binary64, keeping the
 * upper part while CESS >= rho N (beta_t is the last point kept, or the first
 * upper end if none was).  At t = Tmax beta_t is set to 1.  Then the step
 * reweights, records the moments and moves every particle at beta_t (step
 * size eps), as Alg. 1 does.
 * Outputs: beta[Tmax + 1] (entries 0..T), *T, log_g[3 * Tmax] (layout
 * i * Tmax + t - 1), *logZ, lw_out[N], x_out[N * d].
 */
static double lse_shift(int64_t N, const double* lw, const double* ell_v, double a, double* tmp)
{
    for (int64_t j = 0; j < N; ++j) tmp[j] = (a == 0.0) ? lw[j] : lw[j] + a * ell_v[j];
    return logsumexp(tmp, N, 1);
}

int orc_zja(const orc_problem* P, const orc_opts* O, int64_t N, double rho, int Tmax, int iters,
            double eps, uint64_t seed, uint32_t round_k, uint32_t problem_id, double* beta,
            int* T_out, double* log_g, double* logZ, double* lw_out, double* x_out)
{
    if (!P || !O || N < 1 || Tmax < 1 || iters < 1 || !(rho > 0.0 && rho < 1.0) || !beta ||
        !T_out || !log_g || !logZ)
        return ORC_EINVAL;
    int d = P->d;
    rng_key K = {seed, round_k, problem_id};
    if (O->nthreads > 0) omp_set_num_threads(O->nthreads);
    double* X = (double*)malloc(sizeof(double) * (size_t)N * d);
    double* G = (double*)malloc(sizeof(double) * (size_t)N * d);
    double* L = (double*)malloc(sizeof(double) * (size_t)N);
    double* lw = (double*)calloc((size_t)N, sizeof(double));
    double* lg = (double*)malloc(sizeof(double) * (size_t)N);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)N);
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * 6 * d);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < N; ++j) {
            particle p = {X + (size_t)j * d, 0.0, G + (size_t)j * d};
            init_particle(P, O, &K, (uint32_t)j, &p, work);
            L[j] = p.ell;
        }
        free(work);
    }
    const double log_rho = log(rho);
    beta[0] = 0.0;
    int T = 0;
    for (int t = 1; t <= Tmax; ++t) {
        double b0 = beta[t - 1];
        double L0 = lse_shift(N, lw, L, 0.0, tmp);
#define LOG_CESS(db) (2.0 * lse_shift(N, lw, L, (db), tmp) - lse_shift(N, lw, L, 2.0 * (db), tmp) - L0)
        double bt;
        if (LOG_CESS(1.0 - b0) >= log_rho) {
            bt = 1.0;
        } else {
            double lo = b0, hi = 1.0;
            for (int it = 0; it < iters; ++it) {
                double mid = 0.5 * (lo + hi);
                if (LOG_CESS(mid - b0) >= log_rho) lo = mid;
                else hi = mid;
            }
            bt = (lo > b0) ? lo : hi;
        }
#undef LOG_CESS
        if (t == Tmax) bt = 1.0;
        beta[t] = bt;
        for (int64_t j = 0; j < N; ++j) lg[j] = (bt - b0) * L[j];
        double m3[3];
        moments(N, lw, lg, m3, tmp);
        for (int i = 0; i < 3; ++i) log_g[(size_t)i * Tmax + (t - 1)] = m3[i];
        for (int64_t j = 0; j < N; ++j) lw[j] += lg[j];
#pragma omp parallel
        {
            double* work = (double*)malloc(sizeof(double) * 6 * d);
#pragma omp for schedule(static)
            for (int64_t j = 0; j < N; ++j) {
                particle p = {X + (size_t)j * d, L[j], G + (size_t)j * d};
                mh_step(P, O, &K, (uint32_t)j, (uint32_t)t, bt, eps, &p, work, NULL, -1);
                L[j] = p.ell;
            }
            free(work);
        }
        T = t;
        if (bt >= 1.0) break;
    }
    *T_out = T;
    *logZ = logsumexp(lw, N, 1) - log((double)N);
    if (lw_out) memcpy(lw_out, lw, sizeof(double) * (size_t)N);
    if (x_out) memcpy(x_out, X, sizeof(double) * (size_t)N * d);
    free(X); free(G); free(L); free(lw); free(lg); free(tmp);
    return isfinite(*logZ) ? ORC_OK : ORC_ENONFINITE;
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering through computational duality.                         */
/* ------------------------------------------------------------------------ */
/*
 * PT (Sec. "Computational duality with parallel tempering"): K independent
 * copies, each of N' + 1 chains jointly targeting pi_{beta_0} x ... x
 * pi_{beta_N'}, run for T' iterations.  Reading (the section gives the
 * estimators; the swap scheme is that of non-reversible PT, deterministic even
 * and odd swaps): every chain (a replica r of copy k, global index
 * k (N' + 1) + r) starts from eta; iteration t applies the forward kernel at the
 * replica's current temperature (counters (replica, t), step size eps[n] of
 * temperature n), then proposes swaps of the replicas at temperatures
 * (n, n + 1) for every n of the parity of t (even t: n = 0, 2, ...), accepted
 * iff log u < (beta_{n+1} - beta_n)(ell(y at n) - ell(y at n+1)), u from
 * stream 4 with counter (k (N' + 1) + n, t).  Swaps exchange temperatures, not
 * states.  After iteration t:
 *   - the stepping stone terms (beta_n - beta_{n-1}) ell(Y^{n-1}_t), n = 1..N',
 *     pooled over copies: log Z_PT = sum_n [logsumexp_{k,t}(...) - log(K T')]
 *     (eq. (Z_PT) with the K T' samples of each temperature);
 *   - the swap rejection 1 - min(1, alpha) of each proposed pair, averaged per
 *     pair into r_n (Lambda_PT estimate = sum_n r_n);
 *   - round trips: a replica that reached temperature N' after its last visit
 *     to 0 completes one when it returns to 0;
 *   - x_i and x_i^2 of the replica at temperature N' (the target chain).
 * Outputs: *logZ, ss[N'] (the per-temperature log-means), rej[N'], trips (total
 * over copies), tmean[d], tsecond[d] (averages over K T' target-chain states).
 */
#define STREAM_SWAP 4u
int orc_pt(const orc_problem* P, const orc_opts* O, int K, int Np, int Tp, const double* beta,
           const double* eps, uint64_t seed, uint32_t round_k, uint32_t problem_id, double* logZ,
           double* ss, double* rej, int64_t* trips, double* tmean, double* tsecond)
{
    if (!P || !O || K < 1 || Np < 1 || Tp < 1 || !beta || !eps || !logZ || !ss || !rej)
        return ORC_EINVAL;
    if (beta[0] != 0.0 || beta[Np] != 1.0) return ORC_EINVAL;
    for (int n = 1; n <= Np; ++n)
        if (!(beta[n] > beta[n - 1])) return ORC_EINVAL;
    int d = P->d, R = Np + 1;
    rng_key Kk = {seed, round_k, problem_id};
    if (O->nthreads > 0) omp_set_num_threads(O->nthreads);
    /* per copy: stepping-stone terms [Np][Tp], rejection sums [Np], counts [Np],
     * round trips, target sums [d] x 2 */
    double* terms = (double*)malloc(sizeof(double) * (size_t)K * Np * Tp);
    double* rsum = (double*)calloc((size_t)K * Np, sizeof(double));
    int64_t* rcnt = (int64_t*)calloc((size_t)K * Np, sizeof(int64_t));
    int64_t* rt = (int64_t*)calloc((size_t)K, sizeof(int64_t));
    double* f1 = (double*)calloc((size_t)K * d, sizeof(double));
    double* f2 = (double*)calloc((size_t)K * d, sizeof(double));
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
        double* X = (double*)malloc(sizeof(double) * (size_t)R * d);
        double* G = (double*)malloc(sizeof(double) * (size_t)R * d);
        double* L = (double*)malloc(sizeof(double) * R);
        double* work = (double*)malloc(sizeof(double) * 6 * d);
        int* tau = (int*)malloc(sizeof(int) * R);   /* temperature of replica r */
        int* rep = (int*)malloc(sizeof(int) * R);   /* replica at temperature n */
        int* side = (int*)malloc(sizeof(int) * R);  /* 0: last extreme 0, 1: reached N' since */
        for (int r = 0; r < R; ++r) {
            particle p = {X + (size_t)r * d, 0.0, G + (size_t)r * d};
            init_particle(P, O, &Kk, (uint32_t)(k * R + r), &p, work);
            L[r] = p.ell;
            tau[r] = r;
            rep[r] = r;
            side[r] = (r == 0) ? 0 : -1;
        }
        for (int t = 1; t <= Tp; ++t) {
            for (int r = 0; r < R; ++r) {
                particle p = {X + (size_t)r * d, L[r], G + (size_t)r * d};
                int n = tau[r];
                mh_step(P, O, &Kk, (uint32_t)(k * R + r), (uint32_t)t, beta[n], eps[n], &p, work,
                        NULL, -1);
                L[r] = p.ell;
            }
            for (int n = (t % 2 == 0) ? 0 : 1; n + 1 < R; n += 2) {
                int a = rep[n], b = rep[n + 1];
                double la = (beta[n + 1] - beta[n]) * (L[a] - L[b]);
                double u = draw_uniform(&Kk, (uint32_t)(k * R + n), (uint32_t)t, STREAM_SWAP, 0);
                double acc = (la >= 0.0) ? 1.0 : exp(la);
                if (la != la) acc = 0.0;
                rsum[(size_t)k * Np + n] += 1.0 - acc;
                rcnt[(size_t)k * Np + n] += 1;
                if (log(u) < la) {
                    rep[n] = b;
                    rep[n + 1] = a;
                    tau[a] = n + 1;
                    tau[b] = n;
                }
            }
            for (int r = 0; r < R; ++r) {
                if (tau[r] == Np && side[r] == 0) side[r] = 1;
                if (tau[r] == 0) {
                    if (side[r] == 1) rt[k] += 1;
                    side[r] = 0;
                }
            }
            for (int n = 1; n <= Np; ++n)
                terms[((size_t)k * Np + (n - 1)) * Tp + (t - 1)] =
                    (beta[n] - beta[n - 1]) * L[rep[n - 1]];
            const double* y = X + (size_t)rep[Np] * d;
            for (int i = 0; i < d; ++i) {
                f1[(size_t)k * d + i] += y[i];
                f2[(size_t)k * d + i] += y[i] * y[i];
            }
        }
        free(X); free(G); free(L); free(work); free(tau); free(rep); free(side);
    }
    double lz = 0.0;
    double* col = (double*)malloc(sizeof(double) * (size_t)K * Tp);
    for (int n = 0; n < Np; ++n) {
        for (int k = 0; k < K; ++k)
            memcpy(col + (size_t)k * Tp, terms + ((size_t)k * Np + n) * Tp, sizeof(double) * Tp);
        ss[n] = logsumexp(col, (int64_t)K * Tp, 1) - log((double)K * Tp);
        lz += ss[n];
        double a = 0.0;
        int64_t c = 0;
        for (int k = 0; k < K; ++k) {
            a += rsum[(size_t)k * Np + n];
            c += rcnt[(size_t)k * Np + n];
        }
        rej[n] = c > 0 ? a / (double)c : NAN;
    }
    *logZ = lz;
    if (trips) {
        int64_t tot = 0;
        for (int k = 0; k < K; ++k) tot += rt[k];
        *trips = tot;
    }
    for (int i = 0; tmean && tsecond && i < d; ++i) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < K; ++k) {
            a += f1[(size_t)k * d + i];
            b += f2[(size_t)k * d + i];
        }
        tmean[i] = a / ((double)K * Tp);
        tsecond[i] = b / ((double)K * Tp);
    }
    if (!isfinite(lz)) status = ORC_ENONFINITE;
    free(col); free(terms); free(rsum); free(rcnt); free(rt); free(f1); free(f2);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Final-iteration rejuvenation (Sec. "Computing expectations").             */
/* ------------------------------------------------------------------------ */
/*
 * After the last annealing step, resample the final population (weights
 * lw[N], states x[N*d]) and run N MCMC chains for T steps, chain n starting at
 * its resampled particle; the TN states visited estimate expectations under
 * the target.  Readings: the chains use the pass's forward kernel at beta = 1
 * with the last step size eps_T; the event's uniform is the resampling word of
 * step T (stream 3, particle word 0xFFFFFFFF); chain n draws with counters
 * (n, T + s), s = 1..T, so nothing collides with the annealing pass.  Test
 * functions: f(x) = x_i and x_i^2.
 * Outputs: mean[d] and second[d] (averages of x_i and x_i^2 over the TN
 * samples), *accept (fraction of accepted chain moves), x_out[N*d] (chain end
 * states, may be NULL).
 */
int orc_rejuvenate(const orc_problem* P, const orc_opts* O, int64_t N, int T, double eps_T,
                   uint64_t seed, uint32_t round_k, uint32_t problem_id, const double* lw,
                   const double* x, double* mean, double* second, double* accept,
                   double* x_out)
{
    if (!P || !O || N < 1 || T < 1 || !lw || !x || !mean || !second) return ORC_EINVAL;
    int d = P->d;
    rng_key K = {seed, round_k, problem_id};
    if (O->nthreads > 0) omp_set_num_threads(O->nthreads);
    uint32_t w[4];
    draw_block(&K, 0xFFFFFFFFu, (uint32_t)T, STREAM_RESAMPLE, 0, 0, w);
    int32_t* anc = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    double* S1 = (double*)calloc((size_t)N * d, sizeof(double));
    double* S2 = (double*)calloc((size_t)N * d, sizeof(double));
    int64_t* na = (int64_t*)calloc((size_t)N, sizeof(int64_t));
    int st = orc_systematic(N, lw, w[0], anc);
    if (st != ORC_OK) {
        free(anc); free(S1); free(S2); free(na);
        return st;
    }
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * 6 * d);
        double* px = (double*)malloc(sizeof(double) * d);
        double* pg = (double*)malloc(sizeof(double) * d);
#pragma omp for schedule(dynamic, 16)
        for (int64_t n = 0; n < N; ++n) {
            memcpy(px, x + (size_t)anc[n] * d, sizeof(double) * d);
            particle p = {px, ell(P, px), pg};
            if (O->move != MOVE_RWMH) grad_ell(P, px, pg);
            for (int s = 1; s <= T; ++s) {
                na[n] += mh_step(P, O, &K, (uint32_t)n, (uint32_t)(T + s), 1.0, eps_T, &p, work,
                                 NULL, -1);
                for (int i = 0; i < d; ++i) {
                    S1[(size_t)n * d + i] += p.x[i];
                    S2[(size_t)n * d + i] += p.x[i] * p.x[i];
                }
            }
            if (x_out) memcpy(x_out + (size_t)n * d, p.x, sizeof(double) * d);
        }
        free(work);
        free(px);
        free(pg);
    }
    double tot = (double)N * (double)T;
    int64_t acc = 0;
    for (int i = 0; i < d; ++i) {
        double a = 0.0, b = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            a += S1[(size_t)n * d + i];
            b += S2[(size_t)n * d + i];
        }
        mean[i] = a / tot;
        second[i] = b / tot;
    }
    for (int64_t n = 0; n < N; ++n) acc += na[n];
    if (accept) *accept = (double)acc / tot;
    free(anc); free(S1); free(S2); free(na);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 3: OptimiseSchedule.                                                  */
/* ------------------------------------------------------------------------ */
/* Fritsch-Carlson monotone piecewise-cubic Hermite interpolation (PCHIP):
 * knot slopes by the weighted harmonic mean of adjacent secants (zero at a
 * change of sign), shape-preserving three-point end slopes. */
static void pchip_slopes(int m, const double* xs, const double* ys, double* s)
{
    if (m == 2) {
        s[0] = s[1] = (ys[1] - ys[0]) / (xs[1] - xs[0]);
        return;
    }
    double* h = (double*)malloc(sizeof(double) * (m - 1));
    double* del = (double*)malloc(sizeof(double) * (m - 1));
    for (int k = 0; k < m - 1; ++k) {
        h[k] = xs[k + 1] - xs[k];
        del[k] = (ys[k + 1] - ys[k]) / h[k];
    }
    for (int k = 1; k < m - 1; ++k) {
        if (del[k - 1] == 0.0 || del[k] == 0.0 || (del[k - 1] > 0.0) != (del[k] > 0.0)) {
            s[k] = 0.0;
        } else {
            double w1 = 2.0 * h[k] + h[k - 1];
            double w2 = h[k] + 2.0 * h[k - 1];
            s[k] = (w1 + w2) / (w1 / del[k - 1] + w2 / del[k]);
        }
    }
    /* end slopes: non-centred three-point formula, then shape preservation */
    for (int end = 0; end < 2; ++end) {
        double h0, h1, d0, d1;
        if (end == 0) {
            h0 = h[0]; h1 = h[1]; d0 = del[0]; d1 = del[1];
        } else {
            h0 = h[m - 2]; h1 = h[m - 3]; d0 = del[m - 2]; d1 = del[m - 3];
        }
        double sl = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
        if ((sl > 0.0) != (d0 > 0.0) || sl == 0.0) {
            sl = 0.0;
        } else if ((d0 > 0.0) != (d1 > 0.0) && fabs(sl) > fabs(3.0 * d0)) {
            sl = 3.0 * d0;
        }
        if (end == 0) s[0] = sl; else s[m - 1] = sl;
    }
    free(h);
    free(del);
}

static double hermite_eval(int m, const double* xs, const double* ys, const double* s, double x)
{
    int k = 0;
    if (x <= xs[0]) return ys[0];
    if (x >= xs[m - 1]) return ys[m - 1];
    while (k < m - 2 && x >= xs[k + 1]) ++k;
    double h = xs[k + 1] - xs[k];
    double u = (x - xs[k]) / h;
    double u2 = u * u, u3 = u2 * u;
    double h00 = 2.0 * u3 - 3.0 * u2 + 1.0;
    double h10 = u3 - 2.0 * u2 + u;
    double h01 = -2.0 * u3 + 3.0 * u2;
    double h11 = u3 - u2;
    return h00 * ys[k] + h10 * h * s[k] + h01 * ys[k + 1] + h11 * h * s[k + 1];
}

/* Exported so the interpolant can be pinned against a library PCHIP. */
void orc_pchip_eval(int m, const double* xs, const double* ys, int q, const double* xq,
                    double* yq)
{
    double* s = (double*)malloc(sizeof(double) * m);
    pchip_slopes(m, xs, ys, s);
    for (int j = 0; j < q; ++j) yq[j] = hermite_eval(m, xs, ys, s, xq[j]);
    free(s);
}

static void uniform_schedule(int Tn, double* b)
{
    for (int t = 0; t <= Tn; ++t) b[t] = (double)t / (double)Tn;
    b[Tn] = 1.0;
}

/*
 * D_hat_t = log g_hat_{t,2} - 2 log g_hat_{t,1} + log g_hat_{t,0} (clamped at 0:
 * non-negative by Cauchy-Schwarz, a negative value is roundoff),
 * Lambda_hat_t = sum_{s<=t} sqrt(D_hat_s), knots (Lambda_hat_t, beta_t) with
 * repeated abscissae removed (first kept, the final knot always kept),
 * beta*_{t'} = Lambda_hat^{-1}(Lambda_hat_T t'/T').
 * interp: 0 PCHIP, 1 piecewise linear.
 */
int orc_optimise_schedule(int T, const double* beta, const double* log_g, int T_new, int interp,
                          double* beta_new, double* Lambda)
{
    if (T < 1 || T_new < 1 || !beta || !log_g || !beta_new) return ORC_EINVAL;
    double* Lam = (double*)malloc(sizeof(double) * (T + 1));
    Lam[0] = 0.0;
    int finite = 1;
    for (int t = 1; t <= T; ++t) {
        double D = log_g[2 * T + t - 1] - 2.0 * log_g[T + t - 1] + log_g[t - 1];
        if (!isfinite(D)) finite = 0;
        if (!(D > 0.0)) D = 0.0;
        Lam[t] = Lam[t - 1] + sqrt(D);
    }
    if (Lambda) memcpy(Lambda, Lam, sizeof(double) * (T + 1));
    if (!finite || !(Lam[T] > 0.0)) {
        uniform_schedule(T_new, beta_new);
        free(Lam);
        return finite ? ORC_OK : ORC_ENONFINITE;
    }
    /* knots with strictly increasing abscissa */
    double* kx = (double*)malloc(sizeof(double) * (T + 1));
    double* ky = (double*)malloc(sizeof(double) * (T + 1));
    int m = 0;
    for (int t = 0; t <= T; ++t) {
        if (m > 0 && !(Lam[t] > kx[m - 1])) {
            if (t == T) { /* the final knot replaces an equal-abscissa one */
                kx[m - 1] = Lam[t];
                ky[m - 1] = beta[t];
            }
            continue;
        }
        kx[m] = Lam[t];
        ky[m] = beta[t];
        ++m;
    }
    for (int tp = 0; tp <= T_new; ++tp) {
        double u = Lam[T] * (double)tp / (double)T_new;
        double b;
        if (interp == 1) {
            int k = 0;
            while (k < m - 2 && u >= kx[k + 1]) ++k;
            double w = (u - kx[k]) / (kx[k + 1] - kx[k]);
            if (w < 0.0) w = 0.0;
            if (w > 1.0) w = 1.0;
            b = ky[k] + w * (ky[k + 1] - ky[k]);
        } else {
            orc_pchip_eval(m, kx, ky, 1, &u, &b);
        }
        beta_new[tp] = b;
    }
    /* endpoints exact, strictly increasing interior */
    beta_new[0] = 0.0;
    beta_new[T_new] = 1.0;
    for (int tp = 1; tp < T_new; ++tp) {
        if (!(beta_new[tp] > beta_new[tp - 1])) beta_new[tp] = nextafter(beta_new[tp - 1], 2.0);
    }
    for (int tp = T_new - 1; tp >= 1; --tp) {
        if (!(beta_new[tp] < beta_new[tp + 1])) beta_new[tp] = nextafter(beta_new[tp + 1], -1.0);
    }
    free(kx);
    free(ky);
    free(Lam);
    return ORC_OK;
}

/*
 * Deterministic adaptive resampling times on a new schedule (DAR: Sec.
 * "Effective resample size for deterministic adaptive resampling", eq.
 * (DAR-times); AR converges to it as N grows, appendix "Adaptive resampling
 * in the large particle limit").  The true incremental discrepancies are
 * replaced by a prediction from a previous round's moments:
 *   - D_hat_t and Lambda_hat_t on the previous schedule beta[0..T] (as in
 *     Alg. 3, negative D_hat clamped to 0);
 *   - the cumulative barrier as a function of beta, the monotone interpolant
 *     (interp 0: PCHIP, 1: linear) through the knots (beta_t, Lambda_hat_t);
 *   - sqrt D(b, b') ~ Lambda(b') - Lambda(b) (the root-discrepancy estimate
 *     of the dense-schedule analysis), so on the new schedule
 *     D_pred_t = (Lambda(bn_t) - Lambda(bn_{t-1}))^2;
 *   - tau_r is the first t > tau_{r-1} with exp(-sum_{s=tau_{r-1}+1}^t D_pred_s) < nu.
 * flags[t-1] = 1 where t = tau_r < T_new (the event at T_new is the final one
 * of the estimator, not a resampling).  D_pred (may be NULL) gets the
 * predictions.  Non-finite moments: no flags, ORC_ENONFINITE.
 */
int orc_dar_times(int T, const double* beta, const double* log_g, int T_new,
                  const double* beta_new, int interp, double nu, unsigned char* flags,
                  double* D_pred)
{
    if (T < 1 || T_new < 1 || !beta || !log_g || !beta_new || !flags) return ORC_EINVAL;
    if (!(nu > 0.0 && nu < 1.0)) return ORC_EINVAL;
    for (int t = 0; t < T_new; ++t) flags[t] = 0;
    double* Lam = (double*)malloc(sizeof(double) * (T + 1));
    double* at = (double*)malloc(sizeof(double) * (T_new + 1));
    Lam[0] = 0.0;
    int finite = 1;
    for (int t = 1; t <= T; ++t) {
        double D = log_g[2 * T + t - 1] - 2.0 * log_g[T + t - 1] + log_g[t - 1];
        if (!isfinite(D)) finite = 0;
        if (!(D > 0.0)) D = 0.0;
        Lam[t] = Lam[t - 1] + sqrt(D);
    }
    if (!finite) {
        if (D_pred)
            for (int t = 0; t < T_new; ++t) D_pred[t] = NAN;
        free(Lam);
        free(at);
        return ORC_ENONFINITE;
    }
    /* Lambda at the new knots */
    if (interp == 1) {
        for (int tp = 0; tp <= T_new; ++tp) {
            double b = beta_new[tp];
            int k = 0;
            while (k < T - 1 && b >= beta[k + 1]) ++k;
            double w = (b - beta[k]) / (beta[k + 1] - beta[k]);
            if (w < 0.0) w = 0.0;
            if (w > 1.0) w = 1.0;
            at[tp] = Lam[k] + w * (Lam[k + 1] - Lam[k]);
        }
    } else {
        orc_pchip_eval(T + 1, beta, Lam, T_new + 1, beta_new, at);
    }
    const double thr = -log(nu);
    double accum = 0.0;
    for (int t = 1; t <= T_new; ++t) {
        double r = at[t] - at[t - 1];
        double D = r * r;
        if (D_pred) D_pred[t - 1] = D;
        accum += D;
        if (t < T_new && accum > thr) { /* exp(-accum) < nu */
            flags[t - 1] = 1;
            accum = 0.0;
        }
    }
    free(Lam);
    free(at);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: OASMC round loop with Budget and step-size adaptation.            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int budget;          /* 0 fixed, 1 double N, 2 double T (capped), 3 sqrt2 then double T */
    int T1, Tmax;
    int64_t Nmax;
    int eps_adapt;       /* 0: eps_t = eps0; 1: adapt across rounds */
    double eps0, eps_kappa, accept_target;
    int interp;
    int dar;             /* with resampling: 1 = each round resamples at the DAR times
                          * predicted from the previous round (orc_dar_times, threshold
                          * nu of the options); round 1, with no previous round, resamples
                          * at no intermediate step */
} orc_run_opts;

/*
 * Budget(N_k, T_k) -> (N_{k+1}, T_{k+1}).
 *  1: N doubles, T fixed.  2: N fixed, T doubles up to Tmax.
 *  3: the heuristic of the Budget section: N and T grow by sqrt 2 until N
 *     would exceed Nmax, then N stays and T doubles (T capped at Tmax).
 */
static void budget_next(const orc_run_opts* R, int64_t N, int T, int64_t* Nn, int* Tn)
{
    *Nn = N;
    *Tn = T;
    if (R->budget == 1) {
        *Nn = 2 * N;
    } else if (R->budget == 2) {
        *Tn = 2 * T;
    } else if (R->budget == 3) {
        int64_t Ng = (int64_t)llround((double)N * sqrt(2.0));
        if (Ng <= R->Nmax) {
            *Nn = Ng;
            int Tg = (int)lround((double)T * sqrt(2.0));
            *Tn = Tg > T ? Tg : T + 1;
        } else {
            *Tn = 2 * T;
        }
    }
    if (R->Tmax > 0 && *Tn > R->Tmax) *Tn = R->Tmax;
}

/* Piecewise-linear interpolation on knots (bx[j], by[j]), j < m, constant beyond. */
static double pl_interp(int m, const double* bx, const double* by, double x)
{
    if (x <= bx[0]) return by[0];
    if (x >= bx[m - 1]) return by[m - 1];
    int k = 0;
    while (k < m - 2 && x >= bx[k + 1]) ++k;
    double w = (x - bx[k]) / (bx[k + 1] - bx[k]);
    return by[k] + w * (by[k + 1] - by[k]);
}

/*
 * Step sizes: round 1 uses eps_t = eps0 (1 + beta_t kappa)^(-1/2), a scale
 * that follows the posterior width along the path for Gaussian-like targets.
 * Afterwards log eps^{(k+1)}(beta) = log eps^{(k)}(beta) + (acc^{(k)}(beta) - a*),
 * as a piecewise-linear function of beta through the knots beta_t, t >= 1.
 */
static void eps_first(const orc_run_opts* R, int T, const double* beta, double* eps)
{
    for (int t = 1; t <= T; ++t)
        eps[t - 1] = R->eps_adapt ? R->eps0 / sqrt(1.0 + beta[t] * R->eps_kappa) : R->eps0;
}

static void eps_next(const orc_run_opts* R, int T, const double* beta, const double* eps,
                     const double* acc, int Tn, const double* beta_n, double* eps_n)
{
    if (!R->eps_adapt) {
        for (int t = 0; t < Tn; ++t) eps_n[t] = R->eps0;
        return;
    }
    double* kx = (double*)malloc(sizeof(double) * T);
    double* ky = (double*)malloc(sizeof(double) * T);
    for (int t = 1; t <= T; ++t) {
        kx[t - 1] = beta[t];
        ky[t - 1] = log(eps[t - 1]) + (acc[t - 1] - R->accept_target);
    }
    for (int t = 1; t <= Tn; ++t) eps_n[t - 1] = exp(pl_interp(T, kx, ky, beta_n[t]));
    free(kx);
    free(ky);
}

/*
 * Rounds k = 1..rounds.  Round k uses counter field round_k = k.  Outputs are
 * indexed by round with row capacity Tcap: beta[k][Tcap+1], Lambda[k][Tcap+1],
 * log_g[k][3][Tcap], acc[k][Tcap], eps[k][Tcap].
 */
int orc_run(const orc_problem* P, const orc_opts* O, const orc_run_opts* R, int64_t N1,
            int rounds, uint64_t seed, uint32_t problem_id, int Tcap, double* logZ,
            int64_t* Ns, int* Ts, double* beta_out, double* Lambda_out, double* log_g_out,
            double* acc_out, double* eps_out, int* nres_out)
{
    if (!P || !O || !R || N1 < 1 || rounds < 1 || R->T1 < 1 || R->T1 > Tcap) return ORC_EINVAL;
    int64_t N = N1;
    int T = R->T1;
    double* beta = (double*)malloc(sizeof(double) * (Tcap + 1));
    double* eps = (double*)malloc(sizeof(double) * Tcap);
    double* lg = (double*)malloc(sizeof(double) * 3 * Tcap);
    double* acc = (double*)malloc(sizeof(double) * Tcap);
    uniform_schedule(T, beta);
    eps_first(R, T, beta, eps);
    int status = ORC_OK;
    const int dar = R->dar && O->resample;
    unsigned char* flags = (unsigned char*)calloc((size_t)Tcap + 1, 1);
    orc_opts Ok = *O;
    if (dar) {
        Ok.trigger = 3;
        Ok.resample_at = flags;
    }
    for (int k = 1; k <= rounds; ++k) {
        double* lw = (double*)malloc(sizeof(double) * (size_t)N);
        double* xo = (double*)malloc(sizeof(double) * (size_t)N * P->d);
        double lz = 0.0;
        int nres = 0;
        status = orc_asmc(P, &Ok, N, T, beta, eps, seed, (uint32_t)k, problem_id, lg, acc, &lz, lw,
                          xo, &nres, NULL, NULL, NULL, NULL, NULL, 0, NULL);
        free(lw);
        free(xo);
        if (status != ORC_OK && status != ORC_ENONFINITE) break;
        int r = k - 1;
        logZ[r] = lz;
        Ns[r] = N;
        Ts[r] = T;
        nres_out[r] = nres;
        memcpy(beta_out + (size_t)r * (Tcap + 1), beta, sizeof(double) * (T + 1));
        for (int i = 0; i < 3; ++i) /* layout [rounds][3][Tcap] */
            memcpy(log_g_out + ((size_t)r * 3 + i) * Tcap, lg + (size_t)i * T, sizeof(double) * T);
        memcpy(acc_out + (size_t)r * Tcap, acc, sizeof(double) * T);
        memcpy(eps_out + (size_t)r * Tcap, eps, sizeof(double) * T);
        /* Lambda_hat of this round and the next round's schedule (Alg. 3) */
        int64_t Nn;
        int Tn;
        budget_next(R, N, T, &Nn, &Tn);
        if (Tn > Tcap) Tn = Tcap;
        double* bn = (double*)malloc(sizeof(double) * (Tn + 1));
        double* en = (double*)malloc(sizeof(double) * Tn);
        int s2 = orc_optimise_schedule(T, beta, lg, Tn, R->interp, bn,
                                       Lambda_out + (size_t)r * (Tcap + 1));
        if (status == ORC_OK && s2 != ORC_OK) status = s2;
        if (dar) {
            int s3 = orc_dar_times(T, beta, lg, Tn, bn, R->interp, O->nu, flags, NULL);
            if (status == ORC_OK && s3 != ORC_OK) status = s3;
        }
        eps_next(R, T, beta, eps, acc, Tn, bn, en);
        memcpy(beta, bn, sizeof(double) * (Tn + 1));
        memcpy(eps, en, sizeof(double) * Tn);
        free(bn);
        free(en);
        N = Nn;
        T = Tn;
        if (status != ORC_OK) break;
    }
    free(beta);
    free(eps);
    free(lg);
    free(acc);
    free(flags);
    return status;
}

/* Evaluate ell and its gradient (exported for the gradient pins). */
double orc_ell(const orc_problem* P, const double* x, double* grad_or_null)
{
    if (grad_or_null) grad_ell(P, x, grad_or_null);
    return ell(P, x);
}


/* ------------------------------------------------------------------------ */
/* Derivatives of log Z_hat with respect to the mixture's parameters.        */
/* ------------------------------------------------------------------------ */
/*
 * theta = (means[k][i] for k < K, i < d, then log_scales[k] for k < K).
 * With a_k = (m_k - x)/v_k, v_k = exp(2 s_k), r = softmax_k(-|x - m_k|^2/(2 v_k)),
 * g = sum_k r_k a_k, q_k = |x - m_k|^2 / v_k:
 *   grad_x log gamma          = g
 *   hess_x log gamma          = sum_k r_k (a_k a_k^T - I/v_k) - g g^T
 *   d log gamma / d m_k       = -r_k a_k
 *   d log gamma / d s_k       = r_k q_k
 *   d g_i / d m_{k,l}         = r_k (delta_il / v_k - (a_k - g)_i a_{k,l})
 *   d g_i / d s_k             = r_k q_k (a_k - g)_i - 2 r_k a_{k,i}
 * eta does not depend on theta; hess_x ell = hess_x log gamma + I/ref_sigma2.
 * Outputs: H[d*d] (hessian of ell), M[d*np] (d grad_x ell / d theta),
 * dl[np] (d ell / d theta), np = K*d + K.
 */
void orc_gmm_derivs(const orc_problem* P, const double* x, double* H, double* M, double* dl)
{
    int d = P->d, K = P->K, np = K * d + K;
    double* e = (double*)malloc(sizeof(double) * K);
    double* r = (double*)malloc(sizeof(double) * K);
    double* v = (double*)malloc(sizeof(double) * K);
    double* q = (double*)malloc(sizeof(double) * K);
    double* a = (double*)malloc(sizeof(double) * K * d);
    double* g = (double*)calloc(d, sizeof(double));
    double mx = -INFINITY;
    for (int k = 0; k < K; ++k) {
        v[k] = exp(2.0 * P->log_scales[k]);
        double ss = 0.0;
        for (int i = 0; i < d; ++i) {
            double diff = x[i] - P->means[(size_t)k * d + i];
            ss += diff * diff;
            a[(size_t)k * d + i] = -diff / v[k];
        }
        q[k] = ss / v[k];
        e[k] = -ss / (2.0 * v[k]);
        if (e[k] > mx) mx = e[k];
    }
    double z = 0.0;
    for (int k = 0; k < K; ++k) {
        r[k] = exp(e[k] - mx);
        z += r[k];
    }
    for (int k = 0; k < K; ++k) r[k] /= z;
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < d; ++i) g[i] += r[k] * a[(size_t)k * d + i];
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double h = -g[i] * g[j];
            for (int k = 0; k < K; ++k) {
                h += r[k] * a[(size_t)k * d + i] * a[(size_t)k * d + j];
                if (i == j) h -= r[k] / v[k];
            }
            if (i == j) h += 1.0 / P->ref_sigma2;
            H[(size_t)i * d + j] = h;
        }
    for (int i = 0; i < d; ++i) {
        for (int k = 0; k < K; ++k) {
            for (int l = 0; l < d; ++l) {
                double val = -r[k] * (a[(size_t)k * d + i] - g[i]) * a[(size_t)k * d + l];
                if (i == l) val += r[k] / v[k];
                M[(size_t)i * np + k * d + l] = val;
            }
            M[(size_t)i * np + K * d + k] =
                r[k] * q[k] * (a[(size_t)k * d + i] - g[i]) - 2.0 * r[k] * a[(size_t)k * d + i];
        }
    }
    for (int k = 0; k < K; ++k) {
        for (int l = 0; l < d; ++l) dl[k * d + l] = -r[k] * a[(size_t)k * d + l];
        dl[K * d + k] = r[k] * q[k];
    }
    free(e); free(r); free(v); free(q); free(a); free(g);
}

/*
 * Pathwise gradient of log Z_hat (AIS, MALA, mixture target) with the accept
 * decisions held fixed, by forward-mode (tangent) propagation of
 * D x_t = dx_t/dtheta through every step:
 *   log w_T = sum_t (beta_t - beta_{t-1}) ell(x_{t-1}),
 *   x' = x + h (grad log eta(x) + beta grad ell(x)) + eps xi,  h = eps^2/2,
 *   D x' = D x + h (-D x / ref_sigma2 + beta (H D x + M)),
 *   x_t = x' and D x_t = D x' when accepted, else unchanged;
 * grad log Z_hat = sum_n W_n D log w_T^n with W = softmax(log w_T).
 * The rounding of stored states to binary32 is differentiated as the
 * identity.  Decisions are the MH ones of this run unless force_accept is
 * given.  Outputs grad[np], logZ, and optionally the decisions accept[N*T].
 */
int orc_logZ_grad(const orc_problem* P, const orc_opts* O, int64_t N, int T, const double* beta,
                  const double* eps, uint64_t seed, uint32_t round_k, uint32_t problem_id,
                  double* grad, double* logZ, unsigned char* accept)
{
    if (!P || !O || P->family != FAM_GMM || O->move != MOVE_MALA || O->resample) return ORC_EINVAL;
    int d = P->d, np = P->K * d + P->K;
    rng_key K = {seed, round_k, problem_id};
    if (O->nthreads > 0) omp_set_num_threads(O->nthreads);
    double* lw = (double*)malloc(sizeof(double) * (size_t)N);
    double* dlw = (double*)calloc((size_t)N * np, sizeof(double));
#pragma omp parallel
    {
        double* work = (double*)malloc(sizeof(double) * 6 * d);
        double* x = (double*)malloc(sizeof(double) * d);
        double* gx = (double*)malloc(sizeof(double) * d);
        double* Dx = (double*)malloc(sizeof(double) * d * np);
        double* Dxp = (double*)malloc(sizeof(double) * d * np);
        double* H = (double*)malloc(sizeof(double) * d * d);
        double* M = (double*)malloc(sizeof(double) * d * np);
        double* dl = (double*)malloc(sizeof(double) * np);
#pragma omp for schedule(dynamic, 1)
        for (int64_t n = 0; n < N; ++n) {
            particle p = {x, 0.0, gx};
            init_particle(P, O, &K, (uint32_t)n, &p, work);
            for (int c = 0; c < d * np; ++c) Dx[c] = 0.0;
            double w = 0.0;
            double* dw = dlw + (size_t)n * np;
            for (int t = 1; t <= T; ++t) {
                double db = beta[t] - beta[t - 1];
                double h = 0.5 * eps[t - 1] * eps[t - 1];
                orc_gmm_derivs(P, p.x, H, M, dl);
                /* weight and its tangent at the pre-move state */
                w += db * p.ell;
                for (int c = 0; c < np; ++c) {
                    double s = dl[c];
                    for (int i = 0; i < d; ++i) s += p.gell[i] * Dx[(size_t)i * np + c];
                    dw[c] += db * s;
                }
                /* tangent of the proposal from x_{t-1} */
                for (int i = 0; i < d; ++i)
                    for (int c = 0; c < np; ++c) {
                        double hd = 0.0;
                        for (int j = 0; j < d; ++j) hd += H[(size_t)i * d + j] * Dx[(size_t)j * np + c];
                        Dxp[(size_t)i * np + c] = Dx[(size_t)i * np + c] +
                            h * (-Dx[(size_t)i * np + c] / P->ref_sigma2 +
                                 beta[t] * (hd + M[(size_t)i * np + c]));
                    }
                const int forced = O->force_accept ? O->force_accept[(size_t)n * T + (t - 1)] : -1;
                int a = mh_step(P, O, &K, (uint32_t)n, (uint32_t)t, beta[t], eps[t - 1], &p, work,
                                NULL, forced);
                if (accept) accept[(size_t)n * T + (t - 1)] = (unsigned char)a;
                if (a) memcpy(Dx, Dxp, sizeof(double) * d * np);
            }
            lw[n] = w;
        }
        free(work); free(x); free(gx); free(Dx); free(Dxp); free(H); free(M); free(dl);
    }
    double L = logsumexp(lw, N, 1);
    *logZ = L - log((double)N);
    for (int c = 0; c < np; ++c) grad[c] = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        double Wn = exp(lw[n] - L);
        for (int c = 0; c < np; ++c) grad[c] += Wn * dlw[(size_t)n * np + c];
    }
    free(lw);
    free(dlw);
    return isfinite(*logZ) ? ORC_OK : ORC_ENONFINITE;
}
