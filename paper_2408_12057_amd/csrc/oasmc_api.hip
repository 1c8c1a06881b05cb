// oasmc_api.hip -- the C ABI (include/oasmc.h): argument validation, the
// handle-owned workspace, the per-round host driver (Alg. 2), the host schedule
// optimiser (Alg. 3), Budget and step-size adaptation.  All compute of the
// annealing passes runs in the gfx950 kernels; the host only moves O(T)
// vectors per round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/oasmc.h"
#include "kernels.hpp"

using namespace oasmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(OASMC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// One growable device allocation.
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct oasmc_handle_s {
    int device = 0;
    int cus = 256;
    size_t lds_per_block = 0;
    std::vector<Buf> bufs;
    // live kernel timing
    bool prof = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double prof_ms = 0.0, prof_steps = 0.0, prof_flops = 0.0;
    int64_t prof_launches = 0;

    // Returns a device buffer of at least `bytes` in slot `id` (grow-only).
    hipError_t get(int id, size_t bytes, void** out)
    {
        if ((int)bufs.size() <= id) bufs.resize(id + 1);
        Buf& b = bufs[id];
        if (b.bytes < bytes) {
            if (b.p) {
                hipError_t e = hipFree(b.p);
                if (e != hipSuccess) return e;
                b.p = nullptr;
                b.bytes = 0;
            }
            size_t want = std::max<size_t>(bytes, 256);
            hipError_t e = hipMalloc(&b.p, want);
            if (e != hipSuccess) return e;
            b.bytes = want;
        }
        *out = b.p;
        return hipSuccess;
    }
};

namespace {

enum BufId {
    B_BETA, B_EPS, B_PART, B_LOGG, B_ACC, B_SCAL, B_X, B_X2, B_ELL, B_ELL2, B_LW, B_ACCW,
    B_TPART, B_NRES, B_ESS, B_RES, B_C, B_BTOT, B_LWO, B_XO, B_LOGREG, B_COUNT
};

template <typename T>
hipError_t wget(oasmc_handle* h, int id, size_t count, T** p)
{
    void* v = nullptr;
    hipError_t e = h->get(id, count * sizeof(T), &v);
    *p = static_cast<T*>(v);
    return e;
}

int check_schedule(int T, const double* beta)
{
    if (T < 1) return fail(OASMC_EINVAL, "T must be >= 1 (got %d)", T);
    if (!beta) return fail(OASMC_EINVAL, "beta is NULL");
    if (beta[0] != 0.0 || beta[T] != 1.0)
        return fail(OASMC_EINVAL, "schedule must start at 0 and end at 1 (got %g, %g)", beta[0],
                    beta[T]);
    for (int t = 1; t <= T; ++t)
        if (!(beta[t] > beta[t - 1]))
            return fail(OASMC_EINVAL, "schedule not strictly increasing at t=%d", t);
    return OASMC_OK;
}

int check_problem(const oasmc_problem* p, const oasmc_kernel* k)
{
    if (!p || !k) return fail(OASMC_EINVAL, "problem or kernel is NULL");
    if (!(p->ref_sigma2 > 0.0) || !std::isfinite(p->ref_sigma2))
        return fail(OASMC_EINVAL, "ref_sigma2 must be positive and finite");
    if (k->move < OASMC_RWMH || k->move > OASMC_HMC)
        return fail(OASMC_EINVAL, "unknown move %d", k->move);
    if (k->move == OASMC_HMC && k->leapfrog < 1)
        return fail(OASMC_EINVAL, "HMC needs leapfrog >= 1");
    if (k->resample && !(k->nu > 0.0 && k->nu < 1.0))
        return fail(OASMC_EINVAL, "nu must lie in (0, 1)");
    switch (p->family) {
    case OASMC_GAUSS:
        if (!p->mu) return fail(OASMC_EINVAL, "Gaussian target needs mu");
        if (!(p->sigma2 > 0.0) || !std::isfinite(p->sigma2))
            return fail(OASMC_EINVAL, "sigma2 must be positive and finite");
        if (p->d < 1 || p->d > kMaxDValu)
            return fail(OASMC_EUNSUPPORTED, "Gaussian target supports 1 <= d <= %d", kMaxDValu);
        break;
    case OASMC_GMM:
        if (!p->means || !p->log_scales) return fail(OASMC_EINVAL, "mixture needs means, log_scales");
        if (p->K < 1 || p->K > kMaxK) return fail(OASMC_EUNSUPPORTED, "mixture supports 1 <= K <= %d", kMaxK);
        if (p->d < 1 || p->d > kMaxDValu)
            return fail(OASMC_EUNSUPPORTED, "mixture supports 1 <= d <= %d", kMaxDValu);
        break;
    case OASMC_LOGREG:
        if (!p->X || !p->y) return fail(OASMC_EINVAL, "logistic regression needs X and y");
        if (p->n < 1) return fail(OASMC_EINVAL, "logistic regression needs n >= 1");
        if (p->d < 1 || p->d > kMaxDLogreg)
            return fail(OASMC_EUNSUPPORTED, "logistic regression supports 1 <= d <= %d", kMaxDLogreg);
        if (k->move != OASMC_MALA || k->resample)
            return fail(OASMC_EUNSUPPORTED, "logistic regression is built for MALA without resampling");
        break;
    default:
        return fail(OASMC_EINVAL, "unknown family %d", p->family);
    }
    return OASMC_OK;
}

TargetDev target_dev(const oasmc_problem* p)
{
    TargetDev t{};
    t.family = p->family;
    t.d = p->d;
    t.K = p->K;
    t.n = p->n;
    t.mu = p->mu;
    t.sigma2 = p->sigma2;
    t.X = p->X;
    t.y = p->y;
    t.means = p->means;
    t.log_scales = p->log_scales;
    t.ref_mean = p->ref_mean;
    t.ref_sigma2 = p->ref_sigma2;
    return t;
}

// ---------------------------------------------------------------------------
// Alg. 3 on the host: monotone cubic Hermite inverse of the cumulative barrier.
// ---------------------------------------------------------------------------
struct MonotoneCubic {
    std::vector<double> x, y, m;  // knots and knot slopes

    // Fritsch-Carlson slopes: harmonic mean of neighbouring secants with
    // weights (2h_k + h_{k-1}, h_k + 2h_{k-1}), zero at extrema; end slopes
    // from the one-sided three-point formula, limited to keep monotonicity.
    void fit()
    {
        const size_t k = x.size();
        m.assign(k, 0.0);
        if (k == 2) {
            m[0] = m[1] = (y[1] - y[0]) / (x[1] - x[0]);
            return;
        }
        std::vector<double> h(k - 1), sec(k - 1);
        for (size_t i = 0; i + 1 < k; ++i) {
            h[i] = x[i + 1] - x[i];
            sec[i] = (y[i + 1] - y[i]) / h[i];
        }
        for (size_t i = 1; i + 1 < k; ++i) {
            const double a = sec[i - 1], b = sec[i];
            if (a * b <= 0.0) continue;
            const double w1 = 2.0 * h[i] + h[i - 1], w2 = h[i] + 2.0 * h[i - 1];
            m[i] = (w1 + w2) / (w1 / a + w2 / b);
        }
        auto end_slope = [](double h0, double h1, double s0, double s1) {
            double v = ((2.0 * h0 + h1) * s0 - h0 * s1) / (h0 + h1);
            if (v * s0 <= 0.0) return 0.0;
            if (s0 * s1 < 0.0 && std::fabs(v) > 3.0 * std::fabs(s0)) return 3.0 * s0;
            return v;
        };
        m[0] = end_slope(h[0], h[1], sec[0], sec[1]);
        m[k - 1] = end_slope(h[k - 2], h[k - 3], sec[k - 2], sec[k - 3]);
    }

    double operator()(double q) const
    {
        const size_t k = x.size();
        if (q <= x.front()) return y.front();
        if (q >= x.back()) return y.back();
        const size_t i = std::upper_bound(x.begin(), x.end(), q) - x.begin() - 1;
        const double h = x[i + 1] - x[i];
        const double s = (q - x[i]) / h;
        const double s2 = s * s, s3 = s2 * s;
        return (2 * s3 - 3 * s2 + 1) * y[i] + (s3 - 2 * s2 + s) * h * m[i] +
               (3 * s2 - 2 * s3) * y[i + 1] + (s3 - s2) * h * m[i + 1];
        (void)k;
    }
};

void uniform_schedule(int Tn, double* b)
{
    for (int t = 0; t <= Tn; ++t) b[t] = (double)t / (double)Tn;
    b[Tn] = 1.0;
}

int adapt_schedule_impl(int T, const double* beta, const double* log_g, int Tn, int interp,
                        double* beta_new, double* Lambda)
{
    std::vector<double> lam(T + 1, 0.0);
    bool finite = true;
    for (int t = 1; t <= T; ++t) {
        const double D = log_g[2 * T + t - 1] - 2.0 * log_g[T + t - 1] + log_g[t - 1];
        if (!std::isfinite(D)) finite = false;
        lam[t] = lam[t - 1] + (D > 0.0 ? std::sqrt(D) : 0.0);
    }
    if (Lambda) std::copy(lam.begin(), lam.end(), Lambda);
    if (!finite || !(lam[T] > 0.0)) {
        uniform_schedule(Tn, beta_new);
        return finite ? OASMC_OK
                      : fail(OASMC_ENONFINITE, "non-finite moments: schedule reset to uniform");
    }
    MonotoneCubic f;
    for (int t = 0; t <= T; ++t) {
        if (!f.x.empty() && !(lam[t] > f.x.back())) {
            if (t == T) {  // the final knot (Lambda_T, 1) replaces its equal-abscissa twin
                f.x.back() = lam[t];
                f.y.back() = beta[t];
            }
            continue;
        }
        f.x.push_back(lam[t]);
        f.y.push_back(beta[t]);
    }
    if (interp == 0) f.fit();
    for (int tp = 0; tp <= Tn; ++tp) {
        const double u = lam[T] * (double)tp / (double)Tn;
        double b;
        if (interp == 0) {
            b = f(u);
        } else {
            if (u <= f.x.front()) b = f.y.front();
            else if (u >= f.x.back()) b = f.y.back();
            else {
                const size_t i = std::upper_bound(f.x.begin(), f.x.end(), u) - f.x.begin() - 1;
                const double w = (u - f.x[i]) / (f.x[i + 1] - f.x[i]);
                b = f.y[i] + w * (f.y[i + 1] - f.y[i]);
            }
        }
        beta_new[tp] = b;
    }
    beta_new[0] = 0.0;
    beta_new[Tn] = 1.0;
    for (int tp = 1; tp < Tn; ++tp)
        if (!(beta_new[tp] > beta_new[tp - 1])) beta_new[tp] = std::nextafter(beta_new[tp - 1], 2.0);
    for (int tp = Tn - 1; tp >= 1; --tp)
        if (!(beta_new[tp] < beta_new[tp + 1])) beta_new[tp] = std::nextafter(beta_new[tp + 1], -1.0);
    return OASMC_OK;
}

}  // namespace

extern "C" {

const char* oasmc_last_error(void) { return g_err.c_str(); }

int oasmc_handle_create(oasmc_handle** h, int device)
{
    if (!h) return fail(OASMC_EINVAL, "handle pointer is NULL");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(OASMC_EINVAL, "no HIP device %d", device);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    oasmc_handle* p = new oasmc_handle();
    p->lds_per_block = (size_t)prop.sharedMemPerBlock;
    p->device = device;
    p->cus = prop.multiProcessorCount;
    p->bufs.resize(B_COUNT);
    *h = p;
    g_err.clear();
    return OASMC_OK;
}

int oasmc_handle_destroy(oasmc_handle* h)
{
    if (!h) return OASMC_OK;
    hipSetDevice(h->device);
    if (h->ev0) hipEventDestroy(h->ev0);
    if (h->ev1) hipEventDestroy(h->ev1);
    for (auto& b : h->bufs)
        if (b.p) hipFree(b.p);
    delete h;
    return OASMC_OK;
}

int oasmc_adapt_schedule(int32_t T, const double* beta, const double* log_g, int32_t T_new,
                         int32_t interp, double* beta_new, double* Lambda_hat)
{
    int s = check_schedule(T, beta);
    if (s) return s;
    if (!log_g || !beta_new) return fail(OASMC_EINVAL, "log_g or beta_new is NULL");
    if (T_new < 1) return fail(OASMC_EINVAL, "T_new must be >= 1");
    if (interp != 0 && interp != 1) return fail(OASMC_EINVAL, "interp must be 0 or 1");
    return adapt_schedule_impl(T, beta, log_g, T_new, interp, beta_new, Lambda_hat);
}

int oasmc_asmc(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
               int64_t N, int32_t T, const double* beta, const double* eps, uint64_t seed,
               uint32_t round_k, uint32_t problem_id, oasmc_round_out* out, void* stream)
{
    if (!h) return fail(OASMC_EINVAL, "handle is NULL");
    if (!out) return fail(OASMC_EINVAL, "out is NULL");
    int s = check_problem(problem, kernel);
    if (s) return s;
    s = check_schedule(T, beta);
    if (s) return s;
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (!eps) return fail(OASMC_EINVAL, "eps is NULL");
    for (int t = 0; t < T; ++t)
        if (!(eps[t] > 0.0) || !std::isfinite(eps[t]))
            return fail(OASMC_EINVAL, "eps[%d] must be positive and finite", t);
    if (!out->log_g || !out->accept) return fail(OASMC_EINVAL, "out->log_g and out->accept are required");
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;

    SweepArgs a{};
    a.tg = target_dev(problem);
    a.move = kernel->move;
    a.leapfrog = kernel->leapfrog;
    a.N = N;
    a.T = T;
    a.key.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key.k1 = (uint32_t)(seed >> 32);
    a.key.c2 = (round_k & 0xFFFFu) | (problem_id << 16);
    a.lw_out = out->lw;
    a.x_out = out->x;
    a.acc_bits = out->accept_bits;
    a.acc_words = (T + 31) / 32;

    double *dbeta, *deps, *dlogg, *dacc, *dscal;
    HIP_TRY(wget(h, B_BETA, T + 1, &dbeta));
    HIP_TRY(wget(h, B_EPS, T, &deps));
    HIP_TRY(wget(h, B_LOGG, 3 * (size_t)T, &dlogg));
    HIP_TRY(wget(h, B_ACC, T, &dacc));
    HIP_TRY(wget(h, B_SCAL, 8, &dscal));
    HIP_TRY(hipMemcpyAsync(dbeta, beta, sizeof(double) * (T + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(deps, eps, sizeof(double) * T, hipMemcpyHostToDevice, st));
    a.beta = dbeta;
    a.eps = deps;

    std::vector<double> scal(8, 0.0);
    int nres = 0;
    if (!kernel->resample) {
        int64_t ntiles;
        ValuShape shape{};
        if (problem->family == OASMC_LOGREG) {
            if (h->lds_per_block < logreg_shared_bytes())
                return fail(OASMC_EUNSUPPORTED, "device offers %zu bytes of LDS per workgroup, need %zu",
                            h->lds_per_block, logreg_shared_bytes());
            ntiles = logreg_tiles(N);
        } else {
            if (!valu_shape(problem->d, &shape))
                return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
            ntiles = valu_tiles(N, shape);
        }
        const int64_t S = std::min<int64_t>(ntiles, 2048);
        double* part;
        HIP_TRY(wget(h, B_PART, (size_t)S * (T + 1) * 4, &part));
        a.part = part;
        a.S = S;
        a.ntiles = ntiles;
        void* ws = nullptr;
        size_t wb = 0;
        if (problem->family == OASMC_LOGREG) {
            wb = logreg_workspace_bytes(a.tg, N);
            HIP_TRY(h->get(B_LOGREG, wb, &ws));
            HIP_TRY(logreg_prepare(a.tg, ws, st));
        }
        if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
        if (problem->family == OASMC_LOGREG) {
            HIP_TRY(launch_oais_logreg(a, h->cus, ws, wb, st));
        } else {
            const int grid_waves = (int)std::min<int64_t>(S, (int64_t)h->cus * 8);
            HIP_TRY(launch_oais_valu(a, shape, grid_waves, st));
        }
        if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
        HIP_TRY(launch_merge_slots(part, S, T, N, dlogg, dacc, dscal, st));
        HIP_TRY(hipMemcpyAsync(out->log_g, dlogg, sizeof(double) * 3 * T, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(out->accept, dacc, sizeof(double) * T, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(scal.data(), dscal, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h->prof) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
            h->prof_ms += ms;
            h->prof_launches += 1;
            h->prof_steps += (double)N * T;
            if (problem->family == OASMC_LOGREG)
                h->prof_flops += 4.0 * problem->d * (double)problem->n * (double)N * (T + 1);
        }
        if (out->resampled) std::fill(out->resampled, out->resampled + T, 0);
        if (out->ess) {
            // relative ESS of w_{t^-} is not streamed by the AIS pass
            for (int t = 0; t < T; ++t) out->ess[t] = NAN;
        }
    } else {
        ValuShape shape{};
        if (!valu_shape(problem->d, &shape))
            return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
        const int64_t ntiles = valu_tiles(N, shape);
        const int d = problem->d;
        AsmcState z{};
        HIP_TRY(wget(h, B_X, (size_t)N * d, &z.X));
        HIP_TRY(wget(h, B_X2, (size_t)N * d, &z.X2));
        HIP_TRY(wget(h, B_ELL, N, &z.ell));
        HIP_TRY(wget(h, B_ELL2, N, &z.ell2));
        HIP_TRY(wget(h, B_LW, N, &z.lw));
        HIP_TRY(wget(h, B_ACCW, N, &z.accw));
        HIP_TRY(wget(h, B_TPART, (size_t)ntiles * 8, &z.tile_part));
        HIP_TRY(wget(h, B_NRES, 4, &z.nres));
        HIP_TRY(wget(h, B_ESS, T, &z.ess));
        HIP_TRY(wget(h, B_RES, T, &z.resampled));
        HIP_TRY(wget(h, B_C, N, &z.C));
        HIP_TRY(wget(h, B_BTOT, resample_blocks(N), &z.btot));
        z.scal = dscal;
        z.log_g = dlogg;
        z.accept = dacc;
        a.ntiles = ntiles;
        HIP_TRY(launch_zero(dscal, 8, z.nres, 4, st));
        HIP_TRY(launch_asmc_init(a, shape, z, st));
        for (int t = 1; t <= T; ++t) {
            HIP_TRY(launch_asmc_step(a, shape, z, t, kernel->trigger, kernel->nu, st));
            if (t < T) HIP_TRY(launch_resample_step(a, z, t, st));
        }
        std::vector<double> cnt(T);
        HIP_TRY(hipMemcpyAsync(out->log_g, dlogg, sizeof(double) * 3 * T, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(cnt.data(), dacc, sizeof(double) * T, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(scal.data(), dscal, sizeof(double) * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&nres, z.nres, sizeof(int), hipMemcpyDeviceToHost, st));
        if (out->ess)
            HIP_TRY(hipMemcpyAsync(out->ess, z.ess, sizeof(double) * T, hipMemcpyDeviceToHost, st));
        if (out->resampled)
            HIP_TRY(hipMemcpyAsync(out->resampled, z.resampled, sizeof(int) * T,
                                   hipMemcpyDeviceToHost, st));
        if (out->lw) HIP_TRY(hipMemcpyAsync(out->lw, z.lw, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
        if (out->x)
            HIP_TRY(hipMemcpyAsync(out->x, z.X, sizeof(float) * N * d, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int t = 0; t < T; ++t) out->accept[t] = cnt[t] / (double)N;
    }
    out->logZ = scal[0];
    out->n_resample = nres;
    if (!std::isfinite(out->logZ)) return fail(OASMC_ENONFINITE, "log Z_hat is not finite");
    g_err.clear();
    return OASMC_OK;
}

int oasmc_logreg_eval(oasmc_handle* h, const oasmc_problem* problem, int64_t N,
                      const float* theta, double* ell, float* grad, void* stream)
{
    if (!h || !problem || !theta || !ell || !grad) return fail(OASMC_EINVAL, "NULL argument");
    if (problem->family != OASMC_LOGREG) return fail(OASMC_EINVAL, "problem is not logistic regression");
    if (!problem->X || !problem->y || problem->n < 1) return fail(OASMC_EINVAL, "need X, y, n >= 1");
    if (problem->d < 1 || problem->d > kMaxDLogreg)
        return fail(OASMC_EUNSUPPORTED, "logistic regression supports 1 <= d <= %d", kMaxDLogreg);
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (h->lds_per_block < logreg_shared_bytes())
        return fail(OASMC_EUNSUPPORTED, "device offers %zu bytes of LDS per workgroup, need %zu",
                    h->lds_per_block, logreg_shared_bytes());
    HIP_TRY(hipSetDevice(h->device));
    const TargetDev tg = target_dev(problem);
    void* ws;
    HIP_TRY(h->get(B_LOGREG, logreg_workspace_bytes(tg, N), &ws));
    HIP_TRY(logreg_prepare(tg, ws, (hipStream_t)stream));
    HIP_TRY(launch_logreg_eval(tg, theta, N, ell, grad, ws, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    g_err.clear();
    return OASMC_OK;
}

int oasmc_profile(oasmc_handle* h, int32_t enable, double* kernel_ms, int64_t* launches,
                  double* particle_steps, double* flops)
{
    if (!h) return fail(OASMC_EINVAL, "handle is NULL");
    if (kernel_ms) *kernel_ms = h->prof_ms;
    if (launches) *launches = h->prof_launches;
    if (particle_steps) *particle_steps = h->prof_steps;
    if (flops) *flops = h->prof_flops;
    if (enable && !h->prof) {
        HIP_TRY(hipSetDevice(h->device));
        if (!h->ev0) HIP_TRY(hipEventCreate(&h->ev0));
        if (!h->ev1) HIP_TRY(hipEventCreate(&h->ev1));
        h->prof_ms = h->prof_steps = h->prof_flops = 0.0;
        h->prof_launches = 0;
    }
    h->prof = enable != 0;
    g_err.clear();
    return OASMC_OK;
}

int oasmc_resample(oasmc_handle* h, int64_t N, const double* lw, uint32_t u, int32_t* anc,
                   void* stream)
{
    if (!h || !lw || !anc) return fail(OASMC_EINVAL, "NULL argument");
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    uint64_t *C, *bt;
    double* scal;
    HIP_TRY(wget(h, B_C, N, &C));
    HIP_TRY(wget(h, B_BTOT, resample_blocks(N), &bt));
    HIP_TRY(wget(h, B_SCAL, 8, &scal));
    HIP_TRY(launch_resample_plain(N, lw, u, anc, C, bt, scal, st));
    double flag[4];
    HIP_TRY(hipMemcpyAsync(flag, scal, sizeof(flag), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flag[2] == 0.0) return fail(OASMC_ENONFINITE, "no finite log-weight");
    g_err.clear();
    return OASMC_OK;
}

int oasmc_philox(oasmc_handle* h, uint64_t seed, const uint32_t* ctr, uint32_t* out,
                 int64_t count, void* stream)
{
    if (!h || !ctr || !out) return fail(OASMC_EINVAL, "NULL argument");
    if (count < 0) return fail(OASMC_EINVAL, "negative count");
    if (count == 0) return OASMC_OK;
    HIP_TRY(hipSetDevice(h->device));
    HIP_TRY(launch_philox(seed, ctr, out, count, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    g_err.clear();
    return OASMC_OK;
}

// ---------------------------------------------------------------------------
// Alg. 2: the round loop.
// ---------------------------------------------------------------------------
static void budget_step(const oasmc_run_opts* o, int64_t N, int T, int64_t* Nn, int* Tn)
{
    int64_t n2 = N;
    int t2 = T;
    switch (o->budget) {
    case OASMC_BUDGET_DOUBLE_N:
        n2 = N * 2;
        break;
    case OASMC_BUDGET_DOUBLE_T:
        t2 = T * 2;
        break;
    case OASMC_BUDGET_SQRT2: {
        const int64_t grown = (int64_t)std::llround((double)N * std::sqrt(2.0));
        if (grown <= o->N_max) {
            n2 = grown;
            const int tg = (int)std::lround((double)T * std::sqrt(2.0));
            t2 = std::max(tg, T + 1);
        } else {
            t2 = T * 2;
        }
        break;
    }
    default:
        break;
    }
    if (o->T_max > 0) t2 = std::min(t2, o->T_max);
    *Nn = n2;
    *Tn = t2;
}

static double interp_linear_const(const std::vector<double>& xs, const std::vector<double>& ys,
                                  double q)
{
    if (q <= xs.front()) return ys.front();
    if (q >= xs.back()) return ys.back();
    const size_t i = std::upper_bound(xs.begin(), xs.end(), q) - xs.begin() - 1;
    const double w = (q - xs[i]) / (xs[i + 1] - xs[i]);
    return ys[i] + w * (ys[i + 1] - ys[i]);
}

extern "C" int oasmc_run(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                         const oasmc_run_opts* opts, int64_t N1, uint64_t seed, uint32_t problem_id,
                         oasmc_run_out* out, void* stream)
{
    if (!h || !opts || !out) return fail(OASMC_EINVAL, "NULL argument");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (out->rounds < 1) return fail(OASMC_EINVAL, "rounds must be >= 1");
    if (opts->T1 < 1 || opts->T1 > out->Tcap) return fail(OASMC_EINVAL, "need 1 <= T1 <= Tcap");
    if (N1 < 1) return fail(OASMC_EINVAL, "N1 must be >= 1");
    if (opts->budget < 0 || opts->budget > 3) return fail(OASMC_EINVAL, "unknown budget rule");
    if (!(opts->eps0 > 0.0)) return fail(OASMC_EINVAL, "eps0 must be positive");
    if (!out->logZ || !out->N || !out->T || !out->beta || !out->log_g || !out->accept ||
        !out->eps || !out->n_resample || !out->Lambda_hat)
        return fail(OASMC_EINVAL, "every oasmc_run_out array is required");
    const int Tcap = out->Tcap;
    out->rounds_done = 0;
    int64_t N = N1;
    int T = opts->T1;
    std::vector<double> beta(T + 1), eps(T);
    uniform_schedule(T, beta.data());
    for (int t = 1; t <= T; ++t)
        eps[t - 1] = opts->eps_adapt ? opts->eps0 / std::sqrt(1.0 + beta[t] * opts->eps_kappa)
                                     : opts->eps0;
    int status = OASMC_OK;
    for (int k = 1; k <= out->rounds; ++k) {
        std::vector<double> lg(3 * (size_t)T), acc(T);
        oasmc_round_out ro{};
        ro.log_g = lg.data();
        ro.accept = acc.data();
        status = oasmc_asmc(h, problem, kernel, N, T, beta.data(), eps.data(), seed, (uint32_t)k,
                            problem_id, &ro, stream);
        if (status != OASMC_OK && status != OASMC_ENONFINITE) break;
        const int r = k - 1;
        out->logZ[r] = ro.logZ;
        out->N[r] = N;
        out->T[r] = T;
        out->n_resample[r] = ro.n_resample;
        std::copy(beta.begin(), beta.end(), out->beta + (size_t)r * (Tcap + 1));
        std::copy(lg.begin(), lg.end(), out->log_g + (size_t)r * 3 * Tcap);
        std::copy(acc.begin(), acc.end(), out->accept + (size_t)r * Tcap);
        std::copy(eps.begin(), eps.end(), out->eps + (size_t)r * Tcap);
        int64_t Nn;
        int Tn;
        budget_step(opts, N, T, &Nn, &Tn);
        Tn = std::min(Tn, Tcap);
        std::vector<double> bn(Tn + 1), en(Tn);
        const int s2 = adapt_schedule_impl(T, beta.data(), lg.data(), Tn, opts->interp, bn.data(),
                                           out->Lambda_hat + (size_t)r * (Tcap + 1));
        if (status == OASMC_OK && s2 != OASMC_OK) status = s2;
        if (opts->eps_adapt) {
            std::vector<double> kx(T), ky(T);
            for (int t = 1; t <= T; ++t) {
                kx[t - 1] = beta[t];
                ky[t - 1] = std::log(eps[t - 1]) + (acc[t - 1] - opts->accept_target);
            }
            for (int t = 1; t <= Tn; ++t) en[t - 1] = std::exp(interp_linear_const(kx, ky, bn[t]));
        } else {
            std::fill(en.begin(), en.end(), opts->eps0);
        }
        out->rounds_done = k;
        beta.swap(bn);
        eps.swap(en);
        N = Nn;
        T = Tn;
        if (status != OASMC_OK) break;
    }
    if (status == OASMC_OK) g_err.clear();
    return status;
}

}  // extern "C"
