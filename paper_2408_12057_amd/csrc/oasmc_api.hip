// oasmc_api.hip -- the C ABI (include/oasmc.h): argument validation, the
// handle-owned workspace, the per-round host driver (Alg. 2), the host schedule
// optimiser (Alg. 3), Budget and step-size adaptation.  All compute of the
// annealing passes runs in the gfx950 kernels; the host only moves O(T)
// vectors per round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
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

}  // namespace

namespace oasmc {
// Error reporting for entry points defined in other source files.
int record_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
void clear_error() { g_err.clear(); }
}  // namespace oasmc

namespace {

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
    // a captured multi-round graph and the descriptor bytes it was built from;
    // capture runs on a stream of the handle (the null stream cannot capture)
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<char> graph_key;
    // side streams (default priority) on which the kernel classes of a batch
    // round run concurrently, forked from and joined back into the caller's
    // stream by events (captured as parallel branches of the graph)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> fork_join;  // [0]: fork, [1 + i]: join of side stream i
    // live kernel timing
    bool prof = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> evpool;  // event pairs around the sweeps of each round
    double prof_ms = 0.0, prof_steps = 0.0, prof_flops = 0.0;
    int64_t prof_launches = 0;
    // measured launch shapes of the loop-swapped VALU sweep, per problem class
    // (family, move, d, N rounded up to a power of two, leapfrog, K)
    bool autotune = false;
    std::map<std::array<int64_t, 6>, ValuShape> tuned;

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
    B_TPART, B_NRES, B_ESS, B_RES, B_C, B_BTOT, B_LWO, B_XO, B_LOGREG, B_CKPT, B_SEG, B_ABITS,
    B_GPART, B_GRAD, B_DEVRUN, B_DEVDESC, B_G, B_G2, B_BLK, B_RJ_ANC, B_RJ_SUM, B_RJ_OUT,
    B_RJ_LW, B_RJ_X, B_ZSTOP, B_PT_OUT, B_PT_F, B_COUNT
};

template <typename T>
hipError_t wget(oasmc_handle* h, int id, size_t count, T** p)
{
    void* v = nullptr;
    hipError_t e = h->get(id, count * sizeof(T), &v);
    *p = static_cast<T*>(v);
    return e;
}

// Moment slots of an AIS pass over `ntiles` tiles (oasmc_kernel.slots).
int64_t slot_count(int64_t ntiles, int32_t slots)
{
    const int64_t cap = slots > 0 ? (int64_t)slots : 2048;
    return std::min<int64_t>(ntiles, cap);
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
    if (p->family != OASMC_UNID && (!(p->ref_sigma2 > 0.0) || !std::isfinite(p->ref_sigma2)))
        return fail(OASMC_EINVAL, "ref_sigma2 must be positive and finite");
    if (k->move < OASMC_RWMH || k->move > OASMC_RWMH3)
        return fail(OASMC_EINVAL, "unknown move %d", k->move);
    if (k->move == OASMC_HMC && k->leapfrog < 1)
        return fail(OASMC_EINVAL, "HMC needs leapfrog >= 1");
    if (k->slots < 0) return fail(OASMC_EINVAL, "slots must be >= 0 (0 = default)");
    if (k->resample && !(k->nu > 0.0 && k->nu < 1.0))
        return fail(OASMC_EINVAL, "nu must lie in (0, 1)");
    if (k->resample && (k->trigger < 0 || k->trigger > 3))
        return fail(OASMC_EINVAL, "unknown resampling trigger %d", k->trigger);
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
    case OASMC_UNID:
        if (p->d != 2) return fail(OASMC_EUNSUPPORTED, "the Unid target has d = 2");
        if (!(p->binom_n > 0.0) || !(p->binom_k > 0.0) || !(p->binom_k < p->binom_n) ||
            !std::isfinite(p->binom_n))
            return fail(OASMC_EINVAL, "Unid needs 0 < binom_k < binom_n");
        if (!(p->box > 0.0) || !std::isfinite(p->box)) return fail(OASMC_EINVAL, "box must be positive");
        if (k->move != OASMC_RWMH && k->move != OASMC_RWMH3)
            return fail(OASMC_EUNSUPPORTED, "the Unid target is built for RWMH and RWMH3");
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
    t.binom_n = p->binom_n;
    t.binom_k = p->binom_k;
    t.box = p->box;
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

// DAR times on a new schedule from a previous round's moments (eq.
// (DAR-times)): predicted incremental discrepancies as squared differences of
// the interpolated cumulative barrier, an event where their running sum since
// the last event exceeds -log nu.
int dar_times_impl(int T, const double* beta, const double* log_g, int Tn,
                   const double* beta_new, int interp, double nu, int32_t* flags,
                   double* D_pred)
{
    std::fill(flags, flags + Tn, 0);
    MonotoneCubic f;
    f.x.assign(beta, beta + T + 1);
    f.y.assign(T + 1, 0.0);
    for (int t = 1; t <= T; ++t) {
        const double D = log_g[2 * T + t - 1] - 2.0 * log_g[T + t - 1] + log_g[t - 1];
        if (!std::isfinite(D)) {
            if (D_pred) std::fill(D_pred, D_pred + Tn, NAN);
            return fail(OASMC_ENONFINITE, "non-finite moments: no DAR times");
        }
        f.y[t] = f.y[t - 1] + (D > 0.0 ? std::sqrt(D) : 0.0);
    }
    if (interp == 0) f.fit();
    auto lam_at = [&](double b) {
        if (interp == 0) return f(b);
        if (b <= f.x.front()) return f.y.front();
        if (b >= f.x.back()) return f.y.back();
        const size_t i = std::upper_bound(f.x.begin(), f.x.end(), b) - f.x.begin() - 1;
        const double w = (b - f.x[i]) / (f.x[i + 1] - f.x[i]);
        return f.y[i] + w * (f.y[i + 1] - f.y[i]);
    };
    const double thr = -std::log(nu);
    double prev = lam_at(beta_new[0]), sum = 0.0;
    for (int t = 1; t <= Tn; ++t) {
        const double cur = lam_at(beta_new[t]);
        const double D = (cur - prev) * (cur - prev);
        prev = cur;
        if (D_pred) D_pred[t - 1] = D;
        sum += D;
        if (t < Tn && sum > thr) {
            flags[t - 1] = 1;
            sum = 0.0;
        }
    }
    return OASMC_OK;
}

// Shapes (lanes per particle, coordinates per lane) the VALU sweeps are built
// for; a shape holds d when LPP DPL >= d.
const ValuShape kShapes[] = {{1, 4}, {1, 8}, {1, 12}, {1, 16}, {1, 20}, {1, 24}, {2, 16},
                             {4, 8}, {8, 4}, {4, 16}, {8, 8}, {8, 16}, {16, 8}, {16, 16}};

// The launch shape of a loop-swapped VALU sweep.  Without autotuning the
// fixed rule of valu_shape; with it, the shape measured fastest for the
// problem's class: every shape that holds d runs the same short pass (4 steps,
// uniform schedule, all N particles up to 2^20) on the problem itself, twice,
// timed with HIP events; the fastest per particle-step is kept in the handle.
// Results do not depend on the shape except through binary64 summation order
// across a particle's lanes.
int pick_shape(oasmc_handle* h, const oasmc_problem* p, const oasmc_kernel* k, int64_t N,
               ValuShape* s, hipStream_t st)
{
    if (!valu_shape(p->d, N, s)) return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", p->d);
    if (!h->autotune || p->family == OASMC_UNID) return OASMC_OK;
    int64_t nb = 1;
    while (nb < N) nb <<= 1;
    // leapfrog steps matter only to HMC
    const std::array<int64_t, 6> key{p->family, k->move, p->d, nb,
                                     k->move == OASMC_HMC ? k->leapfrog : 0, p->K};
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) {
        *s = it->second;
        return OASMC_OK;
    }
    const int T = 4;
    const int64_t Nt = std::min<int64_t>(N, (int64_t)1 << 20);
    std::vector<double> bh(T + 1), eh(T, 0.1);
    for (int t = 0; t <= T; ++t) bh[t] = (double)t / T;
    double *db, *de;
    HIP_TRY(wget(h, B_BETA, T + 1, &db));
    HIP_TRY(wget(h, B_EPS, T, &de));
    HIP_TRY(hipMemcpyAsync(db, bh.data(), sizeof(double) * (T + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(de, eh.data(), sizeof(double) * T, hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const ValuShape rule = *s;
    ValuShape best = rule;
    float best_ms = 1e30f;
    std::vector<ValuShape> cands{rule};  // the rule's shape first: it wins near ties
    for (const ValuShape& c : kShapes)
        if (c.lpp * c.dpl >= p->d && !(c.lpp == rule.lpp && c.dpl == rule.dpl)) cands.push_back(c);
    for (const ValuShape& c : cands) {
        SweepArgs a{};
        a.tg = target_dev(p);
        a.move = k->move;
        a.leapfrog = k->leapfrog;
        a.N = Nt;
        a.T = T;
        a.beta = db;
        a.eps = de;
        a.key.k0 = 0x7E57u;
        a.ntiles = valu_tiles(Nt, c);
        a.S = slot_count(a.ntiles, 0);
        double* part;
        HIP_TRY(wget(h, B_PART, (size_t)a.S * (T + 1) * 4, &part));
        a.part = part;
        const int gw = (int)std::min<int64_t>(a.S, (int64_t)h->cus * 8);
        float ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(hipEventRecord(e0, st));
            HIP_TRY(launch_oais_valu(a, c, gw, st));
            HIP_TRY(hipEventRecord(e1, st));
            HIP_TRY(hipEventSynchronize(e1));
            float m = 0.f;
            HIP_TRY(hipEventElapsedTime(&m, e0, e1));
            ms = std::min(ms, m);
        }
        if (ms < best_ms * 0.98f) {  // a candidate must beat the best so far by 2%
            best_ms = ms;
            best = c;
        }
    }
    HIP_TRY(hipEventDestroy(e0));
    HIP_TRY(hipEventDestroy(e1));
    h->tuned[key] = best;
    *s = best;
    return OASMC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Device-resident round loop (Alg. 2 with N fixed): every round's sweep,
// merge, OptimiseSchedule and step-size update stay on the GPU; one batch of
// problems (or a single one) is enqueued, optionally as one hipGraph.
// ---------------------------------------------------------------------------
namespace {

struct DevProblem {
    oasmc_problem prob;
    oasmc_kernel kern;
    int64_t N;
    std::vector<int> Ts;  // T of each round, plus the T of the schedule after the last
    int eps_adapt, interp;
    double eps0, eps_kappa, accept_target;
    uint64_t seed;
    uint32_t problem_id;
    // derived
    bool logreg;
    ValuShape shape;
    int kh;
    int64_t ntiles, S;
    int Tcap;
    size_t off_sched, off_out, off_part, off_scratch, off_par, off_data;
};

struct DevOut {  // byte offsets inside a problem's output block
    size_t logZ, log_g, acc, Lambda, status, beta, eps;
};

template <typename T>
T* at(char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

DevOut out_layout(const DevProblem& q, int R, size_t* bytes)
{
    DevOut o{};
    size_t b = 0;
    const size_t Tc = (size_t)q.Tcap;
    o.logZ = b; b += sizeof(double) * R;
    o.log_g = b; b += sizeof(double) * R * 3 * Tc;
    o.acc = b; b += sizeof(double) * R * Tc;
    o.Lambda = b; b += sizeof(double) * R * (Tc + 1);
    o.status = b; b += sizeof(int) * R;
    b = align256(b);
    *bytes = b;
    return o;
}

// schedule block: beta [(R+1)][Tcap+1] then eps [(R+1)][Tcap]
size_t sched_bytes(const DevProblem& q, int R)
{
    return align256(sizeof(double) * (size_t)(R + 1) * ((q.Tcap + 1) + q.Tcap));
}

int run_device(oasmc_handle* h, std::vector<DevProblem>& ps, int R, bool use_graph,
               std::vector<char>& host_sched, std::vector<char>& host_out, hipStream_t st)
{
    const int P = (int)ps.size();
    // layout of the device workspace
    size_t off = 0;
    size_t sched_total = 0, out_total = 0;
    for (auto& q : ps) { q.off_sched = sched_total; sched_total += sched_bytes(q, R); }
    off = sched_total;
    const size_t out_base = off;
    for (auto& q : ps) {
        size_t ob;
        out_layout(q, R, &ob);
        q.off_out = out_base + out_total;
        out_total += ob;
    }
    off += out_total;
    for (auto& q : ps) {
        q.off_part = off;
        off += align256(sizeof(double) * (size_t)q.S * (q.Tcap + 1) * 4);
        q.off_scratch = off;
        off += align256(sizeof(double) * 3 * (size_t)(q.Tcap + 1));
        q.off_par = off;
        if (!q.logreg) {
            const TargetDev tg = target_dev(&q.prob);
            off += align256(sizeof(float) * q.prob.d) + align256(2 * sizeof(double) * kMaxK) +
                   align256(sizeof(double) * lane_param_doubles(tg, q.shape.lpp, q.shape.dpl));
        }
        q.off_data = off;
        if (q.logreg) off += align256(logreg_workspace_bytes(target_dev(&q.prob), q.N, q.kh));
    }
    char* ws;
    {
        void* v;
        HIP_TRY(h->get(B_DEVRUN, off, &v));
        ws = static_cast<char*>(v);
    }
    // descriptors: SweepArgs [R][P], LogregArgs [R][P], ParView [P], RoundDev [R][P],
    // TargetDev [P], BatchParam [P], items per class
    struct ClassKey {
        bool logreg; int fam, move, lpp, dpl, kh;
        bool operator==(const ClassKey& o) const
        {
            return logreg == o.logreg && fam == o.fam && move == o.move && lpp == o.lpp &&
                   dpl == o.dpl && kh == o.kh;
        }
    };
    std::vector<ClassKey> classes;
    std::vector<std::vector<int2>> items;
    std::vector<std::vector<double>> item_cost;
    for (int p = 0; p < P; ++p) {
        const DevProblem& q = ps[p];
        ClassKey k{q.logreg, q.prob.family, q.kern.move, q.shape.lpp, q.shape.dpl, q.kh};
        size_t c = 0;
        while (c < classes.size() && !(classes[c] == k)) ++c;
        if (c == classes.size()) { classes.push_back(k); items.emplace_back(); item_cost.emplace_back(); }
        for (int64_t sl = 0; sl < q.S; ++sl) {
            const int64_t tiles = (q.ntiles - sl + q.S - 1) / q.S;
            items[c].push_back(make_int2(p, (int)sl));
            item_cost[c].push_back((double)tiles * q.Ts[R - 1] * (q.logreg ? q.prob.n : q.prob.d));
        }
    }
    // longest items first, so the static round-robin assignment balances
    for (size_t c = 0; c < classes.size(); ++c) {
        std::vector<size_t> idx(items[c].size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(),
                         [&](size_t a, size_t b) { return item_cost[c][a] > item_cost[c][b]; });
        std::vector<int2> sorted(idx.size());
        for (size_t i = 0; i < idx.size(); ++i) sorted[i] = items[c][idx[i]];
        items[c].swap(sorted);
    }
    size_t dsz = 0;
    const size_t d_sweep = dsz; dsz += align256(sizeof(SweepArgs) * R * P);
    const size_t d_lr = dsz; dsz += align256(sizeof(LogregArgs) * R * P);
    const size_t d_view = dsz; dsz += align256(sizeof(ParView) * P);
    const size_t d_round = dsz; dsz += align256(sizeof(RoundDev) * R * P);
    const size_t d_tg = dsz; dsz += align256(sizeof(TargetDev) * P);
    const size_t d_pp = dsz; dsz += align256(sizeof(BatchParam) * P);
    // one work counter per class, zeroed at the start of every round by a
    // fill kernel (capturable, unlike a memset node)
    const size_t d_next = dsz; dsz += align256(sizeof(uint32_t) * classes.size());
    std::vector<size_t> d_items(classes.size());
    for (size_t c = 0; c < classes.size(); ++c) { d_items[c] = dsz; dsz += align256(sizeof(int2) * items[c].size()); }
    char* dd;
    {
        void* v;
        HIP_TRY(h->get(B_DEVDESC, dsz, &v));
        dd = static_cast<char*>(v);
    }
    std::vector<char> blob(dsz, 0);
    for (int p = 0; p < P; ++p) {
        DevProblem& q = ps[p];
        size_t ob;
        const DevOut o = out_layout(q, R, &ob);
        char* outp = ws + q.off_out;
        double* beta0 = at<double>(ws, q.off_sched);
        double* eps0 = beta0 + (size_t)(R + 1) * (q.Tcap + 1);
        // parameter view (closed-form families): m [d] floats, then 1/(2 v_k) and
        // 1/v_k (kMaxK doubles each), then the lane-layout means of the
        // problem's sweep shape; none for logistic regression
        ParView v{};
        BatchParam bp{};
        if (!q.logreg) {
            char* base = ws + q.off_par;
            bp.m = reinterpret_cast<float*>(base);
            bp.hiv = reinterpret_cast<double*>(base + align256(sizeof(float) * q.prob.d));
            bp.iv = bp.hiv + kMaxK;
            bp.lane = reinterpret_cast<double*>(base + align256(sizeof(float) * q.prob.d) +
                                                align256(2 * sizeof(double) * kMaxK));
            bp.lpp = q.shape.lpp;
            bp.dpl = q.shape.dpl;
            v.m = bp.m;
            v.hiv = bp.hiv;
            v.iv = bp.iv;
            v.mu = (q.prob.family == OASMC_GMM) ? q.prob.means : q.prob.mu;
            v.lm = bp.lane;
            v.lmu = bp.lane + (size_t)bp.lpp * bp.dpl;
        }
        reinterpret_cast<ParView*>(blob.data() + d_view)[p] = v;
        reinterpret_cast<TargetDev*>(blob.data() + d_tg)[p] = target_dev(&q.prob);
        reinterpret_cast<BatchParam*>(blob.data() + d_pp)[p] = bp;
        for (int k = 0; k < R; ++k) {
            const int T = q.Ts[k];
            SweepArgs a{};
            a.tg = target_dev(&q.prob);
            a.move = q.kern.move;
            a.leapfrog = q.kern.leapfrog;
            a.N = q.N;
            a.T = T;
            a.beta = beta0 + (size_t)k * (q.Tcap + 1);
            a.eps = eps0 + (size_t)k * q.Tcap;
            a.key.k0 = (uint32_t)(q.seed & 0xFFFFFFFFu);
            a.key.k1 = (uint32_t)(q.seed >> 32);
            a.key.c2 = ((uint32_t)(k + 1) & 0xFFFFu) | (q.problem_id << 16);
            a.part = at<double>(ws, q.off_part);
            a.S = q.S;
            a.ntiles = q.ntiles;
            a.acc_words = (T + 31) / 32;
            reinterpret_cast<SweepArgs*>(blob.data() + d_sweep)[(size_t)k * P + p] = a;
            LogregArgs la{};
            la.a = a;
            if (q.logreg) logreg_layout(a.tg, q.N, q.kh, ws + q.off_data, &la);
            reinterpret_cast<LogregArgs*>(blob.data() + d_lr)[(size_t)k * P + p] = la;
            RoundDev rd{};
            rd.T = T;
            rd.Tn = q.Ts[k + 1];
            rd.N = q.N;
            rd.S = q.S;
            rd.part = a.part;
            rd.beta = a.beta;
            rd.eps = a.eps;
            rd.log_g = at<double>(outp, o.log_g) + (size_t)k * 3 * q.Tcap;
            rd.acc = at<double>(outp, o.acc) + (size_t)k * q.Tcap;
            rd.logZ = at<double>(outp, o.logZ) + k;
            rd.Lambda = at<double>(outp, o.Lambda) + (size_t)k * (q.Tcap + 1);
            rd.beta_next = beta0 + (size_t)(k + 1) * (q.Tcap + 1);
            rd.eps_next = eps0 + (size_t)(k + 1) * q.Tcap;
            rd.status = at<int>(outp, o.status) + k;
            rd.scratch = at<double>(ws, q.off_scratch);
            rd.interp = q.interp;
            rd.eps_adapt = q.eps_adapt;
            rd.eps0 = q.eps0;
            rd.accept_target = q.accept_target;
            reinterpret_cast<RoundDev*>(blob.data() + d_round)[(size_t)k * P + p] = rd;
        }
    }
    for (size_t c = 0; c < classes.size(); ++c)
        std::copy(items[c].begin(), items[c].end(), reinterpret_cast<int2*>(blob.data() + d_items[c]));

    // the round-1 schedules and step sizes
    host_sched.assign(sched_total, 0);
    for (const auto& q : ps) {
        double* b = reinterpret_cast<double*>(host_sched.data() + q.off_sched);
        double* e = b + (size_t)(R + 1) * (q.Tcap + 1);
        const int T = q.Ts[0];
        uniform_schedule(T, b);
        for (int t = 1; t <= T; ++t)
            e[t - 1] = q.eps_adapt ? q.eps0 / std::sqrt(1.0 + b[t] * q.eps_kappa) : q.eps0;
    }
    HIP_TRY(hipMemcpyAsync(dd, blob.data(), dsz, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(ws, host_sched.data(), sched_total, hipMemcpyHostToDevice, st));
    // per-problem constant data: parameter views and packed regression data
    {
        std::vector<int> vp;
        for (int p = 0; p < P; ++p)
            if (!ps[p].logreg) vp.push_back(p);
        if (!vp.empty()) {
            const TargetDev* tgs = reinterpret_cast<const TargetDev*>(dd + d_tg);
            const BatchParam* bps = reinterpret_cast<const BatchParam*>(dd + d_pp);
            // logistic-regression entries have null pointers and are skipped by family
            HIP_TRY(launch_batch_params(tgs, bps, P, st));
        }
        for (int p = 0; p < P; ++p)
            if (ps[p].logreg) {
                const TargetDev tg = target_dev(&ps[p].prob);
                HIP_TRY(logreg_pack_into(tg, ps[p].N, ps[p].kh, ws + ps[p].off_data, st));
            }
    }
    HIP_TRY(hipStreamSynchronize(st));

    int Tmax = 1;
    for (const auto& q : ps)
        for (int k = 0; k < R; ++k) Tmax = std::max(Tmax, q.Ts[k]);
    // per-round event pairs around the sweep kernels (timed runs, not graphs)
    const bool time_sweeps = h->prof && !use_graph;
    if (time_sweeps)
        while ((int)h->evpool.size() < 2 * R) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            h->evpool.push_back(e);
        }
    // the classes of a round run concurrently on up to kSideStreams streams
    // (their problems' buffers and work counters are disjoint); on the
    // 256-problem batch two streams measured 1% faster than four or eight
    constexpr int kSideStreams = 2;
    const int nside = (P > 1) ? std::min<int>(kSideStreams, (int)classes.size()) : 0;
    while ((int)h->side.size() < nside) {
        hipStream_t ss;
        HIP_TRY(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking));
        h->side.push_back(ss);
    }
    while ((int)h->fork_join.size() < 1 + nside) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->fork_join.push_back(e);
    }
    auto enqueue = [&](hipStream_t s) -> int {
        for (int k = 0; k < R; ++k) {
            // one problem's items (its slots) are equal: the static round
            // robin already balances them, and no counter is needed
            uint32_t* next = P > 1 ? reinterpret_cast<uint32_t*>(dd + d_next) : nullptr;
            const int nc = (int)classes.size();
            for (int c0 = 0; next && c0 < nc; c0 += 64)
                HIP_TRY(launch_zero(nullptr, 0, reinterpret_cast<int*>(next + c0),
                                    std::min(64, nc - c0), s));
            if (time_sweeps) HIP_TRY(hipEventRecord(h->evpool[2 * k], s));
            if (nside > 1) {
                HIP_TRY(hipEventRecord(h->fork_join[0], s));
                for (int i = 0; i < nside; ++i) HIP_TRY(hipStreamWaitEvent(h->side[i], h->fork_join[0], 0));
            }
            for (size_t c = 0; c < classes.size(); ++c) {
                const hipStream_t cs = (nside > 1) ? h->side[c % nside] : s;
                const int64_t n = (int64_t)items[c].size();
                const int2* it = reinterpret_cast<const int2*>(dd + d_items[c]);
                if (classes[c].logreg) {
                    const LogregArgs* la = reinterpret_cast<const LogregArgs*>(dd + d_lr) + (size_t)k * P;
                    const int grid = (int)std::min<int64_t>(n, h->cus);
                    HIP_TRY(launch_oais_logreg_batch(classes[c].kh, la, it, n, next ? next + c : nullptr,
                                                     grid, cs));
                } else {
                    ValuBatch b{};
                    b.args = reinterpret_cast<const SweepArgs*>(dd + d_sweep) + (size_t)k * P;
                    b.views = reinterpret_cast<const ParView*>(dd + d_view);
                    b.items = it;
                    b.nitems = n;
                    b.next = next ? next + c : nullptr;
                    ValuShape sh{classes[c].lpp, classes[c].dpl};
                    const int gw = (int)std::min<int64_t>(n, (int64_t)h->cus * 8);
                    HIP_TRY(launch_oais_valu_batch(classes[c].fam, classes[c].move, sh, b, gw, cs));
                }
            }
            if (nside > 1)
                for (int i = 0; i < nside; ++i) {
                    HIP_TRY(hipEventRecord(h->fork_join[1 + i], h->side[i]));
                    HIP_TRY(hipStreamWaitEvent(s, h->fork_join[1 + i], 0));
                }
            if (time_sweeps) HIP_TRY(hipEventRecord(h->evpool[2 * k + 1], s));
            const RoundDev* rd = reinterpret_cast<const RoundDev*>(dd + d_round) + (size_t)k * P;
            HIP_TRY(launch_round_merge(rd, P, Tmax, s));
            HIP_TRY(launch_round_schedule(rd, P, s));
        }
        return OASMC_OK;
    };

    if (h->prof && use_graph) HIP_TRY(hipEventRecord(h->ev0, st));
    if (use_graph) {
        // reuse the instantiated graph when the descriptors are unchanged
        std::vector<char> key(blob);
        key.insert(key.end(), host_sched.begin(), host_sched.end());
        const char* wsc = reinterpret_cast<const char*>(&ws);
        key.insert(key.end(), wsc, wsc + sizeof(ws));
        if (!h->graph_exec || key != h->graph_key) {
            if (h->graph_exec) {
                HIP_TRY(hipGraphExecDestroy(h->graph_exec));
                h->graph_exec = nullptr;
            }
            hipGraph_t g;
            if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            const int e = enqueue(h->cap_stream);
            hipGraph_t gg = nullptr;
            const hipError_t ce = hipStreamEndCapture(h->cap_stream, &gg);
            if (e != OASMC_OK) {
                if (gg) (void)hipGraphDestroy(gg);  // the enqueue's error is the one reported
                return e;
            }
            if (ce != hipSuccess) return fail(OASMC_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
            g = gg;
            HIP_TRY(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
            HIP_TRY(hipGraphDestroy(g));
            h->graph_key.swap(key);
        }
        HIP_TRY(hipGraphLaunch(h->graph_exec, st));
    } else {
        const int e = enqueue(st);
        if (e != OASMC_OK) return e;
    }
    if (h->prof && use_graph) HIP_TRY(hipEventRecord(h->ev1, st));
    host_out.resize(out_total + sched_total);
    HIP_TRY(hipMemcpyAsync(host_out.data(), ws + out_base, out_total, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(host_out.data() + out_total, ws, sched_total, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->prof) {
        // graphs: the whole replay; otherwise the sweep kernels of each round
        if (use_graph) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
            h->prof_ms += ms;
            h->prof_launches += 1;
        } else {
            for (int k = 0; k < R; ++k) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, h->evpool[2 * k], h->evpool[2 * k + 1]));
                h->prof_ms += ms;
                h->prof_launches += (int64_t)classes.size();
            }
        }
        for (const auto& q : ps)
            for (int k = 0; k < R; ++k) {
                h->prof_steps += (double)q.N * q.Ts[k];
                if (q.logreg) h->prof_flops += 4.0 * q.prob.d * (double)q.prob.n * (double)q.N * (q.Ts[k] + 1);
            }
    }
    return OASMC_OK;
}

// Fills the derived fields of a problem; returns a status.
int prepare_dev_problem(oasmc_handle* h, DevProblem& q, hipStream_t st)
{
    int s = check_problem(&q.prob, &q.kern);
    if (s) return s;
    if (q.kern.resample) return fail(OASMC_EUNSUPPORTED, "the device round loop runs AIS passes");
    if (q.N < 1 || q.N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (!(q.eps0 > 0.0)) return fail(OASMC_EINVAL, "eps0 must be positive");
    q.logreg = (q.prob.family == OASMC_LOGREG);
    if (q.logreg) {
        q.kh = logreg_kh(q.prob.d, q.N, h->cus);
        if (q.kh < 0) return fail(OASMC_EUNSUPPORTED, "no kernel for d=%d", q.prob.d);
        if (h->lds_per_block < logreg_shared_bytes(q.kh))
            return fail(OASMC_EUNSUPPORTED, "device offers %zu bytes of LDS per workgroup, need %zu",
                        h->lds_per_block, logreg_shared_bytes(q.kh));
        q.shape = ValuShape{0, 0};
        q.ntiles = logreg_tiles(q.N, q.kh);
    } else {
        const int ps = pick_shape(h, &q.prob, &q.kern, q.N, &q.shape, st);
        if (ps) return ps;
        q.kh = 0;
        q.ntiles = valu_tiles(q.N, q.shape);
    }
    q.S = slot_count(q.ntiles, q.kern.slots);
    q.Tcap = 1;
    for (int T : q.Ts) q.Tcap = std::max(q.Tcap, T);
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
    // teardown releases everything it can; a failing release leaves nothing
    // for the caller to act on, so the statuses are discarded on purpose
    (void)hipSetDevice(h->device);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    for (auto e : h->evpool) (void)hipEventDestroy(e);
    for (auto e : h->fork_join) (void)hipEventDestroy(e);
    for (auto s : h->side) (void)hipStreamDestroy(s);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (auto& b : h->bufs)
        if (b.p) (void)hipFree(b.p);
    delete h;
    return OASMC_OK;
}

int oasmc_autotune(oasmc_handle* h, int32_t enable, int32_t* n_classes)
{
    if (!h) return fail(OASMC_EINVAL, "handle is NULL");
    h->autotune = enable > 0;
    if (enable < 0) h->tuned.clear();
    if (n_classes) *n_classes = (int32_t)h->tuned.size();
    g_err.clear();
    return OASMC_OK;
}

int oasmc_shape(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                int64_t N, int32_t* lpp, int32_t* dpl, void* stream)
{
    if (!h || !lpp || !dpl) return fail(OASMC_EINVAL, "NULL argument");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (problem->family == OASMC_LOGREG) return fail(OASMC_EUNSUPPORTED, "no VALU shape for logistic regression");
    if (N < 1) return fail(OASMC_EINVAL, "N must be >= 1");
    HIP_TRY(hipSetDevice(h->device));
    ValuShape sh{};
    s = pick_shape(h, problem, kernel, N, &sh, (hipStream_t)stream);
    if (s) return s;
    *lpp = sh.lpp;
    *dpl = sh.dpl;
    g_err.clear();
    return OASMC_OK;
}

int oasmc_dar_times(int32_t T, const double* beta, const double* log_g, int32_t T_new,
                    const double* beta_new, int32_t interp, double nu, int32_t* flags,
                    double* D_pred)
{
    if (T < 1 || T_new < 1) return fail(OASMC_EINVAL, "T and T_new must be >= 1");
    if (!log_g || !beta_new || !flags) return fail(OASMC_EINVAL, "NULL argument");
    if (!(nu > 0.0 && nu < 1.0)) return fail(OASMC_EINVAL, "nu must lie in (0, 1)");
    int s = check_schedule(T, beta);
    if (s) return s;
    s = check_schedule(T_new, beta_new);
    if (s) return s;
    s = dar_times_impl(T, beta, log_g, T_new, beta_new, interp, nu, flags, D_pred);
    if (s == OASMC_OK) g_err.clear();
    return s;
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
        int kh = -1;
        if (problem->family == OASMC_LOGREG) {
            kh = logreg_kh(problem->d, N, h->cus);
            if (kh < 0) return fail(OASMC_EUNSUPPORTED, "no kernel for d=%d", problem->d);
            if (h->lds_per_block < logreg_shared_bytes(kh))
                return fail(OASMC_EUNSUPPORTED, "device offers %zu bytes of LDS per workgroup, need %zu",
                            h->lds_per_block, logreg_shared_bytes(kh));
            ntiles = logreg_tiles(N, kh);
        } else {
            const int ps = pick_shape(h, problem, kernel, N, &shape, st);
            if (ps) return ps;
            ntiles = valu_tiles(N, shape);
        }
        const int64_t S = slot_count(ntiles, kernel->slots);
        double* part;
        HIP_TRY(wget(h, B_PART, (size_t)S * (T + 1) * 4, &part));
        a.part = part;
        a.S = S;
        a.ntiles = ntiles;
        void* ws = nullptr;
        if (problem->family == OASMC_LOGREG) {
            HIP_TRY(h->get(B_LOGREG, logreg_workspace_bytes(a.tg, N, kh), &ws));
            HIP_TRY(logreg_prepare(a.tg, N, kh, ws, st));
        }
        if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
        if (problem->family == OASMC_LOGREG) {
            HIP_TRY(launch_oais_logreg(a, kh, h->cus, ws, st));
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
        if (!valu_shape(problem->d, N, &shape))
            return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
        const int64_t ntiles = valu_tiles(N, shape);
        const int d = problem->d;
        AsmcState z{};
        HIP_TRY(wget(h, B_X, (size_t)N * d, &z.X));
        HIP_TRY(wget(h, B_X2, (size_t)N * d, &z.X2));
        HIP_TRY(wget(h, B_ELL, N, &z.ell));
        HIP_TRY(wget(h, B_ELL2, N, &z.ell2));
        if (uses_grad(kernel->move)) {
            HIP_TRY(wget(h, B_G, (size_t)N * d, &z.G));
            HIP_TRY(wget(h, B_G2, (size_t)N * d, &z.G2));
        }
        HIP_TRY(wget(h, B_LW, N, &z.lw));
        HIP_TRY(wget(h, B_ACCW, N, &z.accw));
        HIP_TRY(wget(h, B_TPART, (size_t)ntiles * 8, &z.tile_part));
        HIP_TRY(wget(h, B_BLK, (size_t)kAsmcMergeBlocks * 8, &z.blk_part));
        HIP_TRY(wget(h, B_NRES, 4, &z.nres));
        HIP_TRY(wget(h, B_ESS, T, &z.ess));
        HIP_TRY(wget(h, B_RES, T, &z.resampled));
        HIP_TRY(wget(h, B_C, N, &z.C));
        HIP_TRY(wget(h, B_BTOT, resample_blocks(N), &z.btot));
        z.ticket = reinterpret_cast<unsigned*>(z.nres + 1);  // cleared with nres below
        z.scal = dscal;
        z.log_g = dlogg;
        z.accept = dacc;
        a.ntiles = ntiles;
        if (kernel->trigger == 3) {
            // times fixed in advance: each segment between two of them runs as
            // a loop-swapped pass (particles in registers, moments streamed
            // into O(T) slots), then its merge and the resampler
            const int64_t S = slot_count(ntiles, kernel->slots);
            double* part;
            HIP_TRY(wget(h, B_PART, (size_t)S * (T + 1) * 4, &part));
            a.part = part;
            a.S = S;
            a.lw_out = nullptr;
            a.x_out = nullptr;
            a.sx = z.X;
            a.sg = z.G;
            a.sell = z.ell;
            a.slw = z.lw;
            a.saccw = z.accw;
            const int grid_waves = (int)std::min<int64_t>(S, (int64_t)h->cus * 8);
            if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
            HIP_TRY(launch_zero(dscal, 8, z.nres, 4, st));
            HIP_TRY(launch_asmc_init(a, shape, z, st));
            int t0 = 0;
            for (int t = 1; t <= T; ++t) {
                const bool ev = t < T && kernel->resample_at && kernel->resample_at[t - 1] != 0;
                if (!ev && t < T) continue;
                a.t_begin = t0;
                a.t_end = t;
                HIP_TRY(launch_oais_valu(a, shape, grid_waves, st));
                HIP_TRY(launch_segment_merge(a, z, st));
                if (t < T) HIP_TRY(launch_resample_step(a, z, t, true, st));
                t0 = t;
            }
            if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
        } else {
            if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
            HIP_TRY(launch_zero(dscal, 8, z.nres, 4, st));
            HIP_TRY(launch_asmc_init(a, shape, z, st));
            for (int t = 1; t <= T; ++t) {
                HIP_TRY(launch_asmc_step(a, shape, z, t, kernel->trigger, kernel->nu, st));
                if (t < T) HIP_TRY(launch_resample_step(a, z, t, false, st));
            }
            if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
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
        if (h->prof) {
            // one "launch" per step: the step's sweep, merge and resampler
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
            h->prof_ms += ms;
            h->prof_launches += T;
            h->prof_steps += (double)N * T;
        }
    }
    out->logZ = scal[0];
    out->n_resample = nres;
    if (!std::isfinite(out->logZ)) return fail(OASMC_ENONFINITE, "log Z_hat is not finite");
    g_err.clear();
    return OASMC_OK;
}

int oasmc_zja(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel, int64_t N,
              double rho, int32_t Tmax, int32_t iters, double eps, uint64_t seed, uint32_t round_k,
              uint32_t problem_id, double* beta, int32_t* T_out, double* log_g, double* logZ,
              double* lw, float* x, void* stream)
{
    if (!h || !beta || !T_out || !logZ) return fail(OASMC_EINVAL, "NULL argument");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (problem->family == OASMC_LOGREG || kernel->resample)
        return fail(OASMC_EUNSUPPORTED, "ZJA is built for AIS on the Gaussian, mixture and Unid families");
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (!(rho > 0.0 && rho < 1.0)) return fail(OASMC_EINVAL, "rho must lie in (0, 1)");
    if (Tmax < 1) return fail(OASMC_EINVAL, "Tmax must be >= 1");
    if (iters < 1 || iters > 60) return fail(OASMC_EINVAL, "iters must lie in [1, 60]");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(OASMC_EINVAL, "eps must be positive");
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    ValuShape shape{};
    if (!valu_shape(problem->d, N, &shape))
        return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
    const int d = problem->d;
    SweepArgs a{};
    a.tg = target_dev(problem);
    a.move = kernel->move;
    a.leapfrog = kernel->leapfrog;
    a.N = N;
    a.T = Tmax;
    a.key.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key.k1 = (uint32_t)(seed >> 32);
    a.key.c2 = (round_k & 0xFFFFu) | (problem_id << 16);
    a.ntiles = valu_tiles(N, shape);
    a.acc_words = (Tmax + 31) / 32;
    double *dbeta, *deps, *dlogg, *dscal;
    int* dstop;
    HIP_TRY(wget(h, B_BETA, (size_t)Tmax + 1, &dbeta));
    HIP_TRY(wget(h, B_EPS, Tmax, &deps));
    HIP_TRY(wget(h, B_LOGG, 3 * (size_t)Tmax, &dlogg));
    HIP_TRY(wget(h, B_SCAL, 8, &dscal));
    HIP_TRY(wget(h, B_ZSTOP, 1, &dstop));
    std::vector<double> eps_h(Tmax, eps), beta0(1, 0.0);
    HIP_TRY(hipMemcpyAsync(deps, eps_h.data(), sizeof(double) * Tmax, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dbeta, beta0.data(), sizeof(double), hipMemcpyHostToDevice, st));
    const int stop0 = Tmax;
    HIP_TRY(hipMemcpyAsync(dstop, &stop0, sizeof(int), hipMemcpyHostToDevice, st));
    a.beta = dbeta;
    a.eps = deps;
    a.t_stop = dstop;
    AsmcState z{};
    HIP_TRY(wget(h, B_X, (size_t)N * d, &z.X));
    HIP_TRY(wget(h, B_ELL, N, &z.ell));
    if (uses_grad(kernel->move)) HIP_TRY(wget(h, B_G, (size_t)N * d, &z.G));
    HIP_TRY(wget(h, B_LW, N, &z.lw));
    HIP_TRY(wget(h, B_ACCW, N, &z.accw));
    HIP_TRY(wget(h, B_TPART, (size_t)a.ntiles * 8, &z.tile_part));
    const double log_rho = std::log(rho);
    if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(launch_asmc_init(a, shape, z, st));
    // steps in chunks; the host looks at the device's stop step after each
    // chunk (steps past it are no-ops on the device)
    constexpr int kChunk = 32;
    int T = Tmax;
    for (int t0 = 1; t0 <= Tmax; t0 += kChunk) {
        const int t1 = std::min(Tmax, t0 + kChunk - 1);
        for (int t = t0; t <= t1; ++t) {
            HIP_TRY(launch_zja_select(N, z.lw, z.ell, dbeta, t, Tmax, log_rho, iters, dstop, dlogg, st));
            HIP_TRY(launch_asmc_move(a, shape, z, t, st));
        }
        int stop = 0;
        HIP_TRY(hipMemcpyAsync(&stop, dstop, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (stop <= t1) {
            T = stop;
            break;
        }
    }
    HIP_TRY(launch_zja_final(N, z.lw, dscal, st));
    if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
    double lz = 0.0;
    HIP_TRY(hipMemcpyAsync(beta, dbeta, sizeof(double) * (T + 1), hipMemcpyDeviceToHost, st));
    if (log_g) HIP_TRY(hipMemcpyAsync(log_g, dlogg, sizeof(double) * 3 * Tmax, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&lz, dscal, sizeof(double), hipMemcpyDeviceToHost, st));
    if (lw) HIP_TRY(hipMemcpyAsync(lw, z.lw, sizeof(double) * N, hipMemcpyDeviceToDevice, st));
    if (x) HIP_TRY(hipMemcpyAsync(x, z.X, sizeof(float) * N * d, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->prof) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->prof_ms += ms;
        h->prof_launches += T;
        h->prof_steps += (double)N * T;
    }
    *T_out = T;
    *logZ = lz;
    if (!std::isfinite(lz)) return fail(OASMC_ENONFINITE, "log Z_hat is not finite");
    g_err.clear();
    return OASMC_OK;
}

int oasmc_pt(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel, int32_t K,
             int32_t Np, int32_t Tp, const double* beta, const double* eps, uint64_t seed,
             uint32_t round_k, uint32_t problem_id, double* logZ, double* ss, double* rej,
             int64_t* trips, double* tmean, double* tsecond, void* stream)
{
    if (!h || !logZ) return fail(OASMC_EINVAL, "NULL argument");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (problem->family == OASMC_LOGREG)
        return fail(OASMC_EUNSUPPORTED, "parallel tempering is built for the Gaussian, mixture and Unid families");
    if (K < 1 || Np < 1 || Tp < 1) return fail(OASMC_EINVAL, "need K, Np, Tp >= 1");
    s = check_schedule(Np, beta);
    if (s) return s;
    if (!eps) return fail(OASMC_EINVAL, "eps is NULL");
    for (int n = 0; n <= Np; ++n)
        if (!(eps[n] > 0.0) || !std::isfinite(eps[n]))
            return fail(OASMC_EINVAL, "eps[%d] must be positive and finite", n);
    const int R = Np + 1;
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    // the sweeps' shape for K (N' + 1) chains (measured when autotuning is on);
    // the rule's shape when the measured one cannot hold a copy in 8 waves
    ValuShape shape{};
    const int ps = pick_shape(h, problem, kernel, (int64_t)K * R, &shape, st);
    if (ps) return ps;
    // a copy runs in one workgroup of at most 8 waves
    if (R > 8 * (kWave / shape.lpp) && !valu_shape(problem->d, (int64_t)K * R, &shape))
        return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
    const int P = kWave / shape.lpp;
    if (R > 8 * P)
        return fail(OASMC_EUNSUPPORTED, "a copy holds at most %d chains at d=%d", 8 * P, problem->d);
    const int d = problem->d;
    PtArgs A{};
    A.a.tg = target_dev(problem);
    A.a.move = kernel->move;
    A.a.leapfrog = kernel->leapfrog;
    A.a.N = (int64_t)K * R;
    A.a.T = Tp;
    A.a.key.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    A.a.key.k1 = (uint32_t)(seed >> 32);
    A.a.key.c2 = (round_k & 0xFFFFu) | (problem_id << 16);
    A.K = K;
    A.Np = Np;
    A.stride = 3 * (int64_t)Np + 2;
    if (pt_shared_bytes(A, shape.lpp, shape.dpl) > h->lds_per_block)
        return fail(OASMC_EUNSUPPORTED, "too many chains for the LDS of one workgroup");
    double *dbeta, *deps, *out, *fpart;
    HIP_TRY(wget(h, B_BETA, (size_t)R, &dbeta));
    HIP_TRY(wget(h, B_EPS, (size_t)R, &deps));
    HIP_TRY(wget(h, B_PT_OUT, (size_t)K * A.stride, &out));
    HIP_TRY(wget(h, B_PT_F, (size_t)K * 16 * 2 * d, &fpart));
    HIP_TRY(hipMemcpyAsync(dbeta, beta, sizeof(double) * R, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(deps, eps, sizeof(double) * R, hipMemcpyHostToDevice, st));
    A.beta = dbeta;
    A.eps = deps;
    A.out = out;
    A.fpart = fpart;
    if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(launch_pt(A, shape, st));
    if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
    std::vector<double> ho((size_t)K * A.stride), hf((size_t)K * 16 * 2 * d);
    HIP_TRY(hipMemcpyAsync(ho.data(), out, sizeof(double) * ho.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hf.data(), fpart, sizeof(double) * hf.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->prof) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->prof_ms += ms;
        h->prof_launches += 1;
        h->prof_steps += (double)K * R * Tp;
    }
    // the copies' outputs in copy order: stepping stones pooled over the K T'
    // terms of each temperature, rejections averaged over the proposals
    double lz = 0.0;
    const double lkt = std::log((double)K * Tp);
    for (int n = 0; n < Np; ++n) {
        double m = -INFINITY, sum = 0.0;
        for (int k = 0; k < K; ++k) {
            const double mk = ho[(size_t)k * A.stride + 2 * n], sk = ho[(size_t)k * A.stride + 2 * n + 1];
            if (!(mk > -INFINITY) || !(sk > 0.0)) continue;
            if (mk > m) {
                sum = sum * std::exp(m - mk) + sk;
                m = mk;
            } else {
                sum += sk * std::exp(mk - m);
            }
        }
        const double v = (sum > 0.0) ? m + std::log(sum) - lkt : -INFINITY;
        if (ss) ss[n] = v;
        lz += v;
        // pair n is proposed at the iterations t of its parity
        const double cnt = (double)K * ((n % 2 == 0) ? (Tp / 2) : ((Tp + 1) / 2));
        double rs = 0.0;
        for (int k = 0; k < K; ++k) rs += ho[(size_t)k * A.stride + 2 * Np + n];
        if (rej) rej[n] = cnt > 0 ? rs / cnt : NAN;
    }
    if (trips) {
        double tr = 0.0;
        for (int k = 0; k < K; ++k) tr += ho[(size_t)k * A.stride + 3 * Np];
        *trips = (int64_t)std::llround(tr);
    }
    if (tmean && tsecond) {
        const int waves = (R + P - 1) / P;
        for (int i = 0; i < d; ++i) {
            double a1 = 0.0, a2 = 0.0;
            for (int k = 0; k < K; ++k)
                for (int w = 0; w < waves; ++w) {
                    a1 += hf[((size_t)k * 16 + w) * 2 * d + i];
                    a2 += hf[((size_t)k * 16 + w) * 2 * d + d + i];
                }
            tmean[i] = a1 / ((double)K * Tp);
            tsecond[i] = a2 / ((double)K * Tp);
        }
    }
    *logZ = lz;
    if (!std::isfinite(lz)) return fail(OASMC_ENONFINITE, "log Z_PT is not finite");
    g_err.clear();
    return OASMC_OK;
}

int oasmc_rejuvenate(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                     int64_t N, int32_t T, double eps_T, uint64_t seed, uint32_t round_k,
                     uint32_t problem_id, const double* lw, const float* x, double* mean,
                     double* second, double* accept, float* x_out, void* stream)
{
    if (!h) return fail(OASMC_EINVAL, "handle is NULL");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (problem->family == OASMC_LOGREG)
        return fail(OASMC_EUNSUPPORTED, "rejuvenation is built for the Gaussian and mixture families");
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (T < 1) return fail(OASMC_EINVAL, "T must be >= 1");
    if (!(eps_T > 0.0) || !std::isfinite(eps_T)) return fail(OASMC_EINVAL, "eps_T must be positive");
    if (!lw || !x || !mean || !second) return fail(OASMC_EINVAL, "NULL argument");
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    ValuShape shape{};
    if (!valu_shape(problem->d, N, &shape))
        return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
    const int d = problem->d;
    RejuvArgs R{};
    R.a.tg = target_dev(problem);
    R.a.move = kernel->move;
    R.a.leapfrog = kernel->leapfrog;
    R.a.N = N;
    R.a.T = T;
    R.a.key.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    R.a.key.k1 = (uint32_t)(seed >> 32);
    R.a.key.c2 = (round_k & 0xFFFFu) | (problem_id << 16);
    R.a.ntiles = valu_tiles(N, shape);
    R.eps = eps_T;
    R.x_in = x;
    R.x_out = x_out;
    int32_t* anc;
    double *tsum, *res, *scal;
    uint64_t *C, *btot;
    HIP_TRY(wget(h, B_RJ_ANC, N, &anc));
    HIP_TRY(wget(h, B_RJ_SUM, (size_t)R.a.ntiles * (2 * d + 1), &tsum));
    HIP_TRY(wget(h, B_RJ_OUT, 2 * (size_t)d + 1, &res));
    HIP_TRY(wget(h, B_SCAL, 8, &scal));
    HIP_TRY(wget(h, B_C, N, &C));
    HIP_TRY(wget(h, B_BTOT, resample_blocks(N), &btot));
    R.anc = anc;
    R.tsum = tsum;
    HIP_TRY(launch_resample_event(N, lw, R.a.key, (uint32_t)T, anc, C, btot, scal, st));
    double flag = 0.0;
    HIP_TRY(hipMemcpyAsync(&flag, scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (flag == 0.0) return fail(OASMC_ENONFINITE, "no finite final weight to resample");
    if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(launch_rejuv(R, shape, st));
    if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
    HIP_TRY(launch_rejuv_reduce(tsum, R.a.ntiles, d, (double)N * (double)T, res, st));
    std::vector<double> hres(2 * (size_t)d + 1);
    HIP_TRY(hipMemcpyAsync(hres.data(), res, sizeof(double) * hres.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->prof) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->prof_ms += ms;
        h->prof_launches += 1;
        h->prof_steps += (double)N * T;
    }
    std::copy(hres.begin(), hres.begin() + d, mean);
    std::copy(hres.begin() + d, hres.begin() + 2 * d, second);
    if (accept) *accept = hres[2 * d];
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
    const int kh = logreg_kh(problem->d, N, h->cus);
    if (kh < 0) return fail(OASMC_EUNSUPPORTED, "no kernel for d=%d", problem->d);
    if (h->lds_per_block < logreg_shared_bytes(kh))
        return fail(OASMC_EUNSUPPORTED, "device offers %zu bytes of LDS per workgroup, need %zu",
                    h->lds_per_block, logreg_shared_bytes(kh));
    HIP_TRY(hipSetDevice(h->device));
    const TargetDev tg = target_dev(problem);
    void* ws;
    HIP_TRY(h->get(B_LOGREG, logreg_workspace_bytes(tg, N, kh), &ws));
    HIP_TRY(logreg_prepare(tg, N, kh, ws, (hipStream_t)stream));
    HIP_TRY(launch_logreg_eval(tg, kh, theta, N, ell, grad, ws, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    g_err.clear();
    return OASMC_OK;
}

int oasmc_target_eval(oasmc_handle* h, const oasmc_problem* problem, int64_t N, const float* x,
                      int32_t lpp, int32_t dpl, double* ell, double* grad, void* stream)
{
    if (!h || !problem || !x || !ell || !grad) return fail(OASMC_EINVAL, "NULL argument");
    if (problem->family == OASMC_LOGREG)
        return fail(OASMC_EINVAL, "logistic regression is evaluated by oasmc_logreg_eval");
    oasmc_kernel k{};
    k.move = problem->family == OASMC_UNID ? OASMC_RWMH : OASMC_MALA;
    k.leapfrog = 1;
    const int cs = check_problem(problem, &k);
    if (cs) return cs;
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    ValuShape shape{};
    if (lpp == 0 && dpl == 0) {
        if (!valu_shape(problem->d, N, &shape))
            return fail(OASMC_EUNSUPPORTED, "no kernel shape for d=%d", problem->d);
    } else {
        bool known = false;
        for (const ValuShape& c : kShapes) known |= (c.lpp == lpp && c.dpl == dpl);
        if (!known || (int64_t)lpp * dpl < problem->d)
            return fail(OASMC_EINVAL, "shape %d x %d is not built or does not hold d=%d", lpp, dpl,
                        problem->d);
        if (problem->family == OASMC_UNID && !(lpp == 1 && dpl == 4))
            return fail(OASMC_EUNSUPPORTED, "the Unid target runs on one lane of 4 coordinates");
        shape = ValuShape{lpp, dpl};
    }
    HIP_TRY(hipSetDevice(h->device));
    EvalArgs E{};
    E.a.tg = target_dev(problem);
    E.a.move = k.move;
    E.a.leapfrog = 1;
    E.a.N = N;
    E.a.ntiles = valu_tiles(N, shape);
    E.x = x;
    E.ell = ell;
    E.grad = grad;
    HIP_TRY(launch_target_eval(E, shape, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    g_err.clear();
    return OASMC_OK;
}

int oasmc_logZ_backward(oasmc_handle* h, const oasmc_problem* problem, const oasmc_kernel* kernel,
                        int64_t N, int32_t T, const double* beta, const double* eps, uint64_t seed,
                        uint32_t round_k, uint32_t problem_id, double* logZ, double* grad,
                        void* stream)
{
    if (!h || !logZ || !grad) return fail(OASMC_EINVAL, "NULL argument");
    int s = check_problem(problem, kernel);
    if (s) return s;
    if (problem->family != OASMC_GMM || kernel->move != OASMC_MALA || kernel->resample)
        return fail(OASMC_EUNSUPPORTED, "the gradient is built for the mixture target with MALA and no resampling");
    ValuShape shape{}, ashape{};
    int kb = 0;
    if (!valu_shape(problem->d, N, &shape) || !adjoint_shape(problem->d, problem->K, N, &ashape, &kb) ||
        shape.lpp != ashape.lpp || shape.dpl != ashape.dpl)
        return fail(OASMC_EUNSUPPORTED, "the gradient supports d <= 32 and K <= 8");
    s = check_schedule(T, beta);
    if (s) return s;
    if (N < 1 || N > ((int64_t)1 << 30)) return fail(OASMC_EINVAL, "N must lie in [1, 2^30]");
    if (!eps) return fail(OASMC_EINVAL, "eps is NULL");
    for (int t = 0; t < T; ++t)
        if (!(eps[t] > 0.0) || !std::isfinite(eps[t]))
            return fail(OASMC_EINVAL, "eps[%d] must be positive and finite", t);
    HIP_TRY(hipSetDevice(h->device));
    hipStream_t st = (hipStream_t)stream;
    const int d = problem->d;
    const int every = 16;
    const int nseg = (T + every - 1) / every;
    const int np = problem->K * d + problem->K;

    SweepArgs a{};
    a.tg = target_dev(problem);
    a.move = kernel->move;
    a.leapfrog = 1;
    a.N = N;
    a.T = T;
    a.key.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key.k1 = (uint32_t)(seed >> 32);
    a.key.c2 = (round_k & 0xFFFFu) | (problem_id << 16);
    a.acc_words = (T + 31) / 32;
    a.ckpt_every = every;
    double *dbeta, *deps, *dlogg, *dacc, *dscal, *dlw, *gpart, *dgrad;
    HIP_TRY(wget(h, B_BETA, T + 1, &dbeta));
    HIP_TRY(wget(h, B_EPS, T, &deps));
    HIP_TRY(wget(h, B_LOGG, 3 * (size_t)T, &dlogg));
    HIP_TRY(wget(h, B_ACC, T, &dacc));
    HIP_TRY(wget(h, B_SCAL, 8, &dscal));
    HIP_TRY(wget(h, B_LWO, N, &dlw));
    HIP_TRY(wget(h, B_CKPT, (size_t)N * nseg * d, &a.ckpt));
    HIP_TRY(wget(h, B_ABITS, (size_t)N * a.acc_words, &a.acc_bits));
    HIP_TRY(hipMemcpyAsync(dbeta, beta, sizeof(double) * (T + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(deps, eps, sizeof(double) * T, hipMemcpyHostToDevice, st));
    a.beta = dbeta;
    a.eps = deps;
    a.lw_out = dlw;
    const int64_t ntiles = valu_tiles(N, shape);
    const int64_t S = slot_count(ntiles, kernel->slots);
    double* part;
    HIP_TRY(wget(h, B_PART, (size_t)S * (T + 1) * 4, &part));
    a.part = part;
    a.S = S;
    a.ntiles = ntiles;
    // forward: the AIS pass with checkpoints and decisions recorded
    const int grid_waves = (int)std::min<int64_t>(S, (int64_t)h->cus * 8);
    if (h->prof) HIP_TRY(hipEventRecord(h->ev0, st));
    HIP_TRY(launch_oais_valu(a, shape, grid_waves, st));
    HIP_TRY(launch_merge_slots(part, S, T, N, dlogg, dacc, dscal, st));
    // reverse
    AdjointArgs A{};
    A.a = a;
    A.lw = dlw;
    A.scal = dscal;
    HIP_TRY(wget(h, B_SEG, (size_t)N * every * d, &A.seg));
    HIP_TRY(wget(h, B_GPART, (size_t)ntiles * np, &gpart));
    HIP_TRY(wget(h, B_GRAD, np, &dgrad));
    A.partial = gpart;
    A.nwaves = ntiles;
    HIP_TRY(launch_adjoint(A, ashape, kb, st));
    HIP_TRY(launch_adjoint_reduce(gpart, ntiles, np, dgrad, st));
    if (h->prof) HIP_TRY(hipEventRecord(h->ev1, st));
    double lz = 0.0;
    HIP_TRY(hipMemcpyAsync(&lz, dscal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(grad, dgrad, sizeof(double) * np, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h->prof) {
        // forward pass, merge, reverse pass and reduction timed as one launch
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->prof_ms += ms;
        h->prof_launches += 1;
        h->prof_steps += (double)N * T;
    }
    *logZ = lz;
    if (!std::isfinite(lz)) return fail(OASMC_ENONFINITE, "log Z_hat is not finite");
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
    const bool rejuv = out->rejuv_mean && out->rejuv_second;
    if (rejuv && problem->family == OASMC_LOGREG)
        return fail(OASMC_EUNSUPPORTED, "rejuvenation is built for the Gaussian and mixture families");
    if (!kernel->resample && !rejuv &&
        (opts->budget == OASMC_BUDGET_FIXED || opts->budget == OASMC_BUDGET_DOUBLE_T)) {
        DevProblem q{};
        q.prob = *problem;
        q.kern = *kernel;
        q.N = N1;
        int T = opts->T1;
        for (int k = 0; k <= out->rounds; ++k) {
            q.Ts.push_back(T);
            if (opts->budget == OASMC_BUDGET_DOUBLE_T) T *= 2;
            if (opts->T_max > 0) T = std::min(T, opts->T_max);
            T = std::min(T, Tcap);
        }
        q.eps_adapt = opts->eps_adapt;
        q.interp = opts->interp;
        q.eps0 = opts->eps0;
        q.eps_kappa = opts->eps_kappa;
        q.accept_target = opts->accept_target;
        q.seed = seed;
        q.problem_id = problem_id;
        int st = prepare_dev_problem(h, q, (hipStream_t)stream);
        if (st) return st;
        HIP_TRY(hipSetDevice(h->device));
        std::vector<DevProblem> ps{q};
        std::vector<char> hs, ho;
        st = run_device(h, ps, out->rounds, false, hs, ho, (hipStream_t)stream);
        if (st) return st;
        const DevProblem& r = ps[0];
        size_t ob;
        const DevOut o = out_layout(r, out->rounds, &ob);
        const char* base = ho.data();
        const char* sched = ho.data() + ob;
        const double* beta_all = reinterpret_cast<const double*>(sched);
        const double* eps_all = beta_all + (size_t)(out->rounds + 1) * (r.Tcap + 1);
        int status = OASMC_OK;
        for (int k = 0; k < out->rounds; ++k) {
            const int T = r.Ts[k];
            out->logZ[k] = reinterpret_cast<const double*>(base + o.logZ)[k];
            out->N[k] = N1;
            out->T[k] = T;
            out->n_resample[k] = 0;
            std::copy(beta_all + (size_t)k * (r.Tcap + 1), beta_all + (size_t)k * (r.Tcap + 1) + T + 1,
                      out->beta + (size_t)k * (Tcap + 1));
            std::copy(eps_all + (size_t)k * r.Tcap, eps_all + (size_t)k * r.Tcap + T,
                      out->eps + (size_t)k * Tcap);
            const double* lg = reinterpret_cast<const double*>(base + o.log_g) + (size_t)k * 3 * r.Tcap;
            for (int i = 0; i < 3; ++i)  // layout [rounds][3][Tcap]
                std::copy(lg + (size_t)i * T, lg + (size_t)(i + 1) * T,
                          out->log_g + ((size_t)k * 3 + i) * Tcap);
            const double* ac = reinterpret_cast<const double*>(base + o.acc) + (size_t)k * r.Tcap;
            std::copy(ac, ac + T, out->accept + (size_t)k * Tcap);
            const double* la = reinterpret_cast<const double*>(base + o.Lambda) + (size_t)k * (r.Tcap + 1);
            std::copy(la, la + T + 1, out->Lambda_hat + (size_t)k * (Tcap + 1));
            if (reinterpret_cast<const int*>(base + o.status)[k] && status == OASMC_OK)
                status = fail(OASMC_ENONFINITE, "non-finite moments in round %d", k + 1);
            if (!std::isfinite(out->logZ[k]) && status == OASMC_OK)
                status = fail(OASMC_ENONFINITE, "log Z_hat is not finite in round %d", k + 1);
            out->rounds_done = k + 1;
            if (status != OASMC_OK) break;
        }
        if (status == OASMC_OK) g_err.clear();
        return status;
    }
    int64_t N = N1;
    int T = opts->T1;
    std::vector<double> beta(T + 1), eps(T);
    uniform_schedule(T, beta.data());
    // DAR: round k >= 2 resamples at the times predicted from round k - 1;
    // round 1 at none before T
    const bool dar = opts->dar && kernel->resample;
    oasmc_kernel kdar = *kernel;
    std::vector<int32_t> flags(T, 0);
    if (dar) {
        kdar.trigger = 3;
        kdar.resample_at = flags.data();
    }
    for (int t = 1; t <= T; ++t)
        eps[t - 1] = opts->eps_adapt ? opts->eps0 / std::sqrt(1.0 + beta[t] * opts->eps_kappa)
                                     : opts->eps0;
    int status = OASMC_OK;
    for (int k = 1; k <= out->rounds; ++k) {
        std::vector<double> lg(3 * (size_t)T), acc(T);
        oasmc_round_out ro{};
        ro.log_g = lg.data();
        ro.accept = acc.data();
        if (rejuv) {
            HIP_TRY(wget(h, B_RJ_LW, N, &ro.lw));
            HIP_TRY(wget(h, B_RJ_X, (size_t)N * problem->d, &ro.x));
        }
        status = oasmc_asmc(h, problem, dar ? &kdar : kernel, N, T, beta.data(), eps.data(), seed,
                            (uint32_t)k, problem_id, &ro, stream);
        if (status != OASMC_OK && status != OASMC_ENONFINITE) break;
        const int r = k - 1;
        if (rejuv) {
            const int s4 = oasmc_rejuvenate(h, problem, kernel, N, T, eps[T - 1], seed, (uint32_t)k,
                                            problem_id, ro.lw, ro.x,
                                            out->rejuv_mean + (size_t)r * problem->d,
                                            out->rejuv_second + (size_t)r * problem->d, nullptr,
                                            nullptr, stream);
            if (status == OASMC_OK && s4 != OASMC_OK) status = s4;
        }
        out->logZ[r] = ro.logZ;
        out->N[r] = N;
        out->T[r] = T;
        out->n_resample[r] = ro.n_resample;
        std::copy(beta.begin(), beta.end(), out->beta + (size_t)r * (Tcap + 1));
        for (int i = 0; i < 3; ++i)  // layout [rounds][3][Tcap]
            std::copy(lg.begin() + (size_t)i * T, lg.begin() + (size_t)(i + 1) * T,
                      out->log_g + ((size_t)r * 3 + i) * Tcap);
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
        if (dar) {
            std::vector<int32_t> fn(Tn, 0);
            const int s3 = dar_times_impl(T, beta.data(), lg.data(), Tn, bn.data(), opts->interp,
                                          kernel->nu, fn.data(), nullptr);
            if (status == OASMC_OK && s3 != OASMC_OK) status = s3;
            flags.swap(fn);
            kdar.resample_at = flags.data();
        }
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

extern "C" int oasmc_run_batch(oasmc_handle* h, const oasmc_batch_problem* probs, int32_t P,
                               int32_t rounds, int32_t use_graph, oasmc_batch_out* out,
                               void* stream)
{
    if (!h || !probs || !out || !out->logZ) return fail(OASMC_EINVAL, "NULL argument");
    if (P < 1) return fail(OASMC_EINVAL, "need at least one problem");
    if (rounds < 1) return fail(OASMC_EINVAL, "rounds must be >= 1");
    HIP_TRY(hipSetDevice(h->device));
    std::vector<DevProblem> ps(P);
    for (int p = 0; p < P; ++p) {
        const oasmc_batch_problem& b = probs[p];
        DevProblem& q = ps[p];
        q.prob = b.problem;
        q.kern = b.kernel;
        q.N = b.N;
        if (b.T < 1) return fail(OASMC_EINVAL, "problem %d: T must be >= 1", p);
        int T = std::max(1, b.T >> (rounds - 1));
        for (int k = 0; k <= rounds; ++k) {
            q.Ts.push_back(T);
            T = std::min(2 * T, b.T);
        }
        q.eps_adapt = b.eps_adapt;
        q.interp = 0;
        q.eps0 = b.eps0;
        q.eps_kappa = b.eps_kappa;
        q.accept_target = b.accept_target;
        q.seed = b.seed;
        q.problem_id = b.problem_id;
        const int st = prepare_dev_problem(h, q, (hipStream_t)stream);
        if (st) {
            std::string m = g_err;
            return fail(st, "problem %d: %s", p, m.c_str());
        }
    }
    std::vector<char> hs, ho;
    const int st = run_device(h, ps, rounds, use_graph != 0, hs, ho, (hipStream_t)stream);
    if (st) return st;
    int status = OASMC_OK;
    for (int p = 0; p < P; ++p) {
        const DevProblem& q = ps[p];
        size_t ob;
        const DevOut o = out_layout(q, rounds, &ob);
        const char* base = ho.data() + (q.off_out - ps[0].off_out);
        for (int k = 0; k < rounds; ++k) {
            out->logZ[(size_t)p * rounds + k] = reinterpret_cast<const double*>(base + o.logZ)[k];
            if (out->Lambda_T)
                out->Lambda_T[(size_t)p * rounds + k] =
                    reinterpret_cast<const double*>(base + o.Lambda)[(size_t)k * (q.Tcap + 1) + q.Ts[k]];
            const int bad = reinterpret_cast<const int*>(base + o.status)[k];
            if (out->status) out->status[(size_t)p * rounds + k] = bad;
            if (bad && status == OASMC_OK)
                status = fail(OASMC_ENONFINITE, "problem %d round %d: non-finite moments", p, k + 1);
        }
    }
    if (status == OASMC_OK) g_err.clear();
    return status;
}
