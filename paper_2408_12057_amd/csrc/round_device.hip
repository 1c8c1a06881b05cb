// round_device.hip -- the between-rounds work of Alg. 2 on the device, one
// workgroup per problem, so that a whole multi-round run (and a batch of
// problems) can be enqueued without host round trips and captured in a
// hipGraph:
//   * merge of the slot partials (the moments of eq. (CESS), acceptance and
//     log Z_hat) in a fixed order that does not depend on the grid;
//   * Alg. 3 (OptimiseSchedule): D_hat_t, Lambda_hat_t = sum sqrt(D_hat_s),
//     monotone cubic (Fritsch-Carlson) inverse of the knots (Lambda_hat_t,
//     beta_t) evaluated at Lambda_hat_T t'/T';
//   * the step-size update between rounds (log eps moved by acceptance minus
//     target, piecewise linear in beta) and the next T from the Budget rule.
// The arithmetic follows the host implementation of oasmc_adapt_schedule
// statement by statement; sequential parts (prefix sums, knot selection,
// monotone fix-ups) run on one lane so their order is fixed.
#include "kernels.hpp"

namespace oasmc {

// Merge the slot partials of one problem (blockIdx.x selects the problem,
// blockIdx.y + k gridDim.y the entry; one wave per entry, a maximum and then
// a sum of exp(x - max) over the slots in a fixed order).
__global__ void __launch_bounds__(kWave) k_round_merge(const RoundDev* __restrict__ rd)
{
    const RoundDev& R = rd[blockIdx.x];
    const int T = R.T;
    const int lane = threadIdx.x;
    for (int e = blockIdx.y; e <= T; e += gridDim.y) {
        double m[3] = {-INFINITY, -INFINITY, -INFINITY};
        double c = 0.0;
        for (int64_t s = lane; s < R.S; s += kWave) {
            const double* p = R.part + ((size_t)s * (T + 1) + e) * 4;
#pragma unroll
            for (int i = 0; i < 3; ++i) m[i] = fmax(m[i], p[i]);
            c += p[3];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) m[i] = wave_max(m[i]);
        double sum[3] = {0.0, 0.0, 0.0};
        for (int64_t s = lane; s < R.S; s += kWave) {
            const double* p = R.part + ((size_t)s * (T + 1) + e) * 4;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (m[i] > -INFINITY && p[i] > -INFINITY) sum[i] += exp(p[i] - m[i]);
        }
        double L[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) L[i] = lse_value(m[i], wave_sum(sum[i]));
        const double cnt = wave_sum(c);
        if (lane == 0) {
            if (e < T) {
#pragma unroll
                for (int i = 0; i < 3; ++i) R.log_g[(size_t)i * T + e] = L[i];
                R.acc[e] = cnt / (double)R.N;
            } else {
                R.logZ[0] = L[0] - log((double)R.N);
            }
        }
    }
}

// Alg. 3 + step sizes + Budget for one problem per workgroup.  Reads
// beta[T+1], eps[T], log_g[3T], acc[T]; writes beta_next[Tn+1],
// eps_next[Tn] and Lambda[T+1].
__global__ void __launch_bounds__(256) k_round_schedule(const RoundDev* __restrict__ rd)
{
    const RoundDev& R = rd[blockIdx.x];
    const int T = R.T;
    const int Tn = R.Tn;  // the Budget rule fixes it in advance (no data dependence)
    __shared__ int s_m, s_finite;
    __shared__ double s_lamT;
    double* kx = R.scratch;            // knots, abscissa  [T+1]
    double* ky = kx + (T + 1);         // knots, ordinate  [T+1]
    double* ks = ky + (T + 1);         // knot slopes      [T+1]
    if (threadIdx.x == 0) {
        // Lambda_hat and the knots, in order
        double lam = 0.0;
        R.Lambda[0] = 0.0;
        int finite = 1;
        for (int t = 1; t <= T; ++t) {
            const double D = R.log_g[2 * T + t - 1] - 2.0 * R.log_g[T + t - 1] + R.log_g[t - 1];
            if (!isfinite(D)) finite = 0;
            lam = lam + (D > 0.0 ? sqrt(D) : 0.0);
            R.Lambda[t] = lam;
        }
        int m = 0;
        for (int t = 0; t <= T; ++t) {
            const double L = R.Lambda[t];
            if (m > 0 && !(L > kx[m - 1])) {
                if (t == T) {
                    kx[m - 1] = L;
                    ky[m - 1] = R.beta[t];
                }
                continue;
            }
            kx[m] = L;
            ky[m] = R.beta[t];
            ++m;
        }
        s_m = m;
        s_finite = finite;
        s_lamT = R.Lambda[T];
    }
    __syncthreads();
    const int m = s_m;
    const double lamT = s_lamT;
    const bool degenerate = !s_finite || !(lamT > 0.0);
    if (!degenerate && R.interp == 0) {
        // Fritsch-Carlson slopes
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            double v = 0.0;
            if (m == 2) {
                v = (ky[1] - ky[0]) / (kx[1] - kx[0]);
            } else if (i > 0 && i < m - 1) {
                const double h0 = kx[i] - kx[i - 1], h1 = kx[i + 1] - kx[i];
                const double a = (ky[i] - ky[i - 1]) / h0, b = (ky[i + 1] - ky[i]) / h1;
                if (a * b > 0.0) {
                    const double w1 = 2.0 * h1 + h0, w2 = h1 + 2.0 * h0;
                    v = (w1 + w2) / (w1 / a + w2 / b);
                }
            } else {
                const int e0 = (i == 0) ? 0 : m - 2;   // interval at the end
                const int e1 = (i == 0) ? 1 : m - 3;   // its neighbour
                const double h0 = kx[e0 + 1] - kx[e0], h1 = kx[e1 + 1] - kx[e1];
                const double s0 = (ky[e0 + 1] - ky[e0]) / h0, s1 = (ky[e1 + 1] - ky[e1]) / h1;
                v = ((2.0 * h0 + h1) * s0 - h0 * s1) / (h0 + h1);
                if (v * s0 <= 0.0) v = 0.0;
                else if (s0 * s1 < 0.0 && fabs(v) > 3.0 * fabs(s0)) v = 3.0 * s0;
            }
            ks[i] = v;
        }
    }
    __syncthreads();
    for (int tp = threadIdx.x; tp <= Tn; tp += blockDim.x) {
        double b;
        if (degenerate) {
            b = (double)tp / (double)Tn;
        } else {
            const double u = lamT * (double)tp / (double)Tn;
            if (u <= kx[0]) {
                b = ky[0];
            } else if (u >= kx[m - 1]) {
                b = ky[m - 1];
            } else {
                int lo = 0, hi = m - 1;  // last knot with kx <= u
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (kx[mid] <= u) lo = mid; else hi = mid;
                }
                const double h = kx[lo + 1] - kx[lo];
                const double s = (u - kx[lo]) / h;
                if (R.interp == 0) {
                    const double s2 = s * s, s3 = s2 * s;
                    b = (2 * s3 - 3 * s2 + 1) * ky[lo] + (s3 - 2 * s2 + s) * h * ks[lo] +
                        (3 * s2 - 2 * s3) * ky[lo + 1] + (s3 - s2) * h * ks[lo + 1];
                } else {
                    b = ky[lo] + s * (ky[lo + 1] - ky[lo]);
                }
            }
        }
        R.beta_next[tp] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* bn = R.beta_next;
        bn[0] = 0.0;
        bn[Tn] = 1.0;
        for (int tp = 1; tp < Tn; ++tp)
            if (!(bn[tp] > bn[tp - 1])) bn[tp] = nextafter(bn[tp - 1], 2.0);
        for (int tp = Tn - 1; tp >= 1; --tp)
            if (!(bn[tp] < bn[tp + 1])) bn[tp] = nextafter(bn[tp + 1], -1.0);
        if (R.status) *R.status = (degenerate && !s_finite) ? 1 : 0;
    }
    __syncthreads();
    // step sizes for the next round
    for (int t = threadIdx.x + 1; t <= Tn; t += blockDim.x) {
        double e;
        if (!R.eps_adapt) {
            e = R.eps0;
        } else {
            const double q = R.beta_next[t];
            // knots (beta_t, log eps_t + acc_t - target), t = 1..T, constant beyond
            double y;
            if (q <= R.beta[1]) {
                y = log(R.eps[0]) + (R.acc[0] - R.accept_target);
            } else if (q >= R.beta[T]) {
                y = log(R.eps[T - 1]) + (R.acc[T - 1] - R.accept_target);
            } else {
                int lo = 1, hi = T;  // last knot with beta <= q
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (R.beta[mid] <= q) lo = mid; else hi = mid;
                }
                const double y0 = log(R.eps[lo - 1]) + (R.acc[lo - 1] - R.accept_target);
                const double y1 = log(R.eps[lo]) + (R.acc[lo] - R.accept_target);
                const double w = (q - R.beta[lo]) / (R.beta[lo + 1] - R.beta[lo]);
                y = y0 + w * (y1 - y0);
            }
            e = exp(y);
        }
        R.eps_next[t - 1] = e;
    }
}

hipError_t launch_round_merge(const RoundDev* rd, int nprob, int Tmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_round_merge, dim3(nprob, std::min(Tmax + 1, 65535)), dim3(kWave), 0, st,
                       rd);
    return hipGetLastError();
}

hipError_t launch_round_schedule(const RoundDev* rd, int nprob, hipStream_t st)
{
    hipLaunchKernelGGL(k_round_schedule, dim3(nprob), dim3(256), 0, st, rd);
    return hipGetLastError();
}

}  // namespace oasmc
