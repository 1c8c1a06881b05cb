// adjoint.hpp -- reverse pass of the pathwise gradient of log Z_hat for the
// equal-weight Gaussian-mixture target with MALA moves and the accept
// decisions of the forward pass held fixed.
//
// theta = (means m_k, log-scales s_k).  With a_k = (m_k - x)/v_k,
// v_k = exp(2 s_k), r = softmax_k(-|x - m_k|^2 / (2 v_k)), g = sum_k r_k a_k,
// q_k = |x - m_k|^2 / v_k (all at the pre-move state x_{t-1}):
//   log w_T = sum_t Delta beta_t ell(x_{t-1}),  grad_x ell = g + (x - m_eta)/s^2
//   x_t = x_{t-1} + h (-(x_{t-1} - m_eta)/s^2 + beta_t grad_x ell) + eps xi  if accepted
// so, with xbar the adjoint of x_t (xbar_T = 0):
//   thetabar += Delta beta_t d ell/d theta      (-r_k a_k ; r_k q_k)
//   accepted:  thetabar += h beta_t M^T xbar     (M = d grad_x ell / d theta)
//              xbar <- xbar + h (-xbar/s^2 + beta_t H xbar)
//   xbar += Delta beta_t grad_x ell
// with H xbar = sum_k r_k (a_k (a_k . xbar) - xbar/v_k) - g (g . xbar) + xbar/s^2,
//   (M^T xbar)_{m_k} = r_k (xbar/v_k - ((a_k - g) . xbar) a_k),
//   (M^T xbar)_{s_k} = r_k q_k ((a_k - g) . xbar) - 2 r_k (a_k . xbar).
// Each 16-step segment is recomputed from its checkpoint with the same
// Philox counters and the stored decisions, written to a per-particle
// scratch buffer, and walked backwards.  grad log Z_hat = sum_n W_n thetabar_n,
// W = softmax(log w_T), summed per wave in a fixed butterfly order.
#pragma once
#include "valu_sweep.hpp"

namespace oasmc {

// Waves per SIMD requested from the compiler: two for lanes of at most 8
// coordinates and blocks of at most 4 components (a few registers spill, the
// second wave hides the binary64 latencies), its own choice for wider shapes
// (which would spill heavily).
template <int DPL, int KB>
struct AdjMinWaves {
    static constexpr int value = (DPL <= 8 && KB <= 4) ? 2 : 1;
};

template <int LPP, int DPL, int KB>
__global__ void __launch_bounds__(256, (AdjMinWaves<DPL, KB>::value)) k_adjoint_gmm(AdjointArgs A)
{
    constexpr int P = kWave / LPP;
    using PT = Particle<kGmm, LPP, DPL>;
    const SweepArgs& a = A.a;
    extern __shared__ __align__(16) char sh_dyn[];
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP, pl = lane / LPP;
    const int64_t wave =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wave >= a.ntiles) return;  // the whole wave leaves together
    const int64_t n64 = wave * P + pl;
    const bool valid = n64 < a.N;
    const int64_t nl = valid ? n64 : a.N - 1;
    const int d = a.tg.d, K = a.tg.K, T = a.T;
    const int every = a.ckpt_every;
    const int nseg = (T + every - 1) / every;
    const int i0 = r * DPL;
    const double Lse = A.scal[0] + log((double)a.N);
    const double W = valid ? exp(A.lw[nl] - Lse) : 0.0;

    double xb[DPL], tm[KB][DPL], ts[KB];
#pragma unroll
    for (int j = 0; j < DPL; ++j) xb[j] = 0.0;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        ts[k] = 0.0;
#pragma unroll
        for (int j = 0; j < DPL; ++j) tm[k][j] = 0.0;
    }
    float* segp = A.seg + (size_t)nl * every * d;
    const uint32_t* bits = a.acc_bits + (size_t)nl * a.acc_words;

    for (int s = nseg - 1; s >= 0; --s) {
        const int t0 = s * every;
        const int Ls = min(every, T - t0);
        // recompute the segment from its checkpoint
        {
            float x[DPL];
            double g[DPL];
            const float* cp = a.ckpt + ((size_t)nl * nseg + s) * d;
#pragma unroll
            for (int j = 0; j < DPL; ++j) x[j] = (i0 + j < d) ? cp[i0 + j] : 0.f;
            double ell = Particle<kGmm, LPP, DPL>::template eval<true>(a.tg, c, pv, r, x, g);
            for (int u = 0; u < Ls; ++u) {
#pragma unroll
                for (int j = 0; j < DPL; ++j)
                    if (i0 + j < d) segp[u * d + i0 + j] = x[j];
                const int t = t0 + u + 1;
                const int bit = (bits[(t - 1) / 32] >> ((t - 1) & 31)) & 1;
                Particle<kGmm, LPP, DPL>::template move<kMala>(
                    a.tg, c, pv, a.key, (uint32_t)nl, (uint32_t)t, r, 1, a.beta[t], a.eps[t - 1], x,
                    ell, g, bit);
            }
        }
        // walk it backwards
        for (int u = Ls - 1; u >= 0; --u) {
            const int t = t0 + u + 1;
            const int bit = (bits[(t - 1) / 32] >> ((t - 1) & 31)) & 1;
            const double db = a.beta[t] - a.beta[t - 1];
            const double bt = a.beta[t];
            const double h = 0.5 * a.eps[t - 1] * a.eps[t - 1];
            // the means in the zero-padded lane layout (re-read each step): the
            // coordinates of a lane beyond d stay exact zeros, no branch needed
            const ParView pq = PT::fresh(pv);
            double xv[DPL];
#pragma unroll
            for (int j = 0; j < DPL; ++j) xv[j] = (i0 + j < d) ? (double)segp[u * d + i0 + j] : 0.0;
            double e[KB], rk[KB], qk[KB];
            double mx = -INFINITY;
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                e[k] = -INFINITY;
                qk[k] = 0.0;
                if (k < K) {
                    double sq = 0.0;
#pragma unroll
                    for (int j = 0; j < DPL; ++j) {
                        const double df = xv[j] - PT::mean(pq, k, r, j);
                        sq = fma(df, df, sq);
                    }
                    sq = group_sum<LPP>(sq);
                    qk[k] = sq * pv.iv[k];
                    e[k] = -sq * pv.hiv[k];
                    mx = fmax(mx, e[k]);
                }
            }
            double z = 0.0;
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                rk[k] = (k < K) ? exp(e[k] - mx) : 0.0;
                z += rk[k];
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) rk[k] /= z;
            double gv[DPL];
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                gv[j] = 0.0;
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k < K) gv[j] += rk[k] * (PT::mean(pq, k, r, j) - xv[j]) * pv.iv[k];
            }
            // weight term: d ell / d theta
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                if (k < K) {
#pragma unroll
                    for (int j = 0; j < DPL; ++j)
                        tm[k][j] -= db * rk[k] * (PT::mean(pq, k, r, j) - xv[j]) * pv.iv[k];
                    ts[k] += db * rk[k] * qk[k];
                }
            }
            if (bit) {
                double ua[KB];
                double ug = 0.0;
#pragma unroll
                for (int j = 0; j < DPL; ++j) ug += gv[j] * xb[j];
                ug = group_sum<LPP>(ug);
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    ua[k] = 0.0;
                    if (k < K) {
                        double sdot = 0.0;
#pragma unroll
                        for (int j = 0; j < DPL; ++j)
                            sdot += (PT::mean(pq, k, r, j) - xv[j]) * pv.iv[k] * xb[j];
                        ua[k] = group_sum<LPP>(sdot);
                    }
                }
                const double hb = h * bt;
                double nx[DPL];
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    double Hu = -gv[j] * ug + xb[j] * c.inv_s2r;
#pragma unroll
                    for (int k = 0; k < KB; ++k)
                        if (k < K) {
                            const double akj = (PT::mean(pq, k, r, j) - xv[j]) * pv.iv[k];
                            Hu += rk[k] * (akj * ua[k] - xb[j] * pv.iv[k]);
                            tm[k][j] += hb * rk[k] * (xb[j] * pv.iv[k] - (ua[k] - ug) * akj);
                        }
                    nx[j] = xb[j] + h * (-xb[j] * c.inv_s2r + bt * Hu);
                }
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (k < K) ts[k] += hb * (rk[k] * qk[k] * (ua[k] - ug) - 2.0 * rk[k] * ua[k]);
#pragma unroll
                for (int j = 0; j < DPL; ++j) xb[j] = nx[j];
            }
#pragma unroll
            for (int j = 0; j < DPL; ++j)
                xb[j] += db * (gv[j] + (xv[j] - PT::ref(pq, r, j)) * c.inv_s2r);
        }
    }
    // weighted sums over the tile's particles (butterfly over particle slots)
    const int np = K * d + K;
    double* part = A.partial + (size_t)wave * np;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            double v = W * tm[k][j];
#pragma unroll
            for (int o = LPP; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
            if (pl == 0 && k < K && i0 + j < d) part[k * d + i0 + j] = v;
        }
        double v = W * ts[k];
#pragma unroll
        for (int o = LPP; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
        if (lane == 0 && k < K) part[K * d + k] = v;
    }
}

template <int LPP, int DPL, int KB>
hipError_t launch_adjoint_t(const AdjointArgs& A, hipStream_t st)
{
    const int64_t blocks = (A.a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((k_adjoint_gmm<LPP, DPL, KB>), dim3((unsigned)blocks), dim3(256),
                       params_bytes_lanes(A.a.tg, LPP, DPL), st, A);
    return hipGetLastError();
}

}  // namespace oasmc
