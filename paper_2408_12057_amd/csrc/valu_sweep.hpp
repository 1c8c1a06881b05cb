// valu_sweep.hpp -- annealing sweeps for the closed-form targets (isotropic
// Gaussian, equal-weight Gaussian mixture) with RWMH, MALA and HMC moves.
//
// These paths are bound by plain VALU arithmetic (Philox rounds, binary64
// Box-Muller, distance and gradient sums), so the design keeps each particle in
// registers: a particle occupies LPP adjacent lanes, each holding DPL of its
// coordinates (fp32 state, binary64 arithmetic).  Per-particle scalars (ell,
// log w, log alpha) are reduced over the LPP lanes with a butterfly so every
// lane of the group holds the same bits and takes the same MH decision.
//
// Two drivers share the particle code:
//  * k_oais_valu -- the AIS case with the particle loop outside the time loop
//    (Sec. "Optimised AIS"): a wave owns a tile of 64/LPP particles for all T
//    steps; the moments g_hat_{t,i} (eq. CESS) are streamed into a fixed number
//    of slots S of O(T) memory each, independent of N and of the grid shape.
//  * k_asmc_step / k_asmc_merge / resampler -- the adaptive-resampling case
//    (Alg. 1 with AR): one launch per step t, state in HBM, a two-level merge
//    in one launch that evaluates the trigger on the device, and the
//    integer-CDF systematic resampler (launched every step, does nothing
//    unless the trigger fired).
#pragma once
#include "kernels.hpp"

namespace oasmc {



__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Precomputed reference/target scalars.
struct Consts {
    double half_inv_s2r;  // 1 / (2 ref_sigma2)
    double inv_s2r;       // 1 / ref_sigma2
    double cst_eta;       // (d/2) log(2 pi ref_sigma2)
    double sref;          // sqrt(ref_sigma2)
    double half_inv_s2;   // Gaussian target: 1/(2 sigma2)
    double inv_s2;        // Gaussian target: 1/sigma2
    double logK;
};

__device__ __forceinline__ Consts make_consts(const TargetDev& tg)
{
    Consts c;
    c.inv_s2r = 1.0 / tg.ref_sigma2;
    c.half_inv_s2r = 0.5 / tg.ref_sigma2;
    c.cst_eta = 0.5 * tg.d * (1.8378770664093454835606594728112 + log(tg.ref_sigma2));
    c.sref = sqrt(tg.ref_sigma2);
    c.half_inv_s2 = 0.5 / tg.sigma2;
    c.inv_s2 = 1.0 / tg.sigma2;
    c.logK = log((double)(tg.K > 0 ? tg.K : 1));
    return c;
}

// Target parameters staged in LDS: reference mean [d], then the Gaussian mean
// [d] or the mixture means [K*d], then the mixture 1/(2 v_k), 1/v_k (the view
// type ParView is declared in kernels.hpp).

__device__ __forceinline__ ParView stage_params(const TargetDev& tg, char* sh)
{
    const int d = tg.d;
    const int nmu = (tg.family == kGmm) ? tg.K * d : d;
    double* hv = reinterpret_cast<double*>(sh);
    double* iv = hv + kMaxK;
    float* m = reinterpret_cast<float*>(iv + kMaxK);
    float* mu = m + d;
    for (int i = threadIdx.x; i < d; i += blockDim.x) m[i] = tg.ref_mean ? tg.ref_mean[i] : 0.f;
    const float* src = (tg.family == kGmm) ? tg.means : tg.mu;
    if (src)
        for (int i = threadIdx.x; i < nmu; i += blockDim.x) mu[i] = src[i];
    // 1/(2 v_k), 1/v_k; zero beyond K (padded components of a block)
    for (int k = threadIdx.x; k < kMaxK; k += blockDim.x) {
        const bool on = tg.family == kGmm && k < tg.K;
        const double v = on ? exp(2.0 * (double)tg.log_scales[k]) : 1.0;
        hv[k] = on ? 0.5 / v : 0.0;
        iv[k] = on ? 1.0 / v : 0.0;
    }
    __syncthreads();
    return ParView{m, mu, hv, iv};
}

inline size_t params_bytes(const TargetDev& tg)
{
    const int nmu = (tg.family == kGmm) ? tg.K * tg.d : tg.d;
    return 2 * kMaxK * sizeof(double) + (size_t)(tg.d + nmu) * sizeof(float);
}


// The same staging followed by the binary64 lane-layout means lm, lmu of the
// shape (LPP, DPL).
template <int LPP, int DPL>
__device__ __forceinline__ ParView stage_params_lanes(const TargetDev& tg, char* sh)
{
    const ParView base = stage_params(tg, sh);
    double* lane = reinterpret_cast<double*>(sh + lane_params_offset(tg));
    const int nl = (int)lane_param_doubles(tg, LPP, DPL);
    for (int e = threadIdx.x; e < nl; e += blockDim.x) lane[e] = lane_param(tg, LPP, DPL, e);
    __syncthreads();
    return ParView{base.m, base.mu, base.hiv, base.iv, lane, lane + LPP * DPL};
}


// ---------------------------------------------------------------------------
// Particle arithmetic for one lane group.
// ---------------------------------------------------------------------------
// Coordinates of a lane beyond d (the tail of the last lanes' slices) hold
// exact zeros in x, z, the momentum and the gradient, and the lane-layout
// means are zero there too, so every coordinate loop runs without a branch:
// a padded coordinate adds +0 to each sum and stays +0 through every move.
template <int FAM, int LPP, int DPL>
struct Particle {
    // reference mean and target mean k at this lane's coordinate j
    static __device__ __forceinline__ double ref(const ParView& pv, int r, int j)
    {
        return pv.lm[j * LPP + r];
    }
    static __device__ __forceinline__ double mean(const ParView& pv, int k, int r, int j)
    {
        return pv.lmu[(k * DPL + j) * LPP + r];
    }
    // The view with an offset the compiler cannot see through (always zero):
    // the means are then re-read from LDS at each evaluation instead of being
    // hoisted out of the time and leapfrog loops into registers, which for
    // K d / LPP beyond a few dozen would spill.
    static __device__ __forceinline__ ParView fresh(const ParView& pv)
    {
        int z0;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z0));
        ParView v = pv;
        v.lm = pv.lm + z0;
        v.lmu = pv.lmu + z0;
        return v;
    }

    // Inside the support (0, box)^2 of the uniform reference (kUnid).
    static __device__ __forceinline__ bool unid_inside(const TargetDev& tg, const float (&x)[DPL])
    {
        return x[0] > 0.f && (double)x[0] < tg.box && x[1] > 0.f && (double)x[1] < tg.box;
    }

    // ell(x) = log gamma(x) - log eta(x); with GRAD also its gradient on this
    // lane's coordinates.  r = lane index inside the group.
    template <bool GRAD>
    static __device__ __forceinline__ double eval(const TargetDev& tg, const Consts& c,
                                                  const ParView& pv0, int r, const float (&x)[DPL],
                                                  double (&g)[DPL])
    {
        const ParView pv = fresh(pv0);
        if constexpr (FAM == kUnid) {
            // d = 2 on one lane: the log-likelihood ratio of Binomial(k | n, x y)
            // against its maximum, log1p forms near the ridge x y = k / n
            (void)r;
            (void)c;
            const double x0 = (double)x[0], x1 = (double)x[1];
            const double u = x0 * x1;
            if (GRAD) {
#pragma unroll
                for (int j = 0; j < DPL; ++j) g[j] = 0.0;
            }
            if (!unid_inside(tg, x) || !(u > 0.0 && u < 1.0)) return -INFINITY;
            const double n = tg.binom_n, k = tg.binom_k, p = k / n;
            return k * log1p((u - p) / p) + (n - k) * log1p(-(u - p) / (1.0 - p));
        } else if constexpr (FAM == kGauss) {
            double ssg = 0.0, sse = 0.0;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const double xv = (double)x[j];
                const double a = xv - mean(pv, 0, r, j);
                const double b = xv - ref(pv, r, j);
                ssg = fma(a, a, ssg);
                sse = fma(b, b, sse);
                if (GRAD) g[j] = -a * c.inv_s2 + b * c.inv_s2r;
            }
            const double part = -ssg * c.half_inv_s2 + sse * c.half_inv_s2r;
            return group_sum<LPP>(part) + c.cst_eta;
        } else {
            // equal-weight mixture of unnormalised isotropic components, streamed
            // over k with a running maximum (log-sum-exp and responsibilities)
            double sse = 0.0;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const double b = (double)x[j] - ref(pv, r, j);
                sse = fma(b, b, sse);
                if (GRAD) g[j] = 0.0;
            }
            sse = group_sum<LPP>(sse);
            if constexpr (LPP > 1) {
                return mixture_multilane<GRAD>(tg, c, pv, r, x, g, sse);
            }
            double mx = -INFINITY, s = 0.0;
#pragma unroll 1
            for (int k = 0; k < tg.K; ++k) {
                double sq = 0.0;
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const double a = (double)x[j] - mean(pv, k, r, j);
                    sq = fma(a, a, sq);
                }
                const double ek = -group_sum<LPP>(sq) * pv.hiv[k];
                double wk;
                if (ek > mx) {
                    const double sc = exp(mx - ek);  // 0 on the first component
                    s *= sc;
                    if (GRAD) {
#pragma unroll
                        for (int j = 0; j < DPL; ++j) g[j] *= sc;
                    }
                    mx = ek;
                    wk = 1.0;
                } else {
                    wk = exp(ek - mx);
                }
                s += wk;
                if (GRAD) {
                    const double f = wk * pv.iv[k];
#pragma unroll
                    for (int j = 0; j < DPL; ++j)
                        g[j] = fma(f, mean(pv, k, r, j) - (double)x[j], g[j]);
                }
            }
            const double lse = mx + log(s) - c.logK;
            if (GRAD) {
                const double inv_s = 1.0 / s;
#pragma unroll
                for (int j = 0; j < DPL; ++j)
                    g[j] = g[j] * inv_s + ((double)x[j] - ref(pv, r, j)) * c.inv_s2r;
            }
            return lse + sse * c.half_inv_s2r + c.cst_eta;
        }
    }

    // The mixture term for a particle spread over LPP > 1 lanes, in two
    // passes: the exponents e_k = -|x - m_k|^2 / (2 v_k) (summed over the
    // lanes, so every lane holds them all), their maximum M, then one
    // exponential per component, computed by the lane k mod LPP only, and
    // log sum_k exp(e_k - M); the gradient gathers the weights from their
    // lanes.  (Streaming over k on every lane would repeat each exponential
    // LPP times.)
    template <bool GRAD>
    static __device__ __forceinline__ double mixture_multilane(const TargetDev& tg, const Consts& c,
                                                               const ParView& pv, int r,
                                                               const float (&x)[DPL],
                                                               double (&g)[DPL], double sse)
    {
        constexpr int KO = (kMaxK + LPP - 1) / LPP;  // components owned by a lane
        const int K = tg.K;
        double eo[KO];
#pragma unroll
        for (int q = 0; q < KO; ++q) eo[q] = -INFINITY;
        // exponents in blocks of kKBlock components without a branch inside a
        // block, so the independent distance chains and reductions of a block
        // interleave; the lane layout and 1/(2 v_k) are zero-padded to whole
        // blocks and a padded component gets e_k = -inf (weight 0)
        double M = -INFINITY;
#pragma unroll
        for (int k0 = 0; k0 < kMaxK; k0 += kKBlock) {
            if (k0 < K) {
                double sq[kKBlock];
#pragma unroll
                for (int u = 0; u < kKBlock; ++u) {
                    sq[u] = 0.0;
#pragma unroll
                    for (int j = 0; j < DPL; ++j) {
                        const double a = (double)x[j] - mean(pv, k0 + u, r, j);
                        sq[u] = fma(a, a, sq[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kKBlock; ++u) {
                    const int k = k0 + u;
                    double ek = -group_sum<LPP>(sq[u]) * pv.hiv[k];
                    if (k >= K) ek = -INFINITY;
                    M = fmax(M, ek);
                    if ((k % LPP) == r) eo[k / LPP] = ek;
                }
            }
        }
        double wo[KO];
        double so = 0.0;
#pragma unroll
        for (int q = 0; q < KO; ++q) {
            wo[q] = (q * LPP + r < K) ? exp(eo[q] - M) : 0.0;
            so += wo[q];
        }
        const double s = group_sum<LPP>(so);
        const double lse = M + log(s) - c.logK;
        if (GRAD) {
            const int base = (int)(threadIdx.x & (kWave - 1)) & ~(LPP - 1);
#pragma unroll
            for (int k = 0; k < kMaxK; ++k) {
                if (k < K) {
                    const double f = __shfl(wo[k / LPP], base + k % LPP, kWave) * pv.iv[k];
#pragma unroll
                    for (int j = 0; j < DPL; ++j)
                        g[j] = fma(f, mean(pv, k, r, j) - (double)x[j], g[j]);
                }
            }
            const double inv_s = 1.0 / s;
#pragma unroll
            for (int j = 0; j < DPL; ++j)
                g[j] = g[j] * inv_s + ((double)x[j] - ref(pv, r, j)) * c.inv_s2r;
        }
        return lse + sse * c.half_inv_s2r + c.cst_eta;
    }

    // Normals of this lane's coordinates 4 bb .. 4 bb + 3 (zero beyond d) of
    // one (particle, step, stream) sequence: block r DPL / 4 + bb of it.  With
    // one lane per particle the block index is the same in every lane, so the
    // second Box-Muller pair of a block that ends beyond d is skipped by a
    // uniform branch; with several lanes per particle the block index differs
    // across the wave, the branch would diverge (no saving) and its extra live
    // values cost the wide layouts registers, so the pair is always formed.
    static __device__ __forceinline__ void normals_block(const RngKey& key, uint32_t n,
                                                         uint32_t t, uint32_t stream, int r,
                                                         int d, int bb, double (&q)[4],
                                                         uint32_t substep = 0u)
    {
        static_assert(DPL % 4 == 0, "lane slices are whole blocks of 4 coordinates");
        const int b = r * (DPL / 4) + bb;
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = 0.0;
        if (4 * b < d) {
            double w[4];
            normals4(key, n, t, stream, (uint32_t)b, w, substep, LPP == 1 ? d - 4 * b : 4);
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = (4 * b + u < d) ? w[u] : 0.0;
        }
    }

    // d normals of one (particle, step, stream) split over the group's lanes.
    static __device__ __forceinline__ void normals(const RngKey& key, uint32_t n, uint32_t t,
                                                   uint32_t stream, int r, int d, double (&z)[DPL])
    {
#pragma unroll
        for (int bb = 0; bb < DPL / 4; ++bb) {
            double q[4];
            normals_block(key, n, t, stream, r, d, bb, q);
#pragma unroll
            for (int u = 0; u < 4; ++u) z[4 * bb + u] = q[u];
        }
    }

    // X_0 ~ eta.
    static __device__ __forceinline__ double init(const TargetDev& tg, const Consts& c,
                                                  const ParView& pv, const RngKey& key, uint32_t n,
                                                  int r, float (&x)[DPL], double (&g)[DPL],
                                                  bool grad)
    {
        if constexpr (FAM == kUnid) {
            // uniform reference: coordinate i from word i of block 0
            const uint4 w = draw_block(key, n, 0u, kStreamInit, 0u, 0u);
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                x[j] = 0.f;
                g[j] = 0.0;
            }
            x[0] = (float)(tg.box * word_uniform(w.x));
            x[1] = (float)(tg.box * word_uniform(w.y));
            return eval<false>(tg, c, pv, r, x, g);
        }
        double z[DPL];
        normals(key, n, 0u, kStreamInit, r, tg.d, z);
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            x[j] = (float)(ref(pv, r, j) + c.sref * z[j]);
            g[j] = 0.0;
        }
        return grad ? eval<true>(tg, c, pv, r, x, g) : eval<false>(tg, c, pv, r, x, g);
    }

    // One MH step targeting pi_beta.  Returns the accept decision (the same on
    // every lane of the group).
    template <int MOVE>
    static __device__ __forceinline__ bool move(const TargetDev& tg, const Consts& c,
                                                const ParView& pv, const RngKey& key, uint32_t n,
                                                uint32_t t, int r, int L, double beta, double eps,
                                                float (&x)[DPL], double& ell, double (&g)[DPL],
                                                int forced = -1)
    {
        // RWMH draws its normals block by block inside the proposal loop
        // (shorter live ranges); MALA and HMC draw them all first
        if constexpr (MOVE == kRwmh3 || FAM == kUnid) {
            // random-walk substeps (one for kRwmh, three with standard
            // deviations eps (0.1, 1, 10) for kRwmh3), each with its own
            // normals and accept uniform (counter substep j); the decision
            // reported is whether any substep was accepted
            constexpr int NS = (MOVE == kRwmh3) ? 3 : 1;
            bool any = false;
#pragma unroll
            for (int sub = 0; sub < NS; ++sub) {
                const double sd = (MOVE == kRwmh3) ? eps * (sub == 0 ? 0.1 : (sub == 1 ? 1.0 : 10.0))
                                                   : eps;
                float xq[DPL];
                double gq[DPL];
                double dle = 0.0;
#pragma unroll
                for (int bb = 0; bb < DPL / 4; ++bb) {
                    double q[4];
                    normals_block(key, n, t, kStreamMove, r, tg.d, bb, q, (uint32_t)sub);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int j = 4 * bb + u;
                        xq[j] = (float)((double)x[j] + sd * q[u]);
                        if constexpr (FAM != kUnid) {
                            const double a = (double)x[j] - ref(pv, r, j);
                            const double b = (double)xq[j] - ref(pv, r, j);
                            dle += a * a - b * b;
                        }
                    }
                }
                const double ellq = eval<false>(tg, c, pv, r, xq, gq);
                double la;
                if constexpr (FAM == kUnid)
                    la = unid_inside(tg, xq) ? beta * (ellq - ell) : -INFINITY;
                else
                    la = group_sum<LPP>(dle) * c.half_inv_s2r + beta * (ellq - ell);
                const uint4 w = draw_block(key, n, t, kStreamAccept, (uint32_t)sub, 0u);
                const bool acc = (forced >= 0) ? (forced != 0) : (log(word_uniform(w.x)) < la);
                if (acc) {
#pragma unroll
                    for (int j = 0; j < DPL; ++j) x[j] = xq[j];
                    ell = ellq;
                }
                any = any || acc;
            }
            return any;
        }
        double z[DPL];
        if constexpr (uses_grad(MOVE)) normals(key, n, t, kStreamMove, r, tg.d, z);
        float xp[DPL];
        double gp[DPL];
        double ellp;
        double log_alpha;
        if constexpr (MOVE == kRwmh) {
            double dle = 0.0;
#pragma unroll
            for (int bb = 0; bb < DPL / 4; ++bb) {
                double q[4];
                normals_block(key, n, t, kStreamMove, r, tg.d, bb, q);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = 4 * bb + u;
                    xp[j] = (float)((double)x[j] + eps * q[u]);
                    const double a = (double)x[j] - ref(pv, r, j);
                    const double b = (double)xp[j] - ref(pv, r, j);
                    dle += a * a - b * b;
                }
            }
            ellp = eval<false>(tg, c, pv, r, xp, gp);
            log_alpha = group_sum<LPP>(dle) * c.half_inv_s2r + beta * (ellp - ell);
        } else if constexpr (MOVE == kMala) {
            const double h = 0.5 * eps * eps;
            double dle = 0.0, fwd = 0.0, bwd = 0.0;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const double xv = (double)x[j];
                const double ga = -(xv - ref(pv, r, j)) * c.inv_s2r + beta * g[j];
                xp[j] = (float)(xv + h * ga + eps * z[j]);
                const double rr = (double)xp[j] - xv - h * ga;
                fwd = fma(rr, rr, fwd);
            }
            ellp = eval<true>(tg, c, pv, r, xp, gp);
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const double xv = (double)x[j];
                const double xpv = (double)xp[j];
                const double gap = -(xpv - ref(pv, r, j)) * c.inv_s2r + beta * gp[j];
                const double rr = xv - xpv - h * gap;
                bwd = fma(rr, rr, bwd);
                const double a = xv - ref(pv, r, j);
                const double b = xpv - ref(pv, r, j);
                dle += a * a - b * b;
            }
            const double inv2e2 = 1.0 / (2.0 * eps * eps);
            log_alpha = group_sum<LPP>(dle) * c.half_inv_s2r + beta * (ellp - ell) -
                        group_sum<LPP>(bwd) * inv2e2 + group_sum<LPP>(fwd) * inv2e2;
        } else {
            // HMC: unit mass, L leapfrog steps; positions are stored (rounded) states.
            double mom[DPL];
            double kin0 = 0.0;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                mom[j] = z[j];
                xp[j] = x[j];
                gp[j] = g[j];
                kin0 += 0.5 * mom[j] * mom[j];
            }
            ellp = ell;
            const double he = 0.5 * eps;
            for (int l = 0; l < L; ++l) {
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const double xv = (double)xp[j];
                    mom[j] += he * (-(xv - ref(pv, r, j)) * c.inv_s2r + beta * gp[j]);
                    xp[j] = (float)(xv + eps * mom[j]);
                }
                ellp = eval<true>(tg, c, pv, r, xp, gp);
#pragma unroll
                for (int j = 0; j < DPL; ++j)
                    mom[j] += he * (-((double)xp[j] - ref(pv, r, j)) * c.inv_s2r + beta * gp[j]);
            }
            double kin1 = 0.0, dle = 0.0;
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                kin1 += 0.5 * mom[j] * mom[j];
                const double a = (double)x[j] - ref(pv, r, j);
                const double b = (double)xp[j] - ref(pv, r, j);
                dle += a * a - b * b;
            }
            log_alpha = group_sum<LPP>(dle) * c.half_inv_s2r + beta * (ellp - ell) -
                        group_sum<LPP>(kin1) + group_sum<LPP>(kin0);
        }
        const uint4 w = draw_block(key, n, t, kStreamAccept, 0u, 0u);
        const bool acc = (forced >= 0) ? (forced != 0) : (log(word_uniform(w.x)) < log_alpha);
        if (acc) {
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                x[j] = xp[j];
                if (uses_grad(MOVE)) g[j] = gp[j];
            }
            ell = ellp;
        }
        return acc;
    }
};

// ---------------------------------------------------------------------------
// OAIS: persistent tiles, streamed moments.
// ---------------------------------------------------------------------------
constexpr int kTC = 8;      // steps buffered before a transposed reduction
constexpr int kWavesPerBlock = 4;

// Minimum waves per SIMD requested from the compiler for the resampling
// variant's step kernel: four for particles with at most 8 coordinates per
// lane (the 128-register budget costs some spills and buys latency hiding:
// for the mixture/HMC step 5% faster than three waves and 30% faster than
// two), the compiler's choice otherwise (wider lanes would spill heavily).
// The AIS sweeps, which keep more state across their time loop, measured
// slower with such a request.
template <int DPL>
struct MinWaves {
    static constexpr int value = DPL <= 8 ? 4 : 1;
};

// log of w_{t-1} (g_t)^i for a record v = (log w_{t-1}, log g_t): g^0 = 1 also
// where g = 0 (log g = -inf, a zero likelihood), so i = 0 takes log w alone.
__device__ __forceinline__ double mom_term(double2 v, int i)
{
    return (i == 0) ? v.x : v.x + (double)i * v.y;
}

// All tiles of one slot of one problem, in tile order (one wave).  The
// moments of a slot therefore accumulate in the same order whichever wave,
// kernel or launch processes the slot.
template <int FAM, int MOVE, int LPP, int DPL>
__device__ __forceinline__ void oais_slot(const SweepArgs& a, const ParView& pv, const Consts& c,
                                          int64_t slot, double2 (&rec)[kTC][kWave / LPP],
                                          uint32_t (&cntb)[kTC])
{
    constexpr int P = kWave / LPP;
    constexpr int PP = (P + 7) / 8;  // particles per reduction lane
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP;
    const int pl = lane / LPP;
    const int T = a.T;
    const int d = a.tg.d;
    const bool grad = uses_grad(MOVE);

    // Fold TC buffered steps of this tile into the slot's accumulators.  For
    // the final entry (fin) the fourth field keeps the largest log w instead
    // of an accepted count.
    auto flush = [&](int64_t slot, bool first, int e0, int cnt, bool fin) {
        wave_sync();
        const int tcl = lane % kTC;
        const int part = lane / kTC;
        // the maximum over the tile's particles first (an xor butterfly over
        // the lanes of one step: every lane ends with the same value), then
        // one exponential per term against it and a butterfly sum: no
        // rescaling exponentials in the merge
        double m[3] = {-INFINITY, -INFINITY, -INFINITY};
        double s[3] = {0.0, 0.0, 0.0};
        if (tcl < cnt) {
#pragma unroll
            for (int q = 0; q < PP; ++q) {
                const int p = part * PP + q;
                if (p < P) {
                    const double2 v = rec[tcl][p];
#pragma unroll
                    for (int i = 0; i < 3; ++i) m[i] = fmax(m[i], mom_term(v, i));
                }
            }
        }
#pragma unroll
        for (int o = kTC; o < kWave; o <<= 1)
#pragma unroll
            for (int i = 0; i < 3; ++i) m[i] = fmax(m[i], __shfl_xor(m[i], o, kWave));
        if (tcl < cnt) {
#pragma unroll
            for (int q = 0; q < PP; ++q) {
                const int p = part * PP + q;
                if (p < P) {
                    const double2 v = rec[tcl][p];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        if (m[i] > -INFINITY) s[i] += exp(mom_term(v, i) - m[i]);
                }
            }
        }
#pragma unroll
        for (int o = kTC; o < kWave; o <<= 1)
#pragma unroll
            for (int i = 0; i < 3; ++i) s[i] += __shfl_xor(s[i], o, kWave);
        if (part == 0 && tcl < cnt) {
            double* e = a.part + ((size_t)slot * (T + 1) + (size_t)(e0 + tcl)) * 4;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double L = lse_value(m[i], s[i]);
                e[i] = first ? L : log_add(e[i], L);
            }
            if (fin)
                e[3] = first ? m[0] : fmax(e[3], m[0]);
            else
                e[3] = (first ? 0.0 : e[3]) + (double)cntb[tcl];
        }
        wave_sync();
    };

    {
        for (int64_t tile = slot; tile < a.ntiles; tile += a.S) {
            const bool first = (tile == slot);
            const int64_t n64 = tile * P + pl;
            const bool valid = n64 < a.N;
            const uint32_t n = (uint32_t)n64;
            float x[DPL];
            double g[DPL];
            double ell, lw;
            uint32_t accw;
            if (a.sx) {
                // a segment between fixed resampling times: the state the
                // previous segment (or the initial draw) left; lanes past N
                // work on a copy of the last particle and write nothing
                const int64_t nl = valid ? n64 : a.N - 1;
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const int i = r * DPL + j;
                    x[j] = (i < d) ? a.sx[(size_t)nl * d + i] : 0.f;
                    g[j] = (grad && i < d) ? a.sg[(size_t)nl * d + i] : 0.0;
                }
                ell = a.sell[nl];
                lw = a.slw[nl];
                accw = a.saccw[nl];
            } else {
                ell = Particle<FAM, LPP, DPL>::init(a.tg, c, pv, a.key, n, r, x, g, grad);
                lw = 0.0;
                accw = 0;
            }
            const int tb = a.t_begin;
            const int te = a.t_end > 0 ? a.t_end : T;
            for (int t = tb + 1; t <= te; ++t) {
                if (a.ckpt && ((t - 1) % a.ckpt_every) == 0 && valid) {
                    const int nseg = (T + a.ckpt_every - 1) / a.ckpt_every;
                    float* cp = a.ckpt + ((size_t)n64 * nseg + (t - 1) / a.ckpt_every) * d;
#pragma unroll
                    for (int j = 0; j < DPL; ++j) {
                        const int i = r * DPL + j;
                        if (i < d) cp[i] = x[j];
                    }
                }
                const double lg = (a.beta[t] - a.beta[t - 1]) * ell;
                const int tc = (t - tb - 1) % kTC;
                if (r == 0)
                    rec[tc][pl] = valid ? make_double2(lw, lg) : make_double2(-INFINITY, 0.0);
                lw += lg;
                const bool acc = Particle<FAM, LPP, DPL>::template move<MOVE>(
                    a.tg, c, pv, a.key, n, (uint32_t)t, r, a.leapfrog, a.beta[t], a.eps[t - 1], x,
                    ell, g);
                const uint64_t bal = __ballot(valid && acc && r == 0);
                if (lane == 0) cntb[tc] = (uint32_t)__popcll(bal);
                accw |= (acc ? 1u : 0u) << ((t - 1) & 31);
                if (((t - 1) & 31) == 31 || t == T) {
                    if (a.acc_bits && valid && r == 0)
                        a.acc_bits[(size_t)n64 * a.acc_words + (t - 1) / 32] = accw;
                    accw = 0;
                }
                if (tc == kTC - 1 || t == te) flush(slot, first, t - 1 - tc, tc + 1, false);
            }
            // final weights -> entry T (log-sum-exp and maximum of log w over the tile)
            if (r == 0) rec[0][pl] = valid ? make_double2(lw, 0.0) : make_double2(-INFINITY, 0.0);
            if (lane == 0) cntb[0] = 0u;
            flush(slot, first, T, 1, true);
            if (valid) {
                if (a.sx) {
#pragma unroll
                    for (int j = 0; j < DPL; ++j) {
                        const int i = r * DPL + j;
                        if (i < d) {
                            a.sx[(size_t)n64 * d + i] = x[j];
                            if (grad) a.sg[(size_t)n64 * d + i] = g[j];
                        }
                    }
                    if (r == 0) {
                        a.sell[n64] = ell;
                        a.slw[n64] = lw;
                        a.saccw[n64] = accw;
                    }
                }
                if (a.lw_out && r == 0) a.lw_out[n64] = lw;
                if (a.x_out) {
#pragma unroll
                    for (int j = 0; j < DPL; ++j) {
                        const int i = r * DPL + j;
                        if (i < d) a.x_out[(size_t)n64 * d + i] = x[j];
                    }
                }
            }
        }
    }
}

template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(256) k_oais_valu(SweepArgs a)
{
    __shared__ double2 sh_rec[kWavesPerBlock][kTC][kWave / LPP];
    __shared__ uint32_t sh_cnt[kWavesPerBlock][kTC];
    extern __shared__ __align__(16) char sh_dyn[];
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t W = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t slot = gw; slot < a.S; slot += W)
        oais_slot<FAM, MOVE, LPP, DPL>(a, pv, c, slot, sh_rec[wv], sh_cnt[wv]);
}

// Many problems of one (family, move, shape) class in one launch: each wave
// walks the work list of (problem, slot) items; target parameters are read
// from global memory through per-problem views.
template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(256) k_oais_valu_batch(const SweepArgs* __restrict__ args,
                                                         const ParView* __restrict__ views,
                                                         const int2* __restrict__ items,
                                                         int64_t nitems, uint32_t* next)
{
    __shared__ double2 sh_rec[kWavesPerBlock][kTC][kWave / LPP];
    __shared__ uint32_t sh_cnt[kWavesPerBlock][kTC];
    // the wave index through readfirstlane, so that the compiler sees the
    // work item, its arguments and its parameter view as wave-uniform (scalar
    // loads into scalar registers instead of per-lane copies in vector
    // registers)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t W = (int64_t)gridDim.x * kWavesPerBlock;
    // each wave claims its next item from the work counter (zero at the
    // launch; items longest first: a greedy balance), or without one takes
    // the static round robin; the claim is read back wave-uniform
    auto claim = [&](int64_t prev) -> int64_t {
        if (next == nullptr) return prev < 0 ? gw : prev + W;
        uint32_t v = 0u;
        if ((threadIdx.x & (kWave - 1)) == 0) v = atomicAdd(next, 1u);
        return (int64_t)__builtin_amdgcn_readfirstlane(v);
    };
    for (int64_t it = claim(-1); it < nitems; it = claim(it)) {
        const int2 item = items[it];
        const SweepArgs a = args[item.x];
        const ParView pv = views[item.x];
        const Consts c = make_consts(a.tg);
        oais_slot<FAM, MOVE, LPP, DPL>(a, pv, c, (int64_t)item.y, sh_rec[wv], sh_cnt[wv]);
    }
}

// ---------------------------------------------------------------------------
// Adaptive-resampling variant: one launch per step.
// ---------------------------------------------------------------------------
template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(256) k_asmc_init(SweepArgs a, AsmcState z)
{
    constexpr int P = kWave / LPP;
    extern __shared__ __align__(16) char sh_dyn[];
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP, pl = lane / LPP;
    const int64_t tile =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t n64 = tile * P + pl;
    if (tile >= a.ntiles || n64 >= a.N) return;
    float x[DPL];
    double g[DPL];
    const double ell = Particle<FAM, LPP, DPL>::init(a.tg, c, pv, a.key, (uint32_t)n64, r, x, g,
                                                     uses_grad(MOVE));
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int i = r * DPL + j;
        if (i < a.tg.d) {
            z.X[(size_t)n64 * a.tg.d + i] = x[j];
            if (uses_grad(MOVE)) z.G[(size_t)n64 * a.tg.d + i] = g[j];
        }
    }
    if (r == 0) {
        z.ell[n64] = ell;
        z.lw[n64] = 0.0;
        z.accw[n64] = 0u;
    }
}

template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(256, MinWaves<DPL>::value)
    k_asmc_step(SweepArgs a, AsmcState z, int t)
{
    if (a.t_stop && t > *a.t_stop) return;  // an online schedule already reached beta = 1
    constexpr int P = kWave / LPP;
    extern __shared__ __align__(16) char sh_dyn[];
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP, pl = lane / LPP;
    const int64_t tile =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (tile >= a.ntiles) return;  // whole wave leaves together
    const int64_t n64 = tile * P + pl;
    const bool valid = n64 < a.N;
    const int d = a.tg.d;
    const int64_t nl = valid ? n64 : a.N - 1;  // invalid lanes work on a copy, write nothing
    // state, ell and (MALA, HMC) grad ell as the previous step left them:
    // after a resampling event at the previous step (its flag is still set:
    // the merge of this step has not run) the gathered copies X2, G2, ell2
    // with log w = 0; this step writes X, G, ell as always, so the gathered
    // state is never copied back (runs without a gather target never resample)
    const bool rs = z.X2 != nullptr && z.scal[2] != 0.0;
    const float* Xs = rs ? z.X2 : z.X;
    const double* Gs = rs ? z.G2 : z.G;
    float x[DPL];
    double g[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int i = r * DPL + j;
        x[j] = (i < d) ? Xs[(size_t)nl * d + i] : 0.f;
        g[j] = (uses_grad(MOVE) && i < d) ? Gs[(size_t)nl * d + i] : 0.0;
    }
    double ell = rs ? z.ell2[nl] : z.ell[nl];
    double lw = rs ? 0.0 : z.lw[nl];
    const double lg = (a.beta[t] - a.beta[t - 1]) * ell;
    // tile statistics: lse of lw, lw+lg, lw+2lg, 2(lw+lg) over the tile's
    // particles: the maximum by an xor butterfly over the particle groups
    // (every lane ends with the same value), then one exponential per lane
    // against it and a butterfly sum
    double m[4], s[4];
    {
        const double v[4] = {lw, lw + lg, lw + 2.0 * lg, 2.0 * (lw + lg)};
#pragma unroll
        for (int i = 0; i < 4; ++i) m[i] = valid ? v[i] : -INFINITY;
#pragma unroll
        for (int o = LPP; o < kWave; o <<= 1)
#pragma unroll
            for (int i = 0; i < 4; ++i) m[i] = fmax(m[i], __shfl_xor(m[i], o, kWave));
#pragma unroll
        for (int i = 0; i < 4; ++i) s[i] = (valid && m[i] > -INFINITY) ? exp(v[i] - m[i]) : 0.0;
#pragma unroll
        for (int o = LPP; o < kWave; o <<= 1)
#pragma unroll
            for (int i = 0; i < 4; ++i) s[i] += __shfl_xor(s[i], o, kWave);
    }
    lw += lg;
    const bool acc = Particle<FAM, LPP, DPL>::template move<MOVE>(
        a.tg, c, pv, a.key, (uint32_t)nl, (uint32_t)t, r, a.leapfrog, a.beta[t], a.eps[t - 1], x,
        ell, g);
    const uint64_t bal = __ballot(valid && acc && r == 0);
    if (lane == 0) {
        double* tp = z.tile_part + (size_t)tile * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) tp[i] = lse_value(m[i], s[i]);
        tp[4] = m[1];  // max of log w_{t^-}
        tp[5] = (double)__popcll(bal);
    }
    if (valid) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int i = r * DPL + j;
            if (i < d) {
                z.X[(size_t)n64 * d + i] = x[j];
                if (uses_grad(MOVE)) z.G[(size_t)n64 * d + i] = g[j];
            }
        }
        if (r == 0) {
            z.ell[n64] = ell;
            z.lw[n64] = lw;
            uint32_t w = z.accw[n64] | ((acc ? 1u : 0u) << ((t - 1) & 31));
            if (((t - 1) & 31) == 31 || t == a.T) {
                if (a.acc_bits) a.acc_bits[(size_t)n64 * a.acc_words + (t - 1) / 32] = w;
                w = 0u;
            }
            z.accw[n64] = w;
        }
    }
}

// ---------------------------------------------------------------------------
// Final-iteration rejuvenation (Sec. "Computing expectations"): after the
// last annealing step the population is resampled and N chains run T steps of
// the forward kernel at beta = 1 (step size eps_T), chain n from particle
// anc[n]; its states feed the expectations.  One wave per tile as in the
// sweep; the chain draws with counters (n, T + s), s = 1..T.  Sums of x_i and
// x_i^2 over the chain are kept per lane (in step order), summed over the
// wave's particles by an xor butterfly and written per tile.
// ---------------------------------------------------------------------------
template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(256) k_rejuv(RejuvArgs R)
{
    constexpr int P = kWave / LPP;
    extern __shared__ __align__(16) char sh_dyn[];
    const SweepArgs& a = R.a;
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP, pl = lane / LPP;
    const int64_t tile =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (tile >= a.ntiles) return;  // whole wave leaves together
    const int64_t n64 = tile * P + pl;
    const bool valid = n64 < a.N;
    const int d = a.tg.d;
    // the host checked the event, so every ancestor is a particle index
    const int64_t src = R.anc[valid ? n64 : a.N - 1];
    float x[DPL];
    double g[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int i = r * DPL + j;
        x[j] = (i < d) ? R.x_in[(size_t)src * d + i] : 0.f;
        g[j] = 0.0;
    }
    double ell = uses_grad(MOVE) ? Particle<FAM, LPP, DPL>::template eval<true>(a.tg, c, pv, r, x, g)
                                 : Particle<FAM, LPP, DPL>::template eval<false>(a.tg, c, pv, r, x, g);
    double s1[DPL], s2[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) s1[j] = s2[j] = 0.0;
    uint32_t na = 0;
    for (int s = 1; s <= a.T; ++s) {
        const bool acc = Particle<FAM, LPP, DPL>::template move<MOVE>(
            a.tg, c, pv, a.key, (uint32_t)n64, (uint32_t)(a.T + s), r, a.leapfrog, 1.0, R.eps, x,
            ell, g);
        na += acc ? 1u : 0u;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const double v = (double)x[j];
            s1[j] += v;
            s2[j] += v * v;
        }
    }
    if (valid && R.x_out) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int i = r * DPL + j;
            if (i < d) R.x_out[(size_t)n64 * d + i] = x[j];
        }
    }
    // sums over the wave's particles (lanes r, r + LPP, ... hold the same coordinates)
    double cnt = (valid && r == 0) ? (double)na : 0.0;
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        if (!valid) s1[j] = s2[j] = 0.0;
#pragma unroll
        for (int o = LPP; o < kWave; o <<= 1) {
            s1[j] += __shfl_xor(s1[j], o, kWave);
            s2[j] += __shfl_xor(s2[j], o, kWave);
        }
    }
    cnt = wave_sum(cnt);
    double* out = R.tsum + (size_t)tile * (2 * d + 1);
    if (pl == 0) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int i = r * DPL + j;
            if (i < d) {
                out[i] = s1[j];
                out[d + i] = s2[j];
            }
        }
        if (r == 0) out[2 * d] = cnt;
    }
}

// ---------------------------------------------------------------------------
// Parallel tempering (Sec. "Computational duality with parallel tempering"):
// one workgroup per PT copy, replica r of the copy on particle slot r of the
// workgroup (LPP lanes), at temperature tau[r].  Iteration t: every replica
// takes one step of the forward kernel at its temperature (counters (replica,
// t)); then one thread per proposed pair (n, n + 1) of the parity of t decides
// the swap of temperatures (stream 4, counter (copy (N' + 1) + n, t)); then
// the stepping-stone terms (one thread per temperature, a running maximum and
// scaled sum), round trips (one thread per replica) and the target chain's
// sums (the replica at N') are taken.  Swaps exchange temperatures, not states.
// ---------------------------------------------------------------------------
constexpr uint32_t kStreamSwap = 4;

// At most 8 waves per copy (512 threads): two waves per SIMD leave the move
// arithmetic its registers (at 1024 threads the compiler caps a lane at 128
// registers and spills several hundred bytes per lane).
constexpr int kPtMaxThreads = 512;

template <int FAM, int MOVE, int LPP, int DPL>
__global__ void __launch_bounds__(kPtMaxThreads) k_pt(PtArgs A)
{
    constexpr int P = kWave / LPP;
    extern __shared__ __align__(16) char sh_dyn[];
    const SweepArgs& a = A.a;
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int R = A.Np + 1;
    const int Np = A.Np;
    size_t off = (params_bytes_lanes(a.tg, LPP, DPL) + 15) & ~(size_t)15;
    double* Lsh = reinterpret_cast<double*>(sh_dyn + off);   // [R] ell of replica r
    double* rsum = Lsh + R;                                   // [Np] summed rejections
    int* tau = reinterpret_cast<int*>(rsum + Np);             // [R] temperature of replica r
    int* rep = tau + R;                                       // [R] replica at temperature n
    int* side = rep + R;                                      // [R] round-trip state
    double* red = reinterpret_cast<double*>(side + R + ((R & 1) ? 1 : 0));  // [16]
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wv = tid / kWave;
    const int r = lane % LPP;
    const int slot = wv * P + lane / LPP;   // replica of this lane group
    const bool live = slot < R;
    const int k = blockIdx.x;
    const uint32_t gid = (uint32_t)(k * R + (live ? slot : 0));
    const int d = a.tg.d;
    for (int i = tid; i < R; i += blockDim.x) {
        tau[i] = i;
        rep[i] = i;
        side[i] = (i == 0) ? 0 : -1;
    }
    for (int i = tid; i < Np; i += blockDim.x) rsum[i] = 0.0;
    float x[DPL];
    double g[DPL];
    double ell = Particle<FAM, LPP, DPL>::init(a.tg, c, pv, a.key, gid, r, x, g, uses_grad(MOVE));
    double f1[DPL], f2[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) f1[j] = f2[j] = 0.0;
    double sm = -INFINITY, ss = 0.0;  // stepping stone of temperature tid (tid < Np)
    double trips = 0.0;               // round trips of replica tid (tid < R)
    __syncthreads();
    for (int t = 1; t <= a.T; ++t) {
        const int n = live ? tau[slot] : 0;
        Particle<FAM, LPP, DPL>::template move<MOVE>(a.tg, c, pv, a.key, gid, (uint32_t)t, r,
                                                     a.leapfrog, A.beta[n], A.eps[n], x, ell, g);
        if (live && r == 0) Lsh[slot] = ell;
        __syncthreads();
        // swaps of the pairs (n, n + 1), n of the parity of t
        {
            const int np = ((t & 1) ? 1 : 0) + 2 * tid;
            if (np + 1 < R) {
                const int ra = rep[np], rb = rep[np + 1];
                const double la = (A.beta[np + 1] - A.beta[np]) * (Lsh[ra] - Lsh[rb]);
                const uint4 w = draw_block(a.key, (uint32_t)(k * R + np), (uint32_t)t, kStreamSwap,
                                           0u, 0u);
                const double acc = (la >= 0.0) ? 1.0 : ((la == la) ? exp(la) : 0.0);
                rsum[np] += 1.0 - acc;
                if (log(word_uniform(w.x)) < la) {
                    rep[np] = rb;
                    rep[np + 1] = ra;
                    tau[ra] = np + 1;
                    tau[rb] = np;
                }
            }
        }
        __syncthreads();
        if (tid < R) {
            const int tr = tau[tid];
            if (tr == Np && side[tid] == 0) side[tid] = 1;
            if (tr == 0) {
                if (side[tid] == 1) trips += 1.0;
                side[tid] = 0;
            }
        }
        if (tid < Np) {
            const double v = (A.beta[tid + 1] - A.beta[tid]) * Lsh[rep[tid]];
            if (v > -INFINITY) {
                if (v > sm) {
                    ss = ss * exp(sm - v) + 1.0;
                    sm = v;
                } else {
                    ss += exp(v - sm);
                }
            }
        }
        if (live && tau[slot] == Np) {
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const double v = (double)x[j];
                f1[j] += v;
                f2[j] += v * v;
            }
        }
        __syncthreads();
    }
    // per-copy outputs: stepping stone (max, scaled sum), rejections, round
    // trips, target-chain sums over the copy's replicas (fixed order)
    double* o = A.out + (size_t)k * A.stride;
    if (tid < Np) {
        o[2 * tid] = sm;
        o[2 * tid + 1] = ss;
        o[2 * Np + tid] = rsum[tid];
    }
    double tr = wave_sum(trips);
    if (lane == 0) red[wv] = tr;
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        if (!live) f1[j] = f2[j] = 0.0;
#pragma unroll
        for (int q = LPP; q < kWave; q <<= 1) {
            f1[j] += __shfl_xor(f1[j], q, kWave);
            f2[j] += __shfl_xor(f2[j], q, kWave);
        }
    }
    double* fo = A.fpart + ((size_t)k * 16 + wv) * 2 * d;
    if (lane < LPP) {
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int i = r * DPL + j;
            if (i < d) {
                fo[i] = f1[j];
                fo[d + i] = f2[j];
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += red[i];
        o[3 * Np] = s;
        o[3 * Np + 1] = (double)(blockDim.x / kWave);
    }
}

// ell and grad ell at given binary32 states: the particle's coordinates are
// loaded into the lane layout (zero beyond d) and evaluated by the sweep's
// Particle::eval, one lane group per particle.
template <int FAM, int LPP, int DPL>
__global__ void __launch_bounds__(256) k_target_eval(EvalArgs E)
{
    constexpr int P = kWave / LPP;
    extern __shared__ __align__(16) char sh_dyn[];
    const SweepArgs& a = E.a;
    const ParView pv = stage_params_lanes<LPP, DPL>(a.tg, sh_dyn);
    const Consts c = make_consts(a.tg);
    const int lane = threadIdx.x & (kWave - 1);
    const int r = lane % LPP, pl = lane / LPP;
    const int64_t tile =
        (int64_t)blockIdx.x * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (tile >= a.ntiles) return;
    // a tile's particles beyond N evaluate zeros and write nothing, so the
    // lane groups of a wave stay converged through the evaluation
    const int64_t n64 = tile * P + pl;
    const bool valid = n64 < a.N;
    const int d = a.tg.d;
    float x[DPL];
    double g[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int i = r * DPL + j;
        x[j] = (valid && i < d) ? E.x[(size_t)n64 * d + i] : 0.f;
    }
    const double ell = Particle<FAM, LPP, DPL>::template eval<true>(a.tg, c, pv, r, x, g);
    if (!valid) return;
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int i = r * DPL + j;
        if (i < d) E.grad[(size_t)n64 * d + i] = g[j];
    }
    if (r == 0) E.ell[n64] = ell;
}

template <int FAM, int MOVE, int LPP, int DPL>
struct Launch {
    static hipError_t oais(const SweepArgs& a, int grid_waves, hipStream_t st)
    {
        const int blocks = (grid_waves + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((k_oais_valu<FAM, MOVE, LPP, DPL>), dim3(blocks), dim3(256),
                           params_bytes_lanes(a.tg, LPP, DPL), st, a);
        return hipGetLastError();
    }
    static hipError_t batch(const SweepArgs* args, const ParView* views, const int2* items,
                            int64_t nitems, uint32_t* next, int grid_waves, hipStream_t st)
    {
        const int blocks = (grid_waves + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((k_oais_valu_batch<FAM, MOVE, LPP, DPL>), dim3(blocks), dim3(256), 0, st,
                           args, views, items, nitems, next);
        return hipGetLastError();
    }
    static hipError_t init(const SweepArgs& a, const AsmcState& z, hipStream_t st)
    {
        const int64_t blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((k_asmc_init<FAM, MOVE, LPP, DPL>), dim3((unsigned)blocks), dim3(256),
                           params_bytes_lanes(a.tg, LPP, DPL), st, a, z);
        return hipGetLastError();
    }
    static hipError_t rejuv(const RejuvArgs& R, hipStream_t st)
    {
        const int64_t blocks = (R.a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((k_rejuv<FAM, MOVE, LPP, DPL>), dim3((unsigned)blocks), dim3(256),
                           params_bytes_lanes(R.a.tg, LPP, DPL), st, R);
        return hipGetLastError();
    }
    static hipError_t pt(const PtArgs& A, hipStream_t st)
    {
        constexpr int P = kWave / LPP;
        const int waves = (A.Np + 1 + P - 1) / P;
        const size_t shb = pt_shared_bytes(A, LPP, DPL);
        hipLaunchKernelGGL((k_pt<FAM, MOVE, LPP, DPL>), dim3((unsigned)A.K), dim3(waves * kWave),
                           shb, st, A);
        return hipGetLastError();
    }
    static hipError_t eval(const EvalArgs& E, hipStream_t st)
    {
        // one instantiation per family: the evaluation does not depend on the move
        if constexpr (MOVE == kMala || (FAM == kUnid && MOVE == kRwmh)) {
            const int64_t blocks = (E.a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
            hipLaunchKernelGGL((k_target_eval<FAM, LPP, DPL>), dim3((unsigned)blocks), dim3(256),
                               params_bytes_lanes(E.a.tg, LPP, DPL), st, E);
            return hipGetLastError();
        } else {
            (void)E;
            (void)st;
            return hipErrorInvalidValue;
        }
    }
    static hipError_t step(const SweepArgs& a, const AsmcState& z, int t, hipStream_t st)
    {
        const int64_t blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
        hipLaunchKernelGGL((k_asmc_step<FAM, MOVE, LPP, DPL>), dim3((unsigned)blocks), dim3(256),
                           params_bytes_lanes(a.tg, LPP, DPL), st, a, z, t);
        return hipGetLastError();
    }
};

template <int FAM, int MOVE>
hipError_t valu_dispatch(int what, const SweepArgs& a, const ValuShape& s, int gw,
                           const AsmcState* z, int t, hipStream_t st, const ValuBatch* b,
                           const void* ext)
{
    const RejuvArgs* rj = static_cast<const RejuvArgs*>(ext);
    const PtArgs* pt = static_cast<const PtArgs*>(ext);
    const EvalArgs* ev = static_cast<const EvalArgs*>(ext);
#define OASMC_CASE(L, D)                                                     \
    if (s.lpp == L && s.dpl == D) {                                          \
        if (what == 0) return Launch<FAM, MOVE, L, D>::oais(a, gw, st);      \
        if (what == 1) return Launch<FAM, MOVE, L, D>::init(a, *z, st);      \
        if (what == 3)                                                       \
            return Launch<FAM, MOVE, L, D>::batch(b->args, b->views, b->items, \
                                                  b->nitems, b->next, gw, st); \
        if (what == 4) return Launch<FAM, MOVE, L, D>::rejuv(*rj, st);       \
        if (what == 5) return Launch<FAM, MOVE, L, D>::pt(*pt, st);          \
        if (what == 6) return Launch<FAM, MOVE, L, D>::eval(*ev, st);        \
        return Launch<FAM, MOVE, L, D>::step(a, *z, t, st);                  \
    }
    OASMC_CASE(1, 4)
    if constexpr (FAM == kUnid) return hipErrorInvalidValue;  // d = 2: one lane of 4 only
    OASMC_CASE(1, 8)
    OASMC_CASE(1, 12)
    OASMC_CASE(1, 16)
    OASMC_CASE(1, 20)
    OASMC_CASE(1, 24)
    OASMC_CASE(2, 16)
    OASMC_CASE(4, 16)
    OASMC_CASE(8, 16)
    OASMC_CASE(16, 16)
    OASMC_CASE(8, 8)
    OASMC_CASE(16, 8)
    OASMC_CASE(4, 8)
    OASMC_CASE(8, 4)
#undef OASMC_CASE
    return hipErrorInvalidValue;
}

}  // namespace oasmc
