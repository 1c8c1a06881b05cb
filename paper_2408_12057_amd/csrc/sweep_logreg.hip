// sweep_logreg.hip -- the loop-swapped AIS sweep with MALA for Bayesian
// logistic regression, where each move evaluates the log-likelihood and its
// gradient for every particle:
//     z = Theta X^T        ([P x d] . [d x n], logits, never stored)
//     ell_p = sum_i y_i z_pi - softplus(z_pi)
//     grad_p = sum_i (y_i - s(z_pi)) X_i   ([P x n] . [n x d])
// Both products run on FP32 MFMA (v_mfma_f32_32x32x2f32).  The first is
// computed transposed (rows of X on M, particles on N) so that its
// accumulator registers, after the fused softplus/sigmoid epilogue, are
// directly the A operand of the second product: no transpose, no LDS round
// trip for the residuals.
//
// Workgroup = one tile of 64 particles for all T steps (512 threads, 8 waves);
// each wave owns 1/8 of the data rows, streams them through its own LDS
// staging buffer in 32-row chunks, and the 8 partial gradients are summed in
// a fixed-order tree through LDS.  Particle states, the cached gradient and
// log-likelihood stay in LDS across steps; X (n x 64 fp32, features packed)
// is re-read from L2 every step.
//
// Feature packing: with KH = ceil(d/2), feature f < KH sits in column f and
// feature f >= KH in column 32 + f - KH, so every lane reads KH contiguous
// columns for the K loop of the first product (instruction s, lane half h ->
// column 32h + s) and the second product's 64 output columns cover all
// features with two 32-wide tiles.
#include <stdlib.h>

#include "kernels.hpp"

namespace oasmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kLP = 64;          // particles per tile
constexpr int kRows = 32;        // data rows per chunk
constexpr int kSt = 72;          // floats per staged row: 64 columns, y, mask, padding
constexpr int kPs = 68;          // floats per particle row in LDS
constexpr int kRowAlign = kRows * 8;

// Two shapes of the same workgroup:
//  PIPE = true : 4 waves (one per SIMD, 512 registers per lane), double-
//                buffered logits so the next chunk's first product overlaps
//                the current chunk's epilogue inside one wave;
//  PIPE = false: 8 waves (two per SIMD, 256 registers per lane), one chunk at
//                a time; the two waves of a SIMD overlap each other instead.
template <bool PIPE>
struct LCfg {
    static constexpr int waves = PIPE ? 4 : 8;
    static constexpr int threads = waves * kWave;
    static constexpr int tpp = threads / kLP;   // threads per particle, scalar phases
    static constexpr int nbuf = PIPE ? 2 : 1;   // LDS staging buffers per wave
    static constexpr int blocks_per_thread = 16 / tpp;
    static constexpr int feats_per_thread = 4 * blocks_per_thread;
};

template <bool PIPE>
struct LogregShared {
    using C = LCfg<PIPE>;
    float theta[kLP][kPs];  // current states (packed columns)
    float prop[kLP][kPs];   // proposals
    float gl[kLP][kPs];     // gradient of ell at theta
    float glp[kLP][kPs];    // gradient of ell at prop
    float stage[C::waves][C::nbuf][kRows][kSt];
    double ll[kLP], llp[kLP], lw[kLP];
    double llpart[C::waves][kLP];
    double fwd[kLP], dle[kLP], logu[kLP];
    float m[64];
    uint32_t cnt;
};

static_assert(sizeof(float) * 4 * 2 * kRows * kSt >= sizeof(float) * 2 * 64 * kWave, "reduction fits");
static_assert(sizeof(float) * 8 * 1 * kRows * kSt >= sizeof(float) * 4 * 64 * kWave, "reduction fits");

__device__ __forceinline__ void lsync() { __syncthreads(); }

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__host__ __device__ __forceinline__ int col_of(int f, int KH) { return f < KH ? f : 32 + f - KH; }

// Packs X (n x d, row-major) into Xp (n_pad x 64) with the column map above
// and y into yp, marking padded rows with y = -1.
__global__ void k_logreg_pack(const float* __restrict__ X, const float* __restrict__ y, int n,
                              int d, int KH, int n_pad, float* __restrict__ Xp,
                              float* __restrict__ yp)
{
    const int64_t total = (int64_t)n_pad * 64;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / 64), c = (int)(e % 64);
        int f = -1;
        if (c < 32) {
            if (c < KH) f = c;
        } else if (c - 32 < d - KH) {
            f = KH + c - 32;
        }
        Xp[e] = (i < n && f >= 0 && f < d) ? X[(int64_t)i * d + f] : 0.f;
        if (c == 0) yp[i] = (i < n) ? y[i] : -1.f;
    }
}

// ell and grad ell at sh.prop for the 64 particles of the tile; results in
// sh.llp (binary64) and sh.glp (packed columns).  All threads participate.
template <int KH, bool PIPE>
__device__ __forceinline__ void contraction(LogregShared<PIPE>& sh, const float* __restrict__ Xp,
                            const float* __restrict__ yp, int n_pad)
{
    constexpr int kLWaves = LCfg<PIPE>::waves;
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int l = tid % kWave;
    const int h = l / 32;
    const int j = l % 32;

    // B operand of the first product: the particles' states.  The pipelined
    // shape keeps them in registers; the 8-wave shape (256 registers per
    // lane) reads them from LDS at each k-step.
    float bth[2][PIPE ? KH : 1];
    if constexpr (PIPE) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int s = 0; s < KH; ++s) bth[g][s] = sh.prop[32 * g + j][32 * h + s];
    }

    floatx16 G[2][2];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int ft = 0; ft < 2; ++ft)
#pragma unroll
            for (int q = 0; q < 16; ++q) G[g][ft][q] = 0.f;
    double llacc[2] = {0.0, 0.0};

    const int rows_w = n_pad / kLWaves;
    const int r0 = w * rows_w;
    const int nchunks = rows_w / kRows;
    const int srow = l / 2, shalf = l % 2;

    // Software pipeline over 32-row chunks.  Chunk c sits in LDS buffer c&1
    // with its logits in registers; each of its 16 row slots q runs
    //   ~KH/16 k-steps of the NEXT chunk's logits   (matrix cores)
    //   the epilogue of slot q                        (VALU)
    //   slot q's share of the gradient product        (matrix cores)
    // so the in-order wave always has independent matrix-core work queued
    // behind its VALU work.  Global loads run two chunks ahead in registers
    // and land in the buffer chunk c releases.
    // one chunk's share of this lane: 8 x 16 bytes of X and (y, row mask)
    struct Slice {
        float4 v0, v1, v2, v3, v4, v5, v6, v7;
        float2 y;
    };
    auto fetch = [&](int c) -> Slice {
        const float4* src =
            reinterpret_cast<const float4*>(Xp + (size_t)(r0 + c * kRows + srow) * 64 + shalf * 32);
        Slice t;
        t.v0 = src[0]; t.v1 = src[1]; t.v2 = src[2]; t.v3 = src[3];
        t.v4 = src[4]; t.v5 = src[5]; t.v6 = src[6]; t.v7 = src[7];
        t.y = make_float2(0.f, 0.f);
        if (l < kRows) {
            const float yr = yp[r0 + c * kRows + l];
            t.y = (yr >= 0.f) ? make_float2(yr, 1.f) : make_float2(0.f, 0.f);
        }
        return t;
    };
    auto put = [&](int buf, const Slice& t) {
        float4* dst = reinterpret_cast<float4*>(&sh.stage[w][buf][srow][shalf * 32]);
        dst[0] = t.v0; dst[1] = t.v1; dst[2] = t.v2; dst[3] = t.v3;
        dst[4] = t.v4; dst[5] = t.v5; dst[6] = t.v6; dst[7] = t.v7;
        if (l < kRows) *reinterpret_cast<float2*>(&sh.stage[w][buf][l][64]) = t.y;
    };
    auto zero = [](floatx16 (&acc)[2]) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[g][q] = 0.f;
    };
    constexpr float kLn2 = 0.693147180559945309f;
    // k-steps [s0, s1) of the first product for the chunk in buffer `buf`
    auto gemm1 = [&](int buf, floatx16 (&acc)[2], int s0, int s1) {
        float(*st)[kSt] = sh.stage[w][buf];
#pragma unroll
        for (int s = s0; s < s1; ++s) {
            const float a = st[j][32 * h + s];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                float bv;
                if constexpr (PIPE) bv = bth[g][s];
                else bv = sh.prop[32 * g + j][32 * h + s];
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc[g], 0, 0, 0);
            }
        }
    };
    // epilogue of row slot q (y and the row mask in columns 64, 65), then the
    // slot's share of the gradient product
    auto slot = [&](float(*stc)[kSt], floatx16 (&cur)[2], int q, float (&llc)[2]) {
        const int i = 8 * (q / 4) + 4 * h + (q % 4);
        const float2 yv = *reinterpret_cast<const float2*>(&stc[i][64]);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const float z = cur[g][q];
            const float e = __expf(-fabsf(z));
            const float ope = 1.0f + e;
            const float inv = __builtin_amdgcn_rcpf(ope);
            const float sig = (z >= 0.f) ? inv : e * inv;
            const float sp = fmaxf(z, 0.f) + kLn2 * __builtin_amdgcn_logf(ope);
            llc[g] = fmaf(yv.y, fmaf(yv.x, z, -sp), llc[g]);
            cur[g][q] = fmaf(-yv.y, sig, yv.x);
        }
#pragma unroll
        for (int ft = 0; ft < 2; ++ft) {
            const float bx = stc[i][32 * ft + j];
#pragma unroll
            for (int g = 0; g < 2; ++g)
                G[g][ft] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[g][q], bx, G[g][ft], 0, 0, 0);
        }
    };

    if constexpr (PIPE) {
        // Chunk c sits in buffer c&1 with its logits in registers; each row
        // slot q runs ~KH/16 k-steps of the NEXT chunk's first product, then
        // its own epilogue and gradient share, so the in-order wave always has
        // independent matrix-core work queued behind its VALU work.  Loads run
        // two chunks ahead and land in the buffer chunk c releases.  The body
        // is branch-free: past the last chunk it recomputes the last chunk
        // and discards the result.
        auto stage_step = [&](int c, floatx16 (&cur)[2], floatx16 (&nxt)[2]) {
            const int b = c & 1;
            float(*stc)[kSt] = sh.stage[w][b];
            const Slice ahead = fetch(min(c + 2, nchunks - 1));
            zero(nxt);
            float llc[2] = {0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                gemm1(b ^ 1, nxt, (q * KH + 15) / 16, ((q + 1) * KH + 15) / 16);
                slot(stc, cur, q, llc);
            }
            llacc[0] += (double)llc[0];
            llacc[1] += (double)llc[1];
            wsync();
            put(b, ahead);
            wsync();
        };
        floatx16 accA[2], accB[2];
        put(0, fetch(0));
        put(1, fetch(min(1, nchunks - 1)));
        wsync();
        zero(accA);
        gemm1(0, accA, 0, KH);
        for (int c = 0; c < nchunks; c += 2) {
            stage_step(c, accA, accB);
            if (c + 1 < nchunks) stage_step(c + 1, accB, accA);
        }
    } else {
        // One buffer per wave: the next chunk's slice waits in registers
        // while the current chunk is consumed.
        floatx16 acc[2];
        Slice ahead = fetch(0);
        for (int c = 0; c < nchunks; ++c) {
            put(0, ahead);
            wsync();
            ahead = fetch(min(c + 1, nchunks - 1));
            zero(acc);
            gemm1(0, acc, 0, KH);
            float llc[2] = {0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 16; ++q) slot(sh.stage[w][0], acc, q, llc);
            llacc[0] += (double)llc[0];
            llacc[1] += (double)llc[1];
            wsync();
        }
    }

    // per-particle log-likelihood: halves of the wave, then waves in order
#pragma unroll
    for (int g = 0; g < 2; ++g) llacc[g] += __shfl_xor(llacc[g], 32, kWave);
    if (h == 0) {
        sh.llpart[w][j] = llacc[0];
        sh.llpart[w][32 + j] = llacc[1];
    }
    lsync();  // every wave is done with its staging buffer

    // gradient: fixed tree (w + w^2), (w + w^1) through LDS
    float* red = &sh.stage[0][0][0][0];
    static_assert(sizeof(sh.stage) >= sizeof(float) * (kLWaves / 2) * 64 * kWave, "reduction fits");
    for (int span = kLWaves / 2; span >= 1; span /= 2) {
        if (w >= span && w < 2 * span) {
            float* dst = red + (size_t)(w - span) * 64 * kWave;
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                    for (int q = 0; q < 16; ++q) dst[((g * 2 + ft) * 16 + q) * kWave + l] = G[g][ft][q];
        }
        lsync();
        if (w < span) {
            const float* src = red + (size_t)w * 64 * kWave;
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                    for (int q = 0; q < 16; ++q) G[g][ft][q] += src[((g * 2 + ft) * 16 + q) * kWave + l];
        }
        lsync();
    }
    if (w == 0) {
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int p = 32 * g + 8 * (q / 4) + 4 * h + (q % 4);
                    sh.glp[p][32 * ft + j] = G[g][ft][q];
                }
    }
    if (tid < kLP) {
        double s = 0.0;
        for (int ww = 0; ww < kLWaves; ++ww) s += sh.llpart[ww][tid];
        sh.llp[tid] = s;
    }
    lsync();
}


// Particle p's thread r (of tpp) handles the normal blocks r, r + tpp,
// r + 2 tpp, ... i.e. the features 4b..4b+3 of those blocks (below d).
template <int TPP>
__device__ __forceinline__ int feat_of(int r, int u) { return 4 * (r + TPP * (u / 4)) + (u % 4); }

// The parameters shared by every tile of a problem: zero the particle arrays
// (columns beyond d stay zero) and stage the reference mean in packed columns.
template <int KH, bool PIPE>
__device__ __forceinline__ void logreg_setup(LogregShared<PIPE>& sh, const SweepArgs& a)
{
    constexpr int kLThreads = LCfg<PIPE>::threads;
    const int tid = threadIdx.x;
    const int d = a.tg.d;
    for (int e = tid; e < kLP * kPs; e += kLThreads) {
        (&sh.theta[0][0])[e] = 0.f;
        (&sh.prop[0][0])[e] = 0.f;
        (&sh.gl[0][0])[e] = 0.f;
        (&sh.glp[0][0])[e] = 0.f;
    }
    for (int c = tid; c < 64; c += kLThreads) {
        int f = -1;
        if (c < 32) { if (c < KH) f = c; }
        else if (c - 32 < d - KH) f = KH + c - 32;
        sh.m[c] = (f >= 0 && f < d && a.tg.ref_mean) ? a.tg.ref_mean[f] : 0.f;
    }
    lsync();
}

// All tiles of one slot of one problem, in tile order (whole workgroup).
template <int KH, bool PIPE>
__device__ __forceinline__ void logreg_slot(LogregShared<PIPE>& sh, const LogregArgs& A,
                                            int64_t slot)
{
    using Cf = LCfg<PIPE>;
    constexpr int kTPP = Cf::tpp;
    constexpr int kBlocksPerThread = Cf::blocks_per_thread;
    constexpr int kFeatPerThread = Cf::feats_per_thread;
    const SweepArgs& a = A.a;
    const int tid = threadIdx.x;
    const int p = tid / kTPP, r = tid % kTPP;
    const int d = a.tg.d;
    const int T = a.T;
    const double s2r = a.tg.ref_sigma2;
    const double inv_s2r = 1.0 / s2r, half_inv_s2r = 0.5 / s2r, sref = sqrt(s2r);
        for (int64_t tile = slot; tile < a.ntiles; tile += a.S) {
            const bool first = (tile == slot);
            const int64_t n64 = tile * kLP + p;
            const bool valid = n64 < a.N;
            const uint32_t n = (uint32_t)n64;
            uint32_t accw = 0;
            // t = 0 draws X_0 ~ eta and caches ell, grad ell (always kept);
            // t >= 1 reweights, proposes, evaluates and corrects.
            for (int t = 0; t <= T; ++t) {
                const double beta = (t > 0) ? a.beta[t] : 0.0;
                const double eps = (t > 0) ? a.eps[t - 1] : 1.0;
                const double hh = 0.5 * eps * eps;
                if (t > 0 && tid < kWave) {
                    // reweight at the pre-move state and stream the moments
                    const int q = tid;
                    const bool vq = (tile * kLP + q) < a.N;
                    const double lwq = sh.lw[q];
                    const double lg = (beta - a.beta[t - 1]) * sh.ll[q];
                    double m3[3], s3[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        m3[i] = vq ? lwq + (double)i * lg : -INFINITY;
                        s3[i] = vq ? 1.0 : 0.0;
                    }
#pragma unroll
                    for (int o = 1; o < kWave; o <<= 1)
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            const double m2 = __shfl_xor(m3[i], o, kWave);
                            const double s2 = __shfl_xor(s3[i], o, kWave);
                            lse_merge(m3[i], s3[i], m2, s2);
                        }
                    if (q == 0) {
                        double* e = a.part + ((size_t)slot * (T + 1) + (t - 1)) * 4;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            const double L = lse_value(m3[i], s3[i]);
                            e[i] = first ? L : log_add(e[i], L);
                        }
                    }
                    sh.lw[q] = lwq + lg;
                }
                if (tid == 0) sh.cnt = 0u;
                // t = 0: x = m + s z;  t >= 1: x' = x + (eps^2/2) grad log pi_beta(x) + eps xi
                {
                    double fwd = 0.0, dle = 0.0;
#pragma unroll
                    for (int blk = 0; blk < kBlocksPerThread; ++blk) {
                        const int b = r + kTPP * blk;
                        if (4 * b < d) {
                            double zz[4];
                            normals4(a.key, n, (uint32_t)t, t > 0 ? kStreamMove : kStreamInit,
                                     (uint32_t)b, zz);
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int f = 4 * b + u;
                                if (f < d) {
                                    const int c = col_of(f, KH);
                                    const double mv = (double)sh.m[c];
                                    if (t == 0) {
                                        sh.prop[p][c] = (float)(mv + sref * zz[u]);
                                    } else {
                                        const double xv = (double)sh.theta[p][c];
                                        const double ga =
                                            -(xv - mv) * inv_s2r + beta * (double)sh.gl[p][c];
                                        const float xp = (float)(xv + hh * ga + eps * zz[u]);
                                        sh.prop[p][c] = xp;
                                        const double rr = (double)xp - xv - hh * ga;
                                        fwd = fma(rr, rr, fwd);
                                        const double d0 = xv - mv, d1 = (double)xp - mv;
                                        dle += d0 * d0 - d1 * d1;
                                    }
                                }
                            }
                        }
                    }
                    fwd = group_sum<kTPP>(fwd);
                    dle = group_sum<kTPP>(dle);
                    if (r == 0) {
                        sh.fwd[p] = fwd;
                        sh.dle[p] = dle;
                        const uint4 wd = draw_block(a.key, n, (uint32_t)t, kStreamAccept, 0u, 0u);
                        sh.logu[p] = (t > 0) ? log(word_uniform(wd.x)) : -INFINITY;
                    }
                }
                lsync();
                contraction<KH, PIPE>(sh, A.Xp, A.yp, A.n_pad);
                // Metropolis-Hastings correction (the initial draw is always kept)
                {
                    double bwd = 0.0;
#pragma unroll
                    for (int u = 0; u < kFeatPerThread; ++u) {
                        const int f = feat_of<kTPP>(r, u);
                        if (f < d) {
                            const int c = col_of(f, KH);
                            const double xv = (double)sh.theta[p][c];
                            const double xpv = (double)sh.prop[p][c];
                            const double gap =
                                -(xpv - (double)sh.m[c]) * inv_s2r + beta * (double)sh.glp[p][c];
                            const double rr = xv - xpv - hh * gap;
                            bwd = fma(rr, rr, bwd);
                        }
                    }
                    bwd = group_sum<kTPP>(bwd);
                    const double inv2e2 = 1.0 / (2.0 * eps * eps);
                    const double log_alpha = sh.dle[p] * half_inv_s2r + beta * (sh.llp[p] - sh.ll[p]) -
                                             bwd * inv2e2 + sh.fwd[p] * inv2e2;
                    const bool acc = (t == 0) || (sh.logu[p] < log_alpha);
                    if (acc) {
#pragma unroll
                        for (int u = 0; u < kFeatPerThread; ++u) {
                            const int f = feat_of<kTPP>(r, u);
                            if (f < d) {
                                const int c = col_of(f, KH);
                                sh.theta[p][c] = sh.prop[p][c];
                                sh.gl[p][c] = sh.glp[p][c];
                            }
                        }
                    }
                    const uint64_t bal = __ballot(acc && valid && r == 0);
                    if ((tid % kWave) == 0) atomicAdd(&sh.cnt, (uint32_t)__popcll(bal));
                    if (r == 0) {
                        if (acc) sh.ll[p] = sh.llp[p];
                        if (t == 0) sh.lw[p] = 0.0;
                        if (t > 0) {
                            accw |= (acc ? 1u : 0u) << ((t - 1) & 31);
                            if (((t - 1) & 31) == 31 || t == T) {
                                if (a.acc_bits && valid)
                                    a.acc_bits[(size_t)n64 * a.acc_words + (t - 1) / 32] = accw;
                                accw = 0;
                            }
                        }
                    }
                }
                lsync();
                if (t > 0 && tid == 0) {
                    double* e = a.part + ((size_t)slot * (T + 1) + (t - 1)) * 4;
                    e[3] = (first ? 0.0 : e[3]) + (double)sh.cnt;
                }
            }
            // log Z_hat contribution of the tile: entry T
            if (tid < kWave) {
                const bool vq = (tile * kLP + tid) < a.N;
                double m = vq ? sh.lw[tid] : -INFINITY, s = vq ? 1.0 : 0.0;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const double m2 = __shfl_xor(m, o, kWave);
                    const double s2 = __shfl_xor(s, o, kWave);
                    lse_merge(m, s, m2, s2);
                }
                if (tid == 0) {
                    double* e = a.part + ((size_t)slot * (T + 1) + T) * 4;
                    const double L = lse_value(m, s);
                    e[0] = first ? L : log_add(e[0], L);
                    e[1] = e[0];
                    e[2] = e[0];
                    e[3] = 0.0;
                }
                if (vq && a.lw_out) a.lw_out[tile * kLP + tid] = sh.lw[tid];
            }
            if (valid && a.x_out) {
#pragma unroll
                for (int u = 0; u < kFeatPerThread; ++u) {
                    const int f = feat_of<kTPP>(r, u);
                    if (f < d) a.x_out[(size_t)n64 * d + f] = sh.theta[p][col_of(f, KH)];
                }
            }
            lsync();
        }
}

template <int KH, bool PIPE>
__global__ void __launch_bounds__(LCfg<PIPE>::threads) k_oais_logreg(LogregArgs A)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared<PIPE>& sh = *reinterpret_cast<LogregShared<PIPE>*>(sh_raw);
    logreg_setup<KH, PIPE>(sh, A.a);
    for (int64_t slot = blockIdx.x; slot < A.a.S; slot += gridDim.x) logreg_slot<KH, PIPE>(sh, A, slot);
}

// Many logistic-regression problems with the same column half-width in one
// launch: each workgroup walks the work list of (problem, slot) items.
template <int KH, bool PIPE>
__global__ void __launch_bounds__(LCfg<PIPE>::threads)
    k_oais_logreg_batch(const LogregArgs* __restrict__ args, const int2* __restrict__ items,
                        int64_t nitems)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared<PIPE>& sh = *reinterpret_cast<LogregShared<PIPE>*>(sh_raw);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 item = items[it];
        const LogregArgs A = args[item.x];
        logreg_setup<KH, PIPE>(sh, A.a);
        logreg_slot<KH, PIPE>(sh, A, (int64_t)item.y);
        lsync();
    }
}

// ell and its gradient for given states (the same contraction as the sweep).
template <int KH, bool PIPE>
__global__ void __launch_bounds__(LCfg<PIPE>::threads) k_logreg_eval(const float* __restrict__ theta,
                                                           int64_t N, int d, const float* Xp,
                                                           const float* yp, int n_pad,
                                                           double* ell, float* grad)
{
    constexpr int kLThreads = LCfg<PIPE>::threads;
    constexpr int kTPP = LCfg<PIPE>::tpp;
    constexpr int kFeatPerThread = LCfg<PIPE>::feats_per_thread;
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared<PIPE>& sh = *reinterpret_cast<LogregShared<PIPE>*>(sh_raw);
    const int tid = threadIdx.x;
    const int p = tid / kTPP, r = tid % kTPP;
    for (int e = tid; e < kLP * kPs; e += kLThreads) (&sh.prop[0][0])[e] = 0.f;
    lsync();
    const int64_t n64 = (int64_t)blockIdx.x * kLP + p;
    const bool valid = n64 < N;
#pragma unroll
    for (int u = 0; u < kFeatPerThread; ++u) {
        const int f = feat_of<kTPP>(r, u);
        if (f < d && valid) sh.prop[p][col_of(f, KH)] = theta[(size_t)n64 * d + f];
    }
    lsync();
    contraction<KH, PIPE>(sh, Xp, yp, n_pad);
    if (valid) {
#pragma unroll
        for (int u = 0; u < kFeatPerThread; ++u) {
            const int f = feat_of<kTPP>(r, u);
            if (f < d) grad[(size_t)n64 * d + f] = sh.glp[p][col_of(f, KH)];
        }
        if (r == 0) ell[n64] = sh.llp[p];
    }
}

// ---------------------------------------------------------------------------
int64_t logreg_tiles(int64_t N) { return (N + kLP - 1) / kLP; }

static int n_pad_of(int n) { return ((n + kRowAlign - 1) / kRowAlign) * kRowAlign; }

size_t logreg_workspace_bytes(const TargetDev& tg, int64_t)
{
    const int np = n_pad_of(tg.n);
    return (size_t)np * 64 * sizeof(float) + (size_t)np * sizeof(float) + 256;
}

// The shape used for a launch.  FP32 MFMA needs two waves per SIMD to reach
// its peak (measured: 156 TFLOP/s with two, 145 with one), so the 8-wave
// workgroup is the default; OASMC_LOGREG_SHAPE=4 selects the pipelined
// 4-wave one.
static bool use_pipe()
{
    const char* v = getenv("OASMC_LOGREG_SHAPE");
    return v && v[0] == '4';
}

size_t logreg_shared_bytes()
{
    return use_pipe() ? sizeof(LogregShared<true>) : sizeof(LogregShared<false>);
}

template <int KH, bool PIPE>
static hipError_t launch_kh2(const LogregArgs& A, int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregShared<PIPE>);
    hipError_t e = hipFuncSetAttribute((const void*)k_oais_logreg<KH, PIPE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_oais_logreg<KH, PIPE>), dim3(grid), dim3(LCfg<PIPE>::threads), shb, st,
                       A);
    return hipGetLastError();
}

template <int KH>
static hipError_t launch_kh(const LogregArgs& A, int grid, hipStream_t st)
{
    return use_pipe() ? launch_kh2<KH, true>(A, grid, st) : launch_kh2<KH, false>(A, grid, st);
}

template <int KH, bool PIPE>
static hipError_t launch_eval_kh2(const float* theta, int64_t N, int d, const float* Xp,
                                  const float* yp, int n_pad, double* ell, float* grad,
                                  hipStream_t st)
{
    const size_t shb = sizeof(LogregShared<PIPE>);
    hipError_t e = hipFuncSetAttribute((const void*)k_logreg_eval<KH, PIPE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_logreg_eval<KH, PIPE>), dim3((unsigned)logreg_tiles(N)),
                       dim3(LCfg<PIPE>::threads), shb, st, theta, N, d, Xp, yp, n_pad, ell, grad);
    return hipGetLastError();
}

template <int KH>
static hipError_t launch_eval_kh(const float* theta, int64_t N, int d, const float* Xp,
                                 const float* yp, int n_pad, double* ell, float* grad,
                                 hipStream_t st)
{
    return use_pipe() ? launch_eval_kh2<KH, true>(theta, N, d, Xp, yp, n_pad, ell, grad, st)
                      : launch_eval_kh2<KH, false>(theta, N, d, Xp, yp, n_pad, ell, grad, st);
}

static void layout(const TargetDev& tg, void* ws, float** Xp, float** yp, int* np)
{
    *np = n_pad_of(tg.n);
    *Xp = static_cast<float*>(ws);
    *yp = *Xp + (size_t)(*np) * 64;
}

// Exact half-widths with a dedicated instantiation; other widths round up.
static int kh_for(int d);

int logreg_kh(int d) { return kh_for(d); }
int logreg_npad(int n) { return n_pad_of(n); }

hipError_t logreg_pack_into(const TargetDev& tg, float* Xp, float* yp, hipStream_t st)
{
    const int kh = kh_for(tg.d);
    if (kh < 0) return hipErrorInvalidValue;
    const int np = n_pad_of(tg.n);
    const int64_t total = (int64_t)np * 64;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_logreg_pack, dim3(blocks), dim3(256), 0, st, tg.X, tg.y, tg.n, tg.d, kh,
                       np, Xp, yp);
    return hipGetLastError();
}

template <int KH, bool PIPE>
static hipError_t launch_batch_kh2(const LogregArgs* args, const int2* items, int64_t nitems,
                                   int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregShared<PIPE>);
    hipError_t e = hipFuncSetAttribute((const void*)k_oais_logreg_batch<KH, PIPE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_oais_logreg_batch<KH, PIPE>), dim3(grid), dim3(LCfg<PIPE>::threads), shb,
                       st, args, items, nitems);
    return hipGetLastError();
}

hipError_t logreg_prepare(const TargetDev& tg, void* ws, hipStream_t st)
{
    float *Xp, *yp;
    int np;
    layout(tg, ws, &Xp, &yp, &np);
    const int kh = kh_for(tg.d);
    if (kh < 0) return hipErrorInvalidValue;
    // columns are packed with the instantiated half-width, so features
    // [0, KH) and [KH, d) land in columns [0, KH) and [32, 32 + d - KH)
    const int64_t total = (int64_t)np * 64;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_logreg_pack, dim3(blocks), dim3(256), 0, st, tg.X, tg.y, tg.n, tg.d, kh,
                       np, Xp, yp);
    return hipGetLastError();
}

#define OASMC_KH_LIST(X) X(4) X(8) X(12) X(16) X(20) X(25) X(32)

static int kh_for(int d)
{
    const int kh = (d + 1) / 2;
    const int list[] = {4, 8, 12, 16, 20, 25, 32};
    for (int v : list)
        if (kh <= v) return v;
    return -1;
}

hipError_t launch_oais_logreg(const SweepArgs& a, int cus, void* ws, size_t, hipStream_t st)
{
    LogregArgs A{};
    A.a = a;
    float *Xp, *yp;
    int np;
    const int kh = kh_for(a.tg.d);
    if (kh < 0) return hipErrorInvalidValue;
    layout(a.tg, ws, &Xp, &yp, &np);
    A.Xp = Xp;
    A.yp = yp;
    A.n_pad = np;
    const int grid = (int)std::min<int64_t>(a.S, (int64_t)cus);
    switch (kh) {
#define OASMC_KH_CASE(K) case K: return launch_kh<K>(A, grid, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_oais_logreg_batch(int kh, const LogregArgs* args, const int2* items,
                                   int64_t nitems, int grid, hipStream_t st)
{
    const bool pipe = use_pipe();
    switch (kh) {
#define OASMC_KH_CASE(K) \
    case K: return pipe ? launch_batch_kh2<K, true>(args, items, nitems, grid, st) \
                        : launch_batch_kh2<K, false>(args, items, nitems, grid, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_logreg_eval(const TargetDev& tg, const float* theta, int64_t N, double* ell,
                              float* grad, void* ws, hipStream_t st)
{
    float *Xp, *yp;
    int np;
    const int kh = kh_for(tg.d);
    if (kh < 0) return hipErrorInvalidValue;
    layout(tg, ws, &Xp, &yp, &np);
    switch (kh) {
#define OASMC_KH_CASE(K) case K: return launch_eval_kh<K>(theta, N, tg.d, Xp, yp, np, ell, grad, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace oasmc
