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
//
// Labels are folded into the rows: row i is stored as s_i X_i with
// s_i = 2 y_i - 1, so the first product gives u_i = s_i z_i and, with
// sigma the logistic function,
//     y_i z_i - softplus(z_i) = log sigma(u_i) = min(u_i, 0) + log max(s_i, 1 - s_i),
//     (y_i - sigma(z_i)) X_i  = s_i (s_i X_i)   with s_i = sigma(-u_i) = 1 / (1 + exp(u_i)),
// i.e. the epilogue needs no labels and the second product takes s directly
// (1 / (1 + exp(u)) has the exact limits 0 and 1 at both ends).  The factor
// max(s, 1 - s) lies in [1/2, 1], so a running product over a chunk's rows
// cannot underflow and its log is taken once per chunk.  The rounding of
// exp(u) reaches ell with the weight sigma(-|u|) of the bounded form (small
// for well-classified rows), not with the weight sigma(u) that
// u - log(1 + exp(u)) would give it (which biases ell by the exponential's
// rounding over many rows).  Padding rows are zero, so u = 0 and they add
// nothing to either product; their factor 1/2 in the running product is
// divided out.
#include "kernels.hpp"

namespace oasmc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
// The packed rows (and the schedule) are read through global-address-space
// pointers: the pointers arrive through a descriptor in memory, so the
// compiler cannot infer the address space, and flat loads would share the LDS
// wait counter (every LDS wait in the chunk loop would then also wait for the
// next chunk's prefetch).
typedef __attribute__((address_space(1))) const float gmem_f;
typedef __attribute__((address_space(1))) const floatx4 gmem_f4;

constexpr int kLP = 64;          // particles per tile
constexpr int kRows = 32;        // data rows per chunk
constexpr int kSt = 68;          // floats per staged row: 64 columns + 4 (bank offset)
constexpr int kPs = 68;          // floats per particle row in LDS
constexpr int kRowAlign = kRows * 8;

// Workgroup shape: 8 waves, two per SIMD (256 registers per lane).
struct LCfg {
    static constexpr int waves = 8;
    static constexpr int threads = waves * kWave;
    static constexpr int tpp = threads / kLP;   // threads per particle, scalar phases
    static constexpr int blocks_per_thread = 16 / tpp;
    static constexpr int feats_per_thread = 4 * blocks_per_thread;
};

struct LogregShared {
    float theta[kLP][kPs];  // current states (packed columns)
    float prop[kLP][kPs];   // proposals
    float gl[kLP][kPs];     // gradient of ell at theta
    float glp[kLP][kPs];    // gradient of ell at prop
    alignas(16) float stage[LCfg::waves][kRows][kSt];  // 128-bit staging stores
    double ll[kLP], llp[kLP], lw[kLP];
    double llpart[LCfg::waves][kLP];
    double fwd[kLP], dle[kLP], logu[kLP];
    float m[64];
    uint32_t cnt;
    uint32_t item;  // the batch item claimed by the workgroup
};

static_assert(sizeof(LogregShared::stage) >= sizeof(float) * (LCfg::waves / 2) * 64 * kWave,
              "the gradient reduction fits in the staging buffers");

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads, so prefetches (the next step's schedule values,
// chunk 0 of the next evaluation) stay in flight across it.  Waves of a tile
// exchange data through LDS only.
__device__ __forceinline__ void lsync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__host__ __device__ __forceinline__ int col_of(int f, int KH) { return f < KH ? f : 32 + f - KH; }

// Packs X (n x d, row-major) into Xp (n_pad x 64) with the column map above,
// each row multiplied by s_i = 2 y_i - 1 (a label y_i != 0 counts as 1);
// padding rows are zero.
__global__ void k_logreg_pack(const float* __restrict__ X, const float* __restrict__ y, int n,
                              int d, int KH, int n_pad, float* __restrict__ Xp)
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
        const bool in = i < n && f >= 0 && f < d;
        const float v = in ? X[(int64_t)i * d + f] : 0.f;
        Xp[e] = (in && y[i] == 0.f) ? -v : v;
    }
}

// Row of the 32-row chunk that accumulator element q of lane half h holds
// (the 32 x 32 output layout of v_mfma_f32_32x32x2f32).
__device__ __forceinline__ int slot_row(int q, int h) { return 8 * (q / 4) + 4 * h + (q % 4); }

// The epilogue of one signed logit u, in two halves:
//   a: w = 1 + exp(u)  (exp(u) = 2^(u log2 e), +inf above about 88)
//   b: s = 1 / w, which replaces u as the second product's operand; min(u, 0)
//      into the running sum and max(s, 1 - s) into the running product whose
//      log2 gives the rest of the chunk's rows' ell (one log per chunk).
// Seven VALU instructions and two transcendentals per logit.  On gfx950 FP32
// matrix-core instructions and VALU instructions do not run concurrently on
// a SIMD (measured: the time of an interleaved sequence is the sum of the
// two), so every VALU instruction here costs matrix-core time; the halves are
// placed between the gradient products only to keep the wave's dependencies
// short.
constexpr float kLog2eF = 1.44269504088896341f;

struct EpiTmp {
    float w;
};

__device__ __forceinline__ void epi_a(float u, EpiTmp& t)
{
    t.w = 1.0f + __builtin_amdgcn_exp2f(u * kLog2eF);
    // an empty volatile asm that consumes and redefines the value pins this
    // half where it is written (the IR passes would otherwise sink it next to
    // its uses in the second half)
    asm volatile("" : "+v"(t.w));
}

__device__ __forceinline__ float epi_b(float u, const EpiTmp& t, float& lin, float& prod)
{
    const float sg = __builtin_amdgcn_rcpf(t.w);
    // min(u, 0) = (u - |u|) / 2 and max(s, 1 - s) = 1/2 + |s - 1/2|: absolute
    // values are free source modifiers, where fminf / fmaxf would add NaN
    // canonicalisations
    lin = fmaf(0.5f, u - fabsf(u), lin);
    prod *= 0.5f + fabsf(sg - 0.5f);
    return sg;
}

// Padding rows among the 16 rows a lane half h holds in a chunk whose first
// L rows are data (rows slot_row(q, h): blocks of 4 at 8 b + 4 h).
__device__ __forceinline__ int padding_rows(int L, int h)
{
    if (L >= kRows) return 0;
    int c = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) c += min(4, max(0, 8 * b + 4 * h + 4 - L));
    return c;
}

// One 32-row chunk's share of a lane: row l / 2, columns 32 (l % 2) ..+31
// (8 x 16 bytes of the packed rows).
struct Slice {
    floatx4 v0, v1, v2, v3, v4, v5, v6, v7;
};

// Rows [r0, r0 + rows_w) of the packed data belong to wave w of the tile.
__device__ __forceinline__ int wave_rows(int n_pad) { return n_pad / LCfg::waves; }

// Loads chunk c of this wave's rows.  The address-space cast is taken on the
// base pointer (a cast of each derived address can fold back into a flat
// access, and flat loads would share the LDS wait counter).
__device__ __forceinline__ Slice fetch_slice(const float* Xp, int n_pad, int c)
{
    const int l = threadIdx.x % kWave;
    const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * wave_rows(n_pad);
    gmem_f* const Xg = (gmem_f*)Xp;
    const gmem_f4* src = (const gmem_f4*)(Xg + (size_t)(r0 + c * kRows + l / 2) * 64 + (l % 2) * 32);
    Slice t;
    t.v0 = src[0]; t.v1 = src[1]; t.v2 = src[2]; t.v3 = src[3];
    t.v4 = src[4]; t.v5 = src[5]; t.v6 = src[6]; t.v7 = src[7];
    return t;
}

__device__ __forceinline__ void put_slice(float (*stc)[kSt], const Slice& t)
{
    const int l = threadIdx.x % kWave;
    floatx4* dst = reinterpret_cast<floatx4*>(&stc[l / 2][(l % 2) * 32]);
    dst[0] = t.v0; dst[1] = t.v1; dst[2] = t.v2; dst[3] = t.v3;
    dst[4] = t.v4; dst[5] = t.v5; dst[6] = t.v6; dst[7] = t.v7;
}

// Feature tiles of the gradient product: the packed halves (features
// [0, KH) in columns 0 .. KH - 1, [KH, 2 KH) in columns 32 .. 32 + KH - 1)
// take one 32-column tile each, or, for KH <= 16, share one tile whose
// column j reads packed column col_of(j, KH) (feature j): half the gradient
// instructions for d <= 32.
template <int KH>
struct GradTiles {
    static constexpr int nft = KH <= 16 ? 1 : 2;
};

// The 32 NFT gradient accumulators of a lane as 8 NFT float4 (element 4 k + i
// is G[g][ft][q] with (g * NFT + ft) * 16 + q = 4 k + i), stored
// lane-interleaved (float4 k of lane l at k * 64 + l) so every 128-bit LDS
// access is conflict-free.
template <int NFT>
__device__ __forceinline__ void store_grad(floatx4* dst, const floatx16 (&G)[2][NFT], int l)
{
#pragma unroll
    for (int k = 0; k < 8 * NFT; ++k) {
        const floatx16& v = G[k / (4 * NFT)][(k / 4) % NFT];
        const int q = 4 * (k % 4);
        dst[k * kWave + l] = floatx4{v[q], v[q + 1], v[q + 2], v[q + 3]};
    }
}

template <int NFT>
__device__ __forceinline__ void add_grad(floatx16 (&G)[2][NFT], const floatx4* src, int l)
{
#pragma unroll
    for (int k = 0; k < 8 * NFT; ++k) {
        floatx16& v = G[k / (4 * NFT)][(k / 4) % NFT];
        const int q = 4 * (k % 4);
        const floatx4 u = src[k * kWave + l];
        v[q] += u[0];
        v[q + 1] += u[1];
        v[q + 2] += u[2];
        v[q + 3] += u[3];
    }
}

// ell and grad ell at sh.prop for the 64 particles of the tile; results in
// sh.llp (binary64) and sh.glp (packed columns).  All threads participate.
// n is the number of data rows.  `first` holds this wave's chunk 0 on entry;
// on exit it holds chunk 0 again, loaded at the end so that the next call
// finds it in registers.
template <int KH>
__device__ __forceinline__ void contraction(LogregShared& sh, const float* __restrict__ Xp, int n,
                                            int n_pad, Slice& first)
{
    constexpr int kLWaves = LCfg::waves;
    constexpr double kLn2 = 0.693147180559945309;
    constexpr int NFT = GradTiles<KH>::nft;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    const int l = tid % kWave;
    const int h = l / 32;
    const int j = l % 32;
    // packed column of this lane's gradient column in each feature tile
    const int cb0 = (NFT == 1) ? col_of(j, KH) : j;

    floatx16 G[2][NFT];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int ft = 0; ft < NFT; ++ft)
#pragma unroll
            for (int q = 0; q < 16; ++q) G[g][ft][q] = 0.f;
    double llacc[2] = {0.0, 0.0};

    const int nchunks = wave_rows(n_pad) / kRows;
    const int r0 = w * wave_rows(n_pad);
    float(*stc)[kSt] = sh.stage[w];

    // the next chunk's slice is loaded into registers while the current
    // chunk is consumed from the wave's LDS staging buffer
    floatx16 acc[2];
    Slice ahead = first;
    for (int c = 0; c < nchunks; ++c) {
        put_slice(stc, ahead);
        wsync();
        ahead = fetch_slice(Xp, n_pad, min(c + 1, nchunks - 1));
        // signed logits of the chunk, transposed: acc[g] = X'_chunk . Theta_g^T
        // (k-step s: lane half h holds column 32 h + s of its row and of its
        // particle)
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[g][q] = 0.f;
#pragma unroll
        for (int s = 0; s < KH; ++s) {
            const float a = stc[j][32 * h + s];
#pragma unroll
            for (int g = 0; g < 2; ++g)
                acc[g] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, sh.prop[32 * g + j][32 * h + s],
                                                            acc[g], 0, 0, 0);
        }
        // row slots: the epilogue of slot q + 1 is issued between the four
        // gradient products of slot q (G[g][ft] += sigma(-u_g)^T X'_ft over
        // its rows)
        float lin[2] = {0.f, 0.f}, prod[2] = {1.f, 1.f};
        EpiTmp t0, t1;
        epi_a(acc[0][0], t0);
        acc[0][0] = epi_b(acc[0][0], t0, lin[0], prod[0]);
        epi_a(acc[1][0], t1);
        acc[1][0] = epi_b(acc[1][0], t1, lin[1], prod[1]);
        if constexpr (NFT == 2) {
            float bx0 = stc[slot_row(0, h)][j], bx1 = stc[slot_row(0, h)][32 + j];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int qn = (q < 15) ? q + 1 : 15;
                const int in = slot_row(qn, h);
                const float nbx0 = stc[in][j], nbx1 = stc[in][32 + j];
                G[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[0][q], bx0, G[0][0], 0, 0, 0);
                if (q < 15) epi_a(acc[0][qn], t0);
                __builtin_amdgcn_sched_barrier(0);
                G[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[1][q], bx0, G[1][0], 0, 0, 0);
                if (q < 15) acc[0][qn] = epi_b(acc[0][qn], t0, lin[0], prod[0]);
                __builtin_amdgcn_sched_barrier(0);
                G[0][NFT - 1] =
                    __builtin_amdgcn_mfma_f32_32x32x2f32(acc[0][q], bx1, G[0][NFT - 1], 0, 0, 0);
                if (q < 15) epi_a(acc[1][qn], t1);
                __builtin_amdgcn_sched_barrier(0);
                G[1][NFT - 1] =
                    __builtin_amdgcn_mfma_f32_32x32x2f32(acc[1][q], bx1, G[1][NFT - 1], 0, 0, 0);
                if (q < 15) acc[1][qn] = epi_b(acc[1][qn], t1, lin[1], prod[1]);
                __builtin_amdgcn_sched_barrier(0);
                bx0 = nbx0;
                bx1 = nbx1;
            }
        } else {
            // one feature tile: the two halves of each slot's epilogue go
            // between its two gradient products
            float bx = stc[slot_row(0, h)][cb0];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int qn = (q < 15) ? q + 1 : 15;
                const float nbx = stc[slot_row(qn, h)][cb0];
                G[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[0][q], bx, G[0][0], 0, 0, 0);
                if (q < 15) {
                    epi_a(acc[0][qn], t0);
                    epi_a(acc[1][qn], t1);
                }
                __builtin_amdgcn_sched_barrier(0);
                G[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[1][q], bx, G[1][0], 0, 0, 0);
                if (q < 15) {
                    acc[0][qn] = epi_b(acc[0][qn], t0, lin[0], prod[0]);
                    acc[1][qn] = epi_b(acc[1][qn], t1, lin[1], prod[1]);
                }
                __builtin_amdgcn_sched_barrier(0);
                bx = nbx;
            }
        }
        // the chunk's data rows: the sum of min(u, 0) plus the log of the
        // product (the padding rows' exact factors of 1/2 divided out), one log
        // per chunk
        const int npad_rows = padding_rows(n - (r0 + c * kRows), h);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const float lp = __builtin_amdgcn_logf(__builtin_amdgcn_ldexpf(prod[g], npad_rows));
            llacc[g] += (double)lin[g] + kLn2 * (double)lp;
        }
        wsync();
    }

    // per-particle log-likelihood: halves of the wave, then waves in order
#pragma unroll
    for (int g = 0; g < 2; ++g) llacc[g] += __shfl_xor(llacc[g], 32, kWave);
    if (h == 0) {
        sh.llpart[w][j] = llacc[0];
        sh.llpart[w][32 + j] = llacc[1];
    }
    lsync();  // every wave is done with its staging buffer

    // gradient: G_w + G_{w+4} on waves 0..3, then wave 0 adds waves 1, 2, 3
    // in that order (fixed tree), through four 16 KB slots of the staging area
    floatx4* red = reinterpret_cast<floatx4*>(&sh.stage[0][0][0]);
    constexpr int kSlot = 8 * NFT * kWave;  // float4 per slot
    if (w >= 4) store_grad(red + (w - 4) * kSlot, G, l);
    if (tid < kLP) {
        double s = 0.0;
        for (int ww = 0; ww < kLWaves; ++ww) s += sh.llpart[ww][tid];
        sh.llp[tid] = s;
    }
    lsync();
    if (w < 4) {
        add_grad(G, red + w * kSlot, l);
        store_grad(red + w * kSlot, G, l);  // slot w is read only by wave w
    }
    lsync();
    // ((slot 0 + slot 1) + slot 2) + slot 3: wave w sums float4 NFT w ..
    // NFT w + NFT - 1 of every lane and writes those gradient entries
#pragma unroll
    for (int kk = 0; kk < NFT; ++kk) {
        const int k = NFT * w + kk;
        floatx4 v = red[k * kWave + l];
#pragma unroll
        for (int sl = 1; sl < 4; ++sl) {
            const floatx4 u = red[sl * kSlot + k * kWave + l];
            v[0] += u[0];
            v[1] += u[1];
            v[2] += u[2];
            v[3] += u[3];
        }
        // float4 k holds G[g][ft][q .. q + 3], (g * NFT + ft) * 16 + q = 4 k
        const int g = k / (4 * NFT), ft = (k / 4) % NFT, q0 = 4 * (k % 4);
        const int col = (NFT == 1) ? cb0 : 32 * ft + j;
#pragma unroll
        for (int i = 0; i < 4; ++i) sh.glp[32 * g + slot_row(q0 + i, h)][col] = v[i];
    }
    // chunk 0 of the next evaluation (the rows do not change between steps)
    first = fetch_slice(Xp, n_pad, 0);
    lsync();
}


// Particle p's thread r (of tpp) handles the normal blocks r, r + tpp,
// r + 2 tpp, ... i.e. the features 4b..4b+3 of those blocks (below d).
template <int TPP>
__device__ __forceinline__ int feat_of(int r, int u) { return 4 * (r + TPP * (u / 4)) + (u % 4); }

// The parameters shared by every tile of a problem: zero the particle arrays
// (columns beyond d stay zero) and stage the reference mean in packed columns.
template <int KH>
__device__ __forceinline__ void logreg_setup(LogregShared& sh, const LogregArgs& A)
{
    constexpr int kLThreads = LCfg::threads;
    const SweepArgs& a = A.a;
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
template <int KH>
__device__ __forceinline__ void logreg_slot(LogregShared& sh, const LogregArgs& A,
                                            int64_t slot)
{
    using Cf = LCfg;
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
    // the schedule through global-address-space pointers (see fetch_slice)
    typedef __attribute__((address_space(1))) const double gmem_d;
    gmem_d* const beta_g = (gmem_d*)a.beta;
    gmem_d* const eps_g = (gmem_d*)a.eps;
    Slice chunk0 = fetch_slice(A.Xp, A.n_pad, 0);
        for (int64_t tile = slot; tile < a.ntiles; tile += a.S) {
            const bool first = (tile == slot);
            const int64_t n64 = tile * kLP + p;
            const bool valid = n64 < a.N;
            const uint32_t n = (uint32_t)n64;
            uint32_t accw = 0;
            // beta_t and eps_t of the next step are loaded one step ahead
            double beta_next = (T >= 1) ? beta_g[1] : 1.0;
            double eps_next = (T >= 1) ? eps_g[0] : 1.0;
            double beta_prev = 0.0;
            // t = 0 draws X_0 ~ eta and caches ell, grad ell (always kept);
            // t >= 1 reweights, proposes, evaluates and corrects.
            for (int t = 0; t <= T; ++t) {
                const double beta = (t > 0) ? beta_next : 0.0;
                const double eps = (t > 0) ? eps_next : 1.0;
                if (t > 0 && t < T) {
                    beta_next = beta_g[t + 1];
                    eps_next = eps_g[t];
                }
                const double hh = 0.5 * eps * eps;
                if (t > 0 && tid < 3 * kWave) {
                    // moment i = wave index of the pre-move weights times
                    // g_t^i: a max and a sum of exps over the 64 particles
                    // (the weights themselves advance in the correction)
                    const int i = __builtin_amdgcn_readfirstlane(tid / kWave), q = tid % kWave;
                    const bool vq = (tile * kLP + q) < a.N;
                    const double lg = (beta - beta_prev) * sh.ll[q];
                    const double x = vq ? (i == 0 ? sh.lw[q] : sh.lw[q] + (double)i * lg) : -INFINITY;
                    double m = x;
#pragma unroll
                    for (int o = 1; o < kWave; o <<= 1) m = fmax(m, __shfl_xor(m, o, kWave));
                    double sum = (m > -INFINITY && vq) ? exp(x - m) : 0.0;
#pragma unroll
                    for (int o = 1; o < kWave; o <<= 1) sum += __shfl_xor(sum, o, kWave);
                    if (q == 0) {
                        double* e = a.part + ((size_t)slot * (T + 1) + (t - 1)) * 4;
                        const double L = lse_value(m, sum);
                        e[i] = first ? L : log_add(e[i], L);
                    }
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
                            normals4<false>(a.key, n, (uint32_t)t, t > 0 ? kStreamMove : kStreamInit,
                                     (uint32_t)b, zz, 0u, d - 4 * b);
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
                        const uint4 wd = draw_block<false>(a.key, n, (uint32_t)t, kStreamAccept, 0u, 0u);
                        sh.logu[p] = (t > 0) ? log(word_uniform(wd.x)) : -INFINITY;
                    }
                }
                lsync();
                contraction<KH>(sh, A.Xp, a.tg.n, A.n_pad, chunk0);
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
                        // the weight advances by the increment the moments
                        // used, at the pre-move log-likelihood
                        sh.lw[p] = (t == 0) ? 0.0 : sh.lw[p] + (beta - beta_prev) * sh.ll[p];
                        if (acc) sh.ll[p] = sh.llp[p];
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
                beta_prev = beta;
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

template <int KH>
__global__ void __launch_bounds__(LCfg::threads) k_oais_logreg(LogregArgs A)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared& sh = *reinterpret_cast<LogregShared*>(sh_raw);
    logreg_setup<KH>(sh, A);
    for (int64_t slot = blockIdx.x; slot < A.a.S; slot += gridDim.x) logreg_slot<KH>(sh, A, slot);
}

// The next work item of a batched launch for the whole workgroup: claimed
// from the work counter (zero at the launch; the items come longest first, so
// each one goes to the first workgroup that becomes idle, a greedy balance of
// items whose lengths differ by their problems' T, N and n), or, without a
// counter, the static round robin.  Every thread calls it; a claim passes
// through LDS (the workgroup's previous reads of `slot` lie behind barriers).
__device__ __forceinline__ int64_t next_item(uint32_t* next, uint32_t& slot, int64_t prev)
{
    if (next == nullptr) return prev < 0 ? (int64_t)blockIdx.x : prev + gridDim.x;
    if (threadIdx.x == 0) slot = atomicAdd(next, 1u);
    lsync();
    return (int64_t)slot;
}

// Many logistic-regression problems with the same column half-width in one
// launch: the workgroups walk the work list of (problem, slot) items, claimed
// from the work counter (DYN) or in the static round robin (one problem,
// whose slots are equal; that instantiation carries no claiming code).
template <int KH, bool DYN>
__global__ void __launch_bounds__(LCfg::threads)
    k_oais_logreg_batch(const LogregArgs* __restrict__ args, const int2* __restrict__ items,
                        int64_t nitems, uint32_t* next)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared& sh = *reinterpret_cast<LogregShared*>(sh_raw);
    for (int64_t it = DYN ? next_item(next, sh.item, -1) : (int64_t)blockIdx.x; it < nitems;
         it = DYN ? next_item(next, sh.item, it) : it + gridDim.x) {
        const int2 item = items[it];
        const LogregArgs A = args[item.x];
        logreg_setup<KH>(sh, A);
        logreg_slot<KH>(sh, A, (int64_t)item.y);
        lsync();
    }
}

// ell and its gradient for given states (the same contraction as the sweep).
template <int KH>
__global__ void __launch_bounds__(LCfg::threads) k_logreg_eval(const float* __restrict__ theta,
                                                           int64_t N, int d, const float* Xp,
                                                           int n, int n_pad,
                                                           double* ell, float* grad)
{
    constexpr int kLThreads = LCfg::threads;
    constexpr int kTPP = LCfg::tpp;
    constexpr int kFeatPerThread = LCfg::feats_per_thread;
    extern __shared__ __align__(16) char sh_raw[];
    LogregShared& sh = *reinterpret_cast<LogregShared*>(sh_raw);
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
    Slice chunk0 = fetch_slice(Xp, n_pad, 0);
    contraction<KH>(sh, Xp, n, n_pad, chunk0);
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
// Wide variant, 64 < d <= 256: the features sit in NP panels of 64 packed
// columns (panel p holds features p F .. p F + F - 1, F = ceil(d / NP), with the
// same split of each panel into two halves of width KHW = ceil(F / 2) as the
// 64-column layout), so the logits' K loop runs over the panels.  A tile has
// 32 particles (one 32-particle group of the MFMA products), so a wave keeps
// the gradient tiles of every panel (NP x 2 x 16 accumulators) and LDS holds
// the states, proposals and one staged panel per wave; the cached gradients
// (at the state and at the proposal) live in HBM, [N][NP 64] in packed column
// order.  Per 32-row chunk a wave stages each panel twice: once for the
// logits, once after the epilogue for the gradient (the second pass re-reads
// the panels from L2), with the global load of the next panel issued one stage
// ahead.  The eight waves' gradient tiles are summed panel by panel in wave
// order through the staging area.
// ---------------------------------------------------------------------------
constexpr int kLPW = 32;  // particles per tile, wide variant

struct LCfgW {
    static constexpr int waves = 8;
    static constexpr int threads = waves * kWave;
    static constexpr int tpp = threads / kLPW;  // threads per particle, scalar phases
};

template <int NP>
struct LogregSharedW {
    // rows of NP 64 + 1 floats: lane (h, j) of an MFMA operand read hits
    // bank j + 32 h (conflict-free on 64 banks)
    float theta[kLPW][NP * 64 + 1];
    float prop[kLPW][NP * 64 + 1];
    alignas(16) float stage[LCfgW::waves][kRows][kSt];
    double ll[kLPW], llp[kLPW], lw[kLPW];
    double llpart[LCfgW::waves][kLPW];
    double fwd[kLPW], dle[kLPW], logu[kLPW];
    float m[NP * 64];
    uint32_t cnt;
    uint32_t item;  // the batch item claimed by the workgroup
};

static_assert(sizeof(LogregSharedW<4>::stage) >= 16 * 8 * LCfgW::waves * kWave,
              "the wide gradient reduction fits in the staging buffers");
static_assert(sizeof(LogregSharedW<4>) <= 160 * 1024, "the wide tile fits in LDS");

// Panel widths of the wide layout.
__host__ __device__ inline int wide_np(int d) { return (d + 63) / 64; }
__host__ __device__ inline int wide_f(int d) { return (d + wide_np(d) - 1) / wide_np(d); }
__host__ __device__ inline int wide_khw(int d) { return (wide_f(d) + 1) / 2; }
__host__ __device__ inline int col_of_wide(int f, int F, int KHW)
{
    const int p = f / F, l = f - p * F;
    return 64 * p + (l < KHW ? l : 32 + l - KHW);
}

__global__ void k_logreg_pack_wide(const float* __restrict__ X, const float* __restrict__ y,
                                   int n, int d, int cols, int n_pad, float* __restrict__ Xp)
{
    const int F = wide_f(d), KHW = wide_khw(d);
    const int64_t total = (int64_t)n_pad * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / cols), c = (int)(e % cols);
        const int p = c / 64, cc = c % 64;
        int l = -1;
        if (cc < 32) {
            if (cc < KHW) l = cc;
        } else if (cc - 32 + KHW < F) {
            l = KHW + cc - 32;
        }
        const int f = p * F + l;
        const bool in = i < n && l >= 0 && f < d;
        const float v = in ? X[(int64_t)i * d + f] : 0.f;
        Xp[e] = (in && y[i] == 0.f) ? -v : v;
    }
}

// The chunk slice of panel p: row l / 2, columns 64 p + 32 (l % 2) .. + 31.
__device__ __forceinline__ Slice fetch_slice_w(const float* Xp, int n_pad, int cols, int c, int p)
{
    const int l = threadIdx.x % kWave;
    const int r0 = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * wave_rows(n_pad);
    gmem_f* const Xg = (gmem_f*)Xp;
    const gmem_f4* src =
        (const gmem_f4*)(Xg + (size_t)(r0 + c * kRows + l / 2) * cols + 64 * p + (l % 2) * 32);
    Slice t;
    t.v0 = src[0]; t.v1 = src[1]; t.v2 = src[2]; t.v3 = src[3];
    t.v4 = src[4]; t.v5 = src[5]; t.v6 = src[6]; t.v7 = src[7];
    return t;
}

// ell and grad ell at sh.prop for the tile's 32 particles: ell into sh.llp,
// the gradient into glp (HBM, packed columns) of particles pbase .. pbase + 31
// (rows past N are written too: the buffers cover whole tiles).
template <int NP>
__device__ __forceinline__ void contraction_w(LogregSharedW<NP>& sh, const float* __restrict__ Xp,
                                              int n, int n_pad, int khw, float* glp, int64_t pbase)
{
    constexpr int kW = LCfgW::waves;
    constexpr int cols = NP * 64;
    constexpr double kLn2 = 0.693147180559945309;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int l = tid % kWave;
    const int h = l / 32;
    const int j = l % 32;
    floatx16 G[NP][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int ft = 0; ft < 2; ++ft)
#pragma unroll
            for (int q = 0; q < 16; ++q) G[p][ft][q] = 0.f;
    double llacc = 0.0;
    const int nchunks = wave_rows(n_pad) / kRows;
    const int r0 = w * wave_rows(n_pad);
    float(*stc)[kSt] = sh.stage[w];
    // 2 NP stages per chunk (the panels for the logits, then again for the
    // gradient); `ahead` holds the next stage's slice, loaded while the
    // current one is consumed from the wave's staging buffer
    Slice ahead = fetch_slice_w(Xp, n_pad, cols, 0, 0);
    for (int c = 0; c < nchunks; ++c) {
        // signed logits of the chunk, transposed, accumulated over the panels
        floatx16 acc;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            put_slice(stc, ahead);
            wsync();
            ahead = fetch_slice_w(Xp, n_pad, cols, c, (p + 1) % NP);
#pragma nounroll
            for (int s = 0; s < khw; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(stc[j][32 * h + s],
                                                           sh.prop[j][64 * p + 32 * h + s], acc,
                                                           0, 0, 0);
            wsync();
        }
        // the epilogue (see epi_a, epi_b): acc becomes sigma(-u)
        {
            float prod = 1.f, lin = 0.f;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                EpiTmp tq;
                epi_a(acc[q], tq);
                acc[q] = epi_b(acc[q], tq, lin, prod);
            }
            const int npad_rows = padding_rows(n - (r0 + c * kRows), h);
            const float lp = __builtin_amdgcn_logf(__builtin_amdgcn_ldexpf(prod, npad_rows));
            llacc += (double)lin + kLn2 * (double)lp;
        }
        // gradient, panel by panel: G[p][ft] += sigma(-u)^T X'_{p, ft}
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            put_slice(stc, ahead);
            wsync();
            if (p + 1 < NP)
                ahead = fetch_slice_w(Xp, n_pad, cols, c, p + 1);
            else
                ahead = fetch_slice_w(Xp, n_pad, cols, min(c + 1, nchunks - 1), 0);
            if (NP == 1 && khw <= 16) {
                // a single panel of at most 32 features: one gradient tile,
                // whose column j reads packed column col_of(j, khw) (feature
                // j): half the gradient instructions (wave-uniform branch)
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    G[p][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                        acc[q], stc[slot_row(q, h)][col_of(j, khw)], G[p][0], 0, 0, 0);
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = slot_row(q, h);
                    G[p][0] =
                        __builtin_amdgcn_mfma_f32_32x32x2f32(acc[q], stc[row][j], G[p][0], 0, 0, 0);
                    G[p][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(acc[q], stc[row][32 + j], G[p][1],
                                                                 0, 0, 0);
                }
            }
            wsync();
        }
    }
    // per-particle log-likelihood: halves of the wave, then the waves in order
    llacc += __shfl_xor(llacc, 32, kWave);
    if (h == 0) sh.llpart[w][j] = llacc;
    lsync();  // every wave is done with its staging buffer
    if (tid < kLPW) {
        double sacc = 0.0;
        for (int ww = 0; ww < kW; ++ww) sacc += sh.llpart[ww][tid];
        sh.llp[tid] = sacc;
    }
    // gradient, panel by panel: every wave stores its 2 tiles (8 float4 per
    // lane, lane-interleaved), then wave w sums float4 w of every lane over the
    // waves in order and writes those entries
    floatx4* red = reinterpret_cast<floatx4*>(&sh.stage[0][0][0]);
    constexpr int kSlot = 8 * kWave;  // float4 per wave slot
    if constexpr (NP == 1) {
        // a single panel; with one gradient tile (khw <= 16) the 4 float4 of
        // tile 0 only, summed by waves 0..3, written at packed column
        // col_of(j, khw) (waves 4..7 would otherwise overwrite real columns
        // 32 .. with the empty second tile)
        const bool one = khw <= 16;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const floatx16& v = G[0][k / 4];
            const int q = 4 * (k % 4);
            if (!one || k < 4)
                red[w * kSlot + k * kWave + l] = floatx4{v[q], v[q + 1], v[q + 2], v[q + 3]};
        }
        lsync();
        if (!one || w < 4) {
            const int k = w;
            floatx4 v = red[k * kWave + l];
            for (int ww = 1; ww < kW; ++ww) {
                const floatx4 u = red[ww * kSlot + k * kWave + l];
                v[0] += u[0];
                v[1] += u[1];
                v[2] += u[2];
                v[3] += u[3];
            }
            const int ft = k / 4, q0 = 4 * (k % 4);
            const int col = one ? col_of(j, khw) : 32 * ft + j;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                glp[(size_t)(pbase + slot_row(q0 + i, h)) * cols + col] = v[i];
        }
        __threadfence_block();
        lsync();
    } else {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const floatx16& v = G[p][k / 4];
                const int q = 4 * (k % 4);
                red[w * kSlot + k * kWave + l] = floatx4{v[q], v[q + 1], v[q + 2], v[q + 3]};
            }
            lsync();
            {
                const int k = w;  // float4 k holds G[p][k / 4][q .. q + 3], q = 4 (k % 4)
                floatx4 v = red[k * kWave + l];
                for (int ww = 1; ww < kW; ++ww) {
                    const floatx4 u = red[ww * kSlot + k * kWave + l];
                    v[0] += u[0];
                    v[1] += u[1];
                    v[2] += u[2];
                    v[3] += u[3];
                }
                const int ft = k / 4, q0 = 4 * (k % 4);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    glp[(size_t)(pbase + slot_row(q0 + i, h)) * cols + 64 * p + 32 * ft + j] = v[i];
            }
            // the stores complete before the barrier: after it, other waves of
            // the tile read these entries (through the CU's shared L1)
            __threadfence_block();
            lsync();
        }
    }
}

template <int NP>
__device__ __forceinline__ void logreg_setup_w(LogregSharedW<NP>& sh, const LogregArgs& A)
{
    const SweepArgs& a = A.a;
    const int tid = threadIdx.x;
    const int d = a.tg.d, F = wide_f(d), KHW = wide_khw(d);
    for (int e = tid; e < kLPW * (NP * 64 + 1); e += LCfgW::threads) {
        (&sh.theta[0][0])[e] = 0.f;
        (&sh.prop[0][0])[e] = 0.f;
    }
    for (int c = tid; c < NP * 64; c += LCfgW::threads) sh.m[c] = 0.f;
    lsync();
    for (int f = tid; f < d; f += LCfgW::threads)
        sh.m[col_of_wide(f, F, KHW)] = a.tg.ref_mean ? a.tg.ref_mean[f] : 0.f;
    lsync();
}

// All tiles of one slot of one problem (the wide counterpart of logreg_slot:
// the same steps, moments, proposals and correction, in the same order).
template <int NP>
__device__ __forceinline__ void logreg_slot_w(LogregSharedW<NP>& sh, const LogregArgs& A,
                                              int64_t slot)
{
    constexpr int kTPP = LCfgW::tpp;
    constexpr int cols = NP * 64;
    const SweepArgs& a = A.a;
    const int tid = threadIdx.x;
    const int p = tid / kTPP, r = tid % kTPP;
    const int d = a.tg.d, F = wide_f(d), KHW = wide_khw(d);
    const int T = a.T;
    const double s2r = a.tg.ref_sigma2;
    const double inv_s2r = 1.0 / s2r, half_inv_s2r = 0.5 / s2r, sref = sqrt(s2r);
    typedef __attribute__((address_space(1))) const double gmem_d;
    gmem_d* const beta_g = (gmem_d*)a.beta;
    gmem_d* const eps_g = (gmem_d*)a.eps;
    const int nblocks = (d + 3) / 4;
    for (int64_t tile = slot; tile < a.ntiles; tile += a.S) {
        const bool first = (tile == slot);
        const int64_t pbase = tile * kLPW;
        const int64_t n64 = pbase + p;
        const bool valid = n64 < a.N;
        const uint32_t n = (uint32_t)n64;
        float* gl = A.gl + (size_t)n64 * cols;     // cached gradient at the state
        float* glpp = A.glp + (size_t)n64 * cols;  // gradient at the proposal
        uint32_t accw = 0;
        double beta_prev = 0.0;
        for (int t = 0; t <= T; ++t) {
            const double beta = (t > 0) ? beta_g[t] : 0.0;
            const double eps = (t > 0) ? eps_g[t - 1] : 1.0;
            const double hh = 0.5 * eps * eps;
            if (t > 0 && tid < 3 * kWave) {
                const int i = __builtin_amdgcn_readfirstlane(tid / kWave), q = tid % kWave;
                const bool vq = q < kLPW && (pbase + q) < a.N;
                const double lg = vq ? (beta - beta_prev) * sh.ll[q] : 0.0;
                const double x = vq ? (i == 0 ? sh.lw[q] : sh.lw[q] + (double)i * lg) : -INFINITY;
                double mm = x;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) mm = fmax(mm, __shfl_xor(mm, o, kWave));
                double sum = (mm > -INFINITY && vq) ? exp(x - mm) : 0.0;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) sum += __shfl_xor(sum, o, kWave);
                if (q == 0) {
                    double* e = a.part + ((size_t)slot * (T + 1) + (t - 1)) * 4;
                    const double L = lse_value(mm, sum);
                    e[i] = first ? L : log_add(e[i], L);
                }
            }
            if (tid == 0) sh.cnt = 0u;
            {
                double fwd = 0.0, dle = 0.0;
                for (int b = r; b < nblocks; b += kTPP) {
                    double zz[4];
                    normals4<false>(a.key, n, (uint32_t)t, t > 0 ? kStreamMove : kStreamInit,
                                    (uint32_t)b, zz, 0u, d - 4 * b);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int f = 4 * b + u;
                        if (f < d) {
                            const int c = col_of_wide(f, F, KHW);
                            const double mv = (double)sh.m[c];
                            if (t == 0) {
                                sh.prop[p][c] = (float)(mv + sref * zz[u]);
                            } else {
                                const double xv = (double)sh.theta[p][c];
                                const double ga = -(xv - mv) * inv_s2r + beta * (double)gl[c];
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
                fwd = group_sum<kTPP>(fwd);
                dle = group_sum<kTPP>(dle);
                if (r == 0) {
                    sh.fwd[p] = fwd;
                    sh.dle[p] = dle;
                    const uint4 wd = draw_block<false>(a.key, n, (uint32_t)t, kStreamAccept, 0u, 0u);
                    sh.logu[p] = (t > 0) ? log(word_uniform(wd.x)) : -INFINITY;
                }
            }
            lsync();
            contraction_w<NP>(sh, A.Xp, a.tg.n, A.n_pad, KHW, A.glp, pbase);
            {
                double bwd = 0.0;
                for (int f = r; f < d; f += kTPP) {
                    const int c = col_of_wide(f, F, KHW);
                    const double xv = (double)sh.theta[p][c];
                    const double xpv = (double)sh.prop[p][c];
                    const double gap = -(xpv - (double)sh.m[c]) * inv_s2r + beta * (double)glpp[c];
                    const double rr = xv - xpv - hh * gap;
                    bwd = fma(rr, rr, bwd);
                }
                bwd = group_sum<kTPP>(bwd);
                const double inv2e2 = 1.0 / (2.0 * eps * eps);
                const double log_alpha = sh.dle[p] * half_inv_s2r + beta * (sh.llp[p] - sh.ll[p]) -
                                         bwd * inv2e2 + sh.fwd[p] * inv2e2;
                const bool acc = (t == 0) || (sh.logu[p] < log_alpha);
                if (acc) {
                    for (int f = r; f < d; f += kTPP) {
                        const int c = col_of_wide(f, F, KHW);
                        sh.theta[p][c] = sh.prop[p][c];
                        gl[c] = glpp[c];
                    }
                }
                const uint64_t bal = __ballot(acc && valid && r == 0);
                if ((tid % kWave) == 0) atomicAdd(&sh.cnt, (uint32_t)__popcll(bal));
                if (r == 0) {
                    sh.lw[p] = (t == 0) ? 0.0 : sh.lw[p] + (beta - beta_prev) * sh.ll[p];
                    if (acc) sh.ll[p] = sh.llp[p];
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
            // the cached-gradient stores complete before the barrier (the next
            // proposals read them from other lanes)
            __threadfence_block();
            lsync();
            if (t > 0 && tid == 0) {
                double* e = a.part + ((size_t)slot * (T + 1) + (t - 1)) * 4;
                e[3] = (first ? 0.0 : e[3]) + (double)sh.cnt;
            }
            beta_prev = beta;
        }
        if (tid < kWave) {
            const bool vq = tid < kLPW && (pbase + tid) < a.N;
            double mm = vq ? sh.lw[tid] : -INFINITY, ss = vq ? 1.0 : 0.0;
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const double m2 = __shfl_xor(mm, o, kWave);
                const double s2 = __shfl_xor(ss, o, kWave);
                lse_merge(mm, ss, m2, s2);
            }
            if (tid == 0) {
                double* e = a.part + ((size_t)slot * (T + 1) + T) * 4;
                const double L = lse_value(mm, ss);
                e[0] = first ? L : log_add(e[0], L);
                e[1] = e[0];
                e[2] = e[0];
                e[3] = 0.0;
            }
            if (vq && a.lw_out) a.lw_out[pbase + tid] = sh.lw[tid];
        }
        if (valid && a.x_out)
            for (int f = r; f < d; f += kTPP)
                a.x_out[(size_t)n64 * d + f] = sh.theta[p][col_of_wide(f, F, KHW)];
        lsync();
    }
}

template <int NP>
__global__ void __launch_bounds__(LCfgW::threads) k_oais_logreg_wide(LogregArgs A)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregSharedW<NP>& sh = *reinterpret_cast<LogregSharedW<NP>*>(sh_raw);
    logreg_setup_w<NP>(sh, A);
    for (int64_t slot = blockIdx.x; slot < A.a.S; slot += gridDim.x) logreg_slot_w<NP>(sh, A, slot);
}

template <int NP, bool DYN>
__global__ void __launch_bounds__(LCfgW::threads)
    k_oais_logreg_wide_batch(const LogregArgs* __restrict__ args, const int2* __restrict__ items,
                             int64_t nitems, uint32_t* next)
{
    extern __shared__ __align__(16) char sh_raw[];
    LogregSharedW<NP>& sh = *reinterpret_cast<LogregSharedW<NP>*>(sh_raw);
    for (int64_t it = DYN ? next_item(next, sh.item, -1) : (int64_t)blockIdx.x; it < nitems;
         it = DYN ? next_item(next, sh.item, it) : it + gridDim.x) {
        const int2 item = items[it];
        const LogregArgs A = args[item.x];
        logreg_setup_w<NP>(sh, A);
        logreg_slot_w<NP>(sh, A, (int64_t)item.y);
        lsync();
    }
}

// ell and its gradient for given states, wide layout (the sweep's contraction).
template <int NP>
__global__ void __launch_bounds__(LCfgW::threads)
    k_logreg_eval_wide(const float* __restrict__ theta, int64_t N, int d, const float* Xp, int n,
                       int n_pad, float* gscratch, double* ell, float* grad)
{
    constexpr int kTPP = LCfgW::tpp;
    constexpr int cols = NP * 64;
    extern __shared__ __align__(16) char sh_raw[];
    LogregSharedW<NP>& sh = *reinterpret_cast<LogregSharedW<NP>*>(sh_raw);
    const int tid = threadIdx.x;
    const int p = tid / kTPP, r = tid % kTPP;
    const int F = wide_f(d), KHW = wide_khw(d);
    for (int e = tid; e < kLPW * (NP * 64 + 1); e += LCfgW::threads) (&sh.prop[0][0])[e] = 0.f;
    lsync();
    const int64_t pbase = (int64_t)blockIdx.x * kLPW;
    const int64_t n64 = pbase + p;
    const bool valid = n64 < N;
    for (int f = r; f < d; f += kTPP)
        if (valid) sh.prop[p][col_of_wide(f, F, KHW)] = theta[(size_t)n64 * d + f];
    lsync();
    contraction_w<NP>(sh, Xp, n, n_pad, KHW, gscratch, pbase);
    if (valid) {
        for (int f = r; f < d; f += kTPP)
            grad[(size_t)n64 * d + f] = gscratch[(size_t)n64 * cols + col_of_wide(f, F, KHW)];
        if (r == 0) ell[n64] = sh.llp[p];
    }
}

// ---------------------------------------------------------------------------
// Layout classes: the 64-column kernel's packed half-width KH (4 .. 32), or
// 1000 + NP for the panel layout with NP panels (1 .. 4).
static int panels_of(int kh) { return kh >= 1000 ? kh - 1000 : 0; }

int logreg_cols(int kh) { return panels_of(kh) ? 64 * panels_of(kh) : 64; }

int64_t logreg_tiles(int64_t N, int kh)
{
    const int lp = panels_of(kh) ? kLPW : kLP;
    return (N + lp - 1) / lp;
}

static int n_pad_of(int n) { return ((n + kRowAlign - 1) / kRowAlign) * kRowAlign; }

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace: the packed rows [n_pad][cols], then (wide layout) the cached
// gradients at the states and at the proposals, [tiles 32][cols] each.
struct WsLayout {
    size_t xp, gl, glp, total;
};

static WsLayout ws_layout(const TargetDev& tg, int64_t N, int kh)
{
    const int cols = logreg_cols(kh);
    const size_t np = (size_t)n_pad_of(tg.n);
    WsLayout L{};
    size_t b = 0;
    L.xp = b; b += a256(np * cols * sizeof(float));
    if (panels_of(kh)) {
        const size_t gb = a256((size_t)logreg_tiles(N, kh) * kLPW * cols * sizeof(float));
        L.gl = b; b += gb;
        L.glp = b; b += gb;
    }
    L.total = b + 256;
    return L;
}

size_t logreg_workspace_bytes(const TargetDev& tg, int64_t N, int kh)
{
    return ws_layout(tg, N, kh).total;
}

void logreg_layout(const TargetDev& tg, int64_t N, int kh, void* ws, LogregArgs* A)
{
    const WsLayout L = ws_layout(tg, N, kh);
    char* base = static_cast<char*>(ws);
    A->n_pad = n_pad_of(tg.n);
    A->Xp = reinterpret_cast<float*>(base + L.xp);
    A->gl = panels_of(kh) ? reinterpret_cast<float*>(base + L.gl) : nullptr;
    A->glp = panels_of(kh) ? reinterpret_cast<float*>(base + L.glp) : nullptr;
}

size_t logreg_shared_bytes(int kh)
{
    switch (panels_of(kh)) {
    case 0: return sizeof(LogregShared);
    case 1: return sizeof(LogregSharedW<1>);
    case 2: return sizeof(LogregSharedW<2>);
    case 3: return sizeof(LogregSharedW<3>);
    default: return sizeof(LogregSharedW<4>);
    }
}

template <int KH>
static hipError_t launch_kh(const LogregArgs& A, int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregShared);
    hipError_t e = hipFuncSetAttribute((const void*)k_oais_logreg<KH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_oais_logreg<KH>), dim3(grid), dim3(LCfg::threads), shb, st, A);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_w(const LogregArgs& A, int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregSharedW<NP>);
    hipError_t e = hipFuncSetAttribute((const void*)k_oais_logreg_wide<NP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_oais_logreg_wide<NP>), dim3(grid), dim3(LCfgW::threads), shb, st, A);
    return hipGetLastError();
}

template <int KH>
static hipError_t launch_eval_kh(const float* theta, int64_t N, int d, const float* Xp,
                                 int n, int n_pad, double* ell, float* grad,
                                 hipStream_t st)
{
    const size_t shb = sizeof(LogregShared);
    hipError_t e = hipFuncSetAttribute((const void*)k_logreg_eval<KH>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_logreg_eval<KH>), dim3((unsigned)logreg_tiles(N, KH)),
                       dim3(LCfg::threads), shb, st, theta, N, d, Xp, n, n_pad, ell, grad);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_eval_w(const float* theta, int64_t N, int d, const LogregArgs& A, int n,
                                double* ell, float* grad, hipStream_t st)
{
    const size_t shb = sizeof(LogregSharedW<NP>);
    hipError_t e = hipFuncSetAttribute((const void*)k_logreg_eval_wide<NP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_logreg_eval_wide<NP>), dim3((unsigned)logreg_tiles(N, 1000 + NP)),
                       dim3(LCfgW::threads), shb, st, theta, N, d, A.Xp, n, A.n_pad, A.glp, ell,
                       grad);
    return hipGetLastError();
}

int logreg_npad(int n) { return n_pad_of(n); }

hipError_t logreg_pack_into(const TargetDev& tg, int64_t N, int kh, void* ws, hipStream_t st)
{
    if (kh < 0) return hipErrorInvalidValue;
    const WsLayout L = ws_layout(tg, N, kh);
    char* base = static_cast<char*>(ws);
    float* Xp = reinterpret_cast<float*>(base + L.xp);
    const int np = n_pad_of(tg.n);
    const int cols = logreg_cols(kh);
    const int64_t total = (int64_t)np * cols;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    if (panels_of(kh))
        hipLaunchKernelGGL(k_logreg_pack_wide, dim3(blocks), dim3(256), 0, st, tg.X, tg.y, tg.n,
                           tg.d, cols, np, Xp);
    else
        hipLaunchKernelGGL(k_logreg_pack, dim3(blocks), dim3(256), 0, st, tg.X, tg.y, tg.n, tg.d,
                           kh, np, Xp);
    return hipGetLastError();
}

template <int KH>
static hipError_t launch_batch_kh(const LogregArgs* args, const int2* items, int64_t nitems,
                                  uint32_t* next, int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregShared);
    const void* f = next ? (const void*)k_oais_logreg_batch<KH, true>
                         : (const void*)k_oais_logreg_batch<KH, false>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    if (next)
        hipLaunchKernelGGL((k_oais_logreg_batch<KH, true>), dim3(grid), dim3(LCfg::threads), shb,
                           st, args, items, nitems, next);
    else
        hipLaunchKernelGGL((k_oais_logreg_batch<KH, false>), dim3(grid), dim3(LCfg::threads), shb,
                           st, args, items, nitems, next);
    return hipGetLastError();
}

template <int NP>
static hipError_t launch_batch_w(const LogregArgs* args, const int2* items, int64_t nitems,
                                 uint32_t* next, int grid, hipStream_t st)
{
    const size_t shb = sizeof(LogregSharedW<NP>);
    const void* f = next ? (const void*)k_oais_logreg_wide_batch<NP, true>
                         : (const void*)k_oais_logreg_wide_batch<NP, false>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
    if (e != hipSuccess) return e;
    if (next)
        hipLaunchKernelGGL((k_oais_logreg_wide_batch<NP, true>), dim3(grid), dim3(LCfgW::threads),
                           shb, st, args, items, nitems, next);
    else
        hipLaunchKernelGGL((k_oais_logreg_wide_batch<NP, false>), dim3(grid), dim3(LCfgW::threads),
                           shb, st, args, items, nitems, next);
    return hipGetLastError();
}

// Packs X and y into the kernel's padded, column-permuted layout in ws
// (features [0, KH) and [KH, d) in columns [0, KH) and [32, 32 + d - KH) of
// the 64-column layout; the panel layout above 64 features).
hipError_t logreg_prepare(const TargetDev& tg, int64_t N, int kh, void* ws, hipStream_t st)
{
    return logreg_pack_into(tg, N, kh, ws, st);
}

#define OASMC_KH_LIST(X) X(4) X(8) X(12) X(16) X(20) X(25) X(32)
#define OASMC_NP_LIST(X) X(1) X(2) X(3) X(4)

// Above 64 features the panel layout with ceil(d / 64) panels.  Up to 64 the
// 64-column kernel (exact half-widths with a dedicated instantiation; other
// widths round up), unless its tiles of 64 particles, one workgroup per CU,
// would leave CUs idle: tiles of 32 (the one-panel layout, about 10% more
// work per particle) then finish sooner, e.g. d = 50 with N = 8192 (128 tiles
// of 64 against 256 tiles of 32 on 256 CUs).  Below 4096 particles both are
// latency-bound and the 64-column kernel is kept.
int logreg_kh(int d, int64_t N, int cus)
{
    if (d < 1 || d > kMaxDLogreg || N < 1) return -1;
    if (d > 64) return 1000 + wide_np(d);
    if (cus > 0 && N >= 4096) {
        const int64_t r64 = ((N + kLP - 1) / kLP + cus - 1) / cus;    // rounds of tiles
        const int64_t r32 = ((N + kLPW - 1) / kLPW + cus - 1) / cus;
        if (0.55 * (double)r32 < (double)r64) return 1001;
    }
    const int kh = (d + 1) / 2;
    const int list[] = {4, 8, 12, 16, 20, 25, 32};
    for (int v : list)
        if (kh <= v) return v;
    return -1;
}

hipError_t launch_oais_logreg(const SweepArgs& a, int kh, int cus, void* ws, hipStream_t st)
{
    LogregArgs A{};
    A.a = a;
    if (kh < 0) return hipErrorInvalidValue;
    logreg_layout(a.tg, a.N, kh, ws, &A);
    const int grid = (int)std::min<int64_t>(a.S, (int64_t)cus);
    switch (kh) {
#define OASMC_KH_CASE(K) case K: return launch_kh<K>(A, grid, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
#define OASMC_NP_CASE(K) case 1000 + K: return launch_w<K>(A, grid, st);
        OASMC_NP_LIST(OASMC_NP_CASE)
#undef OASMC_NP_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_oais_logreg_batch(int kh, const LogregArgs* args, const int2* items,
                                   int64_t nitems, uint32_t* next, int grid, hipStream_t st)
{
    switch (kh) {
#define OASMC_KH_CASE(K) case K: return launch_batch_kh<K>(args, items, nitems, next, grid, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
#define OASMC_NP_CASE(K) \
    case 1000 + K: return launch_batch_w<K>(args, items, nitems, next, grid, st);
        OASMC_NP_LIST(OASMC_NP_CASE)
#undef OASMC_NP_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_logreg_eval(const TargetDev& tg, int kh, const float* theta, int64_t N,
                              double* ell, float* grad, void* ws, hipStream_t st)
{
    if (kh < 0) return hipErrorInvalidValue;
    LogregArgs A{};
    logreg_layout(tg, N, kh, ws, &A);
    switch (kh) {
#define OASMC_KH_CASE(K) \
    case K: return launch_eval_kh<K>(theta, N, tg.d, A.Xp, tg.n, A.n_pad, ell, grad, st);
        OASMC_KH_LIST(OASMC_KH_CASE)
#undef OASMC_KH_CASE
#define OASMC_NP_CASE(K) case 1000 + K: return launch_eval_w<K>(theta, N, tg.d, A, tg.n, ell, grad, st);
        OASMC_NP_LIST(OASMC_NP_CASE)
#undef OASMC_NP_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace oasmc
