// sweep_common.hip -- the kernels shared by every annealing pass: the
// slot-order merge of streamed moments, the per-step merge and trigger of the
// resampling variant, the integer-CDF systematic resampler, raw Philox blocks,
// and the host-side dispatch to the per-(family, move) sweep instantiations.
#include "kernels.hpp"

namespace oasmc {

// Merge the S slot partials of one entry (one wave per entry): each lane
// takes slots lane, lane + 64, ... and the log-sum-exps are a maximum and then
// a sum of exp(x - max), reduced in a fixed order (deterministic, and
// independent of the grid): log_g[i*T + e] for e < T, the accept fraction,
// and log Z_hat from entry T.
__device__ __forceinline__ void merge_entry(const double* __restrict__ part, int64_t S, int T,
                                            int e, double (&L)[3], double& cnt)
{
    const int lane = threadIdx.x;
    double m[3] = {-INFINITY, -INFINITY, -INFINITY};
    double c = 0.0;
    for (int64_t s = lane; s < S; s += kWave) {
        const double* p = part + ((size_t)s * (T + 1) + e) * 4;
#pragma unroll
        for (int i = 0; i < 3; ++i) m[i] = fmax(m[i], p[i]);
        c += p[3];
    }
    double sum[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) m[i] = wave_max(m[i]);
    for (int64_t s = lane; s < S; s += kWave) {
        const double* p = part + ((size_t)s * (T + 1) + e) * 4;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (m[i] > -INFINITY && p[i] > -INFINITY) sum[i] += exp(p[i] - m[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) L[i] = lse_value(m[i], wave_sum(sum[i]));
    cnt = wave_sum(c);
}

__global__ void __launch_bounds__(kWave) k_merge_slots(const double* __restrict__ part, int64_t S,
                                                       int T, int64_t N, double* log_g, double* acc,
                                                       double* logZ)
{
    const int e = blockIdx.x;
    double L[3], cnt;
    merge_entry(part, S, T, e, L, cnt);
    if (threadIdx.x != 0) return;
    if (e < T) {
#pragma unroll
        for (int i = 0; i < 3; ++i) log_g[(size_t)i * T + e] = L[i];
        acc[e] = cnt / (double)N;
    } else {
        logZ[0] = L[0] - log((double)N);
    }
}

// The per-step merge of the resampling variant, in two levels with a fixed
// order (deterministic, independent of timing): block b of the first level
// reduces a contiguous range of tile records to one record (log-sum-exps as a
// maximum and then a sum of exp(x - max)); one wave of the last block to
// finish then merges the block records, records the moments, ESS and CESS,
// decides the event and adds the log Z_hat increment (one launch).
constexpr int kMergeThreads = 256;

__device__ __forceinline__ int merge_blocks(int64_t ntiles)
{
    const int64_t nb = (ntiles + kMergeThreads - 1) / kMergeThreads;
    return (int)(nb < kAsmcMergeBlocks ? nb : kAsmcMergeBlocks);
}

// Second level, by one wave: the block records, the moments, ESS and CESS,
// the event decision and the log Z_hat increment.
__device__ __forceinline__ void asmc_merge_final(const SweepArgs& a, const AsmcState& z, int t,
                                                 int trigger, double nu, int lane)
{
    const int nb = merge_blocks(a.ntiles);
    const double* rec = z.blk_part + (size_t)lane * 8;
    const bool have = lane < nb;
    double L[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) L[i] = wave_lse(have ? rec[i] : -INFINITY);
    const double mx = wave_max(have ? rec[4] : -INFINITY);
    const double total = wave_sum(have ? rec[5] : 0.0);
    if (lane != 0) return;
    const int T = a.T;
    const double logN = log((double)a.N);
    for (int i = 0; i < 3; ++i) z.log_g[(size_t)i * T + (t - 1)] = L[i];
    z.accept[t - 1] = total;
    const double rel_ess = exp(2.0 * L[1] - L[3] - logN);
    const double rel_cess = exp(-(L[2] - 2.0 * L[1] + L[0]));
    z.ess[t - 1] = rel_ess;
    // trigger 2 (SIR) resamples after every step; times fixed in advance
    // (trigger 3) run as segments and never reach this per-step merge
    const bool fire = (trigger == 0)   ? (rel_ess < nu)
                      : (trigger == 1) ? (rel_cess < nu)
                                       : (trigger == 2 && L[1] > -INFINITY);
    z.resampled[t - 1] = 0;
    z.scal[2] = 0.0;
    if (t == T) {
        z.scal[0] += L[1] - logN;
    } else if (fire) {
        z.scal[0] += L[1] - logN;
        z.scal[1] = mx;
        z.scal[2] = 1.0;
        const uint4 wd = draw_block(a.key, 0xFFFFFFFFu, (uint32_t)t, kStreamResample, 0u, 0u);
        z.scal[3] = (double)wd.x;
        z.resampled[t - 1] = 1;
        z.nres[0] += 1;
    }
}

__global__ void __launch_bounds__(kMergeThreads) k_asmc_merge(SweepArgs a, AsmcState z, int t,
                                                                int trigger, double nu)
{
    constexpr int W = kMergeThreads / kWave;
    __shared__ double shm[W][6];
    __shared__ double res[6];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int nb = merge_blocks(a.ntiles);
    const int64_t per = (a.ntiles + nb - 1) / nb;
    const int64_t k0 = (int64_t)blockIdx.x * per;
    const int64_t k1 = (k0 + per < a.ntiles) ? k0 + per : a.ntiles;
    // pass 1: maxima (the four log-sums and the largest log w) and the count
    double m[5] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY, -INFINITY};
    double cnt = 0.0;
    for (int64_t k = k0 + tid; k < k1; k += kMergeThreads) {
        const double* tp = z.tile_part + (size_t)k * 8;
#pragma unroll
        for (int i = 0; i < 5; ++i) m[i] = fmax(m[i], tp[i]);
        cnt += tp[5];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) m[i] = wave_max(m[i]);
    cnt = wave_sum(cnt);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 5; ++i) shm[w][i] = m[i];
        shm[w][5] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) res[i] = shm[0][i];
        for (int ww = 1; ww < W; ++ww) {
#pragma unroll
            for (int i = 0; i < 5; ++i) res[i] = fmax(res[i], shm[ww][i]);
            res[5] += shm[ww][5];
        }
    }
    __syncthreads();
    double M[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) M[i] = res[i];
    // pass 2: sums of exp(L_tile - max)
    double sm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = k0 + tid; k < k1; k += kMergeThreads) {
        const double* tp = z.tile_part + (size_t)k * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (M[i] > -INFINITY && tp[i] > -INFINITY) sm[i] += exp(tp[i] - M[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) sm[i] = wave_sum(sm[i]);
    __syncthreads();  // every thread has read res
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) shm[w][i] = sm[i];
    }
    __syncthreads();
    if (tid == 0) {
        double* out = z.blk_part + (size_t)blockIdx.x * 8;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double acc = shm[0][i];
            for (int ww = 1; ww < W; ++ww) acc += shm[ww][i];
            out[i] = lse_value(M[i], acc);
        }
        out[4] = res[4];
        out[5] = res[5];
    }
    // the last block to finish merges the block records; the arrival counter
    // only elects that block (no block waits for another)
    __shared__ bool last;
    if (tid == 0) {
        __threadfence();  // this block's record before its arrival
        last = atomicAdd(z.ticket, 1u) == (unsigned)(nb - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // the other blocks' records
    if (w == 0) asmc_merge_final(a, z, t, trigger, nu, lane);
    if (tid == 0) z.ticket[0] = 0u;
}

// Merge of one segment between resampling times fixed in advance (one wave
// per entry, the slot order of k_merge_slots): blocks 0 .. t_end - t_begin - 1
// take the entries of steps t_begin + 1 .. t_end (moments, accepted counts; no
// per-step ESS), the last block entry T, whose log-sum-exp of the segment's
// final log-weights gives the log Z_hat factor of this event and whose fourth
// field holds the largest log w (the shift of the resampler's integer
// weights).  Each output element is written by one block.
__global__ void __launch_bounds__(kWave) k_seg_merge(SweepArgs a, AsmcState z)
{
    const int T = a.T;
    const int nsteps = a.t_end - a.t_begin;
    const bool fin = (int)blockIdx.x == nsteps;
    const int e = fin ? T : a.t_begin + (int)blockIdx.x;
    double L[3], cnt;
    merge_entry(a.part, a.S, T, e, L, cnt);
    double mx = -INFINITY;
    if (fin) {
        for (int64_t s = threadIdx.x; s < a.S; s += kWave)
            mx = fmax(mx, a.part[((size_t)s * (T + 1) + T) * 4 + 3]);
        mx = wave_max(mx);
    }
    if (threadIdx.x != 0) return;
    if (!fin) {
#pragma unroll
        for (int i = 0; i < 3; ++i) z.log_g[(size_t)i * T + e] = L[i];
        z.accept[e] = cnt;
        z.ess[e] = NAN;
        z.resampled[e] = (e == a.t_end - 1 && a.t_end < T) ? 1 : 0;
        return;
    }
    z.scal[0] += L[0] - log((double)a.N);
    const bool fire = a.t_end < T && mx > -INFINITY && mx < INFINITY;
    z.scal[2] = fire ? 1.0 : 0.0;
    if (fire) {
        z.scal[1] = mx;
        const uint4 wd = draw_block(a.key, 0xFFFFFFFFu, (uint32_t)a.t_end, kStreamResample, 0u, 0u);
        z.scal[3] = (double)wd.x;
        z.nres[0] += 1;
    }
}

// ---------------------------------------------------------------------------
// Systematic resampling with an exact integer CDF.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;

int64_t resample_blocks(int64_t N) { return (N + kScanBlock - 1) / kScanBlock; }

__device__ __forceinline__ int quant_bits(int64_t N)
{
    int lg = 0;
    while (((int64_t)1 << lg) < N) ++lg;
    return 62 - lg;
}

// Inclusive scan of the block totals (one block, sequential chunks).
__device__ __forceinline__ void scan_block_totals(int64_t nb, uint64_t* btot)
{
    __shared__ uint64_t sh[kScanThreads];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        sh[threadIdx.x] = (b < nb) ? btot[b] : 0;
        __syncthreads();
        for (int o = 1; o < kScanThreads; o <<= 1) {
            const uint64_t v = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += v;
            __syncthreads();
        }
        if (b < nb) btot[b] = sh[threadIdx.x] + carry;
        __syncthreads();
        carry += sh[kScanThreads - 1];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) k_rs_scan_blocks(int64_t nb, const double* scal,
                                                                 uint64_t* btot)
{
    if (scal[2] == 0.0) return;
    scan_block_totals(nb, btot);
}

// q_m and the block-local inclusive prefix; block totals into btot.
// With a ticket, the last block to finish also scans the block totals.
__global__ void __launch_bounds__(kScanThreads) k_rs_quant_scan(int64_t N, const double* lw,
                                                                const double* scal, uint64_t* C,
                                                                uint64_t* btot, unsigned* ticket)
{
    if (scal[2] == 0.0) return;
    __shared__ uint64_t sh[kScanThreads];
    const double mx = scal[1];
    const double scale = ldexp(1.0, quant_bits(N));
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    uint64_t q[kScanItems];
    uint64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t m = base + k;
        q[k] = 0;
        if (m < N) {
            const double v = lw[m];
            if (v == v) q[k] = (uint64_t)floor(exp(v - mx) * scale);
        }
        run += q[k];
        q[k] = run;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread totals (integer: exact)
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint64_t v = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    const uint64_t before = (threadIdx.x > 0) ? sh[threadIdx.x - 1] : 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t m = base + k;
        if (m < N) C[m] = before + q[k];
    }
    if (ticket == nullptr) {
        if (threadIdx.x == kScanThreads - 1) btot[blockIdx.x] = sh[threadIdx.x];
        return;
    }
    __shared__ bool last;
    if (threadIdx.x == kScanThreads - 1) {
        btot[blockIdx.x] = sh[threadIdx.x];
        __threadfence();  // this block's total before its arrival
        last = atomicAdd(ticket, 1u) == (unsigned)(gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // the other blocks' totals
    scan_block_totals((int64_t)gridDim.x, btot);
    if (threadIdx.x == 0) ticket[0] = 0u;
}

// floor(num_hi:num_lo / den) for a quotient below 2^64 (restoring division).
__device__ __forceinline__ uint64_t div128_64(uint64_t hi, uint64_t lo, uint64_t den)
{
    uint64_t q = 0;
    uint64_t rem = hi;  // hi < den is guaranteed by the caller
    for (int b = 63; b >= 0; --b) {
        const bool top = (rem >> 63) != 0;
        rem = (rem << 1) | ((lo >> b) & 1u);
        if (top || rem >= den) {
            rem -= den;
            q |= (uint64_t)1 << b;
        }
    }
    return q;
}

// Ancestor of slot n: min{m : C_m > p_n}, p_n = floor(S (2(n 2^32 + u) + 1) / (N 2^33)).
__device__ __forceinline__ int64_t find_ancestor(int64_t n, int64_t N, uint32_t u,
                                                 const uint64_t* C, const uint64_t* btot,
                                                 int64_t nb)
{
    const uint64_t S = btot[nb - 1];
    const uint64_t mult = 2u * (((uint64_t)n << 32) | (uint64_t)u) + 1u;
    const unsigned __int128 prod = (unsigned __int128)S * (unsigned __int128)mult;
    const uint64_t den = (uint64_t)N << 33;
    const uint64_t pn = div128_64((uint64_t)(prod >> 64), (uint64_t)prod, den);
    // block: first b with btot[b] > pn
    int64_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (btot[mid] > pn) hi = mid; else lo = mid + 1;
    }
    const uint64_t off = (lo > 0) ? btot[lo - 1] : 0;
    int64_t a = lo * kScanBlock;
    int64_t b = (lo + 1) * kScanBlock - 1;
    if (b > N - 1) b = N - 1;
    while (a < b) {
        const int64_t mid = (a + b) >> 1;
        if (C[mid] + off > pn) b = mid; else a = mid + 1;
    }
    return a;
}

__global__ void k_rs_gather(int64_t N, int d, AsmcState z, int64_t nb)
{
    if (z.scal[2] == 0.0) return;
    const uint32_t u = (uint32_t)z.scal[3];
    for (int64_t n = (int64_t)blockIdx.x * blockDim.y + threadIdx.y; n < N;
         n += (int64_t)gridDim.x * blockDim.y) {
        const int64_t an = find_ancestor(n, N, u, z.C, z.btot, nb);
        for (int i = threadIdx.x; i < d; i += blockDim.x) {
            z.X2[(size_t)n * d + i] = z.X[(size_t)an * d + i];
            if (z.G) z.G2[(size_t)n * d + i] = z.G[(size_t)an * d + i];
        }
        if (threadIdx.x == 0) z.ell2[n] = z.ell[an];
    }
}

__global__ void k_rs_commit(int64_t N, int d, AsmcState z)
{
    if (z.scal[2] == 0.0) return;
    const int64_t total = N * (int64_t)d;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        z.X[i] = z.X2[i];
        if (z.G) z.G[i] = z.G2[i];
        if (i < N) {
            z.ell[i] = z.ell2[i];
            z.lw[i] = 0.0;
        }
    }
}

__global__ void k_rs_ancestors(int64_t N, const double* scal, const uint64_t* C,
                               const uint64_t* btot, int64_t nb, int32_t* anc)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    // no finite weight: every ancestor is -1 (the host call also reports it)
    anc[n] = (scal[2] == 0.0) ? -1 : (int32_t)find_ancestor(n, N, (uint32_t)scal[3], C, btot, nb);
}

// Max of lw, the flag and the word for the plain resampling entry point.
__global__ void k_rs_prepare(int64_t N, const double* lw, uint32_t u, double* scal)
{
    __shared__ double sh[256];
    double mx = -INFINITY;
    for (int64_t m = threadIdx.x; m < N; m += 256) {
        const double v = lw[m];
        if (v > mx) mx = v;
    }
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = sh[0];
        const bool ok = (m > -INFINITY) && (m < INFINITY);
        scal[1] = m;
        scal[2] = ok ? 1.0 : 0.0;
        scal[3] = (double)u;
    }
}

__global__ void k_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, uint32_t* out,
                         int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    const uint4 o = philox4x32_10(c, k0, k1);
    out[4 * i] = o.x;
    out[4 * i + 1] = o.y;
    out[4 * i + 2] = o.z;
    out[4 * i + 3] = o.w;
}

// ---------------------------------------------------------------------------
// Host-side dispatch.
// ---------------------------------------------------------------------------
bool valu_shape(int d, int64_t N, ValuShape* s)
{
    if (d < 1 || d > kMaxDValu) return false;
    if (d <= 24) {
        s->lpp = 1;
        s->dpl = ((d + 3) / 4) * 4;
    } else if (d <= 32) {
        s->lpp = 2; s->dpl = 16;
    } else if (d <= 64) {
        s->lpp = 4; s->dpl = 16;
    } else if (d <= 128) {
        // 16 lanes of 8 coordinates rather than 8 of 16: half the registers
        // per lane, two waves per SIMD for the mixture/HMC sweeps (measured
        // 25% faster at d = 100)
        s->lpp = 16; s->dpl = 8;
    } else {
        s->lpp = 16; s->dpl = 16;
    }
    // Few particles: a particle on 4 lanes of 8 coordinates puts more of the
    // GPU to work (fewer lanes than two waves per SIMD otherwise)
    if (d > 8 && d <= 32 && N * s->lpp < kFillLanes) {
        s->lpp = 4;
        s->dpl = 8;
        // fewer still (4 lanes per particle would leave the SIMDs at most half
        // a wave each): 8 lanes of 4 coordinates
        if (N * 4 <= kFillLanes / 4) {
            s->lpp = 8;
            s->dpl = 4;
        }
    }
    return true;
}

int64_t valu_tiles(int64_t N, const ValuShape& s)
{
    const int64_t P = kWave / s.lpp;
    return (N + P - 1) / P;
}

template <int FAM, int MOVE>
hipError_t valu_dispatch(int what, const SweepArgs& a, const ValuShape& s, int gw,
                         const AsmcState* z, int t, hipStream_t st, const ValuBatch* b,
                         const void* ext);
static hipError_t dispatch_all(int what, const SweepArgs& a, const ValuShape& s, int gw,
                               const AsmcState* z, int t, hipStream_t st,
                               const ValuBatch* b = nullptr, const void* rj = nullptr)
{
    const int fam = a.tg.family, mv = a.move;
#define OASMC_FM(F, M) \
    if (fam == F && mv == M) return valu_dispatch<F, M>(what, a, s, gw, z, t, st, b, rj);
    OASMC_FM(kGauss, kRwmh)
    OASMC_FM(kGauss, kMala)
    OASMC_FM(kGauss, kHmc)
    OASMC_FM(kGmm, kRwmh)
    OASMC_FM(kGmm, kMala)
    OASMC_FM(kGmm, kHmc)
    OASMC_FM(kGauss, kRwmh3)
    OASMC_FM(kGmm, kRwmh3)
    OASMC_FM(kUnid, kRwmh)
    OASMC_FM(kUnid, kRwmh3)
#undef OASMC_FM
    return hipErrorInvalidValue;
}

hipError_t launch_asmc_move(const SweepArgs& a, const ValuShape& s, const AsmcState& z, int t,
                            hipStream_t st)
{
    return dispatch_all(2, a, s, 0, &z, t, st);
}

// ---------------------------------------------------------------------------
// ZJA: the online CESS-adaptive schedule of Zhou, Johansen and Aston applied
// to AIS (Sec. "Connection to online conditional ESS optimisation").  One
// workgroup chooses beta_t from log w_{t-1} and ell(X_{t-1}) of every particle:
// CESS(b) / N = g_1^2 / (g_0 g_2), g_i = sum_n w_n exp(i (b - beta_{t-1}) ell_n)
// (eq. CESS); beta_t = 1 if CESS(1) >= rho N, else `iters` halvings of
// (beta_{t-1}, 1] keeping the upper part while CESS >= rho N.  This is the
// per-step communication across all particles that the loop-swapped OAIS pass
// avoids.
// ---------------------------------------------------------------------------
constexpr int kZjaThreads = 1024;

// Log-sum-exps L_i over the particles of log w + i a ell for i = I0 .. 2, in
// two passes (a block maximum, then a block sum of exp(x - max): one
// exponential per term, no data-dependent branch around it); per-thread
// partials in particle order, then the wave's xor butterfly, then the waves in
// order, so every thread ends with the same bits.
template <int I0>
__device__ __forceinline__ void zja_lse(int64_t N, const double* __restrict__ lw,
                                        const double* __restrict__ ell, double a, double (&L)[3],
                                        double* shm)
{
    constexpr int NW = kZjaThreads / kWave;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    auto term = [&](int64_t j, int i) {
        const double v = lw[j];
        return (i == 0) ? v : v + (double)i * a * ell[j];
    };
    double m[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t j = threadIdx.x; j < N; j += kZjaThreads)
#pragma unroll
        for (int i = I0; i < 3; ++i) m[i] = fmax(m[i], term(j, i));
#pragma unroll
    for (int i = I0; i < 3; ++i) {
        m[i] = wave_max(m[i]);
        if (lane == 0) shm[w * 3 + i] = m[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = I0; i < 3; ++i) {
        double mm = -INFINITY;
        for (int ww = 0; ww < NW; ++ww) mm = fmax(mm, shm[ww * 3 + i]);
        m[i] = mm;
    }
    __syncthreads();
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t j = threadIdx.x; j < N; j += kZjaThreads)
#pragma unroll
        for (int i = I0; i < 3; ++i) {
            const double x = term(j, i);
            s[i] += (x > -INFINITY) ? exp(x - m[i]) : 0.0;
        }
#pragma unroll
    for (int i = I0; i < 3; ++i) {
        s[i] = wave_sum(s[i]);
        if (lane == 0) shm[w * 3 + i] = s[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = I0; i < 3; ++i) {
        double ss = 0.0;
        for (int ww = 0; ww < NW; ++ww) ss += shm[ww * 3 + i];
        L[i] = (m[i] > -INFINITY) ? lse_value(m[i], ss) : -INFINITY;
    }
    __syncthreads();  // shm is reused by the next call
}

__global__ void __launch_bounds__(kZjaThreads)
    k_zja_select(int64_t N, const double* __restrict__ lw, const double* __restrict__ ell,
                 double* beta, int t, int Tmax, double log_rho, int iters, int* stop,
                 double* log_g)
{
    if (t > *stop) return;
    __shared__ double shm[(kZjaThreads / kWave) * 3];
    const double b0 = beta[t - 1];
    double L[3];
    zja_lse<0>(N, lw, ell, 1.0 - b0, L, shm);  // L_0 (log of sum w_{t-1}) is fixed for the step
    const double L0 = L[0];
    double bt;
    if (2.0 * L[1] - L[2] - L0 >= log_rho) {
        bt = 1.0;
    } else {
        double lo = b0, hi = 1.0;
        for (int it = 0; it < iters; ++it) {
            const double mid = 0.5 * (lo + hi);
            zja_lse<1>(N, lw, ell, mid - b0, L, shm);
            if (2.0 * L[1] - L[2] - L0 >= log_rho) lo = mid;
            else hi = mid;
        }
        bt = (lo > b0) ? lo : hi;
    }
    if (t == Tmax) bt = 1.0;
    zja_lse<1>(N, lw, ell, bt - b0, L, shm);  // the step's moments at the chosen beta_t
    L[0] = L0;
    if (threadIdx.x == 0) {
        beta[t] = bt;
#pragma unroll
        for (int i = 0; i < 3; ++i) log_g[(size_t)i * Tmax + (t - 1)] = L[i];
        if (bt >= 1.0) *stop = t;
    }
}

__global__ void __launch_bounds__(kZjaThreads) k_zja_final(int64_t N, const double* lw,
                                                           double* logZ)
{
    __shared__ double shm[(kZjaThreads / kWave) * 3];
    double L[3];
    zja_lse<0>(N, lw, lw, 0.0, L, shm);
    if (threadIdx.x == 0) logZ[0] = L[0] - log((double)N);
}

hipError_t launch_zja_select(int64_t N, const double* lw, const double* ell, double* beta, int t,
                             int Tmax, double log_rho, int iters, int* stop, double* log_g,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_zja_select, dim3(1), dim3(kZjaThreads), 0, st, N, lw, ell, beta, t, Tmax,
                       log_rho, iters, stop, log_g);
    return hipGetLastError();
}

hipError_t launch_zja_final(int64_t N, const double* lw, double* logZ, hipStream_t st)
{
    hipLaunchKernelGGL(k_zja_final, dim3(1), dim3(kZjaThreads), 0, st, N, lw, logZ);
    return hipGetLastError();
}

hipError_t launch_pt(const PtArgs& A, const ValuShape& s, hipStream_t st)
{
    return dispatch_all(5, A.a, s, 0, nullptr, 0, st, nullptr, &A);
}

hipError_t launch_rejuv(const RejuvArgs& R, const ValuShape& s, hipStream_t st)
{
    return dispatch_all(4, R.a, s, 0, nullptr, 0, st, nullptr, &R);
}

hipError_t launch_target_eval(const EvalArgs& E, const ValuShape& s, hipStream_t st)
{
    return dispatch_all(6, E.a, s, 0, nullptr, 0, st, nullptr, &E);
}

// Column b of the tile sums over tiles in a fixed order (one wave per column).
__global__ void __launch_bounds__(kWave) k_rejuv_reduce(const double* __restrict__ tsum,
                                                         int64_t ntiles, int d, double samples,
                                                         double* out)
{
    const int b = blockIdx.x;
    const int w = 2 * d + 1;
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < ntiles; k += kWave) v += tsum[(size_t)k * w + b];
    v = wave_sum(v);
    if (threadIdx.x == 0) out[b] = v / samples;
}

hipError_t launch_rejuv_reduce(const double* tsum, int64_t ntiles, int d, double samples,
                               double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_rejuv_reduce, dim3(2 * d + 1), dim3(kWave), 0, st, tsum, ntiles, d,
                       samples, out);
    return hipGetLastError();
}

// The uniform word of the resampling event at step t (particle word 0xFFFFFFFF).
__global__ void k_event_word(RngKey key, uint32_t t, double* scal)
{
    const uint4 wd = draw_block(key, 0xFFFFFFFFu, t, kStreamResample, 0u, 0u);
    scal[3] = (double)wd.x;
}

hipError_t launch_resample_event(int64_t N, const double* lw, const RngKey& key, uint32_t t,
                                 int32_t* anc, uint64_t* C, uint64_t* btot, double* scal,
                                 hipStream_t st)
{
    const int64_t nb = resample_blocks(N);
    hipLaunchKernelGGL(k_rs_prepare, dim3(1), dim3(256), 0, st, N, lw, 0u, scal);
    hipLaunchKernelGGL(k_event_word, dim3(1), dim3(1), 0, st, key, t, scal);
    hipLaunchKernelGGL(k_rs_quant_scan, dim3((unsigned)nb), dim3(kScanThreads), 0, st, N, lw,
                       (const double*)scal, C, btot, (unsigned*)nullptr);
    hipLaunchKernelGGL(k_rs_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, nb,
                       (const double*)scal, btot);
    hipLaunchKernelGGL(k_rs_ancestors, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N,
                       (const double*)scal, (const uint64_t*)C, (const uint64_t*)btot, nb, anc);
    return hipGetLastError();
}

hipError_t launch_oais_valu_batch(int family, int move, const ValuShape& s, const ValuBatch& b,
                                  int grid_waves, hipStream_t st)
{
    SweepArgs a{};
    a.tg.family = family;
    a.move = move;
    return dispatch_all(3, a, s, grid_waves, nullptr, 0, st, &b);
}

__global__ void k_batch_params(const TargetDev* __restrict__ tgs, const BatchParam* __restrict__ bps)
{
    const TargetDev& tg = tgs[blockIdx.x];
    const BatchParam& bp = bps[blockIdx.x];
    // problems without a parameter view (logistic regression) are skipped
    if (tg.family == kLogreg || bp.m == nullptr) return;
    for (int i = threadIdx.x; i < tg.d; i += blockDim.x)
        bp.m[i] = tg.ref_mean ? tg.ref_mean[i] : 0.f;
    // 1/(2 v_k), 1/v_k; zero beyond K (padded components of a block)
    for (int k = threadIdx.x; k < kMaxK; k += blockDim.x) {
        const bool on = tg.family == kGmm && k < tg.K;
        const double v = on ? exp(2.0 * (double)tg.log_scales[k]) : 1.0;
        bp.hiv[k] = on ? 0.5 / v : 0.0;
        bp.iv[k] = on ? 1.0 / v : 0.0;
    }
    const int nl = (int)lane_param_doubles(tg, bp.lpp, bp.dpl);
    for (int e = threadIdx.x; e < nl; e += blockDim.x) bp.lane[e] = lane_param(tg, bp.lpp, bp.dpl, e);
}

hipError_t launch_batch_params(const TargetDev* tgs, const BatchParam* bp, int nprob,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_params, dim3(nprob), dim3(64), 0, st, tgs, bp);
    return hipGetLastError();
}

hipError_t launch_oais_valu(const SweepArgs& a, const ValuShape& s, int grid_waves, hipStream_t st)
{
    return dispatch_all(0, a, s, grid_waves, nullptr, 0, st);
}

hipError_t launch_asmc_init(const SweepArgs& a, const ValuShape& s, const AsmcState& z,
                            hipStream_t st)
{
    return dispatch_all(1, a, s, 0, &z, 0, st);
}

hipError_t launch_asmc_step(const SweepArgs& a, const ValuShape& s, const AsmcState& z, int t,
                            int trigger, double nu, hipStream_t st)
{
    hipError_t e = dispatch_all(2, a, s, 0, &z, t, st);
    if (e != hipSuccess) return e;
    const int64_t nb = std::min<int64_t>((a.ntiles + kMergeThreads - 1) / kMergeThreads,
                                         kAsmcMergeBlocks);
    hipLaunchKernelGGL(k_asmc_merge, dim3((unsigned)nb), dim3(kMergeThreads), 0, st, a, z, t,
                       trigger, nu);
    return hipGetLastError();
}

// Grid cap of the gather and commit kernels of the resampling variant.
constexpr int64_t kIdleGrid = 2048;

hipError_t launch_resample_step(const SweepArgs& a, const AsmcState& z, int t, bool commit,
                                hipStream_t st)
{
    (void)t;
    const int64_t N = a.N;
    const int64_t nb = resample_blocks(N);
    // launched every step and idle unless the trigger fired: grids are capped
    // (grid-stride loops) so that an idle launch stays cheap
    hipLaunchKernelGGL(k_rs_quant_scan, dim3((unsigned)nb), dim3(kScanThreads), 0, st, N,
                       (const double*)z.lw, (const double*)z.scal, z.C, z.btot, z.ticket + 1);
    const int d = a.tg.d;
    const int tx = d >= 32 ? 32 : (d >= 16 ? 16 : (d >= 8 ? 8 : 4));
    const int ty = 256 / tx;
    const int64_t gblocks = std::min<int64_t>((N + ty - 1) / ty, kIdleGrid);
    hipLaunchKernelGGL(k_rs_gather, dim3((unsigned)gblocks), dim3(tx, ty), 0, st, N, d, z, nb);
    if (commit) {
        const int64_t total = N * (int64_t)d;
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, kIdleGrid);
        hipLaunchKernelGGL(k_rs_commit, dim3((unsigned)blocks), dim3(256), 0, st, N, d, z);
    }
    return hipGetLastError();
}

hipError_t launch_segment_merge(const SweepArgs& a, const AsmcState& z, hipStream_t st)
{
    const int nsteps = a.t_end - a.t_begin;
    hipLaunchKernelGGL(k_seg_merge, dim3(nsteps + 1), dim3(kWave), 0, st, a, z);
    return hipGetLastError();
}

hipError_t launch_merge_slots(const double* part, int64_t S, int T, int64_t N, double* log_g,
                              double* acc, double* logZ, hipStream_t st)
{
    hipLaunchKernelGGL(k_merge_slots, dim3(T + 1), dim3(kWave), 0, st, part, S, T, N, log_g, acc,
                       logZ);
    return hipGetLastError();
}

hipError_t launch_resample_plain(int64_t N, const double* lw, uint32_t u, int32_t* anc,
                                 uint64_t* C, uint64_t* btot, double* scal, hipStream_t st)
{
    const int64_t nb = resample_blocks(N);
    hipLaunchKernelGGL(k_rs_prepare, dim3(1), dim3(256), 0, st, N, lw, u, scal);
    hipLaunchKernelGGL(k_rs_quant_scan, dim3((unsigned)nb), dim3(kScanThreads), 0, st, N, lw,
                       (const double*)scal, C, btot, (unsigned*)nullptr);
    hipLaunchKernelGGL(k_rs_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, nb,
                       (const double*)scal, btot);
    hipLaunchKernelGGL(k_rs_ancestors, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N,
                       (const double*)scal, (const uint64_t*)C, (const uint64_t*)btot, nb, anc);
    return hipGetLastError();
}

__global__ void k_zero(double* a, int na, int* b, int nb)
{
    const int i = threadIdx.x;
    if (i < na) a[i] = 0.0;
    if (i < nb) b[i] = 0;
}

hipError_t launch_zero(double* a, int na, int* b, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, a, na, b, nb);
    return hipGetLastError();
}

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t count,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), ctr, out, count);
    return hipGetLastError();
}

}  // namespace oasmc
