// kernels.hpp -- interface between the host driver (oasmc_api.hip) and the
// gfx950 kernels.  Plain structs of device pointers; no torch types.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace oasmc {

enum Family { kGauss = 1, kLogreg = 2, kGmm = 3, kUnid = 4 };
// kRwmh3: the alternation of three random-walk MH substeps with standard
// deviations eps (0.1, 1, 10) per step (the paper's GPU experiments).
enum Move { kRwmh = 1, kMala = 2, kHmc = 3, kRwmh3 = 4 };
// Moves that use grad ell (and keep it with the state).
__host__ __device__ constexpr bool uses_grad(int move) { return move == kMala || move == kHmc; }

constexpr int kMaxK = 16;      // mixture components handled by the VALU kernels
constexpr int kMaxDValu = 256; // dimension handled by the VALU kernels
constexpr int kMaxDLogreg = 256;

// Device description of the target and reference (all pointers device, fp32).
struct TargetDev {
    int family, d, K, n;
    const float* mu;
    double sigma2;
    const float* X;
    const float* y;
    const float* means;
    const float* log_scales;
    const float* ref_mean;  // may be null
    double ref_sigma2;
    // kUnid (d = 2): uniform reference on (0, box)^2; ell = log Binomial(k | n, x y)
    // minus its maximum (at x y = k / n), -inf unless 0 < x y < 1 inside the box
    double binom_n, binom_k, box;
};

// Pointers to a problem's target parameters as the particle code reads them:
// reference mean [d], Gaussian mean [d] or mixture means [K*d], and the
// mixture's 1/(2 v_k), 1/v_k.  lm and lmu hold the same means in binary64 in
// the lane layout of a sweep shape (LPP lanes of DPL coordinates): element
// (k, j, r) at (k DPL + j) LPP + r is coordinate r DPL + j of mean k, zero
// beyond d, so a wave reads them without bank conflicts and padded
// coordinates need no branch.
struct ParView {
    const float* m;
    const float* mu;
    const double* hiv;
    const double* iv;
    const double* lm;   // [DPL][LPP]
    const double* lmu;  // [K or 1][DPL][LPP]
};

// Mixture components handled together by the particle code (the lane layout
// and the per-component constants are zero-padded to whole blocks).
constexpr int kKBlock = 4;
static_assert(kMaxK % kKBlock == 0, "whole blocks of components");
// Means held by the lane layout: the Gaussian mean, or the mixture means
// padded to whole blocks of kKBlock components.
__host__ __device__ inline int lane_means(const TargetDev& tg)
{
    return tg.family == kGmm ? (tg.K + kKBlock - 1) / kKBlock * kKBlock : 1;
}
// Doubles of the lane-layout arrays lm and lmu for one sweep shape.
__host__ __device__ inline size_t lane_param_doubles(const TargetDev& tg, int lpp, int dpl)
{
    return (size_t)(1 + lane_means(tg)) * lpp * dpl;
}

// Offset of the lane-layout arrays behind the staged parameters (8-aligned):
// reference and target means as floats after 1/(2 v_k), 1/v_k.
__host__ __device__ inline size_t lane_params_offset(const TargetDev& tg)
{
    const int nmu = (tg.family == kGmm) ? tg.K * tg.d : tg.d;
    return (2 * kMaxK * sizeof(double) + (size_t)(tg.d + nmu) * sizeof(float) + 7) & ~(size_t)7;
}
// Dynamic LDS of a VALU kernel with the lane-layout parameters of a shape.
__host__ __device__ inline size_t params_bytes_lanes(const TargetDev& tg, int lpp, int dpl)
{
    return lane_params_offset(tg) + lane_param_doubles(tg, lpp, dpl) * sizeof(double);
}

// Arguments of one annealing pass.
struct SweepArgs {
    TargetDev tg;
    int move, leapfrog;
    int64_t N;
    int T;
    const double* beta;  // device [T+1]
    const double* eps;   // device [T]
    RngKey key;
    // per-slot log-domain partials [S][T+1][4]: lse(lw), lse(lw+lg), lse(lw+2lg), count
    double* part;
    int64_t S;
    int64_t ntiles;
    double* lw_out;        // device [N] or null
    float* x_out;          // device [N*d] or null
    uint32_t* acc_bits;    // device [N*acc_words] or null
    int acc_words;
    float* ckpt;           // device [N][ceil(T/ckpt_every)][d] states before steps 1, 1+every, ... or null
    int ckpt_every;
    // A segment between resampling times fixed in advance: the pass runs steps
    // t_begin + 1 .. t_end (t_end = 0 means T) from the particle state in
    // sx [N*d], sg [N*d] (MALA, HMC), sell [N], slw [N], saccw [N] and writes
    // that state back.  sx = null for an AIS pass (start from eta, log w = 0).
    // Entry T of the slot partials then holds the log-sum-exp of log w at the
    // segment's end and, in its fourth field, the largest log w.
    int t_begin, t_end;
    float* sx;
    double* sg;
    double* sell;
    double* slw;
    uint32_t* saccw;
    // Online schedules (ZJA): the per-step kernel of the resampling variant
    // does nothing for steps t > *t_stop (device; null = never stops early).
    const int* t_stop;
};

// Element e of the lane layout of (reference mean, target means) for a shape
// of LPP lanes x DPL coordinates: mean k (0 = reference), coordinate
// r DPL + j, zero beyond d.
__device__ __forceinline__ double lane_param(const TargetDev& tg, int lpp, int dpl, int e)
{
    const int k = e / (dpl * lpp);
    const int rem = e - k * dpl * lpp;
    const int j = rem / lpp;
    const int r = rem - j * lpp;
    const int i = r * dpl + j;
    if (i >= tg.d) return 0.0;
    if (k == 0) return tg.ref_mean ? (double)tg.ref_mean[i] : 0.0;
    if (tg.family == kGmm && k > tg.K) return 0.0;  // padding of the last block
    if (tg.family == kUnid) return 0.0;              // no target means
    const float* src = (tg.family == kGmm) ? tg.means : tg.mu;
    return (double)src[(size_t)(k - 1) * tg.d + i];
}

// Blocks of the first level of the per-step merge in the resampling variant.
constexpr int kAsmcMergeBlocks = 64;

// State of the particle system between steps of the resampling variant.
struct AsmcState {
    float* X;          // [N*d] current states
    float* X2;         // [N*d] gather target
    double* ell;       // [N]
    double* ell2;      // [N]
    double* G;         // [N*d] grad ell at the current states (MALA, HMC), else null
    double* G2;        // [N*d] gather target of G
    double* lw;        // [N]
    uint32_t* accw;    // [N] accept bits of the current 32-step word
    double* tile_part; // [ntiles*8]
    double* blk_part;  // [kAsmcMergeBlocks*8] per-block merge of tile_part
    // scalars updated on the device
    double* scal;      // [0] log Z_hat, [1] max(lw) at event, [2] flag, [3] u word
    int* nres;         // [1]
    unsigned* ticket;  // [2] arrival counters of the per-step merge and of the
                       // resampler's scan; zero between launches (the last
                       // arriving block resets its counter)
    double* log_g;     // [3*T] device
    double* ess;       // [T]
    int* resampled;    // [T]
    double* accept;    // [T] accepted count
    // resampler scratch
    uint64_t* C;       // [N] block-local inclusive prefix of q
    uint64_t* btot;    // [nblocks] inclusive block totals after the scan
};

// Final-iteration rejuvenation (Sec. "Computing expectations"): N chains of
// a.T steps at beta = 1 with step size eps, chain n starting from particle
// anc[n] of the final population x_in; per-tile sums of x_i, x_i^2 over the
// chain states and the accepted count in tsum [ntiles][2 d + 1].
struct RejuvArgs {
    SweepArgs a;          // target, move, leapfrog, N, T = chain length, key, ntiles
    double eps;
    const float* x_in;    // [N*d]
    const int32_t* anc;   // [N]
    double* tsum;         // [ntiles][2 d + 1]
    float* x_out;         // [N*d] chain end states, or null
};

// Parallel tempering: K copies (one workgroup each) of Np + 1 chains at the
// temperatures beta[0..Np] (step sizes eps[0..Np]), a.T iterations; per copy
// out[k * stride ..]: stepping-stone (max, scaled sum) pairs [Np][2], summed
// swap rejections [Np], round trips, the number of waves; fpart [K][16][2d]:
// target-chain sums of x_i, x_i^2 per wave.
struct PtArgs {
    SweepArgs a;          // target, move, leapfrog, key, T = iterations
    int K, Np;
    const double* beta;   // device [Np+1]
    const double* eps;    // device [Np+1]
    double* out;          // device [K][stride]
    int64_t stride;       // >= 3 Np + 2
    double* fpart;        // device [K][16][2d]
};

// ell and grad ell of the closed-form families at given states, evaluated by
// the sweeps' own particle arithmetic in the lane layout of a shape.
struct EvalArgs {
    SweepArgs a;          // target, N, ntiles of the shape
    const float* x;       // device [N][d]
    double* ell;          // device [N]
    double* grad;         // device [N][d]
};

// Validated launch configuration of a VALU sweep.
struct ValuShape {
    int lpp;  // lanes per particle
    int dpl;  // dimensions per lane
};

// Lanes that fill every SIMD of the GPU twice (256 CUs x 4 SIMDs x 64 x 2).
constexpr int64_t kFillLanes = 256 * 4 * 64 * 2;
bool valu_shape(int d, int64_t N, ValuShape* s);

// A batch of problems of one (family, move, shape) class.
struct ValuBatch {
    const SweepArgs* args;   // device [nprob]
    const ParView* views;    // device [nprob]
    const int2* items;       // device [nitems]: (problem, slot), longest first
    int64_t nitems;
    uint32_t* next;          // device work counter, zero at the launch; null: round robin
};
hipError_t launch_oais_valu_batch(int family, int move, const ValuShape& s, const ValuBatch& b,
                                  int grid_waves, hipStream_t st);
// Per-problem parameter buffers of a batched launch (device addresses) and the
// sweep shape whose lane layout lane[] takes.
struct BatchParam {
    float* m;       // [d] reference mean
    double* hiv;    // [kMaxK] 1/(2 v_k)
    double* iv;     // [kMaxK] 1/v_k
    double* lane;   // [lane_param_doubles] lm, then lmu
    int lpp, dpl;
};
// Fills the buffers of every problem with a non-null m (one block each).
hipError_t launch_batch_params(const TargetDev* tgs, const BatchParam* bp, int nprob,
                               hipStream_t st);
int64_t valu_tiles(int64_t N, const ValuShape& s);

hipError_t launch_oais_valu(const SweepArgs& a, const ValuShape& s, int grid_waves,
                            hipStream_t st);
hipError_t launch_asmc_init(const SweepArgs& a, const ValuShape& s, const AsmcState& z,
                            hipStream_t st);
hipError_t launch_asmc_step(const SweepArgs& a, const ValuShape& s, const AsmcState& z, int t,
                            int trigger, double nu, hipStream_t st);
// The resampler after step t: integer CDF, ancestors and the gather into
// X2, G2, ell2 (idle unless the merge flagged an event).  commit copies the
// gathered state back (with log w = 0) for the segment path; the per-step
// path leaves it for the next step kernel to read.
hipError_t launch_resample_step(const SweepArgs& a, const AsmcState& z, int t, bool commit,
                                hipStream_t st);
// Rejuvenation: chains and the per-tile sums, then the fixed-order reduction
// of the tile sums into out [2 d + 1] (averages over N T samples, accepted fraction).
hipError_t launch_rejuv(const RejuvArgs& R, const ValuShape& s, hipStream_t st);
hipError_t launch_pt(const PtArgs& A, const ValuShape& s, hipStream_t st);
// The evaluation kernel is built for the (family, move) pairs (kGauss, kMala),
// (kGmm, kMala) and (kUnid, kRwmh): E.a.move must name that pair's move.
hipError_t launch_target_eval(const EvalArgs& E, const ValuShape& s, hipStream_t st);
// Dynamic LDS of one PT workgroup (staged target parameters, then the
// replicas' ell, rejection sums, temperature maps and a reduction buffer).
__host__ __device__ inline size_t pt_shared_bytes(const PtArgs& A, int lpp, int dpl)
{
    const size_t R = (size_t)A.Np + 1;
    size_t off = params_bytes_lanes(A.a.tg, lpp, dpl);
    off = (off + 15) & ~(size_t)15;
    return off + R * sizeof(double) + (size_t)A.Np * sizeof(double) + 3 * R * sizeof(int) +
           16 * sizeof(double);
}
hipError_t launch_rejuv_reduce(const double* tsum, int64_t ntiles, int d, double samples,
                               double* out, hipStream_t st);
// Systematic resampling of lw[N] for the event word of step t (particle word
// 0xFFFFFFFF, stream 3) of `key`: ancestors anc[N] (all -1 without a finite weight).
hipError_t launch_resample_event(int64_t N, const double* lw, const RngKey& key, uint32_t t,
                                 int32_t* anc, uint64_t* C, uint64_t* btot, double* scal,
                                 hipStream_t st);
// Merge of a segment's slot partials (steps t_begin+1 .. t_end and the segment's
// final log-weights in entry T): moments, accepted counts, the log Z_hat factor
// and, when t_end < T, the resampling event (flag, largest log w, uniform word).
hipError_t launch_segment_merge(const SweepArgs& a, const AsmcState& z, hipStream_t st);
// ZJA (online CESS-adaptive AIS): beta_t by bisection of log CESS on the
// device (one workgroup), then the step's reweight and move without a merge;
// log Z_hat from the final log-weights into logZ[0].
hipError_t launch_zja_select(int64_t N, const double* lw, const double* ell, double* beta, int t,
                             int Tmax, double log_rho, int iters, int* stop, double* log_g,
                             hipStream_t st);
hipError_t launch_asmc_move(const SweepArgs& a, const ValuShape& s, const AsmcState& z, int t,
                            hipStream_t st);
hipError_t launch_zja_final(int64_t N, const double* lw, double* logZ, hipStream_t st);
hipError_t launch_merge_slots(const double* part, int64_t S, int T, int64_t N, double* log_g,
                              double* acc, double* logZ, hipStream_t st);
hipError_t launch_resample_plain(int64_t N, const double* lw, uint32_t u, int32_t* anc,
                                 uint64_t* C, uint64_t* btot, double* scal, hipStream_t st);
// Reverse pass of the pathwise gradient of log Z_hat (mixture target, MALA).
struct AdjointArgs {
    SweepArgs a;          // same target, schedule, keys; ckpt and acc_bits filled by the forward pass
    const double* lw;     // [N] final log-weights of the forward pass
    const double* scal;   // [0] = log Z_hat of the forward pass
    float* seg;           // [N][ckpt_every][d] scratch for one recomputed segment
    double* partial;      // [waves][np] per-wave weighted gradient sums
    int64_t nwaves;
};
bool adjoint_shape(int d, int K, int64_t N, ValuShape* s, int* kb);
hipError_t launch_adjoint(const AdjointArgs& A, const ValuShape& s, int kb, hipStream_t st);
hipError_t launch_adjoint_reduce(const double* partial, int64_t nwaves, int np, double* grad,
                                 hipStream_t st);

// One problem's between-rounds work on the device (Alg. 2 round step).
struct RoundDev {
    int T, Tn;              // this round's and the next round's number of steps
    int64_t N, S;           // particles, slots of the sweep
    const double* part;     // [S][T+1][4] slot partials of the sweep
    const double* beta;     // [T+1] this round's schedule
    const double* eps;      // [T] this round's step sizes
    double* log_g;          // [3T] out
    double* acc;            // [T] out
    double* logZ;           // [1] out
    double* Lambda;         // [T+1] out
    double* beta_next;      // [Tn+1] out
    double* eps_next;       // [Tn] out
    int* status;            // [1] out: 1 when the moments were not finite
    double* scratch;        // [3(T+1)]
    int interp, eps_adapt;
    double eps0, accept_target;
};
hipError_t launch_round_merge(const RoundDev* rd, int nprob, int Tmax, hipStream_t st);
hipError_t launch_round_schedule(const RoundDev* rd, int nprob, hipStream_t st);

hipError_t launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t count,
                         hipStream_t st);

int64_t resample_blocks(int64_t N);

// One logistic-regression problem as its sweep kernel sees it.
struct LogregArgs {
    SweepArgs a;
    const float* Xp;   // packed [n_pad][cols], rows signed by 2 y - 1, padding rows zero
    int n_pad;
    float* gl;         // panel layout: cached gradients at the states, [tiles 32][cols]
    float* glp;        // panel layout: gradients at the proposals, [tiles 32][cols]
};
// Layout class of a problem: the 64-column kernel's half-width KH, or
// 1000 + panels for the panel layout (always above 64 features; below, when
// 64-particle tiles would leave CUs idle); -1 if d is unsupported.  Every
// helper below takes this class.
int logreg_kh(int d, int64_t N, int cus);
int logreg_npad(int n);      // padded row count
int logreg_cols(int kh);     // packed columns
int64_t logreg_tiles(int64_t N, int kh);
size_t logreg_shared_bytes(int kh);
size_t logreg_workspace_bytes(const TargetDev& tg, int64_t N, int kh);
// Points A's data and gradient buffers into a workspace of
// logreg_workspace_bytes(tg, N, kh) bytes.
void logreg_layout(const TargetDev& tg, int64_t N, int kh, void* ws, LogregArgs* A);
// Packs X and y into the class's padded, column-permuted layout in such a
// workspace (logreg_prepare is the same call).
hipError_t logreg_pack_into(const TargetDev& tg, int64_t N, int kh, void* ws, hipStream_t st);
hipError_t logreg_prepare(const TargetDev& tg, int64_t N, int kh, void* ws, hipStream_t st);
hipError_t launch_oais_logreg(const SweepArgs& a, int kh, int cus, void* ws, hipStream_t st);
// items longest first; next: a device work counter that is zero at the launch
// (each workgroup claims the next item when it becomes idle), or null for a
// static round robin over the workgroups
hipError_t launch_oais_logreg_batch(int kh, const LogregArgs* args, const int2* items,
                                   int64_t nitems, uint32_t* next, int grid, hipStream_t st);
hipError_t launch_logreg_eval(const TargetDev& tg, int kh, const float* theta, int64_t N,
                              double* ell, float* grad, void* ws, hipStream_t st);
// Sets / clears the message oasmc_last_error() returns on this thread.
int record_error(int code, const char* fmt, ...);
void clear_error();

// Clears small device scalars with a kernel (no memset nodes, so callers may capture it).
hipError_t launch_zero(double* a, int na, int* b, int nb, hipStream_t st);

}  // namespace oasmc
