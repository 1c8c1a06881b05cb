// device_common.hpp -- device-side building blocks shared by the gfx950 kernels:
// the Philox4x32-10 counter-based generator (Salmon et al., SC'11), binary64
// Box-Muller normals, log-domain accumulation helpers and lane-group
// reductions for 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oasmc {

constexpr int kWave = 64;

// Random-number streams (the fourth counter word carries stream, substep and
// block): initial draw from eta, move normals, accept uniform, resampling.
enum Stream : uint32_t { kStreamInit = 0, kStreamMove = 1, kStreamAccept = 2, kStreamResample = 3 };

struct RngKey {
    uint32_t k0, k1;  // seed low / high words
    uint32_t c2;      // (round & 0xFFFF) | (problem << 16)
};

// Both forms give the same words.  FUSED takes each 32 x 32 -> 64-bit
// product in one multiply (v_mad_u64_u32: fewer quarter-rate instructions,
// used by the VALU sweeps); the split form (low and high halves apart) keeps
// the logistic-regression sweep's register spills off its per-step path
// (1.2% faster there).
template <bool FUSED = true>
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t lo0, hi0, lo1, hi1;
        if constexpr (FUSED) {
            const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
            const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
            lo0 = (uint32_t)p0;
            hi0 = (uint32_t)(p0 >> 32);
            lo1 = (uint32_t)p1;
            hi1 = (uint32_t)(p1 >> 32);
        } else {
            lo0 = 0xD2511F53u * c.x;
            hi0 = __umulhi(0xD2511F53u, c.x);
            lo1 = 0xCD9E8D57u * c.z;
            hi1 = __umulhi(0xCD9E8D57u, c.z);
        }
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

template <bool FUSED = true>
__device__ __forceinline__ uint4 draw_block(const RngKey& key, uint32_t n, uint32_t t,
                                            uint32_t stream, uint32_t substep, uint32_t block)
{
    const uint4 ctr = make_uint4(n, t, key.c2, (stream << 24) | ((substep & 0xFFu) << 16) |
                                                   (block & 0xFFFFu));
    return philox4x32_10<FUSED>(ctr, key.k0, key.k1);
}

// Open-interval uniform from one 32-bit word: (w + 1/2) 2^-32, exact in binary64.
__device__ __forceinline__ double word_uniform(uint32_t w)
{
    return ((double)w + 0.5) * 0x1p-32;
}

// Box-Muller in binary64: (wa, wb) -> (r cos 2 pi u_b, r sin 2 pi u_b), r = sqrt(-2 log u_a).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& zc, double& zs)
{
    const double r = sqrt(-2.0 * log(word_uniform(wa)));
    double s, c;
    sincospi(2.0 * word_uniform(wb), &s, &c);
    zc = r * c;
    zs = r * s;
}

// Normals 4b .. 4b+3 of a (particle, step, stream, substep) sequence.  With
// need = 2 only the first pair is formed (the caller uses normals 4b, 4b+1
// only: coordinates 4b+2 and up lie beyond d); z[2], z[3] are then zero.
template <bool FUSED = true>
__device__ __forceinline__ void normals4(const RngKey& key, uint32_t n, uint32_t t,
                                        uint32_t stream, uint32_t block, double z[4],
                                        uint32_t substep = 0u, int need = 4)
{
    const uint4 w = draw_block<FUSED>(key, n, t, stream, substep, block);
    box_muller(w.x, w.y, z[0], z[1]);
    if (need > 2) {
        box_muller(w.z, w.w, z[2], z[3]);
    } else {
        z[2] = 0.0;
        z[3] = 0.0;
    }
}

// log(exp(a) + exp(b)) with -inf handled.
__device__ __forceinline__ double log_add(double a, double b)
{
    const double m = fmax(a, b);
    if (m == -INFINITY) return -INFINITY;
    return m + log1p(exp(-fabs(a - b)));
}

// (max, scaled sum) pair merge for streaming log-sum-exp.
__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2)
{
    const double M = fmax(m, m2);
    if (M == -INFINITY) {
        m = -INFINITY;
        s = 0.0;
        return;
    }
    s = s * exp(m - M) + s2 * exp(m2 - M);
    m = M;
}

__device__ __forceinline__ double lse_value(double m, double s)
{
    return (s > 0.0) ? m + log(s) : -INFINITY;
}

// A binary64 value from another lane of the same row of 16, by a DPP
// permutation (a VALU move: no LDS traffic, unlike a general shuffle).  Every
// control used here reads a valid lane for every lane, so the moves carry no
// "old" operand (no extra register initialisation per move).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// DPP controls: quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1]
// (lane ^ 2), row_half_mirror (i -> 7 - i within 8), row_mirror (i -> 15 - i).
constexpr int kDppXor1 = 0xB1;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

// Sum over aligned groups of G lanes (G a power of two <= 64).  All lanes of a
// group end with the same bits: each level adds the partial sums of two
// disjoint halves, and the two lanes of a pair add the same operands (the sum
// is commutative), so the tree is that of the xor butterfly.  Levels inside a
// row of 16 lanes use DPP; wider levels use shuffles.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (G >= 2) v += dpp_f64<kDppXor1>(v);
    if constexpr (G >= 4) v += dpp_f64<kDppXor2>(v);
    if constexpr (G >= 8) v += dpp_f64<kDppHalfMirror>(v);
    if constexpr (G >= 16) v += dpp_f64<kDppMirror>(v);
#pragma unroll
    for (int o = 16; o < G; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Wave-wide max and sum (xor butterflies: every lane ends with the same bits).
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// log sum_j exp(v_j) over the values of a wave: the maximum, then the sum of
// exp(v_j - max) (-inf when every value is -inf).  Fixed order.
__device__ __forceinline__ double wave_lse(double v)
{
    const double m = wave_max(v);
    const double s = wave_sum((m > -INFINITY && v > -INFINITY) ? exp(v - m) : 0.0);
    return lse_value(m, s);
}

}  // namespace oasmc
