// adjoint.hip -- dispatch of the reverse pass (see adjoint.hpp) and the
// fixed-order reduction of the per-wave gradient sums.
#include "adjoint.hpp"

namespace oasmc {

bool adjoint_shape(int d, int K, int64_t N, ValuShape* s, int* kb)
{
    // the same particle layout as the forward sweep (valu_shape), so that the
    // recomputed segments repeat its arithmetic exactly
    if (d < 1 || d > 32 || K < 1 || K > 8) return false;
    if (!valu_shape(d, N, s)) return false;
    *kb = (K <= 2) ? 2 : (K <= 4 ? 4 : 8);
    return true;
}

hipError_t launch_adjoint(const AdjointArgs& A, const ValuShape& s, int kb, hipStream_t st)
{
#define OASMC_ADJ(L, D, KB_) \
    if (s.lpp == L && s.dpl == D && kb == KB_) return launch_adjoint_t<L, D, KB_>(A, st);
#define OASMC_ADJ_K(L, D) OASMC_ADJ(L, D, 2) OASMC_ADJ(L, D, 4) OASMC_ADJ(L, D, 8)
    OASMC_ADJ_K(1, 4)
    OASMC_ADJ_K(1, 8)
    OASMC_ADJ_K(1, 12)
    OASMC_ADJ_K(1, 16)
    OASMC_ADJ_K(1, 20)
    OASMC_ADJ_K(1, 24)
    OASMC_ADJ_K(2, 16)
    OASMC_ADJ_K(4, 8)
    OASMC_ADJ_K(8, 4)
#undef OASMC_ADJ_K
#undef OASMC_ADJ
    return hipErrorInvalidValue;
}

// One workgroup per parameter: each thread sums a strided share of the wave
// records in wave order, then a fixed tree over the threads (the same bits
// for a given number of waves).
constexpr int kAdjRedThreads = 256;

__global__ void __launch_bounds__(kAdjRedThreads)
    k_adjoint_reduce(const double* __restrict__ partial, int64_t nwaves, int np, double* grad)
{
    __shared__ double red[kAdjRedThreads];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int64_t w = threadIdx.x; w < nwaves; w += kAdjRedThreads) s += partial[(size_t)w * np + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kAdjRedThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[c] = red[0];
}

hipError_t launch_adjoint_reduce(const double* partial, int64_t nwaves, int np, double* grad,
                                 hipStream_t st)
{
    hipLaunchKernelGGL(k_adjoint_reduce, dim3((unsigned)np), dim3(kAdjRedThreads), 0, st, partial,
                       nwaves, np, grad);
    return hipGetLastError();
}

}  // namespace oasmc
