// Instantiation of the closed-form-target sweeps for one (family, move) pair;
// split into separate translation units so they compile in parallel.
#include "valu_sweep.hpp"

namespace oasmc {
template hipError_t valu_dispatch<kGauss, kRwmh3>(int, const SweepArgs&, const ValuShape&, int,
                                                  const AsmcState*, int, hipStream_t,
                                                  const ValuBatch*, const void*);
}  // namespace oasmc
