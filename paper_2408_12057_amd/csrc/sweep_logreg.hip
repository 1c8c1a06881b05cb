// placeholder: replaced by the MFMA logistic-regression sweep
#include "kernels.hpp"
namespace oasmc {
hipError_t launch_oais_logreg(const SweepArgs&, int, void*, size_t, hipStream_t) { return hipErrorNotSupported; }
size_t logreg_workspace_bytes(const TargetDev&, int64_t) { return 256; }
int64_t logreg_tiles(int64_t N) { return (N + 63) / 64; }
}
