// noalloc.hip -- systematic resampling for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Same kernels and same result as oasmc_resample; the scratch
// (integer CDF, block totals, flag words) lives in a fixed file-scope device
// array instead of the handle's workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/oasmc.h"
#include "kernels.hpp"

using namespace oasmc;

namespace {

// Layout of the scratch array: C[kNoAllocMaxN] (uint64), then the block totals
// (uint64, one per scan block of the largest N), then 8 binary64 flag words.
constexpr int64_t kNoAllocMaxN = OASMC_NOALLOC_MAX_N;
constexpr int64_t kMaxScanBlocks = 512;  // resample_blocks(kNoAllocMaxN), checked below
constexpr size_t kOffC = 0;
constexpr size_t kOffBtot = kOffC + (size_t)kNoAllocMaxN * sizeof(uint64_t);
constexpr size_t kOffScal = kOffBtot + (size_t)kMaxScanBlocks * sizeof(uint64_t);
constexpr size_t kScratchBytes = kOffScal + 8 * sizeof(double);

constexpr int kMaxDevices = 64;

}  // namespace

// One copy per GPU the library runs on, held until the process ends.  In host
// code this name is only a stand-in for the symbol: its device address comes
// from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch, looked up once per device (the
// current device is the caller's).
int scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return record_error(OASMC_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return record_error(OASMC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return record_error(OASMC_EHIP, "hipGetSymbolAddress(scratch) failed: %s",
                         hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return OASMC_OK;
}

}  // namespace

extern "C" int oasmc_resample_noalloc(int64_t N, const double* lw, uint32_t u, int32_t* anc,
                                      void* stream)
{
    if (!lw || !anc) return record_error(OASMC_EINVAL, "NULL argument");
    if (N < 1 || N > kNoAllocMaxN)
        return record_error(OASMC_EINVAL, "N must lie in [1, %lld] (size of the static scratch)",
                     (long long)kNoAllocMaxN);
    if (resample_blocks(kNoAllocMaxN) > kMaxScanBlocks)
        return record_error(OASMC_EINVAL, "scratch layout too small for the scan blocks");
    void* base = nullptr;
    const int rc = scratch_ptr(&base);
    if (rc != OASMC_OK) return rc;
    unsigned char* b = static_cast<unsigned char*>(base);
    uint64_t* C = reinterpret_cast<uint64_t*>(b + kOffC);
    uint64_t* bt = reinterpret_cast<uint64_t*>(b + kOffBtot);
    double* scal = reinterpret_cast<double*>(b + kOffScal);
    // every word of C, the block totals and the flags that the kernels read is
    // written earlier in the same call's kernel sequence, so nothing is
    // cleared; nothing is copied back (the call stays asynchronous)
    const hipError_t e = launch_resample_plain(N, lw, u, anc, C, bt, scal, (hipStream_t)stream);
    if (e != hipSuccess)
        return record_error(OASMC_EHIP, "launch failed: %s", hipGetErrorString(e));
    clear_error();
    return OASMC_OK;
}
