// Allocation-free RMSE: lshmf_rmse without a context, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The FP64 partial sums that lshmf_rmse keeps in the context's arena live
// here in a file-scope device array instead.  Each GPU holds its own copy of
// the array at its own address, looked up once per device with
// hipGetSymbolAddress; host code never passes the array's name to a kernel.
#include <mutex>

#include "common.hpp"

// kRmsePartials FP64 partials: 4 KiB per device, held until the process ends.
static __device__ __align__(256) double scratch[lshmf::kRmsePartials];

namespace lshmf {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
int scratch_of_current_device(double** out)
{
    int dev = -1;
    LSHMF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("lshmf_rmse_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
        return LSHMF_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (p == nullptr) {
            set_error("lshmf_rmse_noalloc: no device address for the scratch array");
            return LSHMF_EDEVICE;
        }
        g_scratch[dev] = static_cast<double*>(p);
    }
    *out = g_scratch[dev];
    return LSHMF_OK;
}

}  // namespace
}  // namespace lshmf

extern "C" int lshmf_rmse_noalloc(const float* d_pred, const uint8_t* d_rc, int64_t n, int32_t rscale,
                                  double* d_out, lshmf_stream_t stream)
{
    using namespace lshmf;
    if (!d_out || n < 0 || (n > 0 && (!d_pred || !d_rc)) || (rscale != 1 && rscale != 2)) {
        set_error("lshmf_rmse_noalloc: bad arguments (need d_out, n >= 0, data pointers when n > 0, "
                  "rscale 1 or 2)");
        return LSHMF_EINVAL;
    }
    // The reduction always uses kRmsePartials partials, whatever n; the
    // array is sized for exactly that many.
    static_assert(sizeof(scratch) >= kRmsePartials * sizeof(double), "scratch holds every partial");
    double* partial = nullptr;
    LSHMF_TRY(scratch_of_current_device(&partial));
    return rmse_with(d_pred, d_rc, n, rscale, partial, d_out, reinterpret_cast<hipStream_t>(stream));
}
