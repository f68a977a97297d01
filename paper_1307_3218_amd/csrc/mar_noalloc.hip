// The solve entry point for callers that cannot allocate device memory: code
// under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// Its workspace is `scratch`, a file-scope device array of MAR_NOALLOC_SCRATCH_BYTES
// that every GPU the library runs on holds until the process ends. In host code
// the array's name is only a host-side stand-in, so its device address is
// taken once per device with hipGetSymbolAddress (with that device current)
// and only that address is ever handed to the solve. Calls on one GPU share the
// array and it keeps the last call's contents; the solve clears what it needs
// cleared itself, exactly as on the context's own (reused) workspace. Calls that
// overlap on one GPU race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mar.h"
#include "mar_internal.h"

namespace {

constexpr size_t kScratchBytes = MAR_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

// Address of `scratch` on device dev (current), looked up at the first call on that device.
hipError_t scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" mar_status mar_solve_async_noalloc(mar_ctx* ctx, const int32_t* d_seeds, int64_t n_seeds, int32_t nu,
                                              double mu, double kT, mar_precision prec, mar_form form, double* d_rho,
                                              double* d_e_band, double* d_e_seed, double* d_n_seed, int32_t* d_nu_eff,
                                              double* d_eps, double* d_weight, void* hip_stream) {
    if (!ctx) return MAR_ERR_STATE;
    const int dev = mar::ctx_device(ctx);
    if (dev < 0 || dev >= kMaxDevices) return mar::ctx_error(ctx, MAR_ERR_STATE, "device index outside [0, 64)");
    if (hipSetDevice(dev) != hipSuccess) return mar::ctx_error(ctx, MAR_ERR_HIP, "hipSetDevice failed");
    void* ws = nullptr;
    if (scratch_address(dev, &ws) != hipSuccess || !ws)
        return mar::ctx_error(ctx, MAR_ERR_HIP, "hipGetSymbolAddress of the static scratch failed");
    return mar::solve_async_ext(ctx, d_seeds, n_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed, d_n_seed,
                                d_nu_eff, d_eps, d_weight, ws, kScratchBytes, hip_stream);
}
