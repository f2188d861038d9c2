// sigma = H c without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The pair kernels' store-and-reduce workspace (one FP64 contribution per
// target determinant, occupied pair of the target and vector, read back by
// the reduce) comes from `scratch`, a file-scope device array of
// kScratchBytes that each device holds from the first context created on it
// until the process ends.  Host code never passes `scratch` itself (its host
// name is a stand-in, not a device address): stpci_create resolves the
// array's address on its device once with hipGetSymbolAddress, and every
// launch takes that address.  Calls on one device share the array, so calls
// that overlap on one device (two streams, two threads) race; the workspace
// is written in full by every sigma before the reduce reads it, so nothing
// has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <sstream>

#include "ctx.hpp"
#include "kernels.hpp"

namespace stp {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device

// With `device` current: resolve the address of this device's copy of the
// array once (later calls return the stored address).
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

static void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace stp

using namespace stp;

extern "C" int64_t stpci_sigma_noalloc_max_bytes(void) { return (int64_t)kScratchBytes; }

extern "C" stpci_status stpci_sigma_noalloc(stpci_ctx* c, const void* c_dev, void* sigma_dev, int n_vec,
                                            stpci_precision prec) {
    if (!c) return STPCI_EINVAL;
    if (c->host_only) return set_err(c, STPCI_ESTATE, "host-only context has no device");
    if (!c_dev || !sigma_dev || n_vec < 1) return set_err(c, STPCI_EINVAL, "bad sigma arguments");
    if (prec != STPCI_FP64 && prec != STPCI_FP32 && prec != STPCI_BF16)
        return set_err(c, STPCI_EINVAL, "unsupported sigma precision");
    // every table must already be on the device: building it would allocate
    if (!c->prepared)
        return set_err(c, STPCI_ESTATE,
                       "device tables not built: call stpci_sigma or stpci_diagonal once after setting the "
                       "integrals and the space");
    if (prec == STPCI_FP32 && !c->have32)
        return set_err(c, STPCI_ESTATE, "FP32 integral copies not built: call stpci_sigma with STPCI_FP32 once");
    if (prec == STPCI_BF16 && !c->have_bf)
        return set_err(c, STPCI_ESTATE, "bfloat16 pair table not built: call stpci_sigma with STPCI_BF16 once");
    stpci_status s = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (s) return s;
    const size_t bytes = (size_t)c->hs.sp.ndets * scalar_bytes(c) * n_vec;
    const char* a = (const char*)c_dev;
    const char* b = (const char*)sigma_dev;
    if (a < b + bytes && b < a + bytes) return set_err(c, STPCI_EINVAL, "c_dev and sigma_dev overlap");
    void* ws = scratch_ptr(c->device);
    if (!ws) return set_err(c, STPCI_EHIP, "the no-allocation scratch array has no address on this device");
    if (c->s2_kernel == 4 && c->pair_store) {
        const size_t need = pair_store_bytes(c->dev, c->cplx);
        if (need > kScratchBytes) {
            std::ostringstream o;
            o << "the pair contribution workspace of this space (" << need
              << " bytes) exceeds the no-allocation scratch array (" << kScratchBytes << " bytes)";
            return set_err(c, STPCI_EINVAL, o.str());
        }
    }
    // no profiling events here: creating them would allocate
    const bool prof = c->profile;
    c->profile = false;
    s = sigma_impl(c, c_dev, sigma_dev, n_vec, prec, ws);
    c->profile = prof;
    return s;
}
