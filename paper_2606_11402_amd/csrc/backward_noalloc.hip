// vecchia_backward without a caller-provided scratch buffer, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  The scratch of the reverse sweep
// and of the theta reduction lives in a file-scope device array of fixed
// size; each GPU the library runs on holds its own copy until the process
// ends.  Its device address is looked up once per device (with that device
// current) and every launch uses that address: in host code the array's name
// is only a host-side stand-in for the symbol.  The kernels are the ones of
// vecchia_backward; nothing here allocates.
#include <mutex>

#include "common.h"
#include "status.h"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;   // w (N doubles) + n0 + per-block partials
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return vecchia_set_error(VECCHIA_EHIP, "vecchia_backward_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "vecchia_backward_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return vecchia_set_error(VECCHIA_EHIP, "vecchia_backward_noalloc: hipGetSymbolAddress: %s",
                                     hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return VECCHIA_OK;
}

}  // namespace

extern "C" int vecchia_backward_noalloc_max_bytes(size_t* bytes) {
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_noalloc_max_bytes: bytes is NULL");
    *bytes = kStaticScratchBytes;
    return VECCHIA_OK;
}

extern "C" int vecchia_backward_noalloc(const vecchia_view* view, const vecchia_kernel* kern, const void* xi,
                                        const void* v, const void* v_bar, const void* xi_bar_in, double logdet_bar,
                                        void* xi_bar, void* v_bar_out, double* theta_bar, void* stream) {
    vecchia_clear_error();
    size_t need = 0;
    int rc = vecchia_backward_scratch_bytes(view, &need);     // validates the view on the host
    if (rc) return rc;
    if (need > kStaticScratchBytes)
        return vecchia_set_error(VECCHIA_ENOMEM,
                                 "vecchia_backward_noalloc: this view needs %zu bytes of scratch, the static buffer "
                                 "holds %zu (about %zu points); use vecchia_backward with a scratch buffer",
                                 need, kStaticScratchBytes, kStaticScratchBytes / 8);
    void* p = nullptr;
    if ((rc = scratch_address(&p))) return rc;
    return vecchia_backward(view, kern, xi, v, v_bar, xi_bar_in, logdet_bar, xi_bar, v_bar_out, theta_bar, p,
                            kStaticScratchBytes, stream);
}
