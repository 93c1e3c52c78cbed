// lat_apply_combo_noalloc: the ROM apply for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Its scratch -- the
// interleaved coefficients, the refinement's per-block error partials and gates, as laid out for
// the LAT_CALL_APPLY_COMBO workspace -- lives in a file-scope device array `scratch` that every
// GPU the library runs on holds until the process ends.  Host code never passes the array's name
// to a kernel: its device address is taken once per device with hipGetSymbolAddress (with that
// device current) and kept here; that address is what the kernels receive.
#include <mutex>

#include "lat_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[LAT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch_addr[kMaxDevices] = {};

// the device address of `scratch` on the current device (resolved on the first call per device)
lat_status scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return LAT_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            std::fprintf(stderr, "liblat: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
            return LAT_E_DEVICE;
        }
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return LAT_OK;
}

}  // namespace

extern "C" lat_status lat_apply_combo_noalloc(const lat_plan *P, const double *K, int32_t n_r, const double *alpha,
                                              const double *X, double *Y, int32_t m, lat_prec prec,
                                              double refine_tol, int32_t transpose, double *err_est,
                                              hipStream_t stream)
{
    if (!P) return LAT_E_ARG;
    size_t need = 0, fast = 0;
    lat_ws_sizes(P, LAT_CALL_APPLY_COMBO, &need, &fast);
    if (need > (size_t)LAT_NOALLOC_SCRATCH_BYTES) {
        std::fprintf(stderr, "liblat: lat_apply_combo_noalloc needs %zu bytes of scratch, above its %zu-byte maximum\n",
                     need, (size_t)LAT_NOALLOC_SCRATCH_BYTES);
        return LAT_E_SHAPE;
    }
    int device = -1;
    LAT_HIP(hipGetDevice(&device));
    if (device != P->device) return LAT_E_ARG;          // the plan's device must be the current one
    void *work = nullptr;
    const lat_status st = scratch_address(device, &work);
    if (st != LAT_OK) return st;
    return lat_apply_combo(P, K, n_r, alpha, X, Y, m, prec, refine_tol, transpose, err_est, work,
                           (size_t)LAT_NOALLOC_SCRATCH_BYTES, stream);
}
