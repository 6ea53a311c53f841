// Allocation-free form of accsk_solve_dense: the same routing and kernels, with
// the whole device workspace carved from one fixed array per GPU instead of
// stream-ordered allocations, for callers that cannot allocate device memory.

#include <algorithm>
#include <mutex>

#include "accsk_common.h"

using namespace accsk;

accsk_status accsk_solve_dense_ws(const float *C, int64_t n, int64_t m, int64_t ldc, const double *a,
                                  const double *b, const accsk_params *p, double *f_out, double *g_out,
                                  accsk_result *res, void *stream, Workspace &ws, accsk_result *pub);
size_t accsk_dense_single_bound(int64_t n, int64_t m, int cu);
accsk_status accsk_check_dense_params(const accsk_params *p);

namespace {

constexpr size_t kScratchBytes = ACCSK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of every accsk_solve_dense_noalloc call on a device.  In host
// code `scratch` names a host-side stand-in, never the device array: kernels
// and copies get the device address from hipGetSymbolAddress (one per device).
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char *g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device (with that device current).
accsk_status scratch_on_current_device(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ACCSK_HIP_ERROR;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ACCSK_HIP_ERROR;
        g_scratch[dev] = (char *)ptr;
    }
    *out = g_scratch[dev];
    return ACCSK_OK;
}

}  // namespace

extern "C" accsk_status accsk_solve_dense_noalloc(const float *C, int64_t n, int64_t m, int64_t ldc,
                                                  const double *a, const double *b, const accsk_params *p,
                                                  double *f_out, double *g_out, accsk_result *res,
                                                  void *stream) {
    if (res) {
        res->status = ACCSK_INVALID_ARG;
        res->converged = 0;
    }
    if (!C || !a || !b || !p || !f_out || !g_out || !res) return ACCSK_INVALID_ARG;
    const accsk_status pst = accsk_check_dense_params(p);
    if (pst != ACCSK_OK) return pst;
    if (n < 1 || m < 1 || ldc < m || m > 8192) return ACCSK_SHAPE;
    int dev = 0, cu = 0;
    ACCSK_HIP_TRY(hipGetDevice(&dev));
    ACCSK_HIP_TRY(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (cu <= 0) return ACCSK_HIP_ERROR;
    // checked before anything is enqueued: no call stops half-way for lack of room
    if (accsk_dense_single_bound(n, m, cu) > kScratchBytes) return ACCSK_SHAPE;
    char *base = nullptr;
    const accsk_status sst = scratch_on_current_device(&base);
    if (sst != ACCSK_OK) return sst;
    Workspace ws;
    ws.base = base;
    ws.cap = kScratchBytes;
    return accsk_solve_dense_ws(C, n, m, ldc, a, b, p, f_out, g_out, res, stream, ws, nullptr);
}
