// Status strings, default parameters and version of libaccsk.
#include "accsk_common.h"

// Homotopy start calibrated on the FP64 oracle (minimum geometric-mean
// iteration count over seeded 256 x 256 problems at eps 1e-1, 1e-2, 1e-3; the
// paper leaves mu0 and m0 open and reports insensitivity to them).
static const double kDefaultMu0 = 0.25;
static const int64_t kDefaultM0 = 5;

extern "C" void accsk_default_params(accsk_params *p) {
    if (!p) return;
    p->method = ACCSK_ACC;
    p->w_rule = ACCSK_W_Y_CONTINUOUS;
    p->eps = 1e-2;
    p->tol = 1e-6;
    p->max_iter = 100000;
    p->mu0 = kDefaultMu0;
    p->m0 = kDefaultM0;
    p->split = 0;
    p->flags = 0;
    p->err_trace = nullptr;
    p->trace_len = 0;
}

extern "C" const char *accsk_status_string(int status) {
    switch (status) {
        case ACCSK_OK: return "ok";
        case ACCSK_INVALID_ARG: return "invalid argument";
        case ACCSK_SHAPE: return "unsupported shape, leading dimension or alignment";
        case ACCSK_NONFINITE: return "non-finite value in the input";
        case ACCSK_NOT_CONVERGED: return "not converged within max_iter";
        case ACCSK_DIVERGED: return "marginal error became non-finite";
        case ACCSK_OOM: return "out of device memory or over the HBM budget";
        case ACCSK_HIP_ERROR: return "HIP runtime error";
        case ACCSK_BUSY: return "queue full";
        default: return "unknown status";
    }
}

extern "C" const char *accsk_version(void) { return "accsk 0.1 gfx950"; }
