// Internal helpers shared by the HIP translation units of libaccsk (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "accsk.h"

namespace accsk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;

// Every grid barrier polls at most this many times, with a sleep between polls
// (a few seconds in total)
// before it gives up and reports ACCSK_HIP_ERROR, so a kernel always drains.
constexpr long kBarrierSpinLimit = 1L << 22;

// FP64 transcendentals used off the streaming loops.  Kept out of line so
// the polynomial constants are not hoisted into registers for the whole
// persistent kernel.
__device__ __attribute__((noinline)) inline double dlog2(double x) { return log2(x); }
__device__ __attribute__((noinline)) inline double dexp2(double x) { return exp2(x); }
__device__ __attribute__((noinline)) inline double dsqrt(double x) { return sqrt(x); }
__device__ __attribute__((noinline)) inline double dexpm1(double x) { return expm1(x); }

// Empty asm barriers that make a value opaque to the optimizer (no code emitted).
template <typename T>
__device__ __forceinline__ void opaque_ptr(T *&p) {
    asm volatile("" : "+s"(p));
}
__device__ __forceinline__ void opaque_int(int &v) { asm volatile("" : "+v"(v)); }

// Deterministic wave-level reductions (fixed xor butterfly, 64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// DPP wave reductions (gfx9 row_shr / row_bcast), result valid in lane 63.
// Lanes whose DPP source is out of range keep `old`, the identity of the op.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const long long vo = __double_as_longlong(old), vv = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)vo, (int)vv, CTRL, ROW_MASK, BANK_MASK, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(vo >> 32), (int)(vv >> 32), CTRL, ROW_MASK, BANK_MASK, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_f32(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK,
                                                      BANK_MASK, false));
}
// row_shr:k = 0x110 + k, row_bcast:15 = 0x142, row_bcast:31 = 0x143
__device__ __forceinline__ double wave_sum_l63(double v) {
    v += dpp_f64<0x111, 0xf, 0xf>(0.0, v);
    v += dpp_f64<0x112, 0xf, 0xf>(0.0, v);
    v += dpp_f64<0x114, 0xf, 0xf>(0.0, v);
    v += dpp_f64<0x118, 0xf, 0xf>(0.0, v);
    v += dpp_f64<0x142, 0xa, 0xf>(0.0, v);
    v += dpp_f64<0x143, 0xc, 0xf>(0.0, v);
    return v;
}
__device__ __forceinline__ float wave_max_l63(float v) {
    v = fmaxf(v, dpp_f32<0x111, 0xf, 0xf>(v, v));
    v = fmaxf(v, dpp_f32<0x112, 0xf, 0xf>(v, v));
    v = fmaxf(v, dpp_f32<0x114, 0xf, 0xf>(v, v));
    v = fmaxf(v, dpp_f32<0x118, 0xf, 0xf>(v, v));
    v = fmaxf(v, dpp_f32<0x142, 0xa, 0xf>(v, v));
    v = fmaxf(v, dpp_f32<0x143, 0xc, 0xf>(v, v));
    return v;
}

// Lane 63's value in every lane (wave-uniform).
__device__ __forceinline__ double wave_bcast63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float wave_bcast63f(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Combine NW <= 16 per-wave partials stored in LDS: lane l loads v[l % 16]
// (identity for l % 16 >= NW), a 16-lane DPP reduction leaves the total in
// lane 15 of every row, and readlane makes it uniform.  Same order everywhere.
template <int NW>
__device__ __forceinline__ double lds_combine_sum(const double *v, int lane) {
    const int r = lane & 15;
    double x = r < NW ? v[r] : 0.0;
    x += dpp_f64<0x111, 0xf, 0xf>(0.0, x);
    x += dpp_f64<0x112, 0xf, 0xf>(0.0, x);
    x += dpp_f64<0x114, 0xf, 0xf>(0.0, x);
    x += dpp_f64<0x118, 0xf, 0xf>(0.0, x);
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, 15);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 15);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int NW>
__device__ __forceinline__ float lds_combine_max(const float *v, int lane) {
    const int r = lane & 15;
    float x = r < NW ? v[r] : -INFINITY;
    x = fmaxf(x, dpp_f32<0x111, 0xf, 0xf>(x, x));
    x = fmaxf(x, dpp_f32<0x112, 0xf, 0xf>(x, x));
    x = fmaxf(x, dpp_f32<0x114, 0xf, 0xf>(x, x));
    x = fmaxf(x, dpp_f32<0x118, 0xf, 0xf>(x, x));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 15));
}

// Barrier over the `nblocks` workgroups of one problem of a cooperative
// launch (all of them are co-resident).  `bar` points at two zeroed
// 64-bit words 128 bytes apart: bar[0] counts arrivals, bar[16] holds the
// number of the last completed barrier.  `gen` counts the barriers this block
// has passed (uniform).
// Every wave first drains its own memory operations (s_waitcnt 0), so after
// the workgroup barrier all of the block's stores have reached L2; one thread
// then makes them visible device-wide (agent release: L2 write-back) and
// arrives.  The block whose arrival completes the count publishes `gen` in the
// flag word; the others poll the flag with relaxed loads (they bypass the
// per-XCD L2 without invalidating it), away from the counter's cache line.
// One agent acquire (L2/L1 invalidate) follows.  Returns false if the wait
// exceeded kBarrierSpinLimit.
__device__ __forceinline__ bool grid_sync(unsigned long long *bar, unsigned long long &gen,
                                          int *lds_flag, unsigned nblocks) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    gen += 1;
    if (threadIdx.x == 0) {
        const unsigned long long target = gen * (unsigned long long)nblocks;
        unsigned long long *flag = bar + 16;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned long long prev =
            __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        if (prev + 1 == target) {
            __hip_atomic_store(flag, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
                __builtin_amdgcn_s_sleep(4);
                if (++spins > kBarrierSpinLimit) {
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *lds_flag = ok;
    }
    __syncthreads();
    return *lds_flag != 0;
}

// Stores/loads of data exchanged between blocks between two grid barriers:
// agent-scope relaxed accesses are coherent across XCDs (written through /
// read past the per-XCD L2), so the barrier's L2 write-back finds little.
__device__ __forceinline__ void xstore(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xstore(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Four floats to bytes [off, off + 16) of a raw buffer, with SC1 set: the
// line is written through the XCD's L2 like xstore's, for per-block results
// too large for single-word stores (column partials: with plain stores, the
// barrier's write-back of 8 MB of dirty partials cost ~6 us per step).
__device__ __forceinline__ void xstore4(__amdgpu_buffer_rsrc_t r, int off, float4 v) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    constexpr int kSC1 = 16;  // cache-policy operand of a raw buffer access: SC1
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, kSC1);
}
__device__ __forceinline__ float xload(const float *p) {
    return __hip_atomic_load(const_cast<float *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xload(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stability monitor: the reduced dual objective f(x) = 1 - <u,a> - <x,b>
// (Lemma coercivity, App. A) falls along plain Sinkhorn (Lemma
// sinkhorn-descent) but not necessarily along Acc-Sinkhorn.  A rise above the
// rounding of f computed from FP32 exponentials counts as an increase.
__device__ __forceinline__ bool fval_rose(double fval, double fprev) {
    return fval > fprev + (1e-8 + 1e-12 * fabs(fval));
}

// Boundedness monitor of the Acc iterates (App. B, Theorem
// thm:condition-boundedness, and the shifted Lyapunov function of its proof),
// evaluated under ACCSK_FLAG_CONDITIONS.  For an iterate (x_k, w_k):
//   p = log(c ./ b) with c the column sums of P at (u(x_k), x_k),
//   xi = grad f(x_k) = c - b = b (e^p - 1),
//   D_k = diag(b (e^p - 1) ./ p) (eq:D: the logarithmic mean of c and b),
//   K_k = D_phi*(0, xi) = sum_j b_j (e^p_j - 1 - p_j),
//   v_k = w_k / alpha - x_k,
//   E_k = f(x_k) + (mu/2) ||v_k||^2_{D_k} - theta/(1 + alpha) K_k, theta = (1/2 + alpha)/(1 + alpha),
// and for consecutive iterates of one homotopy stage the two conditions
//   sum xi_k^2 D_k+1 / D_k^2 < (4 - alpha^2 - 2 alpha^(1/2)) / (2 alpha (1 + alpha)^2) K_k,
//   sum v_k^2 (D_k+1 - D_k)  < alpha^(3/2) sum v_k+1^2 D_k+1,
// and a rise of E above 1e-8 + 1e-12 |f| + 1e-6 ((mu/2) ||v||^2_D + ||xi||_1) (the rounding of
// values formed from FP32 exponentials).  At a stage change the last iterate, with w as handed to
// the new stage and the new alpha and mu, starts the next stage's comparisons.
struct CondTerms {
    double xi, D, K;
};
// xi, D and K of one column from p = log(c_j / b_j): Horner forms of
// b sum p^k/(k+1)! (D) and b sum_{k>=2} p^k/k! (K) for |p| < 1e-2, where
// e^p - 1 - p would cancel; closed forms otherwise.
__device__ inline CondTerms cond_terms(double p, double b) {
    CondTerms t;
    if (fabs(p) < 1e-2) {
        // q = sum_{k=0..8} p^k/(k+1)!  (e^p - 1 = p q);  r = sum_{k=0..7} p^k/(k+2)!  (e^p - 1 - p = p^2 r)
        double r = 1.0 / 3628800.0;
        r = fma(r, p, 1.0 / 362880.0);
        r = fma(r, p, 1.0 / 40320.0);
        r = fma(r, p, 1.0 / 5040.0);
        r = fma(r, p, 1.0 / 720.0);
        r = fma(r, p, 1.0 / 120.0);
        r = fma(r, p, 1.0 / 24.0);
        r = fma(r, p, 1.0 / 6.0);
        r = fma(r, p, 0.5);
        const double q = fma(r, p, 1.0);
        t.xi = b * p * q;
        t.D = b * q;
        t.K = b * p * p * r;
    } else {
        const double em = dexpm1(p);
        t.xi = b * em;
        t.D = t.xi / p;
        t.K = b * (em - p);
    }
    return t;
}
// Running state of the monitor (identical wherever it is kept).
struct CondState {
    double Kb, Eb;          // the last iterate's K and E
    long long n1, n2, nl;   // violations of conditions 1 and 2, rises of E
};
__device__ inline double cond_lyap(double fval, double vd, double K, double alpha, double mu) {
    return fval + 0.5 * mu * vd - (0.5 + alpha) / ((1.0 + alpha) * (1.0 + alpha)) * K;
}
// One new iterate from the sums over its columns: lhs1 = sum xi_b^2 D / D_b^2,
// lhs2 = sum v_b^2 (D - D_b), vd = sum v^2 D, K = sum K_j, l1 = sum |xi|
// (b: the previous iterate).  have: a previous iterate of the same stage exists.
__device__ inline void cond_decide(CondState &s, bool have, double lhs1, double lhs2, double vd, double K,
                                   double l1, double fval, double alpha, double mu) {
    const double E = cond_lyap(fval, vd, K, alpha, mu);
    if (have) {
        const double sa = dsqrt(alpha);
        const double k1 = (4.0 - alpha * alpha - 2.0 * sa) / (2.0 * alpha * (1.0 + alpha) * (1.0 + alpha));
        if (!(lhs1 < k1 * s.Kb)) s.n1++;
        if (!(lhs2 < alpha * sa * vd)) s.n2++;
        if (E > s.Eb + 1e-8 + 1e-12 * fabs(fval) + 1e-6 * (0.5 * mu * vd + l1)) s.nl++;
    }
    s.Kb = K;
    s.Eb = E;
}

// The columns the monitor walks: x, w, S^ in log2 units (S^ not centred), b
// normalized; xib, Db, vb hold grad f, D and v of the previous iterate and
// receive those of the new one.
struct CondCols {
    const double *x, *w, *sh, *b;
    double *xib, *Db, *vb;
};
struct CondSums {
    double lhs1, lhs2, vd, K, l1, vd2;  // vd2: sum v^2 D with v rebased to the next stage
};
namespace {
// Per-thread monitor sums over columns j0 + t, j0 + t + stride, ... < j1.  The
// new iterate's w_k is w as stored (upd 0), (w + c2 x + 2 (sh - mean)) inv_w
// (upd 1, the A2MD w update not yet applied) or alpha x (upd 2, a restart).
// have: compare with the previous iterate; stage: the iterate also starts the
// next stage (v rebased with w * ratio / a_new).  Only the diagnostic
// instantiations of the solver kernels contain it (its FP64 transcendentals
// would otherwise enter the register allocation of the production kernels).
__device__ __forceinline__ CondSums cond_cols(CondCols c, long long j0, long long j1, long long stride,
                                                        int upd, double mean, double c2, double inv_w, double alpha,
                                                        int have, int stage, double ratio, double a_new) {
    CondSums s{0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long j = j0; j < j1; j += stride) {
        const double xv = c.x[j], sh = c.sh[j];
        double w = c.w[j];
        if (upd == 1) w = (w + c2 * xv + 2.0 * (sh - mean)) * inv_w;
        else if (upd == 2) w = alpha * xv;
        const CondTerms t = cond_terms((xv - sh) * kLn2, c.b[j]);
        const double v = (w / alpha - xv) * kLn2;
        if (have) {
            const double xo = c.xib[j], dd = c.Db[j], vo = c.vb[j];
            s.lhs1 += xo * xo * t.D / (dd * dd);
            s.lhs2 += vo * vo * (t.D - dd);
        }
        s.vd += v * v * t.D;
        s.K += t.K;
        s.l1 += fabs(t.xi);
        double vn = v;
        if (stage) {
            vn = (w * ratio / a_new - xv) * kLn2;
            s.vd2 += vn * vn * t.D;
        }
        c.xib[j] = t.xi;
        c.Db[j] = t.D;
        c.vb[j] = vn;
    }
    return s;
}
}  // namespace

// Device-side result record copied back to the host accsk_result.
struct DevResult {
    long long iters;
    long long steps;
    long long fallback;
    long long incr;      // steps at which the reduced dual objective rose (stability monitor)
    long long restarts;  // extrapolation resets (ACCSK_FLAG_RESTART)
    long long cond1, cond2, lyap;  // boundedness monitor counts (-1: not evaluated)
    double err;
    double eot;
    double fval;
    double cost;
    long long t0, t1;    // device wall clock (wall_clock64 ticks) at the start and end of the solve
    int converged;
    int status;
};

// Device wall clock (constant rate, hipDeviceAttributeWallClockRate kHz).
__device__ __forceinline__ long long dev_clock() { return (long long)wall_clock64(); }

// Milliseconds per wall_clock64 tick of the current device (0 if unknown).
inline double wall_tick_ms() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0.0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return 0.0;
    return 1.0 / (double)khz;
}

// Copies a device result record into the public one.  kms < 0: the solve's
// duration is taken from the record's device clock stamps instead of events.
inline void fill_result(accsk_result &o, const DevResult &r, double kms) {
    o.iters = r.iters;
    o.sinkhorn_steps = r.steps;
    o.fallback_steps = r.fallback;
    o.fval_increases = r.incr;
    o.restarts = r.restarts;
    o.cond1_violations = r.cond1;
    o.cond2_violations = r.cond2;
    o.lyap_increases = r.lyap;
    o.marginal_err = r.err;
    o.eot_value = r.eot;
    o.transport_cost = r.cost;
    o.dual_fval = r.fval;
    if (kms < 0.0) {
        const double tick = wall_tick_ms();
        kms = (tick > 0.0 && r.t1 >= r.t0) ? (double)(r.t1 - r.t0) * tick : -1.0;
    }
    o.kernel_ms = kms;
    o.converged = r.converged;
    o.status = r.status;
    if (r.status == ACCSK_OK && !r.converged) o.status = ACCSK_NOT_CONVERGED;
}

// Device form of fill_result for the stream-ordered entry points: the record
// is written by the device, the duration taken from the device clock stamps.
__device__ inline void publish_record(accsk_result *o, const DevResult &r, double tick_ms) {
    o->iters = r.iters;
    o->sinkhorn_steps = r.steps;
    o->fallback_steps = r.fallback;
    o->fval_increases = r.incr;
    o->restarts = r.restarts;
    o->cond1_violations = r.cond1;
    o->cond2_violations = r.cond2;
    o->lyap_increases = r.lyap;
    o->marginal_err = r.err;
    o->eot_value = r.eot;
    o->transport_cost = r.cost;
    o->dual_fval = r.fval;
    o->kernel_ms = (tick_ms > 0.0 && r.t1 >= r.t0) ? (double)(r.t1 - r.t0) * tick_ms : -1.0;
    o->converged = r.converged;
    o->status = (r.status == ACCSK_OK && !r.converged) ? ACCSK_NOT_CONVERGED : r.status;
}

// Host-to-device copy of a small host array through kernel arguments, for the
// stream-ordered entry points: the runtime copies a launch's arguments when
// the launch is enqueued, so the host array may go away as soon as the call
// returns, and nothing waits for earlier work on the stream (a hipMemcpyAsync
// from pageable host memory may).
struct ArgBlob {
    unsigned char b[2048];
};
namespace {
__global__ __launch_bounds__(256) void upload_blob(ArgBlob blob, unsigned nbytes, unsigned char *dst) {
    for (unsigned i = threadIdx.x; i < nbytes; i += 256) dst[i] = blob.b[i];
}
}  // namespace
inline hipError_t upload_args(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const unsigned char *p = (const unsigned char *)src;
    unsigned char *d = (unsigned char *)dst;
    for (size_t off = 0; off < bytes; off += sizeof(ArgBlob)) {
        ArgBlob blob;
        const size_t nb = bytes - off < sizeof(ArgBlob) ? bytes - off : sizeof(ArgBlob);
        for (size_t i = 0; i < nb; i++) blob.b[i] = p[off + i];
        hipLaunchKernelGGL(upload_blob, dim3(1), dim3(256), 0, s, blob, (unsigned)nb, d + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Device workspace of one library call.  By default it is stream-ordered
// (hipMallocAsync / hipFreeAsync on the call's stream).  Over a fixed region
// (base != nullptr) it hands out 256-byte aligned slices in stack order and
// allocates nothing; put() releases a slice and every slice taken after it.
struct Workspace {
    char *base = nullptr;
    size_t cap = 0, top = 0;
    bool fixed() const { return base != nullptr; }
    hipError_t get(void **p, size_t bytes, hipStream_t s) {
        if (!base) return hipMallocAsync(p, bytes, s);
        const size_t b = (bytes + 255) & ~size_t(255);
        if (b > cap - top) return hipErrorOutOfMemory;
        *p = base + top;
        top += b;
        return hipSuccess;
    }
    void put(void *p, hipStream_t s) {
        if (!p) return;
        if (!base) {
            (void)hipFreeAsync(p, s);
            return;
        }
        char *c = (char *)p;
        if (c >= base && c < base + top) top = (size_t)(c - base);
    }
};

}  // namespace accsk

#define ACCSK_HIP_TRY(expr)                                  \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return ACCSK_HIP_ERROR;        \
    } while (0)
