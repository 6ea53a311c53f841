// Batched small-problem solver: one workgroup owns one dense problem (m <= 1024,
// n <= 4096), no grid-wide barrier; every reduction is inside the workgroup.
// The per-workgroup solve is small_body (small_body.h), also used by the
// serving loop.

#include <math.h>

#include <algorithm>
#include <vector>

#include "small_body.h"

namespace accsk {
namespace {

template <int NW, int LPR, int NCL, bool VEC, bool DG>
__global__ __launch_bounds__(64 * NW) void small_solve(const SmallProb *__restrict__ probs, SmallCtl ctl,
                                                       DevResult *__restrict__ results) {
    extern __shared__ double lds[];
    __shared__ double red[NW];
    __shared__ int sflag;
    small_body<NW, LPR, NCL, VEC, DG>(probs[blockIdx.x], ctl, results + blockIdx.x, lds, red, sflag);
}

template <int NW, int LPR, int NCL, bool VEC, bool DG>
hipError_t launch_small(const SmallProb *d_probs, int count, const SmallCtl &ctl, DevResult *d_res, size_t lds,
                        hipStream_t s) {
    hipLaunchKernelGGL((small_solve<NW, LPR, NCL, VEC, DG>), dim3(count), dim3(64 * NW), lds, s, d_probs, ctl,
                       d_res);
    return hipGetLastError();
}

// DG: the diagnostic instantiation (boundedness monitor).
template <bool VEC, bool DG>
hipError_t launch_small_cfg(long long mmax, const SmallProb *d_probs, int count, const SmallCtl &ctl,
                            DevResult *d_res, size_t lds, hipStream_t s) {
    if (mmax <= 64) return launch_small<4, 16, 4, VEC, DG>(d_probs, count, ctl, d_res, lds, s);
    if (mmax <= 128) return launch_small<4, 16, 8, VEC, DG>(d_probs, count, ctl, d_res, lds, s);
    if (mmax <= 256) return launch_small<4, 16, 16, VEC, DG>(d_probs, count, ctl, d_res, lds, s);
    if (mmax <= 512) return launch_small<4, 64, 8, VEC, DG>(d_probs, count, ctl, d_res, lds, s);
    return launch_small<4, 64, 16, VEC, DG>(d_probs, count, ctl, d_res, lds, s);
}

// Stream-ordered calls: each problem's result record, written to the caller's device memory.
__global__ __launch_bounds__(64) void publish_small(const DevResult *__restrict__ res,
                                                   accsk_result *const *__restrict__ pub, int cnt, double tick_ms) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k < cnt) publish_record(pub[k], res[k], tick_ms);
}

}  // namespace
}  // namespace accsk

using namespace accsk;

// Persistent multi-problem solver of accsk_dense.hip (problems that do not fit
// one workgroup).
accsk_status accsk_dense_multi(const accsk_problem *probs, int64_t count, const accsk_params *p,
                               accsk_result *res, hipStream_t s, Workspace &ws, accsk_result *const *pub);

// Dynamic on-chip memory one workgroup may take (of 160 KiB per CU).
static constexpr size_t kSmallLdsMax = 150 * 1024;

// A problem is solved by one workgroup when its whole state (potentials,
// marginals, row shifts, per-wave column sums) fits that workgroup's on-chip
// memory and its columns fit one row strip of the widest configuration.
bool accsk_small_fits(int64_t n, int64_t m) {
    return n >= 1 && m >= 1 && m <= 1024 && n <= 4096 && small_lds_bytes(n, m, 4) <= kSmallLdsMax;
}

// Up to 256 x 256 entries one workgroup per problem is the fastest way to
// solve it.  Above that a group of cooperating workgroups per problem is
// faster as long as the groups are not squeezed to a few workgroups each,
// i.e. for batches of up to 64 problems (measured per step on 500 x 500 and
// 1000 x 1000 problems).
bool accsk_on_one_workgroup(int64_t n, int64_t m, int64_t count) {
    return accsk_small_fits(n, m) && (n * m <= 65536 || count > 64);
}

// One launch, one workgroup per problem.  Over a fixed workspace region the
// kernel time comes from the device clock (no events are created).  pub
// (non-empty: one device record per problem): the stream-ordered form, the
// device writes the records and nothing waits (res unused).
static accsk_status solve_small_batch(const std::vector<accsk_problem> &probs, const SmallCtl &ctl,
                                      accsk_result *res, hipStream_t s, Workspace &ws,
                                      const std::vector<accsk_result *> &pub) {
    const int64_t count = (int64_t)probs.size();
    long long mmax = 0;
    size_t lds = 0;  // each workgroup lays out its own problem: the launch needs the largest one
    bool vec = true;
    std::vector<SmallProb> hp((size_t)count);
    for (int64_t k = 0; k < count; k++) {
        const accsk_problem &q = probs[(size_t)k];
        mmax = std::max<long long>(mmax, q.m);
        lds = std::max(lds, small_lds_bytes(q.n, q.m, 4));
        vec = vec && (q.m % 4 == 0) && (q.ldc % 4 == 0) && ((((uintptr_t)q.C) & 15) == 0);
        hp[(size_t)k] = SmallProb{q.C, q.n, q.m, q.ldc, q.a, q.b, q.f, q.g, q.eps, q.m - 4, nullptr};
    }
    if (lds > kSmallLdsMax) return ACCSK_SHAPE;
    const size_t bytes_p = sizeof(SmallProb) * (size_t)count, bytes_r = sizeof(DevResult) * (size_t)count;
    const bool async = !pub.empty();
    const size_t bytes_q = async ? sizeof(accsk_result *) * (size_t)count : 0;
    // boundedness monitor: [3][m] doubles per problem
    const bool cond = (ctl.flags & ACCSK_FLAG_CONDITIONS) && ctl.method == ACCSK_ACC;
    size_t bytes_c = 0;
    if (cond)
        for (int64_t k = 0; k < count; k++) bytes_c += 3 * (size_t)hp[(size_t)k].m * sizeof(double);
    const size_t o_res = (bytes_p + 255) & ~size_t(255), o_pub = (o_res + bytes_r + 255) & ~size_t(255);
    const size_t o_cond = (o_pub + bytes_q + 255) & ~size_t(255);
    char *buf = nullptr;
    if (ws.get((void **)&buf, o_cond + bytes_c + 256, s) != hipSuccess) return ACCSK_OOM;
    SmallProb *d_probs = (SmallProb *)buf;
    DevResult *d_res = (DevResult *)(buf + o_res);
    if (cond) {
        double *cp = (double *)(buf + o_cond);
        for (int64_t k = 0; k < count; k++) {
            hp[(size_t)k].cond = cp;
            cp += 3 * hp[(size_t)k].m;
        }
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!ws.fixed() && !async) {
        if (hipEventCreate(&ev0) != hipSuccess) ev0 = nullptr;
        if (hipEventCreate(&ev1) != hipSuccess) ev1 = nullptr;
    }
    hipError_t e = async ? upload_args(d_probs, hp.data(), bytes_p, s)
                         : hipMemcpyAsync(d_probs, hp.data(), bytes_p, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && ev0) e = hipEventRecord(ev0, s);
    if (e == hipSuccess)
        e = cond ? (vec ? launch_small_cfg<true, true>(mmax, d_probs, (int)count, ctl, d_res, lds, s)
                        : launch_small_cfg<false, true>(mmax, d_probs, (int)count, ctl, d_res, lds, s))
                 : (vec ? launch_small_cfg<true, false>(mmax, d_probs, (int)count, ctl, d_res, lds, s)
                        : launch_small_cfg<false, false>(mmax, d_probs, (int)count, ctl, d_res, lds, s));
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    if (async) {
        accsk_result **d_pub = (accsk_result **)(buf + o_pub);
        if (e == hipSuccess) e = upload_args(d_pub, pub.data(), bytes_q, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(publish_small, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, s,
                               (const DevResult *)d_res, (accsk_result *const *)d_pub, (int)count, wall_tick_ms());
            e = hipGetLastError();
        }
        ws.put(buf, s);
        return e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
    }
    std::vector<DevResult> hr((size_t)count);
    if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), d_res, bytes_r, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float kms = -1.f;
    if (e == hipSuccess && ev0 && ev1 && hipEventElapsedTime(&kms, ev0, ev1) != hipSuccess) kms = -1.f;
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ws.put(buf, s);
    if (e != hipSuccess) return ACCSK_HIP_ERROR;
    // with events: the whole batch's launch; else the problem's own device clock
    for (int64_t k = 0; k < count; k++) fill_result(res[k], hr[(size_t)k], ws.fixed() ? -1.0 : (double)kms);
    return ACCSK_OK;
}

// accsk_solve_batch with its workspace (a fixed region: no allocation).  pub
// (null, or `count` device result records): the stream-ordered form, where the
// device writes the records, nothing waits, and res is unused.
accsk_status accsk_solve_batch_ws(const accsk_problem *probs, int64_t count, const accsk_params *p,
                                  accsk_result *res, void *stream, Workspace &ws, accsk_result *const *pub) {
    if (!probs || !(res || pub) || !p || count < 0) return ACCSK_INVALID_ARG;
    if (count == 0) return ACCSK_OK;
    if (p->err_trace && count > 1) return ACCSK_INVALID_ARG;  // one trace buffer: one problem
    if ((p->flags & ACCSK_FLAG_CONDITIONS) && count > 1) return ACCSK_INVALID_ARG;  // the monitor: one problem
    SmallCtl ctl;
    accsk_status st = small_ctl_from_params(p, &ctl);
    if (st != ACCSK_OK) return st;
    std::vector<accsk_problem> small, big;
    std::vector<int64_t> small_idx, big_idx;
    for (int64_t k = 0; k < count; k++) {
        const accsk_problem &q = probs[k];
        if (!q.C || !q.a || !q.b || !q.f || !q.g) return ACCSK_INVALID_ARG;
        if (!small_finite_pos(q.eps)) return ACCSK_INVALID_ARG;
        if (q.n < 1 || q.m < 1 || q.ldc < q.m || q.m > 8192) return ACCSK_SHAPE;
        if (accsk_on_one_workgroup(q.n, q.m, count)) {
            small.push_back(q);
            small_idx.push_back(k);
        } else {
            big.push_back(q);
            big_idx.push_back(k);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (pub) {
        for (int64_t k = 0; k < count; k++)
            if (!pub[k]) return ACCSK_INVALID_ARG;
        std::vector<accsk_result *> ps, pb;
        for (int64_t k : small_idx) ps.push_back(pub[k]);
        for (int64_t k : big_idx) pb.push_back(pub[k]);
        if (!small.empty()) {
            st = solve_small_batch(small, ctl, nullptr, s, ws, ps);
            if (st != ACCSK_OK) return st;
        }
        if (!big.empty()) st = accsk_dense_multi(big.data(), (int64_t)big.size(), p, nullptr, s, ws, pb.data());
        return st;
    }
    std::vector<accsk_result> rs(small.size()), rb(big.size());
    const std::vector<accsk_result *> none;
    if (!small.empty()) {
        st = solve_small_batch(small, ctl, rs.data(), s, ws, none);
        if (st != ACCSK_OK) return st;
    }
    if (!big.empty()) {
        st = accsk_dense_multi(big.data(), (int64_t)big.size(), p, rb.data(), s, ws, nullptr);
        if (st != ACCSK_OK) return st;
    }
    for (size_t k = 0; k < small.size(); k++) res[small_idx[k]] = rs[k];
    for (size_t k = 0; k < big.size(); k++) res[big_idx[k]] = rb[k];
    accsk_status worst = ACCSK_OK;
    for (int64_t k = 0; k < count; k++) {
        const int stk = res[k].status;
        if (stk == ACCSK_OK) continue;
        if (worst == ACCSK_OK || (worst == ACCSK_NOT_CONVERGED && stk != ACCSK_NOT_CONVERGED))
            worst = (accsk_status)stk;
    }
    return worst;
}

extern "C" accsk_status accsk_solve_batch(const accsk_problem *probs, int64_t count, const accsk_params *p,
                                          accsk_result *res, void *stream) {
    Workspace ws;  // stream-ordered allocations
    return accsk_solve_batch_ws(probs, count, p, res, stream, ws, nullptr);
}

// Strided batch: host records (res) or, stream-ordered, device records (dres).
static accsk_status solve_batch_strided(const float *C, int64_t batch, int64_t n, int64_t m, int64_t ldc,
                                        int64_t stride_c, const double *a, const double *b, const double *eps,
                                        const accsk_params *p, double *f_out, double *g_out, accsk_result *res,
                                        accsk_result *dres, void *stream) {
    if (!C || !a || !b || !p || !f_out || !g_out || !(res || dres) || batch < 0) return ACCSK_INVALID_ARG;
    if (batch == 0) return ACCSK_OK;
    if (n < 1 || m < 1 || ldc < m || stride_c < (n - 1) * ldc + m) return ACCSK_SHAPE;
    std::vector<accsk_problem> probs((size_t)batch);
    for (int64_t k = 0; k < batch; k++)
        probs[(size_t)k] = accsk_problem{C + k * stride_c, n, m, ldc, a + k * n, b + k * m, f_out + k * n,
                                         g_out + k * m, eps ? eps[k] : p->eps};
    Workspace ws;  // stream-ordered allocations
    if (!dres) return accsk_solve_batch_ws(probs.data(), batch, p, res, stream, ws, nullptr);
    std::vector<accsk_result *> pub((size_t)batch);
    for (int64_t k = 0; k < batch; k++) pub[(size_t)k] = dres + k;
    return accsk_solve_batch_ws(probs.data(), batch, p, nullptr, stream, ws, pub.data());
}

extern "C" accsk_status accsk_solve_batch_strided(const float *C, int64_t batch, int64_t n, int64_t m, int64_t ldc,
                                                  int64_t stride_c, const double *a, const double *b,
                                                  const double *eps, const accsk_params *p, double *f_out,
                                                  double *g_out, accsk_result *res, void *stream) {
    if (!res) return ACCSK_INVALID_ARG;
    return solve_batch_strided(C, batch, n, m, ldc, stride_c, a, b, eps, p, f_out, g_out, res, nullptr, stream);
}

extern "C" accsk_status accsk_solve_batch_strided_async(const float *C, int64_t batch, int64_t n, int64_t m,
                                                        int64_t ldc, int64_t stride_c, const double *a,
                                                        const double *b, const double *eps, const accsk_params *p,
                                                        double *f_out, double *g_out, accsk_result *res,
                                                        void *stream) {
    if (!res) return ACCSK_INVALID_ARG;
    return solve_batch_strided(C, batch, n, m, ldc, stride_c, a, b, eps, p, f_out, g_out, nullptr, res, stream);
}

// Upper bound of the workspace of one-workgroup launches over `count` problems
// (descriptors and result records).
// (descriptors, result records, device record pointers and the boundedness monitor's [3][m] doubles).
size_t accsk_small_workspace_bound(int64_t count, int64_t m) {
    return (sizeof(SmallProb) + sizeof(DevResult) + sizeof(void *) + 3 * (size_t)m * sizeof(double)) * (size_t)count +
           1024;
}
