// Serving loop: a persistent kernel that solves point-cloud OT requests of
// uneven (n, m, eps) as they arrive (continuous batching).
//
// Device side (one launch, kept running while there is work):
//  * workgroup 0 is the dispatcher: it polls the host ring's publish counter
//    (pinned host memory) and forwards it to a device-side counter `avail`;
//  * every other workgroup is a worker: it claims the next published request
//    (compare-and-swap on the device counter `head`), reads its descriptor
//    from the host ring, builds the request's cost matrix into its HBM arena
//    block (FP64 dot products or BF16-split matrix cores, cost_tiles.h), runs
//    the one-workgroup solver (small_body.h: the paper's Sec. 2 row solve,
//    Sec. 4 Algorithms A2MD / A2MD-homotopy, stop on eq:l1tol), and posts the
//    result record to the host ring.  A request's potentials, iterate and
//    extrapolation state stay on the device (LDS and HBM) for its whole solve,
//    and each request stops on its own test.
//  * Every wait is bounded: the dispatcher stops the launch after an idle
//    period (no new request) or on shutdown, workers leave once the stop flag
//    is set and nothing published is left, and a worker that sees no new work
//    for a longer period leaves on its own.  The host relaunches on demand.
// Host side: admission by HBM footprint (first fit in a fixed arena; requests
// that do not fit yet wait, later ones that fit may go first), a ring of
// descriptors in pinned host memory, and a progress thread that admits,
// reaps results and relaunches.
//
// Results do not depend on which other requests are in flight: each request is
// computed by one workgroup with a fixed order of operations.

#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cost_tiles.h"
#include "small_body.h"

namespace accsk {
namespace {

constexpr int kRing = 4096;     // descriptor ring entries
constexpr int kServeNW = 4;     // waves per workgroup
constexpr int kServeTPB = 64 * kServeNW;
constexpr long long kServeMaxN = 512, kServeMaxM = 512, kServeMaxD = 512;
constexpr int kServeKC = 32;  // features staged per chunk (FP64 cost path)
constexpr size_t kArenaAlign = 256;

struct ServeDesc {
    const float *X, *Y;
    float *C;  // arena block, n x ldc
    const double *a, *b;
    double *f, *g;
    long long n, m, d, ldc;
    double inv_s, eps;
    long long kind, split;
    unsigned long long ticket;
};
constexpr int kDescWords = sizeof(ServeDesc) / 8;
static_assert(sizeof(ServeDesc) % 8 == 0, "descriptor is read as 64-bit words");

struct ServeDone {
    unsigned long long t_claim, t_end;  // device wall clock
    DevResult r;
    unsigned long long ticket;  // written last
    unsigned long long pad[3];
};

struct HostRing {
    unsigned long long tail;  // number of published descriptors (host writes)
    unsigned long long pad0[15];
    unsigned long long shutdown;  // host sets 1 to stop the launch
    unsigned long long pad1[15];
    ServeDesc desc[kRing];
    ServeDone done[kRing];
};

struct DevQueue {
    unsigned long long avail;  // published count seen by the dispatcher
    unsigned long long pad0[15];
    unsigned long long head;  // next index to claim
    unsigned long long pad1[15];
    unsigned long long stop;  // set by the dispatcher when the launch ends
    unsigned long long pad2[15];
};

__device__ __forceinline__ unsigned long long ld_sys(const unsigned long long *p) {
    return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_sys(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned long long ld_dev(const unsigned long long *p) {
    return __hip_atomic_load(const_cast<unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Builds the request's cost matrix C (n x ldc, pad columns set to 0) with the
// whole workgroup.  FP64 path: 64 x 64 tiles with chunks of the X and Y rows
// staged in LDS.  Matrix-core path: norms first (FP64, into sm as doubles),
// then one 16 x 16 tile per wave.
template <int KIND>
__device__ void serve_build_cost(const ServeDesc &D, float *sm) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const long long n = D.n, m = D.m, d = D.d, ldc = D.ldc;
    const long long tn = (n + 15) / 16, tm = (m + 15) / 16;
    if (D.split == 0) {
        // 64 x 64 tiles, thread (tr, tc) owns rows tr + 16p and columns tc + 16q
        // (p, q < 4); features staged kServeKC at a time (row stride kServeKC + 1
        // against bank conflicts).  Each entry is the same in-order FP64 sum as
        // in cross_fp64.
        constexpr int LS = kServeKC + 1;
        float *xs = sm, *ys = sm + 64 * LS;
        const int tr = tid >> 4, tc = tid & 15;
        const long long tn64 = (n + 63) / 64, tm64 = (m + 63) / 64;
        for (long long t = 0; t < tn64 * tm64; t++) {
            const long long i0 = (t / tm64) * 64, j0 = (t % tm64) * 64;
            double acc[4][4];
#pragma unroll
            for (int p = 0; p < 4; p++)
#pragma unroll
                for (int q = 0; q < 4; q++) acc[p][q] = 0.0;
            for (long long k0 = 0; k0 < d; k0 += kServeKC) {
                const int kc = (int)std::min<long long>(kServeKC, d - k0);
                __syncthreads();
                for (int e = tid; e < 64 * kc; e += kServeTPB) {
                    const int rr = e / kc, k = e % kc;
                    xs[rr * LS + k] = (i0 + rr < n) ? D.X[(i0 + rr) * d + k0 + k] : 0.f;
                    ys[rr * LS + k] = (j0 + rr < m) ? D.Y[(j0 + rr) * d + k0 + k] : 0.f;
                }
                __syncthreads();
                for (int k = 0; k < kc; k++) {
                    double xv[4], yv[4];
#pragma unroll
                    for (int p = 0; p < 4; p++) xv[p] = xs[(tr + 16 * p) * LS + k];
#pragma unroll
                    for (int q = 0; q < 4; q++) yv[q] = ys[(tc + 16 * q) * LS + k];
#pragma unroll
                    for (int p = 0; p < 4; p++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            if (KIND == ACCSK_SQEUCLID) {
                                const double tt = xv[p] - yv[q];
                                acc[p][q] = fma(tt, tt, acc[p][q]);
                            } else {
                                acc[p][q] = fma(xv[p], yv[q], acc[p][q]);
                            }
                        }
                }
            }
#pragma unroll
            for (int p = 0; p < 4; p++)
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const long long i = i0 + tr + 16 * p, j = j0 + tc + 16 * q;
                    if (i < n && j < ldc) D.C[i * ldc + j] = j < m ? finish_fp64<KIND>(acc[p][q], D.inv_s) : 0.f;
                }
        }
    } else {
        double *nx = reinterpret_cast<double *>(sm), *ny = nx + kServeMaxN;
        if (KIND == ACCSK_SQEUCLID) {
            for (long long i = wid; i < n; i += kServeNW) {
                const double v = row_norm_wave(D.X + i * d, d, lane);
                if (lane == 0) nx[i] = v;
            }
            for (long long j = wid; j < m; j += kServeNW) {
                const double v = row_norm_wave(D.Y + j * d, d, lane);
                if (lane == 0) ny[j] = v;
            }
        }
        __syncthreads();
        for (long long t = wid; t < tn * tm; t += kServeNW) {
            const long long i0 = (t / tm) * 16, j0 = (t % tm) * 16;
            const int rr = lane & 15;
            const long long ia = std::min(i0 + rr, n - 1), jb = std::min(j0 + rr, m - 1);
            double g[4];
            if (D.split == 2) mfma_cross_tile<2>(D.X + ia * d, D.Y + jb * d, d, lane, g);
            else mfma_cross_tile<3>(D.X + ia * d, D.Y + jb * d, d, lane, g);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const long long i = i0 + (lane >> 4) * 4 + q, j = j0 + (lane & 15);
                if (i < n && j < ldc)
                    D.C[i * ldc + j] =
                        j < m ? finish_mfma<KIND>(g[q], KIND == ACCSK_SQEUCLID ? nx[i] : 0.0,
                                                  KIND == ACCSK_SQEUCLID ? ny[j] : 0.0, D.inv_s)
                              : 0.f;
            }
        }
    }
    // C is read back by this workgroup's loads: drain the stores, then an
    // agent-scope fence makes them visible past the per-CU caches.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __threadfence();
    __syncthreads();
}

// Thread 0 of a worker: claim the next published request.  Returns its index,
// or -1 when the launch is over (stop flag set and nothing left, or no new
// work for `idle` wall-clock ticks).
__device__ long long serve_claim(DevQueue *q, long long idle) {
    long long t0 = wall_clock64();
    unsigned long long seen = ld_dev(&q->avail);
    int nap = 1;
    for (;;) {
        const unsigned long long h = ld_dev(&q->head);
        const unsigned long long av = __hip_atomic_load(&q->avail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (h < av) {
            unsigned long long expect = h;
            if (__hip_atomic_compare_exchange_strong(&q->head, &expect, h + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return (long long)h;
            continue;
        }
        if (av != seen) {  // new work was published (taken by others): still busy
            seen = av;
            t0 = wall_clock64();
            nap = 1;
        }
        if (__hip_atomic_load(&q->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) {
            // the final `avail` was stored before `stop`
            if (ld_dev(&q->head) >= __hip_atomic_load(&q->avail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT))
                return -1;
            continue;
        }
        if (wall_clock64() - t0 > idle) return -1;
        // back off while idle (polls of the shared counters by hundreds of
        // idle workgroups slow down the busy ones): ~3.4 us doubling to ~27 us
        for (int k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(127);
        nap = nap < 8 ? 2 * nap : 8;
    }
}

// Thread 0 of workgroup 0: forward the host's publish counter.
__device__ void serve_dispatch(HostRing *ring, DevQueue *q, long long idle) {
    unsigned long long pub = ld_dev(&q->avail);
    long long t_last = wall_clock64();
    for (;;) {
        const unsigned long long tail = ld_sys(&ring->tail);
        const unsigned long long sd = ld_sys(&ring->shutdown);
        if (tail > pub) {
            pub = tail;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // descriptors were written before tail
            __hip_atomic_store(&q->avail, pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            t_last = wall_clock64();
        } else if (sd || wall_clock64() - t_last > idle) {
            __hip_atomic_store(&q->stop, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        __builtin_amdgcn_s_sleep(16);
    }
}

__global__ __launch_bounds__(kServeTPB) void serve_loop(HostRing *ring, DevQueue *q, SmallCtl ctl,
                                                        long long idle_disp, long long idle_work) {
    extern __shared__ double lds[];
    __shared__ double red[kServeNW];
    __shared__ int sflag;
    __shared__ long long s_idx;
    __shared__ unsigned long long s_desc[kDescWords];
    __shared__ DevResult s_res;
    __shared__ long long s_t0;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        if (tid == 0) serve_dispatch(ring, q, idle_disp);
        return;
    }
    for (;;) {
        if (tid == 0) s_idx = serve_claim(q, idle_work);
        __syncthreads();
        const long long idx = s_idx;
        if (idx < 0) break;
        const int slot = (int)(idx % kRing);
        if (tid < kDescWords) s_desc[tid] = ld_sys(reinterpret_cast<const unsigned long long *>(&ring->desc[slot]) + tid);
        if (tid == 0) s_t0 = wall_clock64();
        __syncthreads();
        ServeDesc D;
        memcpy(&D, s_desc, sizeof(ServeDesc));
        if (D.kind == ACCSK_SQEUCLID) serve_build_cost<ACCSK_SQEUCLID>(D, reinterpret_cast<float *>(lds));
        else serve_build_cost<ACCSK_COSINE>(D, reinterpret_cast<float *>(lds));
        const SmallProb P{D.C, D.n, D.m, D.ldc, D.a, D.b, D.f, D.g, D.eps, D.ldc - 4};
        // at most 8 columns per lane keeps the kernel's registers low enough
        // for several resident workgroups per compute unit
        if (D.m <= 64) small_body<kServeNW, 16, 4, true>(P, ctl, &s_res, lds, red, sflag);
        else if (D.m <= 128) small_body<kServeNW, 16, 8, true>(P, ctl, &s_res, lds, red, sflag);
        else if (D.m <= 256) small_body<kServeNW, 64, 4, true>(P, ctl, &s_res, lds, red, sflag);
        else small_body<kServeNW, 64, 8, true>(P, ctl, &s_res, lds, red, sflag);
        // f, g (device) and the result record (host) must be visible before the ticket
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
            ServeDone *o = &ring->done[slot];
            const unsigned long long *rw = reinterpret_cast<const unsigned long long *>(&s_res);
            unsigned long long *ow = reinterpret_cast<unsigned long long *>(&o->r);
            for (int k = 0; k < (int)(sizeof(DevResult) / 8); k++) st_sys(ow + k, rw[k]);
            st_sys(&o->t_claim, (unsigned long long)s_t0);
            st_sys(&o->t_end, (unsigned long long)wall_clock64());
            __threadfence_system();
            __hip_atomic_store(&o->ticket, D.ticket, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
    }
}
static_assert(sizeof(DevResult) % 8 == 0, "result record is written as 64-bit words");

size_t serve_lds_bytes() {
    const size_t solve = small_lds_bytes(kServeMaxN, kServeMaxM, kServeNW);
    const size_t stage = 2 * 64 * (size_t)(kServeKC + 1) * sizeof(float);
    const size_t norms = 2 * (size_t)kServeMaxN * sizeof(double);
    return std::max(solve, std::max(stage, norms));
}

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace accsk

using namespace accsk;

struct accsk_server {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    bool launched = false;
    int workers = 0;
    size_t lds = 0;
    long long idle_disp = 0, idle_work = 0;
    double wall_rate = 100e6;  // device wall clock, ticks per second
    SmallCtl ctl{};
    int split = 0;
    char *arena = nullptr;
    size_t budget = 0;
    std::map<size_t, size_t> free_blocks;  // offset -> size
    HostRing *ring = nullptr;
    DevQueue *dq = nullptr;

    struct Rec {
        accsk_request req;
        size_t bytes = 0, off = 0;
        int state = 0;  // 0 waiting, 1 in flight, 2 done
        long long ring_idx = -1;
        accsk_result res{};
        double t_submit = 0, t_admit = 0, t_done = 0;
        bool space_waited = false;  // a first-fit search found no arena block for it
    };
    std::mutex mu;
    std::condition_variable cv;
    std::unordered_map<unsigned long long, Rec> recs;
    std::deque<unsigned long long> waiting;
    std::vector<unsigned long long> slot_ticket;  // ring slot -> ticket in flight (0 = free)
    std::vector<long long> inflight_idx;          // ring indices in flight
    unsigned long long next_ticket = 1;
    unsigned long long published = 0;
    std::thread th;
    std::atomic<bool> quit{false};
    accsk_status fault = ACCSK_OK;
    long long launches = 0;
    // admission by footprint: requests that waited for arena space, first-fit
    // searches that failed, requests admitted ahead of an earlier one that did
    // not fit, peak arena bytes in use and peak requests in flight
    long long space_waited = 0, fit_failures = 0, overtakes = 0, peak_inflight = 0;
    size_t in_use = 0, peak_in_use = 0;

    bool alloc(size_t bytes, size_t *off) {
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t o2 = it->first + bytes;
                free_blocks.erase(it);
                if (rest) free_blocks[o2] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_blocks.erase(nx);
        }
        if (it != free_blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_blocks.erase(it);
            }
        }
    }

    // Called with mu held.
    void reap() {
        for (size_t k = 0; k < inflight_idx.size();) {
            const long long idx = inflight_idx[k];
            const int slot = (int)(idx % kRing);
            const unsigned long long tk = slot_ticket[slot];
            volatile unsigned long long *tp = &ring->done[slot].ticket;
            if (*tp != tk) {
                k++;
                continue;
            }
            std::atomic_thread_fence(std::memory_order_acquire);
            const ServeDone &o = ring->done[slot];
            Rec &r = recs[tk];
            const DevResult &d = o.r;
            r.res.iters = d.iters;
            r.res.sinkhorn_steps = d.steps;
            r.res.fallback_steps = d.fallback;
            r.res.fval_increases = d.incr;
            r.res.restarts = d.restarts;
            r.res.cond1_violations = r.res.cond2_violations = r.res.lyap_increases = -1;  // not evaluated here
            r.res.marginal_err = d.err;
            r.res.eot_value = d.eot;
            r.res.transport_cost = d.cost;
            r.res.dual_fval = d.fval;
            r.res.kernel_ms = 1e3 * (double)(o.t_end - o.t_claim) / wall_rate;
            r.res.converged = d.converged;
            r.res.status = d.status;
            if (d.status == ACCSK_OK && !d.converged) r.res.status = ACCSK_NOT_CONVERGED;
            r.state = 2;
            r.t_done = now_seconds();
            release(r.off, r.bytes);
            in_use -= r.bytes;
            slot_ticket[slot] = 0;
            inflight_idx[k] = inflight_idx.back();
            inflight_idx.pop_back();
        }
    }

    // Called with mu held: publish waiting requests that fit, in order.
    void admit() {
        bool any = false;
        for (auto it = waiting.begin(); it != waiting.end();) {
            const int slot = (int)(published % kRing);
            if (slot_ticket[slot] != 0) break;  // ring entry still in flight
            Rec &r = recs[*it];
            size_t off;
            if (!alloc(r.bytes, &off)) {
                fit_failures++;
                if (!r.space_waited) {
                    r.space_waited = true;
                    space_waited++;
                }
                ++it;
                continue;
            }
            if (it != waiting.begin()) overtakes++;  // an earlier request is still waiting for space
            in_use += r.bytes;
            peak_in_use = std::max(peak_in_use, in_use);
            r.off = off;
            r.state = 1;
            r.ring_idx = (long long)published;
            r.t_admit = now_seconds();
            const accsk_request &q = r.req;
            ServeDesc D;
            D.X = q.X;
            D.Y = q.Y;
            D.C = reinterpret_cast<float *>(arena + off);
            D.a = q.a;
            D.b = q.b;
            D.f = q.f_out;
            D.g = q.g_out;
            D.n = q.n;
            D.m = q.m;
            D.d = q.d;
            D.ldc = (q.m + 3) / 4 * 4;
            D.inv_s = 1.0 / q.cost_scale;
            D.eps = q.eps;
            D.kind = q.kind;
            D.split = split;
            D.ticket = *it;
            ring->done[slot].ticket = 0;
            memcpy(&ring->desc[slot], &D, sizeof(D));
            slot_ticket[slot] = *it;
            inflight_idx.push_back((long long)published);
            peak_inflight = std::max(peak_inflight, (long long)inflight_idx.size());
            published++;
            any = true;
            it = waiting.erase(it);
        }
        if (any) {
            std::atomic_thread_fence(std::memory_order_release);
            reinterpret_cast<std::atomic<unsigned long long> *>(&ring->tail)->store(published,
                                                                                   std::memory_order_release);
        }
    }

    // Called with mu held: make sure a launch is running while work is in flight.
    void ensure_running() {
        if (inflight_idx.empty() || fault != ACCSK_OK) return;
        if (launched) {
            const hipError_t e = hipEventQuery(done_ev);
            if (e == hipErrorNotReady) return;
            if (e != hipSuccess) {
                fault = ACCSK_HIP_ERROR;
                return;
            }
            launched = false;
        }
        // previous launch (if any) has ended: clear its stop flag and start again
        hipError_t e = hipMemsetAsync(&dq->stop, 0, sizeof(unsigned long long), stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(serve_loop, dim3(workers + 1), dim3(kServeTPB), lds, stream, ring, dq, ctl, idle_disp,
                               idle_work);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(done_ev, stream);
        if (e != hipSuccess) {
            fault = ACCSK_HIP_ERROR;
            return;
        }
        launched = true;
        launches++;
    }

    void loop() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!quit.load()) {
            reap();
            admit();
            ensure_running();
            if (inflight_idx.empty() && waiting.empty()) {
                cv.wait_for(lk, std::chrono::milliseconds(2));
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            }
        }
    }
};

extern "C" accsk_status accsk_server_create(size_t hbm_budget, int max_slots, const accsk_params *p,
                                            accsk_server **out) {
    if (!out || !p) return ACCSK_INVALID_ARG;
    *out = nullptr;
    if (p->err_trace || p->trace_len != 0) return ACCSK_INVALID_ARG;  // no per-step trace when serving
    if (p->flags & ACCSK_FLAG_CONDITIONS) return ACCSK_INVALID_ARG;    // nor the boundedness monitor
    SmallCtl ctl;
    accsk_status st = small_ctl_from_params(p, &ctl);
    if (st != ACCSK_OK) return st;
    if (p->split != 0 && p->split != 2 && p->split != 3) return ACCSK_INVALID_ARG;
    if (hbm_budget < kArenaAlign || max_slots < 0) return ACCSK_INVALID_ARG;
    accsk_server *s = new accsk_server();
    s->ctl = ctl;
    s->split = p->split;
    s->budget = hbm_budget / kArenaAlign * kArenaAlign;
    s->lds = serve_lds_bytes();
    int cus = 0, rate_khz = 0;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
        hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess) {
        delete s;
        return ACCSK_HIP_ERROR;
    }
    if (rate_khz > 0) s->wall_rate = 1e3 * rate_khz;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, serve_loop, kServeTPB, s->lds) != hipSuccess || occ < 1) {
        delete s;
        return ACCSK_HIP_ERROR;
    }
    // one dispatcher plus the workers must all be resident at once
    const int cap = std::min(occ, 3) * cus - 1;
    s->workers = max_slots > 0 ? std::min(max_slots, cap) : cap;
    s->idle_disp = (long long)(0.25 * s->wall_rate);  // 250 ms without a new request ends the launch
    s->idle_work = (long long)(1.0 * s->wall_rate);
    s->slot_ticket.assign(kRing, 0);
    bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void **)&s->ring, sizeof(HostRing), hipHostMallocCoherent | hipHostMallocMapped) ==
                  hipSuccess &&
              hipMalloc((void **)&s->dq, sizeof(DevQueue)) == hipSuccess &&
              hipMemset(s->dq, 0, sizeof(DevQueue)) == hipSuccess;
    if (ok && hipMalloc((void **)&s->arena, s->budget) != hipSuccess) {
        accsk_server_destroy(s);
        return ACCSK_OOM;
    }
    if (!ok) {
        accsk_server_destroy(s);
        return ACCSK_HIP_ERROR;
    }
    memset(s->ring, 0, sizeof(HostRing));
    s->free_blocks[0] = s->budget;
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return ACCSK_OK;
}

extern "C" accsk_status accsk_server_submit(accsk_server *s, const accsk_request *q, uint64_t *ticket) {
    if (!s || !q || !ticket) return ACCSK_INVALID_ARG;
    if (!q->X || !q->Y || !q->a || !q->b || !q->f_out || !q->g_out) return ACCSK_INVALID_ARG;
    if (q->kind != ACCSK_SQEUCLID && q->kind != ACCSK_COSINE) return ACCSK_INVALID_ARG;
    if (!small_finite_pos(q->cost_scale) || !small_finite_pos(q->eps)) return ACCSK_INVALID_ARG;
    if (q->n < 1 || q->m < 1 || q->d < 1 || q->n > kServeMaxN || q->m > kServeMaxM || q->d > kServeMaxD)
        return ACCSK_SHAPE;
    const size_t bytes = ((size_t)q->n * (size_t)((q->m + 3) / 4 * 4) * sizeof(float) + kArenaAlign - 1) /
                         kArenaAlign * kArenaAlign;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fault != ACCSK_OK) return s->fault;
    if (bytes > s->budget) return ACCSK_OOM;
    const unsigned long long t = s->next_ticket++;
    accsk_server::Rec r;
    r.req = *q;
    r.bytes = bytes;
    r.t_submit = now_seconds();
    s->recs.emplace(t, r);
    s->waiting.push_back(t);
    *ticket = t;
    s->admit();
    s->ensure_running();
    s->cv.notify_one();
    return ACCSK_OK;
}

extern "C" accsk_status accsk_server_poll(accsk_server *s, uint64_t ticket, accsk_result *res, int *done,
                                          double *times) {
    if (!s || !done) return ACCSK_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) return ACCSK_INVALID_ARG;
    if (it->second.state != 2) {
        *done = 0;
        return s->fault;
    }
    *done = 1;
    if (res) *res = it->second.res;
    if (times) {
        times[0] = it->second.t_submit;
        times[1] = it->second.t_admit;
        times[2] = it->second.t_done;
    }
    s->recs.erase(it);
    return ACCSK_OK;
}

extern "C" accsk_status accsk_server_info(accsk_server *s, int64_t *info) {
    if (!s || !info) return ACCSK_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    info[0] = s->workers;
    info[1] = (int64_t)s->waiting.size();
    info[2] = (int64_t)s->inflight_idx.size();
    info[3] = s->launches;
    size_t fr = 0;
    for (auto &kv : s->free_blocks) fr += kv.second;
    info[4] = (int64_t)fr;
    return ACCSK_OK;
}

extern "C" accsk_status accsk_server_admission(accsk_server *s, int64_t *stats) {
    if (!s || !stats) return ACCSK_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    stats[0] = s->space_waited;
    stats[1] = s->fit_failures;
    stats[2] = s->overtakes;
    stats[3] = (int64_t)s->peak_in_use;
    stats[4] = s->peak_inflight;
    stats[5] = (int64_t)s->budget;
    return ACCSK_OK;
}

extern "C" double accsk_clock_seconds(void) { return now_seconds(); }

extern "C" accsk_status accsk_server_destroy(accsk_server *s) {
    if (!s) return ACCSK_INVALID_ARG;
    accsk_status st = ACCSK_OK;
    if (s->th.joinable()) {
        s->quit.store(true);
        s->cv.notify_one();
        s->th.join();
    }
    if (s->ring) reinterpret_cast<std::atomic<unsigned long long> *>(&s->ring->shutdown)->store(1);
    if (s->stream) {
        // the launch ends once the dispatcher sees the shutdown flag
        if (hipStreamSynchronize(s->stream) != hipSuccess) st = ACCSK_HIP_ERROR;
    }
    if (s->arena) (void)hipFree(s->arena);
    if (s->dq) (void)hipFree(s->dq);
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->done_ev) (void)hipEventDestroy(s->done_ev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return st;
}
