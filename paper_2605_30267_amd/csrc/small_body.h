// One-workgroup dense solver body, shared by the batched small-problem kernel
// and the serving loop (both instantiate it in their own translation unit).
//
// Layout of the work inside a workgroup of NW waves:
//  * a row is handled by LPR lanes (16 or 64); a wave therefore works on
//    64/LPR rows at a time, the workgroup on NW*64/LPR rows;
//  * lane li of a row owns the float4 column groups li, li+LPR, ... (NCL
//    columns), so the loads of one row are contiguous;
//  * row max and row sum are DPP reductions over the LPR lanes (a butterfly
//    inside a 16-lane row; for a 64-lane row a chain into lane 63 and a
//    readlane), so every lane of the row holds the result and no barrier is
//    needed per row;
//  * column sums are accumulated per lane in FP64 and combined across the
//    rows of a wave (xor shuffles) and across waves (LDS, fixed order) once
//    per Sinkhorn step.
// The iterate x, the extrapolation variable w, log2 b, and the per-row
// quantities live in LDS for the whole solve (paper Sec. 4, Algorithms A2MD
// and A2MD-homotopy; Sec. 2 eq:u-update for the row solve).
#pragma once

#include <math.h>

#include "accsk_common.h"

namespace accsk {
namespace {

struct SmallProb {
    const float *C;
    long long n, m, ldc;
    const double *a, *b;
    double *f, *g;
    double eps;
    long long vlim;  // VEC loads: last float4 start inside every row (m - 4, or ldc - 4 for padded rows)
    double *cond;    // ACCSK_FLAG_CONDITIONS (Acc): [3][m] grad f, D and v of the last iterate, else null
};

struct SmallCtl {
    double tol, tol_stop, mu0;
    long long max_iter, m0;
    int method, w_rule, flags;
    double *trace;  // optional per-step error trace (launches of one problem)
    long long trace_len;
};

// ---- butterfly reductions over the LPR lanes of a row (all lanes get the result)
__device__ __forceinline__ float bfly16_max(float v) {
    v = fmaxf(v, dpp_f32<0xB1, 0xf, 0xf>(v, v));   // quad_perm [1,0,3,2]
    v = fmaxf(v, dpp_f32<0x4E, 0xf, 0xf>(v, v));   // quad_perm [2,3,0,1]
    v = fmaxf(v, dpp_f32<0x141, 0xf, 0xf>(v, v));  // row_half_mirror
    v = fmaxf(v, dpp_f32<0x140, 0xf, 0xf>(v, v));  // row_mirror
    return v;
}
__device__ __forceinline__ double bfly16_sum(double v) {
    v += dpp_f64<0xB1, 0xf, 0xf>(v, v);
    v += dpp_f64<0x4E, 0xf, 0xf>(v, v);
    v += dpp_f64<0x141, 0xf, 0xf>(v, v);
    v += dpp_f64<0x140, 0xf, 0xf>(v, v);
    return v;
}
// Row reductions over the LPR lanes of a row; every lane gets the result.
// LPR = 16: DPP butterfly inside the 16-lane row.  LPR = 64 (the row is the
// whole wave): DPP row_shr / row_bcast chain into lane 63, then readlane; no
// LDS permutes, whose latency would dominate a row.
template <int LPR>
__device__ __forceinline__ float row_max(float v) {
    if (LPR == 64) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_max_l63(v)), 63));
    return bfly16_max(v);
}
template <int LPR>
__device__ __forceinline__ double row_sum(double v) {
    if (LPR == 64) {
        const long long b = __double_as_longlong(wave_sum_l63(v));
        const int lo = __builtin_amdgcn_readlane((int)b, 63);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    return bfly16_sum(v);
}

// Deterministic workgroup sum: wave butterfly, then a fixed-order sum of the
// per-wave values.  `red` holds NW doubles; every thread gets the total.
template <int NW>
__device__ __forceinline__ double wg_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; w++) s += red[w];
    return s;
}
template <int NW>
__device__ __forceinline__ double wg_max(double v, double *red) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = -INFINITY;
#pragma unroll
    for (int w = 0; w < NW; w++) s = fmax(s, red[w]);
    return s;
}

// The solve of one problem by one workgroup of 64*NW threads.  lds: dynamic
// on-chip memory of small_lds_bytes(n, m, NW); red: NW doubles; sflag: one int
// (both on-chip).  The result record is written by thread 0 to *res.
// DG: the diagnostic instantiation, which also runs the boundedness monitor
// (P.cond, ACCSK_FLAG_CONDITIONS); other instantiations carry none of its code.
template <int NW, int LPR, int NCL, bool VEC, bool DG = false>
__device__ __forceinline__ void small_body(const SmallProb &P, const SmallCtl &ctl, DevResult *res, double *lds,
                                           double *red, int &sflag) {
    constexpr int TPB = 64 * NW;
    constexpr int RPW = 64 / LPR;  // rows per wave in flight
    constexpr int RS = NW * RPW;   // rows per workgroup in flight
    constexpr int NK = NCL / 4;    // float4 groups per lane
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int li = lane % LPR, rg = lane / LPR, slot = wid * RPW + rg;
    const int n = (int)P.n, m = (int)P.m;
    const long long ldc = P.ldc;
    const int vlim = (int)P.vlim;
    const double eps = P.eps;
    const double kap2 = kLog2e / eps;

    double *xl = lds;           // [m] x log2 e
    double *wl = xl + m;        // [m] w log2 e
    double *lb2 = wl + m;       // [m] log2 b (normalized)
    double *bn = lb2 + m;       // [m] b (normalized)
    double *la2 = bn + m;       // [n] log2 a (normalized)
    double *rowM = la2 + n;     // [n] row shift of the last strip
    double *rowS = rowM + n;    // [n] row sum of the last strip
    double *afac = rowS + n;    // [n] a_i / max a
    double *wpart = afac + n;   // [NW][m] per-wave column sums

    if (tid == 0) res->t0 = dev_clock();
    // ---------------- set-up: validation, unit mass (eq:Fc), logs ----------------
    int bad = 0;
    double sa = 0.0, sb = 0.0;
    for (int i = tid; i < n; i += TPB) {
        const double v = P.a[i];
        bad |= !isfinite(v) ? 2 : (!(v > 0.0) ? 1 : 0);
        sa += v;
    }
    for (int j = tid; j < m; j += TPB) {
        const double v = P.b[j];
        bad |= !isfinite(v) ? 2 : (!(v > 0.0) ? 1 : 0);
        sb += v;
    }
    if (tid == 0) sflag = 0;
    __syncthreads();
    if (bad) atomicOr(&sflag, bad);
    sa = wg_sum<NW>(sa, red);
    sb = wg_sum<NW>(sb, red);
    const int badall = sflag;
    if (badall) {
        if (tid == 0) {
            DevResult r{};
            r.err = NAN;
            r.eot = NAN;
            r.fval = NAN;
            r.cost = NAN;
            r.status = (badall & 2) ? ACCSK_NONFINITE : ACCSK_INVALID_ARG;
            r.cond1 = r.cond2 = r.lyap = -1;
            r.t0 = res->t0;
            r.t1 = dev_clock();
            *res = r;
        }
        return;
    }
    double mx = -INFINITY;
    for (int i = tid; i < n; i += TPB) {
        const double l2 = log2(P.a[i] / sa);
        la2[i] = l2;
        mx = fmax(mx, l2);
    }
    for (int j = tid; j < m; j += TPB) {
        const double v = P.b[j] / sb;
        bn[j] = v;
        lb2[j] = log2(v);
        xl[j] = 0.0;
        wl[j] = 0.0;
    }
    const double La2 = wg_max<NW>(mx, red);
    const double maxa = exp2(La2);
    for (int i = tid; i < n; i += TPB) afac[i] = exp2(la2[i] - La2);
    __syncthreads();

    double mu = ctl.mu0, alpha = sqrt(2.0 * ctl.mu0);
    long long mstage = ctl.m0, kin = 0, it = 0, steps = 0, fallbacks = 0, incr = 0, restarts = 0;
    double fprev = 0.0;
    bool first = true;
    int status = ACCSK_OK;
    double err = 0.0, mass = 0.0, xb2 = 0.0;
    const int nrows_iter = (n + RS - 1) / RS;
    const bool mon = DG && P.cond != nullptr && ctl.method == ACCSK_ACC;
    CondState cs{0.0, 0.0, 0, 0, 0};

    for (;;) {
        // ---------------- strip: row solve and column sums from one read ----------------
        double xr[NCL];
#pragma unroll
        for (int k = 0; k < NK; k++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int col = 4 * (li + LPR * k) + e;
                xr[k * 4 + e] = col < m ? xl[col] : -INFINITY;
            }
        double colacc[NCL];
#pragma unroll
        for (int q = 0; q < NCL; q++) colacc[q] = 0.0;

        auto load_row = [&](int r, float4 (&v)[NK]) {
            const int i = min(r, n - 1);
            const float *row = P.C + (long long)i * ldc;
#pragma unroll
            for (int k = 0; k < NK; k++) {
                const int c0 = 4 * (li + LPR * k);
                if (VEC) {
                    v[k] = *reinterpret_cast<const float4 *>(row + min(c0, vlim));
                } else {
                    v[k].x = row[min(c0 + 0, m - 1)];
                    v[k].y = row[min(c0 + 1, m - 1)];
                    v[k].z = row[min(c0 + 2, m - 1)];
                    v[k].w = row[min(c0 + 3, m - 1)];
                }
            }
        };
        float4 nxt[NK];
        load_row(slot, nxt);
        for (int itr = 0; itr < nrows_iter; itr++) {
            const int r = slot + itr * RS;
            float4 cur[NK];
#pragma unroll
            for (int k = 0; k < NK; k++) cur[k] = nxt[k];
            if (itr + 1 < nrows_iter) load_row(r + RS, nxt);
            const bool rv = r < n;
            double t[NCL];
            double mloc = -INFINITY;
#pragma unroll
            for (int k = 0; k < NK; k++) {
                const float cv[4] = {cur[k].x, cur[k].y, cur[k].z, cur[k].w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    t[k * 4 + e] = fma(-(double)cv[e], kap2, xr[k * 4 + e]);
                    mloc = fmax(mloc, t[k * 4 + e]);
                }
            }
            const double M = (double)row_max<LPR>((float)mloc);
            float ev[NCL];
#pragma unroll
            for (int q = 0; q < NCL; q++) ev[q] = __builtin_amdgcn_exp2f((float)(t[q] - M));
            float pv[NCL];
#pragma unroll
            for (int q = 0; q < NCL; q++) pv[q] = ev[q];
#pragma unroll
            for (int h = 1; h < NCL; h <<= 1)
#pragma unroll
                for (int q = 0; q + h < NCL; q += 2 * h) pv[q] += pv[q + h];
            const double S = row_sum<LPR>((double)pv[0]);
            // P_ij / max a = e_ij * 2^(log2 a_i - La2) / S_i   (u_i from eq:u-update)
            const int ri = min(r, n - 1);
            const float rfac = rv ? (float)afac[ri] * __builtin_amdgcn_rcpf((float)S) : 0.f;
#pragma unroll
            for (int q = 0; q < NCL; q++) colacc[q] += (double)(ev[q] * rfac);
            if (li == 0 && rv) {
                rowM[r] = M;
                rowS[r] = S;
            }
        }
        // combine the rows of a wave, then the waves (fixed order)
#pragma unroll
        for (int q = 0; q < NCL; q++) {
            double v = colacc[q];
            if (RPW >= 2) v += __shfl_xor(v, 16, 64);
            if (RPW >= 4) v += __shfl_xor(v, 32, 64);
            colacc[q] = v;
        }
        if (rg == 0) {
#pragma unroll
            for (int k = 0; k < NK; k++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int col = 4 * (li + LPR * k) + e;
                    if (col < m) wpart[wid * m + col] = colacc[k * 4 + e];
                }
        }
        __syncthreads();

        // ---------------- column side: S^_j, error, mass ----------------
        double aS = 0.0, aE = 0.0, aC = 0.0, aXB = 0.0;
        int nfb = 0;
        for (int j = tid; j < m; j += TPB) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; w++) s += wpart[w * m + j];
            nfb += (s < 0x1p-64) ? 1 : 0;
            const double lc2 = La2 + log2(s);  // log2 c_j
            const double c = s * maxa;
            const double sh = lb2[j] - lc2 + xl[j];
            wpart[j] = sh;  // wave 0's slot is free now: keep S^_j there
            aS += sh;
            aE += fabs(c - bn[j]);
            aC += c;
            aXB += xl[j] * bn[j];
        }
        __syncthreads();
        if (tid == 0) sflag = 0;
        __syncthreads();
        if (nfb) atomicAdd(&sflag, nfb);
        __syncthreads();
        if (sflag > 0) {
            // Exact column pass (a column with almost no mass): running max per column.
            fallbacks++;
            for (int i = tid; i < n; i += TPB) rowM[i] = la2[i] - (rowM[i] + log2(rowS[i]));  // u_i log2 e
            __syncthreads();
            aS = aE = aC = aXB = 0.0;
            for (int j = tid; j < m; j += TPB) {
                double cmx = -INFINITY, cs = 0.0;
                for (int i = 0; i < n; i++) {
                    const double a2 = fma(-(double)P.C[(long long)i * ldc + j], kap2, rowM[i]);
                    if (a2 > cmx) {
                        cs = cs * exp2(cmx - a2) + 1.0;
                        cmx = a2;
                    } else {
                        cs += exp2(a2 - cmx);
                    }
                }
                const double lc2 = cmx + log2(cs) + xl[j];
                const double c = exp2(lc2);
                const double sh = lb2[j] - lc2 + xl[j];
                wpart[j] = sh;
                aS += sh;
                aE += fabs(c - bn[j]);
                aC += c;
                aXB += xl[j] * bn[j];
            }
            __syncthreads();
            // restore the row shift/sum form: u = la2 - (M + log2 S) with M = la2 - u, S = 1
            for (int i = tid; i < n; i += TPB) {
                rowM[i] = la2[i] - rowM[i];
                rowS[i] = 1.0;
            }
        }
        const double sumS = wg_sum<NW>(aS, red);
        err = wg_sum<NW>(aE, red);
        mass = wg_sum<NW>(aC, red);
        xb2 = wg_sum<NW>(aXB, red);
        // <u,a> (log2 units) for the reduced dual objective f(x) = 1 - <u,a> - <x,b>
        double aU = 0.0;
        for (int i = tid; i < n; i += TPB) aU += afac[i] * maxa * (la2[i] - (rowM[i] + log2(rowS[i])));
        const double fval = 1.0 - (wg_sum<NW>(aU, red) + xb2) * kLn2;
        const double mean = sumS / (double)m;
        steps++;
        if (tid == 0 && ctl.trace && steps <= ctl.trace_len) xstore(&ctl.trace[steps - 1], err);
        if (!isfinite(err)) {
            status = (steps == 1) ? ACCSK_NONFINITE : ACCSK_DIVERGED;
            break;
        }
        // ---------------- update (Sinkhorn or Algorithm A2MD with homotopy) ----------------
        const double fp = fprev;
        fprev = fval;
        if (ctl.method == ACCSK_SINKHORN) {
            if (steps > 1 && fval_rose(fval, fp)) incr++;
            if (err < ctl.tol_stop || it >= ctl.max_iter) break;
            for (int j = tid; j < m; j += TPB) xl[j] = wpart[j] - mean;
            it++;
        } else {
            if (!first) {
                const double c2 = alpha * alpha - 2.0, inv = 1.0 / (1.0 + alpha);
                for (int j = tid; j < m; j += TPB) wl[j] = (wl[j] + c2 * xl[j] + 2.0 * (wpart[j] - mean)) * inv;
                it++;
                kin++;
                if (fval_rose(fval, fp)) {
                    incr++;
                    if (ctl.flags & ACCSK_FLAG_RESTART) {  // safeguard: reset the extrapolation, w <- alpha x
                        for (int j = tid; j < m; j += TPB) wl[j] = alpha * xl[j];
                        restarts++;
                    }
                }
            }
            if (DG && mon) {  // (every thread reads only the columns it wrote in the update above)
                // Boundedness monitor: the new iterate is (x, w_k), w_k as carried to the next x update
                const bool stage = !(err < ctl.tol_stop || it >= ctl.max_iter) && !first && kin == mstage;
                const double a_new = dsqrt(mu), ratio = ctl.w_rule == ACCSK_W_Y_CONTINUOUS ? a_new / alpha : 1.0;
                const CondCols cc{xl, wl, wpart, bn, P.cond, P.cond + m, P.cond + 2 * m};
                const CondSums cv = cond_cols(cc, tid, m, TPB, 0, 0.0, 0.0, 0.0, alpha, first ? 0 : 1,
                                              stage ? 1 : 0, ratio, a_new);
                double s6[6] = {cv.lhs1, cv.lhs2, cv.vd, cv.K, cv.l1, cv.vd2};
#pragma unroll
                for (int q = 0; q < 6; q++) s6[q] = wg_sum<NW>(s6[q], red);
                cond_decide(cs, !first, s6[0], s6[1], s6[2], s6[3], s6[4], fval, alpha, mu);
                if (stage) cs.Eb = cond_lyap(fval, s6[5], s6[3], a_new, 0.5 * mu);
            }
            if (err < ctl.tol_stop || it >= ctl.max_iter) break;
            if (!first && kin == mstage) {
                const double mu_new = mu / 2.0;
                if (ctl.w_rule == ACCSK_W_Y_CONTINUOUS) {
                    const double ratio = sqrt(2.0 * mu_new) / alpha;
                    for (int j = tid; j < m; j += TPB) wl[j] *= ratio;
                }
                mu = mu_new;
                alpha = sqrt(2.0 * mu);
                mstage = (long long)floor(1.4142135623730951 * (double)mstage) + 1;
                kin = 0;
            }
            first = false;
            const double inv = 1.0 / (1.0 + alpha);
            for (int j = tid; j < m; j += TPB) xl[j] = (wl[j] + (wpart[j] - mean)) * inv;
        }
        __syncthreads();
    }
    __syncthreads();

    // ---------------- outputs ----------------
    double ua = 0.0;
    for (int i = tid; i < n; i += TPB) {
        const double u2 = la2[i] - (rowM[i] + log2(rowS[i]));
        P.f[i] = eps * kLn2 * u2;
        ua += exp2(la2[i]) * u2;
        rowM[i] = u2;
    }
    for (int j = tid; j < m; j += TPB) P.g[j] = eps * kLn2 * xl[j];
    ua = wg_sum<NW>(ua, red);
    // <C,P> at the returned potentials (FP32 exponentials, FP64 sums)
    double cst = 0.0;
    if (!(ctl.flags & ACCSK_FLAG_NO_COST)) {
        for (int i = wid; i < n; i += NW) {
            const float *row = P.C + (long long)i * ldc;
            const double u2 = rowM[i];
            for (int j = lane; j < m; j += 64) {
                const float c = row[j];
                const float pij = __builtin_amdgcn_exp2f((float)(fma(-(double)c, kap2, u2 + xl[j])));
                cst += (double)(c * pij);
            }
        }
        cst = wg_sum<NW>(cst, red);
    }
    if (tid == 0) {
        DevResult r;
        r.iters = it;
        r.steps = steps;
        r.fallback = fallbacks;
        r.incr = incr;
        r.restarts = restarts;
        r.err = err;
        const double ua_ln = ua * kLn2, xb_ln = xb2 * kLn2;
        r.fval = 1.0 - ua_ln - xb_ln;
        r.eot = eps * (ua_ln + xb_ln - mass);
        r.cost = (ctl.flags & ACCSK_FLAG_NO_COST) ? NAN : cst;
        r.converged = (status == ACCSK_OK && err < ctl.tol_stop) ? 1 : 0;
        r.status = status;
        r.cond1 = mon ? cs.n1 : -1;
        r.cond2 = mon ? cs.n2 : -1;
        r.lyap = mon ? cs.nl : -1;
        r.t0 = res->t0;
        r.t1 = dev_clock();
        *res = r;
    }
}


// On-chip bytes of small_body for a problem of n rows and m columns.
inline size_t small_lds_bytes(long long n, long long m, int nw) {
    return (size_t)(4 * m + 4 * n + (long long)nw * m) * sizeof(double);
}

inline bool small_finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validates the solver parameters and fills SmallCtl (stop at tol * (1 - 1/16),
// the margin for the FP32-exponential error estimate).
inline accsk_status small_ctl_from_params(const accsk_params *p, SmallCtl *c) {
    if (!p) return ACCSK_INVALID_ARG;
    if (!small_finite_pos(p->tol) || p->max_iter < 0) return ACCSK_INVALID_ARG;
    if (p->method != ACCSK_SINKHORN && p->method != ACCSK_ACC) return ACCSK_INVALID_ARG;
    if (p->method == ACCSK_ACC && !(p->mu0 > 0.0 && p->mu0 < 1.0 && p->m0 >= 1)) return ACCSK_INVALID_ARG;
    if (p->w_rule != ACCSK_W_LITERAL && p->w_rule != ACCSK_W_Y_CONTINUOUS) return ACCSK_INVALID_ARG;
    if (p->trace_len < 0 || (p->trace_len > 0 && !p->err_trace)) return ACCSK_INVALID_ARG;
    c->tol = p->tol;
    c->tol_stop = p->tol * (1.0 - 1.0 / 16.0);
    c->mu0 = p->mu0;
    c->max_iter = p->max_iter;
    c->m0 = p->m0;
    c->method = p->method;
    c->w_rule = p->w_rule;
    c->flags = p->flags;
    c->trace = p->trace_len > 0 ? p->err_trace : nullptr;
    c->trace_len = p->trace_len;
    return ACCSK_OK;
}

}  // namespace
}  // namespace accsk
