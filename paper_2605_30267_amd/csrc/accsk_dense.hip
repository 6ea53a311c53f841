// Dense explicit-cost solver: log-domain Sinkhorn and Acc-Sinkhorn on gfx950.
//
// One cooperative (persistent) launch runs the whole solve.  Per Sinkhorn step
// (paper Sec. 2 eq:u-update with the normalized column step eq:normalized-sinkhorn):
//
//  1. Strip pass.  Block b owns a contiguous range of whole rows and keeps the
//     iterate x (and w) for every column in registers, thread t holding the
//     float4 column groups t, t+TPB, ...  For each of its rows i it
//       - forms t_ij = x_j - C_ij/eps in FP64 (log2 units) from one read of the row,
//       - takes the exact row maximum and the row sum of exp2(t_ij - max) in FP32,
//       - gets u_i = log a_i - LSE_j(t_ij)   (exact row solve, eq:u-update),
//       - adds exp(u_i + x_j - C_ij/eps) / max_k a_k to its per-column sums.
//     The shift log(max a) - x_j is an upper bound of every u_i - C_ij/eps
//     (because x_j - C_ij/eps <= LSE_j), so these terms are <= 1 and the column
//     log-sum-exp needs no second read of C.
//  2. Grid barrier; block b combines the per-block sums of its column slice:
//     c_j = max a * s_j, S^_j = log b_j - log c_j + x_j, |c_j - b_j|.
//  3. Grid barrier; every block forms the same totals (fixed order) and applies
//     the same update to the x/w it holds: mean removal (P_Nperp), then plain
//     Sinkhorn x <- S or Algorithm A2MD with the homotopy of A2MD-homotopy.
//  If a column sum falls below 2^-64 (almost no mass in that column, early at
//  small eps), an exact pass with a running column maximum redoes the column
//  side of that step (one more read of C).
//
// All reductions have a fixed order, so results are bitwise reproducible.

#include <math.h>

#include <algorithm>
#include <vector>

#include "accsk_common.h"

namespace accsk {
namespace {

constexpr int kNS = 8;  // block scalar slots: 0 <u,a>, 1 sum S^, 2 err, 3 mass, 4 <x,b>, 5 fallback

// Scalars carried from one Sinkhorn step to the next (identical in every thread).
struct LoopState {
    double mu, alpha, err, mass, xb2, fprev;
    long long mstage, kin, it, steps, fallbacks, incr, restarts;
    int first;
};

struct DenseArgs {
    const float *C;
    long long n, m, ldc;
    const double *a_in, *b_in;
    double *an, *la2, *bn, *lnb;  // normalized marginals, log2 a, log b
    double *u;                    // [n] row potentials (log2 units)
    double *rsum;                 // [n] row sums of exp2(t - max) of the last strip pass
    float *partf;                 // [G*m] per-block column sums (fast path)
    double *part;                 // [G*m] per-block column sums (exact pass)
    double *partmax;              // [G*m] per-block column maxima (exact pass)
    double *shat;                 // [m] log b - ell
    double *bscal;                // [2][G][kNS]
    double *uapart;               // [G] per-block <u,a> at exit
    double *gscal;                // [0] = max_i log2 a_i, [1] = max_i a_i
    int *status;                  // setup status
    unsigned long long *bar;      // grid barrier counter
    DevResult *res;
    accsk_result *pub;  // stream-ordered calls: the caller's device result record (else null)
    double *f_out, *g_out;
    double eps, kappa, tol, tol_stop, mu0;
    long long max_iter, m0;
    int method, w_rule, serpentine, restart;
    double *cond;  // ACCSK_FLAG_CONDITIONS: [3][m] grad f, D and v of the last iterate (block 0), else null
};

// ---------------------------------------------------------------------------
// Marginal set-up: validation, unit mass (eq:Fc), log2 a, log b, max log2 a.
// One block of 1024 threads; deterministic block reductions.
// ---------------------------------------------------------------------------
__device__ double block_sum_1024(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < 16; k++) s += red[k];
    return s;
}
__device__ double block_max_1024(double v, double *red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = -INFINITY;
    for (int k = 0; k < 16; k++) s = fmax(s, red[k]);
    return s;
}

__global__ __launch_bounds__(1024) void setup_marginals(const DenseArgs *__restrict__ probs) {
    const DenseArgs A = probs[blockIdx.x];
    __shared__ double red[16];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    int lbad = 0;
    double s = 0.0;
    for (long long i = tid; i < A.n; i += 1024) {
        double v = A.a_in[i];
        if (!isfinite(v)) lbad |= 2;
        else if (!(v > 0.0)) lbad |= 1;
        s += v;
    }
    if (lbad) atomicOr(&bad, lbad);
    const double sa = block_sum_1024(s, red);
    double mx = -INFINITY;
    for (long long i = tid; i < A.n; i += 1024) {
        double v = A.a_in[i] / sa;
        A.an[i] = v;
        double l2 = log2(v);
        A.la2[i] = l2;
        mx = fmax(mx, l2);
    }
    mx = block_max_1024(mx, red);
    lbad = 0;
    s = 0.0;
    for (long long j = tid; j < A.m; j += 1024) {
        double v = A.b_in[j];
        if (!isfinite(v)) lbad |= 2;
        else if (!(v > 0.0)) lbad |= 1;
        s += v;
    }
    if (lbad) atomicOr(&bad, lbad);
    const double sb = block_sum_1024(s, red);
    for (long long j = tid; j < A.m; j += 1024) {
        double v = A.b_in[j] / sb;
        A.bn[j] = v;
        A.lnb[j] = log(v);
    }
    __syncthreads();
    if (tid < 32) A.bar[tid] = 0ull;  // the grid barrier's counter and flag lines (256 bytes)
    if (tid == 0) {
        A.gscal[0] = mx;
        A.gscal[1] = exp2(mx);
        A.status[0] = (bad & 2) ? ACCSK_NONFINITE : ((bad & 1) ? ACCSK_INVALID_ARG : ACCSK_OK);
        A.res->t0 = dev_clock();
    }
}

// ---------------------------------------------------------------------------
// The persistent solve kernel.
// TPB threads per block, NG float4 column groups per thread (m <= 4*TPB*NG).
// ---------------------------------------------------------------------------
template <int TPB, int NG, bool VEC>
struct RowIO {
    // Loads the thread's NG float4 column groups of one row as they are: every
    // address is clamped into the row, so loads never leave the buffer, and no
    // value is selected at load time (a select would force an immediate wait
    // on the prefetch).  Columns >= m are masked by the caller through x = -inf.
    // VEC: m % 4 == 0 and 16-byte aligned rows, one dwordx4 per group.
    static __device__ __forceinline__ void load(const float *__restrict__ row, int m, int tid,
                                                float4 (&v)[NG]) {
#pragma unroll
        for (int k = 0; k < NG; k++) {
            const int c0 = 4 * (tid + k * TPB);
            if (VEC) {
                v[k] = *reinterpret_cast<const float4 *>(row + min(c0, m - 4));
            } else {
                v[k].x = row[min(c0 + 0, m - 1)];
                v[k].y = row[min(c0 + 1, m - 1)];
                v[k].z = row[min(c0 + 2, m - 1)];
                v[k].w = row[min(c0 + 3, m - 1)];
            }
        }
    }
};

__device__ __forceinline__ float f4get(const float4 &v, int e) {
    return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

// All potentials inside the kernel are kept in log2 units (value * log2 e):
// xl = x log2 e, wl = w log2 e, so exp(.) becomes exp2(.) with no extra
// multiply per entry.  Algorithm A2MD is linear in (x, w, S), so it runs
// unchanged in these units.
//
// Dynamic LDS layout: wl[m] | xl[m] | la2s[rpb] | rowM[rpb] | rowS[rpb] | rowL[rpb] | rowA[rpb]
// | (WK > 0) the waves' column sums [m]  (doubles).
// x and w live in LDS between steps (the strip pass and the update walk them
// in different thread orders, with workgroup barriers between the phases), so
// no per-column state is carried in registers across steps.
// WK = 0: every row is spread over the whole workgroup (TPB * NG * 4 >= m
// columns, RB rows per batch, row sums reduced across waves).  WK > 0: each
// wave owns whole rows, lane l holding columns 4 (l + 64 k) + e for k < WK
// (m <= 256 WK); row sums stay inside the wave and the waves' column sums are
// combined once per step.
// TR: write the per-step error trace (trace / trace_len); CD (with TR): also run
// the boundedness monitor (ACCSK_FLAG_CONDITIONS).  Separate instantiations,
// so that other solves carry no diagnostic code at all.
// With 32 columns per lane (WK = 8) the wave-rows pass holds one row in
// flight and is capped at two waves per SIMD (256 registers, a few spills):
// 224 instead of 268 us per step on 64 problems of 2048 x 2048.  Without
// 16-byte loads the cap would spill ~90 registers, so it applies to VEC only.
template <int TPB, int NG, int RB, bool VEC, int WK = 0, bool TR = false, bool CD = false>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(WK >= 8 && VEC ? 2 : 1)))
void dense_solve(const DenseArgs *__restrict__ probs, int gp, double *__restrict__ trace, long long trace_len) {
    // gp workgroups per problem; problem p owns blocks [p*gp, (p+1)*gp)
    const DenseArgs A = probs[blockIdx.x / gp];
    constexpr int NW = TPB / 64;
    constexpr int NC = NG * 4;  // columns per thread
    __shared__ float red_max[RB][NW];
    __shared__ double red_sum[RB][NW];
    __shared__ double sred[NW][64];
    __shared__ double tot[kNS];
    __shared__ int bflag;
    extern __shared__ double dyn_lds[];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int G = gp, bid = blockIdx.x % gp;
    if (A.status[0] != ACCSK_OK) {  // uniform across the problem's blocks: no barrier is entered
        if (bid == 0 && tid == 0) {
            DevResult r{};
            r.err = NAN;
            r.eot = NAN;
            r.fval = NAN;
            r.cost = NAN;
            r.status = A.status[0];
            r.cond1 = r.cond2 = r.lyap = -1;
            r.t0 = A.res->t0;
            r.t1 = dev_clock();
            *A.res = r;
        }
        return;
    }

    const long long n = A.n, m = A.m;
    const long long rpb = (n + G - 1) / G;
    const long long r0 = std::min(n, (long long)bid * rpb);
    const long long r1 = std::min(n, r0 + rpb);
    const int nr = (int)(r1 - r0);
    const long long spb = (m + G - 1) / G;
    const long long j0 = std::min(m, (long long)bid * spb);
    const long long j1 = std::min(m, j0 + spb);

    double *wl_lds = dyn_lds;
    double *xl_lds = dyn_lds + m;
    double *la2s = dyn_lds + 2 * m;
    double *rowM = la2s + rpb;
    double *rowS = rowM + rpb;
    double *rowL = rowS + rpb;  // shift for the next step (row log-sum-exp, log2 units)
    double *rowA = rowL + rpb;  // a_i / max a (FP64, rounded once per use to FP32)

    const double kap2 = A.kappa * kLog2e;  // C_ij/eps in log2 units
    const double La2 = A.gscal[0];

#pragma unroll
    for (int k = 0; k < NG; k++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const long long col = 4ll * (tid + k * TPB) + e;
            if (col < m) {  // each thread owns its columns of x and w
                wl_lds[col] = 0.0;
                xl_lds[col] = 0.0;
            }
        }
    for (int r = tid; r < nr; r += TPB) {
        la2s[r] = A.la2[r0 + r];
        rowL[r] = INFINITY;  // unknown: the first step takes the exact row maximum
        rowA[r] = dexp2(la2s[r] - A.gscal[0]);
    }
    // max a, read after every combine: kept on chip (a load from global memory
    // there would follow the barrier's cache invalidation and wait a full round trip)
    __shared__ double maxa_lds;
    if (tid == 0) maxa_lds = A.gscal[1];
    __syncthreads();

    // Loop-carried scalars (the same in every thread) stay in LDS between update
    // phases, so they occupy no registers during the streaming pass.
    __shared__ LoopState ls;
    __shared__ CondState lcs;  // boundedness monitor (diagnostic instantiation, block 0)
    if (CD && tid == 0) lcs = CondState{0.0, 0.0, 0, 0, 0};
    if (tid == 0) {
        ls.mu = A.mu0;
        ls.alpha = dsqrt(2.0 * A.mu0);
        ls.err = ls.mass = ls.xb2 = ls.fprev = 0.0;
        ls.mstage = A.m0;
        ls.kin = ls.it = ls.steps = ls.fallbacks = ls.incr = ls.restarts = 0;
        ls.first = 1;
    }
    __syncthreads();
    unsigned long long gen = 0;
    int status = ACCSK_OK;

    // u_i log2 e = log2 a_i - (M_i + log2 S_i) for this block's rows, from the
    // shift and sum of the last strip pass (needed by the exact column pass and
    // at exit only).  Returns this block's sum_i a_i u_i (log2 units) in tid 0.
    auto materialize_u = [&]() -> double {
        double ua = 0.0;
        for (int r = tid; r < nr; r += TPB) {
            const double u2 = la2s[r] - (rowM[r] + dlog2(rowS[r]));
            A.u[r0 + r] = u2;
            ua += A.an[r0 + r] * u2;
        }
        ua = wave_sum(ua);
        __syncthreads();
        if (lane == 0) sred[wid][0] = ua;
        __syncthreads();
        double tot_ua = 0.0;
        if (tid == 0)
            for (int q = 0; q < NW; q++) tot_ua += sred[q][0];
        __syncthreads();
        return tot_ua;
    };

    for (long long step = 0;; step++) {
        const int par = (int)(step & 1);
        // Opaque copies of the base pointers and of the thread's first column:
        // addresses derived from them are recomputed each step instead of being
        // hoisted out of the step loop and kept live (which spills registers).
        DenseArgs L = A;
        opaque_ptr(L.partf);
        opaque_ptr(L.part);
        opaque_ptr(L.partmax);
        opaque_ptr(L.shat);
        opaque_ptr(L.bn);
        opaque_ptr(L.lnb);
        opaque_ptr(L.u);
        opaque_ptr(L.la2);
        opaque_ptr(L.an);
        opaque_ptr(L.bscal);
        int ctid = tid;
        opaque_int(ctid);
        double *bs = L.bscal + (size_t)par * G * kNS;
        // ---------------- strip pass ----------------
        double xl[NC];  // this thread's x (log2 units); -inf masks columns >= m
#pragma unroll
        for (int k = 0; k < NG; k++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int col = 4 * (ctid + k * TPB) + e;
                xl[k * 4 + e] = (col < m) ? xl_lds[col] : -INFINITY;
            }
        double colacc[NC];
#pragma unroll
        for (int q = 0; q < NC; q++) colacc[q] = 0.0;
        const bool rev = A.serpentine && (step & 1);
        const int nbat = (nr + RB - 1) / RB;

        // local row index of row q of batch bb (serpentine order), clamped for loading
        auto rloc = [&](int bb, int q) {
            const int r = bb * RB + q;
            const int rc = r < nr ? r : nr - 1;
            return rev ? nr - 1 - rc : rc;
        };
        // One batch of RB rows.  Row side: shift M_i, e_ij = exp2(t_ij - M_i),
        // S_i = sum_j e_ij (block reduction).  The shift is the row's log-sum-exp
        // from the previous step (kept in LDS); if the sum leaves [2^-40, 2^40]
        // (first step, or x moved a lot) the batch is redone with the exact row
        // maximum.  Column side: P_ij / max a = e_ij * 2^(log2 a_i - La2) / S_i,
        // one FMA per entry.
        auto batch = [&](int bb, const float4 (&cur)[RB][NG]) {
            double t[RB][NC];
            double M[RB];
            bool exact_rows = false;
#pragma unroll
            for (int q = 0; q < RB; q++) {
                M[q] = rowL[rloc(bb, q)];
                exact_rows |= !(M[q] < INFINITY);
#pragma unroll
                for (int k = 0; k < NG; k++)
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        t[q][k * 4 + e] = fma(-(double)f4get(cur[q][k], e), kap2, xl[k * 4 + e]);
            }
            float ev[RB][NC];
            double S[RB];
            auto row_sums = [&]() {
#pragma unroll
                for (int q = 0; q < RB; q++) {
#pragma unroll
                    for (int c = 0; c < NC; c++) ev[q][c] = __builtin_amdgcn_exp2f((float)(t[q][c] - M[q]));
                    // FP32 pairwise within the thread, FP64 across lanes and waves
                    float pv[NC];
#pragma unroll
                    for (int c = 0; c < NC; c++) pv[c] = ev[q][c];
#pragma unroll
                    for (int h = 1; h < NC; h <<= 1)
#pragma unroll
                        for (int c = 0; c + h < NC; c += 2 * h) pv[c] += pv[c + h];
                    const double sw = wave_sum_l63((double)pv[0]);
                    if (lane == 63) red_sum[q][wid] = sw;
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < RB; q++) S[q] = lds_combine_sum<NW>(red_sum[q], lane);
            };
            if (!exact_rows) {
                row_sums();
#pragma unroll
                for (int q = 0; q < RB; q++) exact_rows |= !(S[q] >= 0x1p-40 && S[q] <= 0x1p40);
                __syncthreads();  // red_sum is reused below
            }
            if (exact_rows) {  // block-uniform
#pragma unroll
                for (int q = 0; q < RB; q++) {
                    double mloc = -INFINITY;
#pragma unroll
                    for (int c = 0; c < NC; c++) mloc = fmax(mloc, t[q][c]);
                    // the shift only needs to be near the row maximum: reduce it in FP32
                    const float mw = wave_max_l63((float)mloc);
                    if (lane == 63) red_max[q][wid] = mw;
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < RB; q++) M[q] = (double)lds_combine_max<NW>(red_max[q], lane);
                row_sums();
            }
            float cterm[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) cterm[c] = 0.f;
#pragma unroll
            for (int q = 0; q < RB; q++) {
                const int rl = rloc(bb, q);
                const bool rv = bb * RB + q < nr;
                const float rfac = rv ? (float)rowA[rl] * __builtin_amdgcn_rcpf((float)S[q]) : 0.f;
#pragma unroll
                for (int c = 0; c < NC; c++) cterm[c] = fmaf(ev[q][c], rfac, cterm[c]);
                if (tid == 0 && rv) {
                    rowM[rl] = M[q];
                    rowS[rl] = S[q];
                    rowL[rl] = M[q] + (double)__builtin_amdgcn_logf((float)S[q]);  // next step's shift
                }
            }
#pragma unroll
            for (int c = 0; c < NC; c++) colacc[c] += (double)cterm[c];
        };
        // ping-pong prefetch buffers: batch bb computes on one while bb+1 loads into the other
        float4 bufA[RB][NG], bufB[RB][NG];
        auto load_batch = [&](int bb, float4 (&dst)[RB][NG]) {
#pragma unroll
            for (int q = 0; q < RB; q++)
                RowIO<TPB, NG, VEC>::load(A.C + (r0 + rloc(bb, q)) * A.ldc, (int)m, ctid, dst[q]);
        };
        if constexpr (WK == 0) {
            if (nbat > 0) load_batch(0, bufA);
            for (int bb = 0; bb < nbat; bb += 2) {
                if (bb + 1 < nbat) load_batch(bb + 1, bufB);
                batch(bb, bufA);
                if (bb + 1 < nbat) {
                    if (bb + 2 < nbat) load_batch(bb + 2, bufA);
                    batch(bb + 1, bufB);
                }
            }
            __syncthreads();
        } else {
            // ---- each wave owns rows wid, wid + NW, ... of the block (in traversal order) ----
            constexpr int WC = 4 * WK;  // columns per lane
            double cacc[WC];            // this lane's column sums of P / max a, FP64
#pragma unroll
            for (int q = 0; q < WC; q++) cacc[q] = 0.0;
            const int nrw = nr > wid ? (nr - wid + NW - 1) / NW : 0;
            auto wrow = [&](int k) {
                const int r = wid + k * NW;
                return rev ? nr - 1 - r : r;
            };
            auto wload = [&](int k, float4 (&dst)[WK]) {
                RowIO<64, WK, VEC>::load(A.C + (r0 + wrow(k)) * A.ldc, (int)m, lane, dst);
            };
            // One row: the same shift rule as the workgroup-wide pass (previous
            // step's log-sum-exp, exact maximum when the sum leaves [2^-40, 2^40]),
            // with every reduction inside the wave.  The row's values are dead once
            // its exponentials are formed (the exact-maximum redo reloads the row),
            // so both share registers.
            auto row_sum = [&](const float4 (&cur)[WK], double M, float (&ev)[WC]) -> double {
#pragma unroll
                for (int kk = 0; kk < WK; kk++) {
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const int col = 4 * (lane + 64 * kk) + e;
                        const double xc = col < m ? xl_lds[col] : -INFINITY;
                        ev[kk * 4 + e] =
                            __builtin_amdgcn_exp2f((float)(fma(-(double)f4get(cur[kk], e), kap2, xc) - M));
                    }
                }
                // FP32 pairwise within the lane, FP64 across lanes
                float pv[WC];
#pragma unroll
                for (int c = 0; c < WC; c++) pv[c] = ev[c];
#pragma unroll
                for (int h = 1; h < WC; h <<= 1)
#pragma unroll
                    for (int c = 0; c + h < WC; c += 2 * h) pv[c] += pv[c + h];
                return wave_bcast63(wave_sum_l63((double)pv[0]));
            };
            auto wrow_pass = [&](int k, const float4 (&cur)[WK]) {
                const int rl = wrow(k);
                double M = rowL[rl];
                float ev[WC];
                double S = 0.0;
                bool exact = !(M < INFINITY);
                if (!exact) {
                    S = row_sum(cur, M, ev);
                    exact = !(S >= 0x1p-40 && S <= 0x1p40);
                }
                if (exact) {  // wave-uniform
                    float4 re[WK];
                    wload(k, re);
                    double mloc = -INFINITY;
#pragma unroll
                    for (int kk = 0; kk < WK; kk++)
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int col = 4 * (lane + 64 * kk) + e;
                            const double xc = col < m ? xl_lds[col] : -INFINITY;
                            mloc = fmax(mloc, fma(-(double)f4get(re[kk], e), kap2, xc));
                        }
                    M = (double)wave_bcast63f(wave_max_l63((float)mloc));
                    S = row_sum(re, M, ev);
                }
                const double rfac = rowA[rl] / S;
#pragma unroll
                for (int c = 0; c < WC; c++) cacc[c] = fma((double)ev[c], rfac, cacc[c]);
                if (lane == 0) {
                    rowM[rl] = M;
                    rowS[rl] = S;
                    rowL[rl] = M + (double)__builtin_amdgcn_logf((float)S);  // next step's shift
                }
            };
            if constexpr (WK >= 8) {
                // one row in flight per wave; the other waves of the SIMD hide its latency
                for (int k = 0; k < nrw; k++) {
                    float4 wA[WK];
                    wload(k, wA);
                    wrow_pass(k, wA);
                }
            } else {
                float4 wA[WK], wB[WK];
                if (nrw > 0) wload(0, wA);
                for (int k = 0; k < nrw; k += 2) {
                    if (k + 1 < nrw) wload(k + 1, wB);
                    wrow_pass(k, wA);
                    if (k + 1 < nrw) {
                        if (k + 2 < nrw) wload(k + 2, wA);
                        wrow_pass(k + 1, wB);
                    }
                }
            }
            // the waves' column sums, added in wave order through on-chip memory
            double *cl = dyn_lds + 2 * m + 5 * rpb;  // m doubles past the row arrays
            for (int w = 0; w < NW; w++) {
                if (wid == w) {
#pragma unroll
                    for (int kk = 0; kk < WK; kk++)
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int col = 4 * (lane + 64 * kk) + e;
                            if (col < m) cl[col] = (w == 0 ? 0.0 : cl[col]) + cacc[kk * 4 + e];
                        }
                }
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < NG; k++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int col = 4 * (ctid + k * TPB) + e;
                    colacc[k * 4 + e] = col < m ? cl[col] : 0.0;
                }
        }
        // per-block column sums: FP64-accumulated, rounded once to FP32, written
        // through L2 (other XCDs read them after the barrier)
#pragma unroll
        for (int k = 0; k < NG; k++) {
            const int c0 = 4 * (ctid + k * TPB);
            float *dst = L.partf + (size_t)bid * m + c0;
            const float4 v = make_float4((float)colacc[k * 4 + 0], (float)colacc[k * 4 + 1],
                                         (float)colacc[k * 4 + 2], (float)colacc[k * 4 + 3]);
            if (VEC && c0 + 3 < m) {
                // raw buffer over this block's partial row: stores past its end are dropped
                const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)(L.partf + (size_t)bid * m), (short)0, (int)(m * 4), 0x00020000);
                xstore4(wrs, c0 * 4, v);
            } else {
                if (c0 + 0 < m) xstore(dst + 0, v.x);
                if (c0 + 1 < m) xstore(dst + 1, v.y);
                if (c0 + 2 < m) xstore(dst + 2, v.z);
                if (c0 + 3 < m) xstore(dst + 3, v.w);
            }
        }
        if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }

        // ---------------- slice combine ----------------
        bool exact = false;
        for (int pass = 0; pass < 2; pass++) {
            if (pass == 1) {
                if (!exact) break;
                (void)materialize_u();
                // Exact column pass: running maximum per column over this block's rows.
                double cm[NC];
                float cs[NC];
#pragma unroll
                for (int q = 0; q < NC; q++) { cm[q] = -INFINITY; cs[q] = 0.f; }
                for (long long rr = 0; rr < nr; rr++) {
                    const long long i = r0 + rr;
                    float4 cv[NG];
                    RowIO<TPB, NG, VEC>::load(A.C + i * A.ldc, (int)m, ctid, cv);
                    const double u2 = L.u[i];
#pragma unroll
                    for (int k = 0; k < NG; k++)
#pragma unroll
                        for (int e = 0; e < 4; e++) {
                            const int q = k * 4 + e;
                            const double a2 = fma(-(double)f4get(cv[k], e), kap2, u2);
                            if (a2 > cm[q]) {
                                cs[q] = cs[q] * __builtin_amdgcn_exp2f((float)(cm[q] - a2)) + 1.f;
                                cm[q] = a2;
                            } else {
                                cs[q] += __builtin_amdgcn_exp2f((float)(a2 - cm[q]));
                            }
                        }
                }
#pragma unroll
                for (int k = 0; k < NG; k++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const long long col = 4ll * (ctid + k * TPB) + e;
                        if (col < m) {
                            L.part[(size_t)bid * m + col] = (double)cs[k * 4 + e];
                            L.partmax[(size_t)bid * m + col] = cm[k * 4 + e];
                        }
                    }
                if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
                if (tid == 0) ls.fallbacks++;
            }
            double aS = 0.0, aE = 0.0, aC = 0.0, aXB = 0.0, aFB = 0.0;
            // columns of the slice in chunks of CW; thread t sums the partials of
            // blocks b = grp, grp + NGRP, ... for column cb + (t % CW)
            constexpr int CW = TPB >= 64 ? 32 : TPB;
            constexpr int NGRP = TPB / CW;
            double *sflat = &sred[0][0];
            const int coff = tid % CW, grp = tid / CW;
            for (long long cb = j0; cb < j1; cb += CW) {
                const long long j = cb + coff;
                double acc = 0.0, pm = -INFINITY;
                // read-only marginal data of the column, fetched while the partials are in flight
                double lnbj = 0.0, bnj = 0.0;
                if (tid < CW && j < j1) {
                    lnbj = L.lnb[j];
                    bnj = L.bn[j];
                }
                if (pass == 0) {
                    // the partials were written by blocks on other XCDs and miss in L2:
                    // keep PU loads in flight per thread, summed in block order
                    if (j < j1) {
                        constexpr int PU = 8;
                        // raw buffer over the G x m partials: one offset register per thread,
                        // the stride between a thread's partials in a scalar register, and
                        // reads past the last block return 0
                        const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
                            (void *)L.partf, (short)0, (int)((long long)G * m * 4), 0x00020000);
                        const int bstride = (int)((long long)NGRP * m * 4);
                        for (int b0 = grp; b0 < G; b0 += PU * NGRP) {
                            const int vo = (int)(((long long)b0 * m + j) * 4);
                            float v[PU];
#pragma unroll
                            for (int u = 0; u < PU; u++)
                                v[u] = __builtin_bit_cast(float,
                                                          __builtin_amdgcn_raw_buffer_load_b32(prs, vo, u * bstride, 0));
#pragma unroll
                            for (int u = 0; u < PU; u++) acc += (double)v[u];
                        }
                    }
                } else {
                    if (j < j1)
                        for (int b = grp; b < G; b += NGRP) pm = fmax(pm, L.partmax[(size_t)b * m + j]);
                    sflat[tid] = pm;
                    __syncthreads();
                    pm = -INFINITY;
#pragma unroll
                    for (int q = 0; q < NGRP; q++) pm = fmax(pm, sflat[q * CW + coff]);
                    __syncthreads();
                    if (j < j1)
                        for (int b = grp; b < G; b += NGRP) {
                            const double mb = L.partmax[(size_t)b * m + j];
                            if (mb > -INFINITY) acc += L.part[(size_t)b * m + j] * dexp2(mb - pm);
                        }
                }
                sflat[tid] = acc;
                __syncthreads();
                if (tid < CW && j < j1) {
                    double sc = 0.0;
#pragma unroll
                    for (int q = 0; q < NGRP; q++) sc += sflat[q * CW + tid];
                    const double xj = xl_lds[j];
                    double lc2, c;  // log2 c_j and c_j, c_j = column sum of P at (u(x), x)
                    if (pass == 0) {
                        lc2 = La2 + dlog2(sc);
                        c = sc * maxa_lds;
                        if (sc < 0x1p-64) aFB += 1.0;
                    } else {
                        lc2 = pm + dlog2(sc) + xj;
                        c = dexp2(lc2);
                    }
                    const double sh = lnbj * kLog2e - lc2 + xj;  // (log b_j - ell_j) log2 e
                    xstore(&L.shat[j], sh);
                    aS += sh;
                    aE += fabs(c - bnj);
                    aC += c;
                    aXB += xj * bnj;
                }
                __syncthreads();
            }
            if (wid == 0) {
                // <u,a> over this block's rows (log2 units) for the reduced dual objective:
                // u_i = log2 a_i - rowL_i, rowL_i = M_i + log2 S_i with an FP32 log2 of a row
                // sum near 1 (the shift is the previous step's log-sum-exp)
                double aU = 0.0;  // a_i = rowA_i max a: on-chip, no load after the barrier
                for (int r = lane; r < nr; r += 64) aU += rowA[r] * (la2s[r] - rowL[r]);
                aU = wave_sum(aU) * maxa_lds;
                aS = wave_sum(aS);
                aE = wave_sum(aE);
                aC = wave_sum(aC);
                aXB = wave_sum(aXB);
                aFB = wave_sum(aFB);
                if (lane == 0) {
                    double *p = bs + (size_t)bid * kNS;
                    xstore(&p[0], aU);
                    xstore(&p[1], aS);
                    xstore(&p[2], aE);
                    xstore(&p[3], aC);
                    xstore(&p[4], aXB);
                    xstore(&p[5], aFB);
                }
            }
            if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
            // totals, identical in every block
            for (int sidx = wid; sidx < 6; sidx += NW) {
                double v = 0.0;
                constexpr int TU = 4;  // loads in flight per lane, summed in block order
                const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
                    (void *)bs, (short)0, (int)((long long)G * kNS * 8), 0x00020000);
                for (int b0 = lane; b0 < G; b0 += TU * 64) {
                    const int vo = (int)(((long long)b0 * kNS + sidx) * 8);
                    double t4[TU];
#pragma unroll
                    for (int u = 0; u < TU; u++)
                        t4[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                               trs, vo, u * 64 * kNS * 8, 0));
#pragma unroll
                    for (int u = 0; u < TU; u++) v += t4[u];
                }
                v = wave_sum(v);
                if (lane == 0) tot[sidx] = v;
            }
            __syncthreads();
            exact = (pass == 0) && (tot[5] > 0.0);
            __syncthreads();
        }
        if (status != ACCSK_OK) break;

        // ---------------- update (every block, identical) ----------------
        // Elementwise over the m columns of x and w (on chip) and S(x): thread t
        // takes columns t + TPB q, so a wave's LDS accesses are consecutive
        // doubles.  (The strip layout, four adjacent columns per thread, puts
        // lanes 32 bytes apart: an 8-way bank conflict on every access.)
        auto ucol = [&](int q) -> int { return ctid + TPB * q; };  // m <= TPB * NC <= 8192
        const int mi = (int)m;
        LoopState st = ls;  // uniform copy, live only in this phase
        st.err = tot[2];
        const double mean = tot[1] / (double)m;
        st.mass = tot[3];
        st.xb2 = tot[4];
        st.steps++;
        if constexpr (TR) {
            if (bid == 0 && tid == 0 && st.steps <= trace_len) xstore(&trace[st.steps - 1], st.err);
        }
        const double fval = 1.0 - (tot[0] + tot[4]) * kLn2;  // f(x) = 1 - <u,a> - <x,b> at this step's x
        bool stop = false;
        if (!isfinite(st.err)) {
            status = (st.steps == 1) ? ACCSK_NONFINITE : ACCSK_DIVERGED;
            stop = true;
        } else if (A.method == ACCSK_SINKHORN) {
            // plain Sinkhorn, eq:normalized-sinkhorn: x <- S(x)
            if (st.steps > 1 && fval_rose(fval, st.fprev)) st.incr++;
            if (st.err < A.tol_stop || st.it >= A.max_iter) {
                stop = true;
            } else {
#pragma unroll
                for (int q = 0; q < NC; q++) {
                    const int col = ucol(q);
                    if (col < mi) xl_lds[col] = L.shat[col] - mean;
                }
                st.it++;
            }
        } else {
            // Algorithm A2MD: S is Sinkhorn(x) at the current x; the w update
            // below uses it as Sinkhorn(x_{k+1}) and the next x update reuses it.
            // The step's decisions are uniform, so they are taken first; then
            // one pass over the thread's columns reads S, w and x once each.
            const bool upd_w = !st.first;
            const double alpha0 = st.alpha, mu0s = st.mu;
            const double c2 = alpha0 * alpha0 - 2.0, inv_w = 1.0 / (1.0 + alpha0);
            bool reset = false;  // safeguard: reset the extrapolation, w <- alpha x
            if (upd_w) {
                st.it++;
                st.kin++;
                if (fval_rose(fval, st.fprev)) {
                    st.incr++;
                    if (A.restart) {
                        reset = true;
                        st.restarts++;
                    }
                }
            }
            double ratio = 1.0;  // w scale at a stage change (exact no-op otherwise)
            bool stage = false;
            if (st.err < A.tol_stop || st.it >= A.max_iter) {
                stop = true;
            } else {
                if (!st.first && st.kin == st.mstage) {
                    // Algorithm A2MD-homotopy: mu <- mu/2, m <- floor(sqrt(2) m) + 1
                    stage = true;
                    const double mu_new = st.mu / 2.0;
                    if (A.w_rule == ACCSK_W_Y_CONTINUOUS) ratio = dsqrt(2.0 * mu_new) / st.alpha;
                    st.mu = mu_new;
                    st.alpha = dsqrt(2.0 * st.mu);
                    st.mstage = (long long)floor(1.4142135623730951 * (double)st.mstage) + 1;
                    st.kin = 0;
                }
                st.first = 0;
            }
            if (CD && A.cond && bid == 0) {
                // Boundedness monitor over all m columns, before x and w are overwritten: the new
                // iterate is (x, w_k) with w_k the value carried to the next x update.
                const CondCols cc{xl_lds, wl_lds, L.shat, L.bn, A.cond, A.cond + m, A.cond + 2 * m};
                const CondSums cs = cond_cols(cc, tid, mi, TPB, upd_w ? (reset ? 2 : 1) : 0, mean, c2, inv_w,
                                              alpha0, upd_w ? 1 : 0, stage ? 1 : 0, ratio, st.alpha);
                const double s6[6] = {cs.lhs1, cs.lhs2, cs.vd, cs.K, cs.l1, cs.vd2};
#pragma unroll
                for (int q = 0; q < 6; q++) {
                    const double v = wave_sum(s6[q]);
                    if (lane == 0) sred[wid][q] = v;
                }
                __syncthreads();
                if (tid == 0) {
                    double r6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    for (int wq = 0; wq < NW; wq++)
#pragma unroll
                        for (int q = 0; q < 6; q++) r6[q] += sred[wq][q];
                    cond_decide(lcs, upd_w, r6[0], r6[1], r6[2], r6[3], r6[4], fval, alpha0, mu0s);
                    if (stage) lcs.Eb = cond_lyap(fval, r6[5], r6[3], st.alpha, st.mu);
                }
            }
            const double inv_x = 1.0 / (1.0 + st.alpha);
#pragma unroll
            for (int q = 0; q < NC; q++) {
                const int col = ucol(q);
                if (col < mi) {
                    const double S = L.shat[col] - mean;
                    double w = wl_lds[col];
                    if (upd_w) {
                        const double xv = xl_lds[col];
                        w = reset ? alpha0 * xv : (w + c2 * xv + 2.0 * S) * inv_w;
                    }
                    w *= ratio;
                    wl_lds[col] = w;
                    if (!stop) xl_lds[col] = (w + S) * inv_x;
                }
            }
        }
        st.fprev = fval;
        __syncthreads();  // every thread has read ls
        if (tid == 0) ls = st;
        __syncthreads();
        if (stop) break;
    }

    // ---------------- outputs ----------------
    __syncthreads();
    const LoopState fin = ls;
    double eot = 0.0, fval = 0.0;
    if (status == ACCSK_OK || status == ACCSK_DIVERGED) {
        const double ua_blk = materialize_u();  // u at the returned iterate, this block's rows
        if (tid == 0) xstore(&A.uapart[bid], ua_blk);
        for (long long i = r0 + tid; i < r1; i += TPB) A.f_out[i] = A.eps * kLn2 * A.u[i];
        if (bid == 0) {
#pragma unroll
            for (int k = 0; k < NG; k++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const long long col = 4ll * (tid + k * TPB) + e;
                    if (col < m) A.g_out[col] = A.eps * kLn2 * xl_lds[col];
                }
        }
        if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) status = ACCSK_HIP_ERROR;
        if (bid == 0 && tid == 0 && status != ACCSK_HIP_ERROR) {
            double ua2 = 0.0;
            for (int b = 0; b < G; b++) ua2 += A.uapart[b];
            const double ua_ln = ua2 * kLn2, xb_ln = fin.xb2 * kLn2;
            fval = 1.0 - ua_ln - xb_ln;               // f(x) = 1 - <u,a> - <x,b>
            eot = A.eps * (ua_ln + xb_ln - fin.mass);  // <f,a> + <g,b> - eps sum P
        }
    }
    if (bid == 0 && tid == 0) {
        DevResult r;
        r.iters = fin.it;
        r.steps = fin.steps;
        r.fallback = fin.fallbacks;
        r.incr = fin.incr;
        r.restarts = fin.restarts;
        r.err = fin.err;
        r.eot = eot;
        r.fval = fval;
        r.cost = NAN;
        r.converged = (status == ACCSK_OK && fin.err < A.tol_stop) ? 1 : 0;
        r.status = status;
        const bool mon = CD && A.cond && A.method == ACCSK_ACC;
        r.cond1 = mon ? lcs.n1 : -1;
        r.cond2 = mon ? lcs.n2 : -1;
        r.lyap = mon ? lcs.nl : -1;
        r.t0 = A.res->t0;
        r.t1 = dev_clock();
        *A.res = r;
    }
}

// ---------------------------------------------------------------------------
// FP64 evaluation of (f, g): row/col L1 errors, dual value, <C,P>, sum P.
// ---------------------------------------------------------------------------
constexpr int kEvalTPB = 256;

__global__ __launch_bounds__(kEvalTPB) void eval_rows(const float *__restrict__ C, long long n,
                                                      long long m, long long ldc, double inv_eps,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ f,
                                                      const double *__restrict__ g,
                                                      double *__restrict__ rowscal) {
    __shared__ double red[kEvalTPB / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int G = gridDim.x, bid = blockIdx.x;
    double re = 0.0, mass = 0.0, cost = 0.0;
    for (long long i = bid; i < n; i += G) {
        double rs = 0.0, rc = 0.0;
        const double fi = f[i];
        for (long long j = tid; j < m; j += kEvalTPB) {
            const double c = (double)C[i * ldc + j];
            const double p = exp((fi + g[j] - c) * inv_eps);
            rs += p;
            rc += c * p;
        }
        rs = wave_sum(rs);
        rc = wave_sum(rc);
        if (lane == 0) {
            red[wid][0] = rs;
            red[wid][1] = rc;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < kEvalTPB / 64; q++) {
                s0 += red[q][0];
                s1 += red[q][1];
            }
            re += fabs(s0 - a[i]);
            mass += s0;
            cost += s1;
        }
        __syncthreads();
    }
    if (tid == 0) {
        rowscal[bid * 3 + 0] = re;
        rowscal[bid * 3 + 1] = mass;
        rowscal[bid * 3 + 2] = cost;
    }
}

// Column sums of P over the row slab blockIdx.y (coalesced along j).
__global__ __launch_bounds__(kEvalTPB) void eval_colpart(const float *__restrict__ C, long long n,
                                                         long long m, long long ldc, double inv_eps,
                                                         const double *__restrict__ f,
                                                         const double *__restrict__ g,
                                                         double *__restrict__ colpart) {
    const long long j = (long long)blockIdx.x * kEvalTPB + threadIdx.x;
    const int RS = gridDim.y;
    const long long rpb = (n + RS - 1) / RS;
    const long long i0 = (long long)blockIdx.y * rpb, i1 = std::min(n, i0 + rpb);
    if (j >= m) return;
    const double gj = g[j];
    double s = 0.0;
    for (long long i = i0; i < i1; i++) s += exp((f[i] + gj - (double)C[i * ldc + j]) * inv_eps);
    colpart[(size_t)blockIdx.y * m + j] = s;
}

__global__ __launch_bounds__(kEvalTPB) void eval_cols(long long m, int G, const double *__restrict__ b,
                                                      const double *__restrict__ colpart,
                                                      double *__restrict__ colerr) {
    const long long j = (long long)blockIdx.x * kEvalTPB + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
    for (int q = 0; q < G; q++) s += colpart[(size_t)q * m + j];
    colerr[j] = fabs(s - b[j]);
}

__global__ __launch_bounds__(1024) void eval_final(long long n, long long m, int G, double eps,
                                                   const double *__restrict__ a,
                                                   const double *__restrict__ b,
                                                   const double *__restrict__ f,
                                                   const double *__restrict__ g,
                                                   const double *__restrict__ rowscal,
                                                   const double *__restrict__ colerr,
                                                   double *__restrict__ out, DevResult *res, accsk_result *pub) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    double re = 0.0, mass = 0.0, cost = 0.0, ce = 0.0, fa = 0.0, gb = 0.0;
    for (int q = tid; q < G; q += 1024) {
        re += rowscal[q * 3 + 0];
        mass += rowscal[q * 3 + 1];
        cost += rowscal[q * 3 + 2];
    }
    for (long long j = tid; j < m; j += 1024) {
        ce += colerr[j];
        gb += g[j] * b[j];
    }
    for (long long i = tid; i < n; i += 1024) fa += f[i] * a[i];
    re = block_sum_1024(re, red);
    mass = block_sum_1024(mass, red);
    cost = block_sum_1024(cost, red);
    ce = block_sum_1024(ce, red);
    fa = block_sum_1024(fa, red);
    gb = block_sum_1024(gb, red);
    if (tid == 0) {
        out[0] = re;
        out[1] = ce;
        out[2] = fa + gb - eps * mass;
        out[3] = cost;
        out[4] = mass;
        if (res) {
            res->cost = cost;
            res->eot = fa + gb - eps * mass;
        }
        if (pub) {
            pub->transport_cost = cost;
            pub->eot_value = fa + gb - eps * mass;
        }
    }
}

// Stream-ordered calls: each problem's result record, written to the caller's device memory.
__global__ __launch_bounds__(64) void publish_dense(const DenseArgs *__restrict__ probs, int cnt, double tick_ms) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k < cnt && probs[k].pub) publish_record(probs[k].pub, *probs[k].res, tick_ms);
}

// an = a / sum a, bn = b / sum b (one workgroup; FP64 sums).
__global__ __launch_bounds__(1024) void normalize_pair(const double *__restrict__ a, long long n,
                                                       const double *__restrict__ b, long long m,
                                                       double *__restrict__ an, double *__restrict__ bn) {
    __shared__ double red[16];
    const int tid = threadIdx.x;
    double sa = 0.0, sb = 0.0;
    for (long long i = tid; i < n; i += 1024) sa += a[i];
    for (long long j = tid; j < m; j += 1024) sb += b[j];
    sa = block_sum_1024(sa, red);
    sb = block_sum_1024(sb, red);
    for (long long i = tid; i < n; i += 1024) an[i] = a[i] / sa;
    for (long long j = tid; j < m; j += 1024) bn[j] = b[j] / sb;
}

// ---------------------------------------------------------------------------
// Plan rows from potentials.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void plan_rows(const float *__restrict__ C, long long m, long long ldc,
                                                 double inv_eps, const double *__restrict__ f,
                                                 const double *__restrict__ g, long long row0,
                                                 long long rows, float *__restrict__ P, long long ldp) {
    const long long r = blockIdx.y;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows || j >= m) return;
    const long long i = row0 + r;
    P[r * ldp + j] = (float)exp((f[i] + g[j] - (double)C[i * ldc + j]) * inv_eps);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

int device_cu_count() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cu;
}

// res / pub (either may be null): the device result record whose dual value
// and <C,P> the evaluation replaces.
accsk_status run_eval(const float *C, long long n, long long m, long long ldc, double eps, const double *a,
                      const double *b, const double *f, const double *g, double *out_dev, DevResult *res,
                      hipStream_t s, Workspace &ws, accsk_result *pub = nullptr) {
    const int G = (int)std::min<long long>(n, 1024);
    const int RS = (int)std::min<long long>(n, 64);
    double *buf = nullptr;
    const size_t bytes = ((size_t)RS * m + (size_t)G * 3 + m) * 8;
    if (ws.get((void **)&buf, bytes, s) != hipSuccess) return ACCSK_OOM;
    double *colpart = buf, *rowscal = buf + (size_t)RS * m, *colerr = rowscal + (size_t)G * 3;
    hipLaunchKernelGGL(eval_rows, dim3(G), dim3(kEvalTPB), 0, s, C, n, m, ldc, 1.0 / eps, a, f, g, rowscal);
    hipLaunchKernelGGL(eval_colpart, dim3((unsigned)((m + kEvalTPB - 1) / kEvalTPB), RS), dim3(kEvalTPB), 0, s,
                       C, n, m, ldc, 1.0 / eps, f, g, colpart);
    hipLaunchKernelGGL(eval_cols, dim3((unsigned)((m + kEvalTPB - 1) / kEvalTPB)), dim3(kEvalTPB), 0, s, m, RS,
                       b, colpart, colerr);
    hipLaunchKernelGGL(eval_final, dim3(1), dim3(1024), 0, s, n, m, G, eps, a, b, f, g, rowscal, colerr,
                       out_dev, res, pub);
    hipError_t e = hipGetLastError();
    ws.put(buf, s);
    return e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}


struct HostProb {
    const float *C;
    long long n, m, ldc;
    const double *a, *b;
    double *f, *g;
    double eps;
    accsk_result *pub;  // stream-ordered calls: device result record (else null)
};

// Solves problems [k0, k1) of `hp` with one cooperative launch, gp workgroups
// per problem.  Results go to res[k0..k1) (the call waits for the stream), or,
// when the problems carry device result records (pub), are written there by
// the device and nothing waits.  Over a fixed workspace region, and for
// device records, the kernel time comes from the device clock (no events).
template <int TPB, int NG, int RB, bool VEC, int WK = 0, bool TR = false, bool CD = false>
accsk_status dense_chunk(const std::vector<HostProb> &hp, int k0, int k1, const accsk_params *p,
                         accsk_result *res, hipStream_t s, int num_cu, Workspace &ws) {
    const int cnt = k1 - k0;
    long long nmax = 0, mmax = 0, nmin = 1LL << 62;
    for (int k = k0; k < k1; k++) {
        nmax = std::max(nmax, hp[k].n);
        mmax = std::max(mmax, hp[k].m);
        nmin = std::min(nmin, hp[k].n);
    }
    // Blocks per problem.  A step costs the streaming of the block's rows plus
    // two grid barriers and a combine of gp column partials, both of which
    // grow with gp: about 16 rows and at most 64K entries of C per block, at
    // most one block per CU, was the measured optimum from 100 x 50 to
    // 8192 x 8192.  The problems of one launch must all be co-resident.
    int occ = 0;
    const long long mextra = WK > 0 ? mmax : 0;  // column sums of the wave-rows pass
    const size_t dyn_probe = (size_t)(2 * mmax + mextra + 5) * sizeof(double);
    ACCSK_HIP_TRY(
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, dense_solve<TPB, NG, RB, VEC, WK, TR, CD>, TPB, dyn_probe));
    if (occ < 1) return ACCSK_SHAPE;
    const long long total = (long long)std::min(occ, 2) * num_cu;
    const long long want = std::max((nmax + 15) / 16, (nmax * mmax + 65535) / 65536);
    long long gp = std::min<long long>({want, (long long)num_cu, total / cnt, nmax});
    gp = std::max<long long>(gp, 1);
    long long rpb_max = 0;
    for (int k = k0; k < k1; k++) rpb_max = std::max(rpb_max, (hp[k].n + gp - 1) / gp);
    const size_t dyn = (size_t)(2 * mmax + mextra + 5 * rpb_max) * sizeof(double);
    if (dyn > 150 * 1024) return ACCSK_SHAPE;
    int occ2 = 0;
    ACCSK_HIP_TRY(
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, dense_solve<TPB, NG, RB, VEC, WK, TR, CD>, TPB, dyn));
    if (occ2 < 1 || (long long)cnt * gp > (long long)occ2 * num_cu) return ACCSK_SHAPE;

    // workspace: shared arrays first (args, results, scalars, barriers), then per-problem slices
    size_t off = 0;
    const size_t o_args = off; off = align_up(off + sizeof(DenseArgs) * cnt);
    const size_t o_res = off; off = align_up(off + sizeof(DevResult) * cnt);
    const size_t o_gscal = off; off = align_up(off + 8 * 8 * (size_t)cnt);
    const size_t o_stat = off; off = align_up(off + 64 * (size_t)cnt);
    const size_t o_bar = off; off = align_up(off + 256 * (size_t)cnt);
    std::vector<size_t> o_prob(cnt);
    const bool cond = (p->flags & ACCSK_FLAG_CONDITIONS) && p->method == ACCSK_ACC;
    for (int q = 0; q < cnt; q++) {
        const HostProb &h = hp[k0 + q];
        const size_t n = h.n, m = h.m;
        o_prob[q] = off;
        off = align_up(off + 4 * n * 8);                    // an, la2, u, rsum
        off = align_up(off + 3 * m * 8);                    // bn, lnb, shat
        off = align_up(off + (size_t)gp * m * 4);           // partf
        off = align_up(off + 2 * (size_t)gp * m * 8);       // part, partmax
        off = align_up(off + (2 * (size_t)gp * kNS + gp) * 8);  // bscal, uapart
        if (cond) off = align_up(off + 3 * m * 8);          // boundedness monitor
    }
    char *base = nullptr;
    if (ws.get((void **)&base, off, s) != hipSuccess) return ACCSK_OOM;
    std::vector<DenseArgs> args(cnt);
    for (int q = 0; q < cnt; q++) {
        const HostProb &h = hp[k0 + q];
        const size_t n = h.n, m = h.m;
        DenseArgs &A = args[q];
        A = DenseArgs{};
        A.C = h.C;
        A.n = h.n;
        A.m = h.m;
        A.ldc = h.ldc;
        A.a_in = h.a;
        A.b_in = h.b;
        A.f_out = h.f;
        A.g_out = h.g;
        A.eps = h.eps;
        A.kappa = 1.0 / h.eps;
        A.tol = p->tol;
        // The stop test compares an error computed from FP32 exponential sums;
        // stopping 1/16 below tol keeps the FP64-evaluated error under tol.
        A.tol_stop = p->tol * (1.0 - 1.0 / 16.0);
        A.mu0 = p->mu0;
        A.max_iter = p->max_iter;
        A.m0 = p->m0;
        A.method = p->method;
        A.w_rule = p->w_rule;
        A.serpentine = (p->flags & ACCSK_FLAG_NO_SERPENTINE) ? 0 : 1;
        A.restart = (p->flags & ACCSK_FLAG_RESTART) ? 1 : 0;
        char *q0 = base + o_prob[q];
        A.an = (double *)q0;
        A.la2 = A.an + n;
        A.u = A.la2 + n;
        A.rsum = A.u + n;
        q0 += align_up(4 * n * 8);
        A.bn = (double *)q0;
        A.lnb = A.bn + m;
        A.shat = A.lnb + m;
        q0 += align_up(3 * m * 8);
        A.partf = (float *)q0;
        q0 += align_up((size_t)gp * m * 4);
        A.part = (double *)q0;
        A.partmax = A.part + (size_t)gp * m;
        q0 += align_up(2 * (size_t)gp * m * 8);
        A.bscal = (double *)q0;
        A.uapart = A.bscal + 2 * (size_t)gp * kNS;
        q0 += align_up((2 * (size_t)gp * kNS + gp) * 8);
        A.cond = cond ? (double *)q0 : nullptr;
        A.res = (DevResult *)(base + o_res) + q;
        A.pub = h.pub;
        A.gscal = (double *)(base + o_gscal) + 8 * q;
        A.status = (int *)(base + o_stat + 64 * (size_t)q);
        A.bar = (unsigned long long *)(base + o_bar + 256 * (size_t)q);
    }
    DenseArgs *d_args = (DenseArgs *)(base + o_args);
    const bool async = hp[k0].pub != nullptr;  // all problems of a call, or none
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!ws.fixed() && !async) {
        if (hipEventCreate(&ev0) != hipSuccess) ev0 = nullptr;
        if (hipEventCreate(&ev1) != hipSuccess) ev1 = nullptr;
    }
    // (setup_marginals also zeroes each problem's barrier words)
    hipError_t e = async ? upload_args(d_args, args.data(), sizeof(DenseArgs) * cnt, s)
                         : hipMemcpyAsync(d_args, args.data(), sizeof(DenseArgs) * cnt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(setup_marginals, dim3(cnt), dim3(1024), 0, s, (const DenseArgs *)d_args);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ev0) e = hipEventRecord(ev0, s);
    if (e == hipSuccess) {
        int gpi = (int)gp;
        double *tr = TR ? p->err_trace : nullptr;  // traced launches hold one problem
        long long tl = TR ? p->trace_len : 0;
        void *kargs[] = {&d_args, &gpi, &tr, &tl};
        e = hipLaunchCooperativeKernel((const void *)dense_solve<TPB, NG, RB, VEC, WK, TR, CD>, dim3((unsigned)(cnt * gp)),
                                       dim3(TPB), kargs, dyn, s);
    }
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    accsk_status st = e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
    if (st == ACCSK_OK && !(p->flags & ACCSK_FLAG_NO_COST)) {
        for (int q = 0; q < cnt && st == ACCSK_OK; q++) {
            const DenseArgs &A = args[q];
            // <C,P> and the dual value at the returned potentials, FP64, with normalized marginals
            st = run_eval(A.C, A.n, A.m, A.ldc, A.eps, A.an, A.bn, A.f_out, A.g_out, A.gscal + 1, A.res, s, ws);
        }
    }
    if (async) {
        if (st == ACCSK_OK) {
            hipLaunchKernelGGL(publish_dense, dim3((unsigned)((cnt + 63) / 64)), dim3(64), 0, s,
                               (const DenseArgs *)d_args, cnt, wall_tick_ms());
            if (hipGetLastError() != hipSuccess) st = ACCSK_HIP_ERROR;
        }
        ws.put(base, s);
        return st;
    }
    std::vector<DevResult> hr(cnt);
    if (st == ACCSK_OK) {
        e = hipMemcpyAsync(hr.data(), base + o_res, sizeof(DevResult) * cnt, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = ACCSK_HIP_ERROR;
    }
    float kms = -1.f;
    if (st == ACCSK_OK && ev0 && ev1 && hipEventElapsedTime(&kms, ev0, ev1) != hipSuccess) kms = -1.f;
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ws.put(base, s);
    if (st != ACCSK_OK) return st;
    for (int q = 0; q < cnt; q++) fill_result(res[k0 + q], hr[q], (double)kms);
    return ACCSK_OK;
}

template <bool VEC, bool TR, bool CD>
accsk_status dense_chunk_cfg_t(long long mmax, const std::vector<HostProb> &hp, int k0, int k1,
                               const accsk_params *p, accsk_result *res, hipStream_t s, int cu, Workspace &ws) {
    // Up to 1024 columns each wave owns whole rows (4 to 16 columns per lane):
    // 20-34 % faster per step than rows spread over the workgroup, whose
    // cross-wave row reductions cost more than the row's arithmetic.  With
    // 2048 columns the wave-rows kernel needs 328 registers (one wave per SIMD):
    // it wins only when a launch holds 16 or more problems (never a traced one).
    if (mmax <= 256) return dense_chunk<256, 1, 1, VEC, 1, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
    if (mmax <= 512) return dense_chunk<256, 1, 1, VEC, 2, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
    if (mmax <= 1024) return dense_chunk<256, 1, 1, VEC, 4, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
    if (mmax <= 2048) {
        if constexpr (!TR)
            if (k1 - k0 >= 16) return dense_chunk<256, 2, 1, VEC, 8>(hp, k0, k1, p, res, s, cu, ws);
        return dense_chunk<512, 1, 4, VEC, 0, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
    }
    if (mmax <= 4096) return dense_chunk<1024, 1, 2, VEC, 0, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
    return dense_chunk<1024, 2, 1, VEC, 0, TR, CD>(hp, k0, k1, p, res, s, cu, ws);
}

// A launch with the per-step trace or the boundedness monitor holds one
// problem (the batch entry points refuse them for several) and runs the
// diagnostic instantiation.
template <bool VEC>
accsk_status dense_chunk_cfg(long long mmax, const std::vector<HostProb> &hp, int k0, int k1,
                             const accsk_params *p, accsk_result *res, hipStream_t s, int cu, Workspace &ws) {
    if ((p->flags & ACCSK_FLAG_CONDITIONS) && p->method == ACCSK_ACC && k1 - k0 == 1)
        return dense_chunk_cfg_t<VEC, true, true>(mmax, hp, k0, k1, p, res, s, cu, ws);
    if (p->err_trace && p->trace_len > 0 && k1 - k0 == 1)
        return dense_chunk_cfg_t<VEC, true, false>(mmax, hp, k0, k1, p, res, s, cu, ws);
    return dense_chunk_cfg_t<VEC, false, false>(mmax, hp, k0, k1, p, res, s, cu, ws);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Validates the shared parameters (everything except eps).
accsk_status check_params(const accsk_params *p) {
    if (!p) return ACCSK_INVALID_ARG;
    if (!finite_pos(p->tol) || p->max_iter < 0) return ACCSK_INVALID_ARG;
    if (p->method != ACCSK_SINKHORN && p->method != ACCSK_ACC) return ACCSK_INVALID_ARG;
    if (p->method == ACCSK_ACC && !(p->mu0 > 0.0 && p->mu0 < 1.0 && p->m0 >= 1)) return ACCSK_INVALID_ARG;
    if (p->w_rule != ACCSK_W_LITERAL && p->w_rule != ACCSK_W_Y_CONTINUOUS) return ACCSK_INVALID_ARG;
    if (p->trace_len < 0 || (p->trace_len > 0 && !p->err_trace)) return ACCSK_INVALID_ARG;
    return ACCSK_OK;
}

}  // namespace
}  // namespace accsk

using namespace accsk;

// Routing rule of the batch solver (accsk_small.hip).
bool accsk_on_one_workgroup(int64_t n, int64_t m, int64_t count);

// Tiled solver of accsk_tiled.hip (m > 8192, or costs formed on the fly).
accsk_status accsk_tiled_solve(const float *C, int64_t ldc, const float *X, const float *Y, int64_t d, int kind,
                               double cost_scale, int64_t n, int64_t m, const double *a, const double *b,
                               const accsk_params *p, double eps, double *f_out, double *g_out, accsk_result *res,
                               hipStream_t s, accsk_result *pub);

// Persistent multi-problem path, also used by the batch entry point for
// problems with more than 1024 columns.  Over a fixed workspace region a
// problem that would need the tiled solver is refused (SHAPE).  pub (null, or
// `count` device result records): the stream-ordered form, res unused.
accsk_status accsk_dense_multi(const accsk_problem *probs, int64_t count, const accsk_params *p,
                               accsk_result *res, hipStream_t s, Workspace &ws, accsk_result *const *pub) {
    using namespace accsk;
    const int cu = device_cu_count();
    if (cu <= 0) return ACCSK_HIP_ERROR;
    std::vector<HostProb> hp((size_t)count);
    for (int64_t k = 0; k < count; k++) {
        const accsk_problem &q = probs[k];
        hp[(size_t)k] = HostProb{q.C, q.n, q.m, q.ldc, q.a, q.b, q.f, q.g, q.eps, pub ? pub[k] : nullptr};
    }
    // At most one CU's worth of problems per cooperative launch.  A launch
    // whose row blocks do not fit on chip (many rows per block) is split in
    // halves; a single problem that still does not fit goes to the tiled
    // solver, whose on-chip footprint does not depend on n or m.
    int64_t k0 = 0;
    while (k0 < count) {
        int64_t k1 = std::min<int64_t>(count, k0 + cu);
        accsk_status st = ACCSK_SHAPE;
        while (true) {
            long long mmax = 0;
            bool vec = true;
            for (int64_t k = k0; k < k1; k++) {
                const HostProb &h = hp[(size_t)k];
                mmax = std::max(mmax, h.m);
                vec = vec && (h.ldc % 4) == 0 && (h.m % 4) == 0 && (((uintptr_t)h.C) & 15) == 0;
            }
            st = vec ? dense_chunk_cfg<true>(mmax, hp, (int)k0, (int)k1, p, res, s, cu, ws)
                     : dense_chunk_cfg<false>(mmax, hp, (int)k0, (int)k1, p, res, s, cu, ws);
            if (st != ACCSK_SHAPE || k1 - k0 == 1) break;
            k1 = k0 + (k1 - k0) / 2;
        }
        if (st == ACCSK_SHAPE) {
            if (ws.fixed()) return ACCSK_SHAPE;
            const HostProb &h = hp[(size_t)k0];
            st = accsk_tiled_solve(h.C, h.ldc, nullptr, nullptr, 0, 0, 1.0, h.n, h.m, h.a, h.b, p, h.eps, h.f, h.g,
                                   res ? &res[k0] : nullptr, s, h.pub);
            // per-problem outcomes are in res[k0] (or its device record); only call failures stop the batch
            if (st == ACCSK_OOM || st == ACCSK_HIP_ERROR || st == ACCSK_SHAPE) return st;
            st = ACCSK_OK;
        }
        if (st != ACCSK_OK) return st;
        k0 = k1;
    }
    return ACCSK_OK;
}

size_t accsk_tiled_workspace_bound(int64_t n, int64_t m, int cu);
size_t accsk_small_workspace_bound(int64_t count, int64_t m);

// Upper bound of the workspace of the FP64 evaluation pass (run_eval) on n x m.
static size_t eval_workspace_bound(long long m) { return (size_t)(64 * m + 3 * 1024 + m) * 8 + 256; }

// Upper bound of the workspace accsk_solve_dense takes for one n x m problem
// (m <= 8192) on its one-workgroup or cooperative route, slices rounded to
// 256 bytes as Workspace hands them out; the tiled route is not counted.
size_t accsk_dense_single_bound(int64_t n, int64_t m, int cu) {
    using namespace accsk;
    const size_t un = (size_t)n, um = (size_t)m;
    const size_t eval = align_up(((size_t)std::min<int64_t>(n, 64) * um + (size_t)std::min<int64_t>(n, 1024) * 3 + um) * 8);
    // one workgroup: descriptors and results, then (released) the FP64 re-evaluation
    const size_t small = std::max(align_up(accsk_small_workspace_bound(1, m)), align_up((un + um + 8) * 8) + eval);
    // cooperative launch of one problem, gp <= min(CUs, n) workgroups, plus the evaluation
    const size_t gp = (size_t)std::max<int64_t>(1, std::min<int64_t>(cu, n));
    const size_t coop = align_up(align_up(sizeof(DenseArgs)) + align_up(sizeof(DevResult)) + align_up(8 * 8) +
                                 align_up(64) + align_up(256) + align_up(4 * un * 8) + align_up(3 * um * 8) +
                                 align_up(gp * um * 4) + align_up(2 * gp * um * 8) + align_up((2 * gp * kNS + gp) * 8) +
                                 align_up(3 * um * 8)) +
                        eval;
    return std::max(small, coop);
}

extern "C" accsk_status accsk_workspace_bytes(int64_t n, int64_t m, int64_t count, size_t *bytes) {
    using namespace accsk;
    if (!bytes || count < 1) return ACCSK_INVALID_ARG;
    if (n < 1 || m < 1) return ACCSK_SHAPE;
    const int cu = device_cu_count();
    if (cu <= 0) return ACCSK_HIP_ERROR;
    // one-workgroup launches (+ the FP64 re-evaluation of a single problem)
    size_t b = accsk_small_workspace_bound(count, m) + (size_t)(n + m + 8) * 8 + eval_workspace_bound(m);
    if (m <= 8192) {
        // one cooperative launch holds k <= min(count, CUs) problems with k * gp <= 2 CUs
        const size_t k = (size_t)std::min<int64_t>(count, cu), G = 2 * (size_t)cu;
        size_t d = align_up(sizeof(DenseArgs) * k) + align_up(sizeof(DevResult) * k) + align_up(64 * k) +
                   align_up(64 * k) + align_up(256 * k);
        d += k * (align_up(4 * (size_t)n * 8) + 2 * align_up(3 * (size_t)m * 8) + 3 * 256);  // (+ the monitor)
        d += G * (size_t)m * (4 + 16) + (2 * G * kNS + G) * 8 + 2 * k * 256;
        d += eval_workspace_bound(m);  // allocated while the launch's workspace is still held
        b = std::max(b, d);
    }
    // tiled solver: m > 8192, or a problem whose row blocks do not fit on chip
    b = std::max(b, accsk_tiled_workspace_bound(n, m, cu));
    *bytes = b;
    return ACCSK_OK;
}

// Host validation of a single dense solve's parameters (eps included).
accsk_status accsk_check_dense_params(const accsk_params *p) {
    using namespace accsk;
    if (!p || !finite_pos(p->eps)) return ACCSK_INVALID_ARG;
    return check_params(p);
}

// Batch solve of accsk_small.hip with its workspace.
accsk_status accsk_solve_batch_ws(const accsk_problem *probs, int64_t count, const accsk_params *p,
                                  accsk_result *res, void *stream, accsk::Workspace &ws, accsk_result *const *pub);

// accsk_solve_dense with its workspace.  Over a fixed region the tiled solver
// (m > 8192, or row blocks too large for on-chip memory) is not used (SHAPE).
// pub: null, or the device result record of the stream-ordered form (then res
// is unused and nothing waits for the stream).
accsk_status accsk_solve_dense_ws(const float *C, int64_t n, int64_t m, int64_t ldc, const double *a,
                                  const double *b, const accsk_params *p, double *f_out, double *g_out,
                                  accsk_result *res, void *stream, accsk::Workspace &ws, accsk_result *pub) {
    using namespace accsk;
    if (res) {
        res->status = ACCSK_INVALID_ARG;
        res->converged = 0;
    }
    if (!C || !a || !b || !p || !f_out || !g_out || !(res || pub)) return ACCSK_INVALID_ARG;
    if (!finite_pos(p->eps)) return ACCSK_INVALID_ARG;
    accsk_status st = check_params(p);
    if (st != ACCSK_OK) return st;
    if (n < 1 || m < 1 || ldc < m) return ACCSK_SHAPE;
    if (m > 8192) {
        if (ws.fixed()) return ACCSK_SHAPE;
        st = accsk_tiled_solve(C, ldc, nullptr, nullptr, 0, 0, 1.0, n, m, a, b, p, p->eps, f_out, g_out, res,
                               (hipStream_t)stream, pub);
        return st;
    }
    // A batch of one: one workgroup up to 256 x 256 entries, else a group of
    // cooperating workgroups (or the tiled solver when its row blocks do not
    // fit on chip).
    accsk_problem q{C, n, m, ldc, a, b, f_out, g_out, p->eps};
    accsk_result *const pubs[1] = {pub};
    st = accsk_solve_batch_ws(&q, 1, p, res, stream, ws, pub ? pubs : nullptr);
    if ((st != ACCSK_OK && st != ACCSK_NOT_CONVERGED) || (p->flags & ACCSK_FLAG_NO_COST) ||
        !accsk_on_one_workgroup(n, m, 1))
        return st;
    // The workgroup reports <C,P> and the dual value from its FP32 exponentials;
    // re-evaluate both in FP64 at the returned potentials, as the other solvers do.
    hipStream_t s = (hipStream_t)stream;
    double *buf = nullptr;
    if (ws.get((void **)&buf, (size_t)(n + m + 8) * 8, s) != hipSuccess) return ACCSK_OOM;
    double *an = buf, *bn = buf + n, *out = buf + n + m;
    hipLaunchKernelGGL(normalize_pair, dim3(1), dim3(1024), 0, s, a, n, b, m, an, bn);
    accsk_status se = hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
    if (se == ACCSK_OK) se = run_eval(C, n, m, ldc, p->eps, an, bn, f_out, g_out, out, nullptr, s, ws, pub);
    if (pub) {  // the evaluation has replaced the values in the device record
        ws.put(buf, s);
        return se;
    }
    double h[5] = {0, 0, 0, 0, 0};
    if (se == ACCSK_OK) {
        hipError_t e = hipMemcpyAsync(h, out, 5 * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) se = ACCSK_HIP_ERROR;
    }
    ws.put(buf, s);
    if (se != ACCSK_OK) return se;
    res->eot_value = h[2];
    res->transport_cost = h[3];
    return st;
}

extern "C" accsk_status accsk_solve_dense(const float *C, int64_t n, int64_t m, int64_t ldc, const double *a,
                                          const double *b, const accsk_params *p, double *f_out,
                                          double *g_out, accsk_result *res, void *stream) {
    accsk::Workspace ws;  // stream-ordered allocations
    return accsk_solve_dense_ws(C, n, m, ldc, a, b, p, f_out, g_out, res, stream, ws, nullptr);
}

extern "C" accsk_status accsk_solve_dense_async(const float *C, int64_t n, int64_t m, int64_t ldc, const double *a,
                                                const double *b, const accsk_params *p, double *f_out,
                                                double *g_out, accsk_result *res, void *stream) {
    if (!res) return ACCSK_INVALID_ARG;
    accsk::Workspace ws;  // stream-ordered allocations
    return accsk_solve_dense_ws(C, n, m, ldc, a, b, p, f_out, g_out, nullptr, stream, ws, res);
}

extern "C" accsk_status accsk_plan_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                                         const double *f, const double *g, int64_t row0, int64_t rows,
                                         float *P, int64_t ldp, void *stream) {
    if (!C || !f || !g || !P) return ACCSK_INVALID_ARG;
    if (!finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (n < 1 || m < 1 || ldc < m || ldp < m || row0 < 0 || rows < 0 || row0 + rows > n) return ACCSK_SHAPE;
    if (rows == 0) return ACCSK_OK;
    if (rows > 65535) {
        for (int64_t r = 0; r < rows; r += 65535) {
            accsk_status st = accsk_plan_dense(C, n, m, ldc, eps, f, g, row0 + r, std::min<int64_t>(65535, rows - r),
                                               P + r * ldp, ldp, stream);
            if (st != ACCSK_OK) return st;
        }
        return ACCSK_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    dim3 grid((unsigned)((m + 255) / 256), (unsigned)rows);
    hipLaunchKernelGGL(plan_rows, grid, dim3(256), 0, s, C, m, ldc, 1.0 / eps, f, g, row0, rows, P, ldp);
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

extern "C" accsk_status accsk_eval_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                                         const double *a, const double *b, const double *f, const double *g,
                                         double *out, void *stream) {
    if (!C || !a || !b || !f || !g || !out) return ACCSK_INVALID_ARG;
    if (!finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (n < 1 || m < 1 || ldc < m) return ACCSK_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    double *dout = nullptr;
    Workspace ws;
    if (hipMallocAsync((void **)&dout, 8 * 8, s) != hipSuccess) return ACCSK_OOM;
    accsk_status st = run_eval(C, n, m, ldc, eps, a, b, f, g, dout, nullptr, s, ws);
    if (st == ACCSK_OK) {
        hipError_t e = hipMemcpyAsync(out, dout, 5 * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = ACCSK_HIP_ERROR;
    }
    (void)hipFreeAsync(dout, s);
    return st;
}
