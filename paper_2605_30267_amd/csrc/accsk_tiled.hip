// Tiled solver for large problems: explicit FP32 costs with m > 8192, and
// costs formed on the fly from point clouds, never materialized: the FP64
// argument on the matrix cores for d <= 3, FP64 dot products for 3 < d <= 16,
// the BF16x3 matrix-core cross term for 16 < d <= 128.
//
// One cooperative (persistent) launch runs the whole solve (paper Sec. 2 row
// solve eq:u-update, normalized column step eq:normalized-sinkhorn; Sec. 4
// Algorithms A2MD / A2MD-homotopy; stop on eq:l1tol).  Per Sinkhorn step:
//
//  A. Row sweep.  Block b owns rows [r0, r1); each wave owns RW of them at a
//     time, its lanes walk the columns in chunks staged in LDS.  The shift of
//     row i is its log-sum-exp of the previous step (exact row maximum on the
//     first step or when the sum leaves [2^-40, 2^40]).  Gives u_i.
//  B. Column sweep.  Each lane owns CPL columns of a chunk and walks all rows
//     of the block (staged in LDS), summing 2^(t_ij + u_i - L_j) = P_ij / 2^L_j
//     with L_j the column's log2-sum of the previous step: one FP32
//     exponential per entry, FP64 accumulation.
//  Then, as in the dense solver: grid barrier, combine of the per-block column
//  sums over the block's column slice (S^_j, |c_j - b_j|), grid barrier,
//  totals, update of the block's slice of x and w (Sinkhorn or Algorithm A2MD
//  with the homotopy), grid barrier.
// Exponent arguments (log2 units) are formed in FP64:
//  * explicit C: t_ij = x_j - C_ij / eps;
//  * points: t_ij = xh_j + r_i + sum_k xt_ik y_jk, with the norms folded into a
//    column term xh_j = x_j - kappa_s |y_j|^2 (cosine: x_j - kappa_s) and a row
//    term r_i = -kappa_s |x_i|^2 (cosine: 0), xt_i = 2 kappa_s x_i (cosine:
//    kappa_s x_i), kappa_s = log2(e) / (eps s).  C_ij is never stored.
//  * points with d <= 3 (D = 3): the whole argument, row and column terms
//    included, from one v_mfma_f64_16x16x4f64 per 16 x 16 tile (K = 4 holds
//    the three coordinates and the column term), all FP64.
//  * points with 16 < d <= 128 (D = 32, 64, 128): the sums over k above are
//    x_i . y_j from v_mfma_f32_16x16x32_bf16 on a 3-piece BF16 split of X and
//    Y (split 3: six products, split 2: three), accumulated in FP32 (two
//    independent chains, small products first); the rest of the argument is
//    FP64 as above.
//    In both cases each wave owns a 16-row tile of the block's rows (its
//    operands stay in registers), the block stages chunks of columns in LDS in
//    the operand layout (double-buffered), and both sweeps walk the same tiles.
// If a combined column sum leaves [2^-64, 2^64] (the column mass changed that
// much in one step), an exact column sweep with a per-column maximum redoes the
// column side of that step.

#include <math.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "accsk_common.h"
#include "cost_tiles.h"

namespace accsk {
namespace {

constexpr int kTT = 512;          // threads per block (explicit costs, FP64 sweeps)
constexpr int kTW = kTT / 64;     // waves per block

// Block shape of tiled_solve<D>: the BF16 matrix-core sweeps run 256 threads (one
// wave per SIMD, up to 512 registers each, so that a wave can hold two row tiles);
// everything else 512.
template <int D>
struct TBlk {
    static constexpr int TT = D >= 32 ? 256 : kTT;
    static constexpr int TW = TT / 64;
    static constexpr int ROWS = 16 * TW * (D >= 32 ? 2 : 1);  // rows per block and round (matrix-core sweeps)
};
constexpr int kF64CH = 1024;      // columns per staged chunk, FP64 matrix-core sweeps (d <= 3)
constexpr int kTNS = 8;           // block scalar slots: 0 <u,a>, 1 sum S^, 2 err, 3 mass, 4 <x,b>, 5 fallback
constexpr int kTRB = 256;         // rows staged per row group of the column sweep

template <int D>
struct TCfg {
    static constexpr int DD = D > 0 ? D : 1;                                   // array extent
    static constexpr int RW = D == 0 ? 8 : (D <= 3 ? 8 : (D <= 8 ? 4 : 2));   // rows per wave, row sweep
    static constexpr int CH = D <= 3 ? 2048 : (D <= 8 ? 1024 : 512);           // columns per chunk
    static constexpr int CPL = CH / kTT;                                       // columns per lane, column sweep
    static constexpr int RG = kTW * RW;                                        // rows per group, row sweep
};

template <int D>
size_t tiled_lds_bytes() {
    if (D >= 32) {  // two buffers of Y pieces [tiles][D/32 chunks][3 pieces][64 lanes] x 16 B, column terms, wave sums
        const size_t mch = D == 128 ? 64 : 128;
        return 2 * (mch / 16) * (D / 32) * 3 * 64 * 16 + 2 * mch * sizeof(double) +
               2 * (size_t)TBlk<D>::TW * mch * sizeof(float);
    }
    if (D == 3)  // two buffers of [tiles][64] FP64 B operands, two of the waves' column values
        return 2 * (size_t)(kF64CH / 16) * 64 * sizeof(double) + 2 * (size_t)TBlk<D>::TW * kF64CH * sizeof(float);
    using Cf = TCfg<D>;
    const size_t cols = (size_t)Cf::CH * (Cf::DD + 1) * sizeof(double);
    const size_t rows = (size_t)kTRB * (Cf::DD + 1) * sizeof(double);
    return std::max(cols, rows);
}

struct TiledArgs {
    const float *C;   // explicit cost (D == 0)
    long long ldc;
    const float *X, *Y;  // points (D > 0): n x d, m x d
    long long d;
    int kind;
    double inv_s;
    long long n, m;
    const double *a_in, *b_in;
    double *an, *la2, *xnrm, *rowL, *rowU;   // [n]
    double *bn, *lnb, *ynrm, *xg, *wg, *shat;  // [m]
    double *colL;                            // [m] log2 of the last column sums (column sweep shift)
    float *partf;                            // [G][m]
    double *part, *partmax;                  // [G][m] exact column sweep
    double *bscal;                           // [2][G][kTNS]
    double *uapart, *costpart;               // [G]
    double *gscal;                           // 0: max log2 a, 1: max a
    int *status;
    unsigned long long *bar;
    DevResult *res;
    accsk_result *pub;  // stream-ordered calls: the caller's device result record (else null)
    double *f_out, *g_out;
    double eps, tol, tol_stop, mu0;
    long long max_iter, m0;
    int method, w_rule, flags;
    int split;      // matrix-core cross term (D >= 32): 2 or 3 BF16 pieces
    const bf16x8 *Xpk, *Ypk;  // (D >= 32) X and Y split into BF16 pieces in the operand layout (split_pieces)
    double *cond;   // ACCSK_FLAG_CONDITIONS (Acc): [3][m] grad f, D and v of the last iterate (slice-owned)
    double *cscal;  // [2][G][8] per-block sums of the boundedness monitor, by step parity
};

// Boundedness monitor of the tiled solver: every block sums its column slice;
// block 0 takes the decision after the next grid barrier, when all sums are in.
struct CondPending {
    CondState cs;
    double fval, alpha, mu, a_new, mu_new;
    int have, stage, par, valid;
};

__device__ double tblock_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) s += red[k];
    __syncthreads();
    return s;
}
__device__ double tblock_max(double v, double *red) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = -INFINITY;
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) s = fmax(s, red[k]);
    __syncthreads();
    return s;
}

// Marginals (unit mass, eq:Fc), logs, max log2 a, and FP64 squared norms of
// the points.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void tiled_setup(const TiledArgs *__restrict__ pa) {
    const TiledArgs A = *pa;
    __shared__ double red[16];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    int lbad = 0;
    double s = 0.0;
    for (long long i = tid; i < A.n; i += 1024) {
        const double v = A.a_in[i];
        lbad |= !isfinite(v) ? 2 : (!(v > 0.0) ? 1 : 0);
        s += v;
    }
    for (long long j = tid; j < A.m; j += 1024) {
        const double v = A.b_in[j];
        lbad |= !isfinite(v) ? 2 : (!(v > 0.0) ? 1 : 0);
    }
    if (lbad) atomicOr(&bad, lbad);
    const double sa = tblock_sum(s, red);
    double mx = -INFINITY;
    for (long long i = tid; i < A.n; i += 1024) {
        const double v = A.a_in[i] / sa;
        A.an[i] = v;
        const double l2 = log2(v);
        A.la2[i] = l2;
        mx = fmax(mx, l2);
        double nn = 0.0;
        if (A.X)
            for (long long k = 0; k < A.d; k++) {
                const double xv = A.X[i * A.d + k];
                nn = fma(xv, xv, nn);
            }
        A.xnrm[i] = nn;
    }
    mx = tblock_max(mx, red);
    s = 0.0;
    for (long long j = tid; j < A.m; j += 1024) s += A.b_in[j];
    const double sb = tblock_sum(s, red);
    for (long long j = tid; j < A.m; j += 1024) {
        const double v = A.b_in[j] / sb;
        A.bn[j] = v;
        A.lnb[j] = log(v);
        double nn = 0.0;
        if (A.Y)
            for (long long k = 0; k < A.d; k++) {
                const double yv = A.Y[j * A.d + k];
                nn = fma(yv, yv, nn);
            }
        A.ynrm[j] = nn;
        A.xg[j] = 0.0;
        A.wg[j] = 0.0;
        A.colL[j] = mx;  // first step: shift max log2 a, every term <= 1
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

// FP64 sum / maximum over the 16 lanes of a DPP row (quad_perm [1,0,3,2], [2,3,0,1],
// row_half_mirror, row_mirror); every lane of the row gets the result, in the same order.
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_f64<0xB1, 0xf, 0xf>(v, v);
    v += dpp_f64<0x4E, 0xf, 0xf>(v, v);
    v += dpp_f64<0x141, 0xf, 0xf>(v, v);
    v += dpp_f64<0x140, 0xf, 0xf>(v, v);
    return v;
}
__device__ __forceinline__ double row16_max(double v) {
    v = fmax(v, dpp_f64<0xB1, 0xf, 0xf>(v, v));
    v = fmax(v, dpp_f64<0x4E, 0xf, 0xf>(v, v));
    v = fmax(v, dpp_f64<0x141, 0xf, 0xf>(v, v));
    v = fmax(v, dpp_f64<0x140, 0xf, 0xf>(v, v));
    return v;
}

// gfx950 cross-lane exchanges (a row is 16 lanes): v_permlane32_swap_b32 swaps the
// upper 32 lanes of a with the lower 32 lanes of b, v_permlane16_swap_b32 the odd rows
// of a with the even rows of b.  Written as instructions (the compiler's builtins
// return the first register only); a VALU result needs two wait states before either
// reads it.
__device__ __forceinline__ void swap_lanes32(float &a, float &b) {
    asm("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap_rows16(float &a, float &b) {
    asm("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
// Column sums of four 16 x 16 tiles with no LDS traffic: in lane l, p<g> is tile g's
// partial sum of column l % 16 over the rows that lane group l / 16 holds.  Returns, in
// lane l, the whole column l % 16 of tile {0, 2, 1, 3}[l / 16], added as
// (groups 0 + 2) + (groups 1 + 3).
__device__ __forceinline__ float col_sums4(float p0, float p1, float p2, float p3) {
    swap_lanes32(p0, p1);  // p0 = [p0 lanes 0-31, p1 lanes 0-31], p1 = [p0 lanes 32-63, p1 lanes 32-63]
    swap_lanes32(p2, p3);
    float x = p0 + p1, y = p2 + p3;  // rows: tile 0 (groups 0+2, 1+3), tile 1 (0+2, 1+3); y: tiles 2, 3
    swap_rows16(x, y);               // x = rows 0 of x, y, rows 2 of x, y; y = the rows 1 and 3
    return x + y;
}
__device__ __forceinline__ int col_sums4_tile(int lane) { return ((lane >> 4) & 1) * 2 + (lane >> 5); }

__device__ __forceinline__ double readlane63_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// TR: write the per-step error trace (trace / trace_len).  A separate
// instantiation, so that untraced solves carry no trace code at all.
// The arguments come by value, in the kernel argument segment: pointers read
// from there are known to address global memory, so loads and stores through
// them are global_* instructions.  (Through a pointer to a copy in device memory
// they would be flat_* instructions, which count on the LDS counter as well: every
// wait for an LDS read would then also wait for the outstanding global loads.)
template <int D, bool TR = false, bool CD = false>
__global__ __launch_bounds__(TBlk<D>::TT) __attribute__((amdgpu_waves_per_eu(D >= 32 ? 1 : 2)))
void tiled_solve(const TiledArgs A, double *__restrict__ trace, long long trace_len) {
    constexpr int TT = TBlk<D>::TT, TW = TBlk<D>::TW;
    using Cf = TCfg<D>;
    constexpr int RW = Cf::RW, CH = Cf::CH, CPL = Cf::CPL, RG = Cf::RG, DD = Cf::DD;
    extern __shared__ double tl[];
    __shared__ double tot[kTNS];
    __shared__ double sred[TW * 64];
    __shared__ int bflag, sflag;
    __shared__ CondPending cpend;  // used by block 0 only

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int G = gridDim.x, bid = blockIdx.x;
    if (A.status[0] != ACCSK_OK) {
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
    const long long n = A.n, m = A.m, d = A.d;
    // (matrix-core sweeps: whole 16-row tiles per block)
    const long long rpb = (D == 3 || D >= 32) ? ((n + G - 1) / G + 15) / 16 * 16 : (n + G - 1) / G;
    const long long r0 = std::min(n, (long long)bid * rpb), r1 = std::min(n, r0 + rpb);
    const long long nr = r1 - r0;
    const long long spb = (m + G - 1) / G;
    const long long j0 = std::min(m, (long long)bid * spb), j1 = std::min(m, j0 + spb);
    const double kap2 = kLog2e / A.eps;      // 1/eps in log2 units
    const double ks = kap2 * A.inv_s;        // points: log2 e / (eps s)
    const bool sq = A.kind == ACCSK_SQEUCLID;
    const double coef = sq ? 2.0 * ks : ks;  // cross-term coefficient
    const double La2 = A.gscal[0];

    for (long long i = r0 + tid; i < r1; i += TT) A.rowL[i] = INFINITY;

    // ---- helpers -------------------------------------------------------
    // row constant r_i (log2 units) of the folded argument
    auto row_const = [&](long long i) -> double { return (D > 0 && sq) ? -ks * A.xnrm[i] : 0.0; };
    // column term xh_j of the folded argument at the current x
    auto col_term = [&](long long j) -> double {
        const double x2 = A.xg[j];
        if (D == 0) return x2;
        return sq ? x2 - ks * A.ynrm[j] : x2 - ks;
    };
    // argument t_ij + rc for a row (xt, rc) and a column (y, xh); explicit: cij
    auto arg_pts = [&](const double (&xt)[DD], double rc, const double (&y)[DD], double xh) -> double {
        double t = xh + rc;
#pragma unroll
        for (int k = 0; k < DD; k++) t = fma(xt[k], y[k], t);
        return t;
    };

    double *ysl = tl;                  // [DD][CH] staged y (SoA), row sweep
    double *xhl = tl + (size_t)DD * CH;  // [CH] staged xh
    double *xtl = tl;                  // [DD][kTRB] staged xt, column sweep
    double *rhl = tl + (size_t)DD * kTRB;  // [kTRB] staged row term

    constexpr bool MF = D == 3 || D >= 32;  // matrix-core sweeps (further below)
    auto stage_cols = [&](long long ja, int len) {
        if constexpr (!MF) {
            for (int c = tid; c < len; c += TT) {
                const long long j = ja + c;
                if (D > 0)
#pragma unroll
                    for (int k = 0; k < D; k++) ysl[(size_t)k * CH + c] = k < d ? (double)A.Y[j * d + k] : 0.0;
                xhl[c] = col_term(j);
            }
        }
    };

    // ---- row sweep: u for the block's rows --------------------------------
    auto row_sweep = [&]() {
        if constexpr (!MF) {
            for (long long g0 = 0; g0 < nr; g0 += RG) {
                double xt[RW][DD];
                double rc0[RW], shift[RW];
                bool rv[RW];
                long long ri[RW];
                int unknown = 0;
#pragma unroll
                for (int q = 0; q < RW; q++) {
                    const long long lr = g0 + wid * RW + q;
                    rv[q] = lr < nr;
                    ri[q] = r0 + std::min(lr, nr - 1);
#pragma unroll
                    for (int k = 0; k < DD; k++)
                        xt[q][k] = (D > 0 && k < d) ? coef * (double)A.X[ri[q] * d + k] : 0.0;
                    rc0[q] = row_const(ri[q]);
                    shift[q] = A.rowL[ri[q]];
                    unknown |= (rv[q] && !(shift[q] < INFINITY)) ? 1 : 0;
                }
                __syncthreads();
                if (tid == 0) sflag = 0;
                __syncthreads();
                if (unknown) atomicOr(&sflag, 1);
                __syncthreads();
                bool need_max = sflag != 0;
                double S[RW];
                for (int attempt = 0; attempt < 2; attempt++) {
                    if (need_max) {
                        // exact row maximum of the argument
                        double mx[RW];
#pragma unroll
                        for (int q = 0; q < RW; q++) mx[q] = -INFINITY;
                        for (long long ja = 0; ja < m; ja += CH) {
                            const int len = (int)std::min<long long>(CH, m - ja);
                            __syncthreads();
                            stage_cols(ja, len);
                            __syncthreads();
                            for (int c = lane; c < len; c += 64) {
                                double y[DD];
#pragma unroll
                                for (int k = 0; k < DD; k++) y[k] = D > 0 ? ysl[(size_t)k * CH + c] : 0.0;
                                const double xh = xhl[c];
#pragma unroll
                                for (int q = 0; q < RW; q++) {
                                    double t;
                                    if (D == 0) t = fma(-(double)A.C[ri[q] * A.ldc + ja + c], kap2, xh);
                                    else t = arg_pts(xt[q], rc0[q], y, xh);
                                    mx[q] = fmax(mx[q], t);
                                }
                            }
                        }
#pragma unroll
                        for (int q = 0; q < RW; q++) shift[q] = wave_max(mx[q]);
                    }
                    double acc[RW];
#pragma unroll
                    for (int q = 0; q < RW; q++) acc[q] = 0.0;
                    for (long long ja = 0; ja < m; ja += CH) {
                        const int len = (int)std::min<long long>(CH, m - ja);
                        __syncthreads();
                        stage_cols(ja, len);
                        __syncthreads();
                        float sp[RW];
#pragma unroll
                        for (int q = 0; q < RW; q++) sp[q] = 0.f;
                        for (int c = lane; c < len; c += 64) {
                            double y[DD];
#pragma unroll
                            for (int k = 0; k < DD; k++) y[k] = D > 0 ? ysl[(size_t)k * CH + c] : 0.0;
                            const double xh = xhl[c];
#pragma unroll
                            for (int q = 0; q < RW; q++) {
                                double t;
                                if (D == 0) t = fma(-(double)A.C[ri[q] * A.ldc + ja + c], kap2, xh) - shift[q];
                                else t = arg_pts(xt[q], rc0[q] - shift[q], y, xh);
                                sp[q] += __builtin_amdgcn_exp2f((float)t);
                            }
                        }
#pragma unroll
                        for (int q = 0; q < RW; q++) acc[q] += (double)sp[q];
                    }
                    int bad = 0;
#pragma unroll
                    for (int q = 0; q < RW; q++) {
                        S[q] = readlane63_f64(wave_sum_l63(acc[q]));
                        bad |= (rv[q] && !(S[q] >= 0x1p-40 && S[q] <= 0x1p40)) ? 1 : 0;
                    }
                    __syncthreads();
                    if (tid == 0) sflag = 0;
                    __syncthreads();
                    if (bad) atomicOr(&sflag, 1);
                    __syncthreads();
                    if (sflag == 0 || need_max) break;
                    need_max = true;  // redo the group with the exact maximum
                }
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < RW; q++) {
                        if (!rv[q]) continue;
                        const double lse = shift[q] + dlog2(S[q]);  // log2-sum-exp of the row (without r_i)
                        A.rowL[ri[q]] = lse;
                        A.rowU[ri[q]] = A.la2[ri[q]] - lse;  // u_i = log a_i - LSE_j t_ij, log2 units
                    }
                }
            }
            __syncthreads();
        }
    };

    // ---- column sweep: per-block column sums ---------------------------------
    // EXACT = false: sum of 2^(t_ij + u_i - L_j) into partf, with L_j the
    // column's log2-sum of the previous step (max log2 a on the first step), so
    // the dominant terms have arguments near 0 and keep FP32 exponential
    // accuracy; the combined sum is checked against [2^-64, 2^64].
    // EXACT = true: per-column maximum m_j of t_ij + u_i over the block's rows,
    // then sum of 2^(t_ij + u_i - m_j) into part / partmax.
    auto col_sweep = [&](bool exact) {
        if constexpr (!MF) {
            for (long long ja = 0; ja < m; ja += CH) {
                double y[CPL][DD], xh[CPL];
                long long jc[CPL];
                bool cv[CPL];
#pragma unroll
                for (int p = 0; p < CPL; p++) {
                    const long long c = (long long)wid * 64 * CPL + lane + 64 * p;
                    cv[p] = ja + c < m;
                    jc[p] = std::min(ja + c, m - 1);
#pragma unroll
                    for (int k = 0; k < DD; k++) y[p][k] = (D > 0 && k < d) ? (double)A.Y[jc[p] * d + k] : 0.0;
                    xh[p] = col_term(jc[p]);
                }
                double cmx[CPL], acc[CPL];
#pragma unroll
                for (int p = 0; p < CPL; p++) {
                    cmx[p] = exact ? -INFINITY : A.colL[jc[p]];
                    acc[p] = 0.0;
                }
                for (int sweep = exact ? 0 : 1; sweep < 2; sweep++) {
                    for (long long rb0 = 0; rb0 < nr; rb0 += kTRB) {
                        const int rl = (int)std::min<long long>(kTRB, nr - rb0);
                        __syncthreads();
                        for (int r = tid; r < rl; r += TT) {
                            const long long i = r0 + rb0 + r;
#pragma unroll
                            for (int k = 0; k < DD; k++)
                                xtl[(size_t)k * kTRB + r] = (D > 0 && k < d) ? coef * (double)A.X[i * d + k] : 0.0;
                            rhl[r] = row_const(i) + A.rowU[i];
                        }
                        __syncthreads();
                        float sp[CPL];
#pragma unroll
                        for (int p = 0; p < CPL; p++) sp[p] = 0.f;
                        for (int r = 0; r < rl; r++) {
                            double xt[DD];
#pragma unroll
                            for (int k = 0; k < DD; k++) xt[k] = D > 0 ? xtl[(size_t)k * kTRB + r] : 0.0;
                            const double rh = rhl[r];
#pragma unroll
                            for (int p = 0; p < CPL; p++) {
                                double t;
                                if (D == 0) t = fma(-(double)A.C[(r0 + rb0 + r) * A.ldc + jc[p]], kap2, xh[p]) + rh;
                                else t = arg_pts(xt, rh, y[p], xh[p]);
                                if (sweep == 0) cmx[p] = (t > cmx[p] || t != t) ? t : cmx[p];  // NaN propagates
                                else sp[p] += __builtin_amdgcn_exp2f((float)(t - cmx[p]));
                            }
                            if ((r & 7) == 7) {
#pragma unroll
                                for (int p = 0; p < CPL; p++) {
                                    acc[p] += (double)sp[p];
                                    sp[p] = 0.f;
                                }
                            }
                        }
#pragma unroll
                        for (int p = 0; p < CPL; p++) acc[p] += (double)sp[p];
                    }
                }
#pragma unroll
                for (int p = 0; p < CPL; p++) {
                    if (!cv[p]) continue;
                    if (exact) {
                        A.part[(size_t)bid * m + jc[p]] = acc[p];
                        A.partmax[(size_t)bid * m + jc[p]] = cmx[p];
                    } else {
                        xstore(&A.partf[(size_t)bid * m + jc[p]], (float)acc[p]);
                    }
                }
            }
        }
    };

    // ---- matrix-core sweeps (D = 3 and D >= 32) --------------------------------
    // Both sweeps walk the columns in chunks of MCH staged in LDS, two buffers: the
    // next chunk is loaded while the current one is used.  Each wave owns RT
    // 16-row tiles per round (BF16 engine: two, so that every B operand read from
    // LDS feeds both) and computes 16 x 16 tiles of the exponent argument on the
    // matrix cores:
    //  * D >= 32 (BF16 engine): x_i . y_j from v_mfma_f32_16x16x32_bf16 on the
    //    BF16 pieces (split_pieces layout: unit ((T KC + kc) 3 + piece) 64 + lane
    //    holds features kc 32 + (lane / 16) 8 + [0, 8) of point 16 T + lane % 16),
    //    then arg = coef (x_i . y_j) + (row term + column term) in FP64.  Lane l
    //    holds column l % 16 and rows 4 (l / 16) + q.  The pieces of the next chunk
    //    go straight from global memory into LDS (global_load_lds_dwordx4).
    //  * D = 3 (FP64 engine): the whole argument from one v_mfma_f64_16x16x4f64,
    //    A = [xt_i, 1] (k = 0..3), B = [y_j, column term], accumulator input = the
    //    row term, all FP64.  Lane l holds column l % 16 and rows l / 16 + 4 q.
    // The column term carries the sweep's column shift: xh_j - s_j, -inf past m.
    constexpr bool BF = D >= 32;
    constexpr int KC = BF ? D / 32 : 1;                   // 32-wide K chunks (BF16 engine)
    constexpr int MCH = BF ? (D == 128 ? 64 : 128) : kF64CH;  // columns per chunk
    constexpr int NTC = MCH / 16;                         // column tiles per chunk
    static_assert(NTC % 4 == 0, "the column sums reduce four tiles at a time");
    constexpr int BU = BF ? NTC * KC * 3 * 64 : NTC * 64; // B units per buffer (16 B BF16 pieces, 8 B FP64)
    constexpr int PF = BF ? BU / TT : 1;                  // direct loads per thread and chunk
    constexpr int RT = BF ? 2 : 1;                        // 16-row tiles per wave and round
    static_assert(!MF || !BF || BU % TT == 0, "chunk units per thread");
    constexpr int CPT = (MCH + TT - 1) / TT;              // staged columns per thread
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    bf16x8 *ylp = reinterpret_cast<bf16x8 *>(tl);                       // BF16: [2][BU]
    double *yl64 = tl;                                                  // FP64: [2][NTC][64]
    double *colt = BF ? reinterpret_cast<double *>(ylp + 2 * BU) : tl + 2 * BU;  // BF16: [2][MCH] column terms
    // [2][TW][MCH] per-wave column values (sums are FP32 already), two buffers so that a
    // chunk's cross-wave combine can wait until the next chunk's barrier
    float *mcp = reinterpret_cast<float *>(BF ? colt + 2 * MCH : tl + 2 * BU);
    const int split = A.split;
    const int ntile = (int)((nr + 15) / 16);  // the block's 16-row tiles (r0 is a multiple of 16)
    const int nround = (ntile + TW * RT - 1) / (TW * RT);
    // the block-relative tile of row tile rt of this wave in a round
    auto wtile = [&](int round, int rt) -> int { return (round * TW + wid) * RT + rt; };
    const long long ytiles = (m + 15) / 16, xtiles = (n + 15) / 16;
    // block-relative row of (lane, q) in the wave's tile
    auto trow = [&](int q) -> int { return BF ? 4 * (lane >> 4) + q : (lane >> 4) + 4 * q; };

    // Column data of the next chunk, in registers until it is committed to LDS
    // (columns tid + c TT; index clamped, columns past m get the term -inf).
    double pxg[CPT], pyn[CPT], psh[CPT];
    float py[CPT][3];
    bool pvalid[CPT];
    auto fetch = [&](long long ja, int buf, auto col_shift) {
        if constexpr (BF) {
            // this thread's share of the chunk's pieces, straight into LDS buffer buf
            // (wave w's lanes fill units u TT + 64 w + [0, 64))
            const long long t0 = ja / 16;
            const long long last = (ytiles - t0) * KC * 3 * 64 - 1;
            const bf16x8 *src = A.Ypk + t0 * KC * 3 * 64;
#pragma unroll
            for (int u = 0; u < PF; u++) {
                const long long unit = std::min<long long>((long long)u * TT + tid, last);
                __builtin_amdgcn_global_load_lds(
                    (__attribute__((address_space(1))) const void *)(src + unit),
                    (__attribute__((address_space(3))) void *)(ylp + (size_t)buf * BU + u * TT + wid * 64), 16, 0, 0);
            }
        }
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int col = tid + c * TT;
            if (col >= MCH) continue;
            const long long jj = std::min(ja + col, m - 1);
            pvalid[c] = ja + col < m;
            pxg[c] = A.xg[jj];
            pyn[c] = sq ? A.ynrm[jj] : 0.0;
            psh[c] = col_shift(jj);
            if constexpr (!BF) {
#pragma unroll
                for (int k = 0; k < 3; k++) py[c][k] = k < d ? A.Y[jj * d + k] : 0.f;
            }
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int c = 0; c < CPT; c++) {
            const int col = tid + c * TT;
            if (col >= MCH) continue;
            const double ct = pvalid[c] ? (sq ? pxg[c] - ks * pyn[c] : pxg[c] - ks) - psh[c] : -INFINITY;
            if constexpr (BF) {
                colt[buf * MCH + col] = ct;
            } else {
                double *bt = yl64 + (size_t)buf * BU + (col >> 4) * 64 + (col & 15);
#pragma unroll
                for (int k = 0; k < 3; k++) bt[16 * k] = (double)py[c][k];
                bt[48] = ct;
            }
        }
    };
    // all m columns chunk by chunk; body(ja, buf) uses the chunk staged in LDS buffer buf
    auto for_chunks = [&](auto col_shift, auto body) {
        __syncthreads();  // every wave has left the previous walk's buffers
        fetch(0, 0, col_shift);
        int buf = 0;
        for (long long ja = 0; ja < m; ja += MCH) {
            // this thread's loads of the chunk (direct-to-LDS pieces and column data) are in
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            commit(buf);
            // the chunk is complete in LDS, and every wave has left chunk ja - MCH, whose
            // buffer the next fetch refills
            __syncthreads();
            if (ja + MCH < m) fetch(ja + MCH, buf ^ 1, col_shift);
            body(ja, buf);
            buf ^= 1;
        }
    };

    // A operands of the wave's tile: global row tile r0 / 16 + tile (clamped: an idle
    // wave's results are not used)
    struct AOps {
        bf16x8 h[KC], m_[KC], l[KC];
        double a64;
    };
    auto load_a = [&](int tile, AOps &ao) {
        if constexpr (BF) {
            const long long T = std::min<long long>(r0 / 16 + tile, xtiles - 1);
            const bf16x8 *src = A.Xpk + (T * KC * 3) * 64 + lane;
#pragma unroll
            for (int kc = 0; kc < KC; kc++) {
                ao.h[kc] = src[(kc * 3) * 64];
                ao.m_[kc] = src[(kc * 3 + 1) * 64];
                ao.l[kc] = src[(kc * 3 + 2) * 64];
            }
        } else {
            const long long i = r0 + std::min<long long>((long long)tile * 16 + (lane & 15), nr - 1);
            const int k = lane >> 4;
            ao.a64 = k == 3 ? 1.0 : (k < d ? coef * (double)A.X[i * d + k] : 0.0);
        }
    };
    // BF16 engine: x_i . y_j of one column tile from its B operands (read from LDS by
    // load_b): the products go into two independent accumulators (small products first in
    // each), summed at the end.  S3: the six products of split 3, else the three of split 2.
    struct BOps {
        bf16x8 h[KC], m_[KC], l[KC];
    };
    auto load_b = [&](auto S3, const bf16x8 *bt, BOps &bo) {
#pragma unroll
        for (int kc = 0; kc < KC; kc++) {
            bo.h[kc] = bt[(kc * 3) * 64];
            bo.m_[kc] = bt[(kc * 3 + 1) * 64];
            if constexpr (decltype(S3)::value) bo.l[kc] = bt[(kc * 3 + 2) * 64];
        }
    };
    auto bf_tile = [&](auto S3, const BOps &bo, const AOps &ao) -> floatx4 {
        floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (decltype(S3)::value) {
#pragma unroll
            for (int kc = 0; kc < KC; kc++) {
                c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.m_[kc], bo.m_[kc], c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.h[kc], bo.l[kc], c1, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.l[kc], bo.h[kc], c0, 0, 0, 0);
            }
        }
#pragma unroll
        for (int kc = 0; kc < KC; kc++) {
            c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.h[kc], bo.m_[kc], c1, 0, 0, 0);
            c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.m_[kc], bo.h[kc], c0, 0, 0, 0);
        }
#pragma unroll
        for (int kc = 0; kc < KC; kc++) {
            if (kc & 1) c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.h[kc], bo.h[kc], c0, 0, 0, 0);
            else c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ao.h[kc], bo.h[kc], c1, 0, 0, 0);
        }
        return c0 + c1;
    };
    // For every column tile t of the staged chunk: arg[rt][q] = the exponent argument of
    // (row trow(q) of the wave's row tile rt, column 16 t + lane % 16), given the row terms
    // rt_[rt][q] (BF16: added in FP64 after the product; FP64: the accumulator input); then
    // use(t, arg).
    auto for_tiles = [&](auto S3, int buf, const AOps (&ao)[RT], const double (&rt_)[RT][4], auto use) {
        if constexpr (BF) {
            const bf16x8 *b0 = ylp + (size_t)buf * BU + lane;
            const double *ct = colt + buf * MCH + (lane & 15);
            // Software pipeline over the chunk's column tiles: the B operands are read two
            // tiles ahead, and tile t + 1's products are issued before tile t's FP64
            // epilogue, so that one wave keeps the matrix cores and the VALU busy together.
            BOps bo[3];
            floatx4 cc[RT], cn[RT];
            load_b(S3, b0, bo[0]);
            if (NTC > 1) load_b(S3, b0 + KC * 3 * 64, bo[1]);
#pragma unroll
            for (int r = 0; r < RT; r++) cc[r] = bf_tile(S3, bo[0], ao[r]);
#pragma unroll
            for (int t = 0; t < NTC; t++) {
                if (t + 2 < NTC) load_b(S3, b0 + (t + 2) * KC * 3 * 64, bo[(t + 2) % 3]);
                if (t + 1 < NTC) {
#pragma unroll
                    for (int r = 0; r < RT; r++) cn[r] = bf_tile(S3, bo[(t + 1) % 3], ao[r]);
                }
                const double x0 = ct[t * 16];
                double arg[RT][4];
#pragma unroll
                for (int r = 0; r < RT; r++)
#pragma unroll
                    for (int q = 0; q < 4; q++) arg[r][q] = fma(coef, (double)cc[r][q], rt_[r][q] + x0);
                use(t, arg);
#pragma unroll
                for (int r = 0; r < RT; r++) cc[r] = cn[r];
            }
        } else {
            f64x4 cin[RT];
#pragma unroll
            for (int r = 0; r < RT; r++) cin[r] = f64x4{rt_[r][0], rt_[r][1], rt_[r][2], rt_[r][3]};
            const double *b0 = yl64 + (size_t)buf * BU + lane;
            constexpr int G4 = 4;  // column tiles per group: RT x G4 independent products in flight
#pragma unroll
            for (int t0 = 0; t0 < NTC; t0 += G4) {
                f64x4 dv[G4][RT];
#pragma unroll
                for (int g = 0; g < G4; g++) {
                    const double bv = b0[(t0 + g) * 64];
#pragma unroll
                    for (int r = 0; r < RT; r++)
                        dv[g][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(ao[r].a64, bv, cin[r], 0, 0, 0);
                }
#pragma unroll
                for (int g = 0; g < G4; g++) {
                    double arg[RT][4];
#pragma unroll
                    for (int r = 0; r < RT; r++)
#pragma unroll
                        for (int q = 0; q < 4; q++) arg[r][q] = dv[g][r][q];
                    use(t0 + g, arg);
                }
            }
        }
    };
    // run f with the split as a compile-time constant (FP64 engine: no split)
    auto with_split = [&](auto f) {
        if (BF && split == 2) f(std::integral_constant<bool, false>{});
        else f(std::integral_constant<bool, true>{});
    };
    auto zero_shift = [](long long) { return 0.0; };

    // Row sweep: the same rule as row_sweep (previous log-sum-exp as the shift,
    // exact row maximum when unknown or when the sum leaves [2^-40, 2^40]).
    auto mrow_sweep = [&]() {
        if constexpr (MF) {
            for (int round = 0; round < nround; round++) {
                bool act[RT];
                AOps ao[RT];
                double rc[RT][4], shift[RT][4];
                long long ri[RT][4];
                bool rv[RT][4];
                int unknown = 0;
#pragma unroll
                for (int r = 0; r < RT; r++) {
                    const int tile = wtile(round, r);
                    act[r] = tile < ntile;
                    load_a(tile, ao[r]);
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const long long lr = (long long)tile * 16 + trow(q);
                        rv[r][q] = act[r] && lr < nr;
                        ri[r][q] = r0 + std::max(0LL, std::min(lr, nr - 1));
                        rc[r][q] = row_const(ri[r][q]);
                        shift[r][q] = rv[r][q] ? A.rowL[ri[r][q]] : 0.0;
                        unknown |= (rv[r][q] && !(shift[r][q] < INFINITY)) ? 1 : 0;
                    }
                }
                const bool wact = act[0];  // the wave has work this round (its first tile is in range)
                __syncthreads();
                if (tid == 0) sflag = 0;
                __syncthreads();
                if (unknown) atomicOr(&sflag, 1);
                __syncthreads();
                bool need_max = sflag != 0;
                double S[RT][4];
                for (int attempt = 0; attempt < 2; attempt++) {
                    if (need_max) {
                        double mx[RT][4];
#pragma unroll
                        for (int r = 0; r < RT; r++)
#pragma unroll
                            for (int q = 0; q < 4; q++) mx[r][q] = -INFINITY;
                        with_split([&](auto S3) {
                            for_chunks(zero_shift, [&](long long, int buf) {
                                if (!wact) return;
                                for_tiles(S3, buf, ao, rc, [&](int, const double (&arg)[RT][4]) {
#pragma unroll
                                    for (int r = 0; r < RT; r++)
#pragma unroll
                                        for (int q = 0; q < 4; q++) mx[r][q] = fmax(mx[r][q], arg[r][q]);
                                });
                            });
                        });
#pragma unroll
                        for (int r = 0; r < RT; r++)
#pragma unroll
                            for (int q = 0; q < 4; q++) shift[r][q] = row16_max(mx[r][q]);
                    }
                    double acc[RT][4], base[RT][4];
#pragma unroll
                    for (int r = 0; r < RT; r++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            acc[r][q] = 0.0;
                            base[r][q] = rc[r][q] - shift[r][q];
                        }
                    with_split([&](auto S3) {
                        for_chunks(zero_shift, [&](long long, int buf) {
                            if (!wact) return;
                            float sp[RT][4];
#pragma unroll
                            for (int r = 0; r < RT; r++)
#pragma unroll
                                for (int q = 0; q < 4; q++) sp[r][q] = 0.f;
                            for_tiles(S3, buf, ao, base, [&](int, const double (&arg)[RT][4]) {
#pragma unroll
                                for (int r = 0; r < RT; r++)
#pragma unroll
                                    for (int q = 0; q < 4; q++) sp[r][q] += __builtin_amdgcn_exp2f((float)arg[r][q]);
                            });
#pragma unroll
                            for (int r = 0; r < RT; r++)
#pragma unroll
                                for (int q = 0; q < 4; q++) acc[r][q] += (double)sp[r][q];
                        });
                    });
                    int bad = 0;
#pragma unroll
                    for (int r = 0; r < RT; r++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            S[r][q] = row16_sum(acc[r][q]);
                            bad |= (rv[r][q] && !(S[r][q] >= 0x1p-40 && S[r][q] <= 0x1p40)) ? 1 : 0;
                        }
                    __syncthreads();
                    if (tid == 0) sflag = 0;
                    __syncthreads();
                    if (bad) atomicOr(&sflag, 1);
                    __syncthreads();
                    if (sflag == 0 || need_max) break;
                    need_max = true;  // redo the round with the exact maximum
                }
                if ((lane & 15) == 0) {
#pragma unroll
                    for (int r = 0; r < RT; r++)
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            if (!rv[r][q]) continue;
                            const double lse = shift[r][q] + dlog2(S[r][q]);
                            A.rowL[ri[r][q]] = lse;
                            A.rowU[ri[r][q]] = A.la2[ri[r][q]] - lse;
                        }
                }
            }
            __syncthreads();
        }
    };

    // Column sweep: per-block column sums as col_sweep (EXACT = false: shift L_j,
    // the column's log2-sum of the previous step; EXACT = true: the block's column
    // maximum, then the sums).  A tile's 16 rows are added in FP32 (4 per lane,
    // then across the lane groups), the waves' tiles and the rounds in FP64 in a
    // fixed order.  Several rounds accumulate in part (FP64) before partf is written.
    auto mcol_sweep = [&](bool exact) {
        if constexpr (MF) {
            // one pass over the block's rows; MXS (compile time): the maximum pass of the
            // exact sweep, else a sum pass
            auto col_pass = [&](auto MXS) {
                constexpr bool mxs = decltype(MXS)::value;
                auto shift_src = [&](long long j) {
                    return exact ? (mxs ? 0.0 : A.partmax[(size_t)bid * m + j]) : A.colL[j];
                };
                if (nround == 0) {  // a block without rows: its partials are the identity
                    for (long long j = tid; j < m; j += TT) {
                        const size_t o = (size_t)bid * m + j;
                        if (mxs) A.partmax[o] = -INFINITY;
                        else if (exact) A.part[o] = 0.0;
                        else xstore(&A.partf[o], 0.0f);
                    }
                }
                for (int round = 0; round < nround; round++) {
                    bool act[RT];
                    AOps ao[RT];
                    double rh[RT][4];
#pragma unroll
                    for (int r = 0; r < RT; r++) {
                        const int tile = wtile(round, r);
                        act[r] = tile < ntile;
                        load_a(tile, ao[r]);
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const long long lr = (long long)tile * 16 + trow(q);
                            const long long i = r0 + std::max(0LL, std::min(lr, nr - 1));
                            rh[r][q] = (act[r] && lr < nr) ? row_const(i) + A.rowU[i] : -INFINITY;
                        }
                    }
                    const bool wact = act[0];
                    // a chunk's column values (mcp buffer pb) added over the waves in a fixed
                    // order, into the block's partials
                    auto combine = [&](long long ja, int pb) {
                        const float *mc = mcp + pb * TW * MCH;
                        for (int c = tid; c < MCH; c += TT) {
                            const long long j = ja + c;
                            if (j >= m) continue;
                            double tv = mxs ? -INFINITY : 0.0;
                            for (int w = 0; w < TW; w++) {
                                const double x = mc[w * MCH + c];
                                if (mxs) tv = (x > tv || x != x) ? x : tv;
                                else tv += x;
                            }
                            const size_t o = (size_t)bid * m + j;
                            if (mxs) {
                                A.partmax[o] = round == 0 ? tv : fmax(A.partmax[o], tv);
                            } else if (exact) {
                                A.part[o] = round == 0 ? tv : A.part[o] + tv;
                            } else if (nround == 1) {
                                xstore(&A.partf[o], (float)tv);
                            } else {
                                const double s2 = round == 0 ? tv : A.part[o] + tv;
                                A.part[o] = s2;
                                if (round == nround - 1) xstore(&A.partf[o], (float)s2);
                            }
                        }
                    };
                    with_split([&](auto S3) {
                        long long jlast = 0;
                        int blast = 0;
                        for_chunks(shift_src, [&](long long ja, int buf) {
                            // every wave has passed this chunk's barrier, so the previous
                            // chunk's values are complete
                            if (ja > 0) combine(ja - MCH, buf ^ 1);
                            float *mw = mcp + (buf * TW + wid) * MCH;
                            if (wact) {
                                float p4[4];          // the current group of four tiles' partial sums
                                float cs[NTC / 4];    // the chunk's column sums, stored after its last tile
                                for_tiles(S3, buf, ao, rh, [&](int t, const double (&arg)[RT][4]) {
                                    if constexpr (mxs) {
                                        double v = -INFINITY;
#pragma unroll
                                        for (int r = 0; r < RT; r++)
#pragma unroll
                                            for (int q = 0; q < 4; q++)
                                                v = (arg[r][q] > v || arg[r][q] != arg[r][q]) ? arg[r][q] : v;  // NaN propagates
                                        double u = __shfl_xor(v, 16, 64);
                                        v = (u > v || u != u) ? u : v;
                                        u = __shfl_xor(v, 32, 64);
                                        v = (u > v || u != u) ? u : v;
                                        // a shift: any value near the maximum serves, as the same
                                        // one is used for the sums and the combine
                                        if (lane < 16) mw[t * 16 + lane] = (float)v;
                                    } else {
                                        float p = __builtin_amdgcn_exp2f((float)arg[0][0]);
#pragma unroll
                                        for (int r = 0; r < RT; r++)
#pragma unroll
                                            for (int q = 0; q < 4; q++)
                                                if (r + q > 0) p += __builtin_amdgcn_exp2f((float)arg[r][q]);
                                        p4[t & 3] = p;
                                        // tiles t - 3 .. t: across the lane groups at once
                                        if ((t & 3) == 3) cs[t >> 2] = col_sums4(p4[0], p4[1], p4[2], p4[3]);
                                    }
                                });
                                if constexpr (!mxs) {
#pragma unroll
                                    for (int k = 0; k < NTC / 4; k++)
                                        mw[(4 * k + col_sums4_tile(lane)) * 16 + (lane & 15)] = cs[k];
                                }
                            } else {
                                for (int c = lane; c < MCH; c += 64) mw[c] = mxs ? -INFINITY : 0.f;
                            }
                            jlast = ja;
                            blast = buf;
                        });
                        __syncthreads();
                        combine(jlast, blast);
                    });
                }
                __syncthreads();
            };
            if (exact) col_pass(std::integral_constant<bool, true>{});
            col_pass(std::integral_constant<bool, false>{});
        }
    };

    double mu = A.mu0, alpha = dsqrt(2.0 * A.mu0);
    long long mstage = A.m0, kin = 0, it = 0, steps = 0, fallbacks = 0, incr = 0, restarts = 0;
    double fprev = 0.0;
    bool first = true;
    unsigned long long gen = 0;
    int status = ACCSK_OK;
    double err = 0.0, last_mass = 0.0, last_xb2 = 0.0, eot = 0.0, fval = 0.0, cost_total = NAN;
    const bool mon = CD && A.cond != nullptr && A.method == ACCSK_ACC;  // diagnostic instantiation only
    if (mon && bid == 0 && tid == 0) {
        cpend.cs = CondState{0.0, 0.0, 0, 0, 0};
        cpend.valid = 0;
    }
    // Block 0, after a grid barrier: the decision for the iterate whose slice sums are complete.
    auto cond_settle = [&]() {
        if (!(mon && bid == 0 && tid == 0 && cpend.valid)) return;
        const double *cs = A.cscal + (size_t)cpend.par * G * 8;
        double r6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int b = 0; b < G; b++)
            for (int q = 0; q < 6; q++) r6[q] += xload(&cs[(size_t)b * 8 + q]);
        CondState c = cpend.cs;
        cond_decide(c, cpend.have != 0, r6[0], r6[1], r6[2], r6[3], r6[4], cpend.fval, cpend.alpha, cpend.mu);
        if (cpend.stage) c.Eb = cond_lyap(cpend.fval, r6[5], r6[3], cpend.a_new, cpend.mu_new);
        cpend.cs = c;
        cpend.valid = 0;
    };

    for (long long step = 0;; step++) {
        const int par = (int)(step & 1);
        double *bs = A.bscal + (size_t)par * G * kTNS;
        if constexpr (MF) {
            mrow_sweep();
            mcol_sweep(false);
        } else {
            row_sweep();
            col_sweep(false);
        }
        if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
        cond_settle();

        bool exact = false;
        for (int pass = 0; pass < 2; pass++) {
            if (pass == 1) {
                if (!exact) break;
                if constexpr (MF) mcol_sweep(true);
                else col_sweep(true);
                if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
                fallbacks++;
            }
            // combine the column slice [j0, j1): thread t sums blocks grp, grp + NGRP, ... of column cb + t % CW
            constexpr int CW = 32, NGRP = TT / CW;
            const int coff = tid % CW, grp = tid / CW;
            double aS = 0.0, aE = 0.0, aC = 0.0, aXB = 0.0, aFB = 0.0;
            for (long long cb = j0; cb < j1; cb += CW) {
                const long long j = cb + coff;
                double acc = 0.0, pm = -INFINITY;
                if (pass == 0) {
                    // the partials come from blocks on other XCDs and miss in L2: a raw buffer
                    // (one offset register, the stride in a scalar register, reads past the
                    // last block return 0) keeps PU loads in flight, summed in block order
                    if (j < j1) {
                        constexpr int PU = 8;
                        const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
                            (void *)A.partf, (short)0, (int)((long long)G * m * 4), 0x00020000);
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
                        for (int b = grp; b < G; b += NGRP) pm = fmax(pm, A.partmax[(size_t)b * m + j]);
                    sred[tid] = pm;
                    __syncthreads();
                    pm = -INFINITY;
                    for (int q = 0; q < NGRP; q++) pm = fmax(pm, sred[q * CW + coff]);
                    __syncthreads();
                    if (j < j1)
                        for (int b = grp; b < G; b += NGRP) {
                            const double mb = A.partmax[(size_t)b * m + j];
                            if (mb != -INFINITY) acc += A.part[(size_t)b * m + j] * dexp2(mb - pm);  // NaN kept
                        }
                }
                sred[tid] = acc;
                __syncthreads();
                if (tid < CW && j < j1) {
                    double sc = 0.0;
                    for (int q = 0; q < NGRP; q++) sc += sred[q * CW + tid];
                    const double xj = A.xg[j];
                    double lc2, c;  // log2 c_j and c_j, the column sum of P at (u(x), x)
                    if (pass == 0) {
                        lc2 = A.colL[j] + dlog2(sc);
                        // out of range -> exact sweep; NaN (a non-finite input) goes on to the error test
                        if (sc < 0x1p-64 || sc > 0x1p64) aFB += 1.0;
                    } else {
                        lc2 = pm + dlog2(sc);
                    }
                    c = dexp2(lc2);
                    A.colL[j] = lc2;  // next step's shift (only this block reads or writes column j here)
                    // c_j = sum_i 2^(t_ij + u_i) = exp(x_j + ell_j):  S^_j = log b_j - ell_j
                    const double sh = A.lnb[j] * kLog2e - lc2 + xj;
                    A.shat[j] = sh;
                    aS += sh;
                    aE += fabs(c - A.bn[j]);
                    aC += c;
                    aXB += xj * A.bn[j];
                }
                __syncthreads();
            }
            if (wid == 0) {
                // <u,a> over this block's rows (log2 units) for the reduced dual objective
                double aU = 0.0;
                for (long long i = r0 + lane; i < r1; i += 64) aU += A.an[i] * A.rowU[i];
                aU = wave_sum(aU);
                aS = wave_sum(aS);
                aE = wave_sum(aE);
                aC = wave_sum(aC);
                aXB = wave_sum(aXB);
                aFB = wave_sum(aFB);
                if (lane == 0) {
                    double *pp = bs + (size_t)bid * kTNS;
                    xstore(&pp[0], aU);
                    xstore(&pp[1], aS);
                    xstore(&pp[2], aE);
                    xstore(&pp[3], aC);
                    xstore(&pp[4], aXB);
                    xstore(&pp[5], aFB);
                }
            }
            if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
            for (int sidx = wid; sidx < 6; sidx += TW) {
                double v = 0.0;
                for (int b = lane; b < G; b += 64) v += bs[(size_t)b * kTNS + sidx];
                v = wave_sum(v);
                if (lane == 0) tot[sidx] = v;
            }
            __syncthreads();
            exact = (pass == 0) && (tot[5] > 0.0);
            __syncthreads();
        }
        if (status != ACCSK_OK) break;

        err = tot[2];
        if constexpr (TR) {
            if (bid == 0 && tid == 0 && steps < trace_len) xstore(&trace[steps], err);
        }
        const double mean = tot[1] / (double)m;
        last_mass = tot[3];
        last_xb2 = tot[4];
        steps++;
        if (!isfinite(err)) {
            status = (steps == 1) ? ACCSK_NONFINITE : ACCSK_DIVERGED;
            break;
        }
        // update of this block's slice of x and w (same scalars in every block)
        const double fval = 1.0 - (tot[0] + tot[4]) * kLn2;  // f(x) = 1 - <u,a> - <x,b>
        const double fp = fprev;
        fprev = fval;
        bool stop = false;
        if (A.method == ACCSK_SINKHORN) {
            if (steps > 1 && fval_rose(fval, fp)) incr++;
            if (err < A.tol_stop || it >= A.max_iter) stop = true;
            else {
                for (long long j = j0 + tid; j < j1; j += TT) xstore(&A.xg[j], A.shat[j] - mean);
                it++;
            }
        } else {
            if (!first) {
                const double c2 = alpha * alpha - 2.0, inv = 1.0 / (1.0 + alpha);
                for (long long j = j0 + tid; j < j1; j += TT)
                    A.wg[j] = (A.wg[j] + c2 * A.xg[j] + 2.0 * (A.shat[j] - mean)) * inv;
                it++;
                kin++;
                if (fval_rose(fval, fp)) {
                    incr++;
                    if (A.flags & ACCSK_FLAG_RESTART) {  // safeguard: reset the extrapolation, w <- alpha x
                        for (long long j = j0 + tid; j < j1; j += TT) A.wg[j] = alpha * A.xg[j];
                        restarts++;
                    }
                }
            }
            if (CD && mon) {
                // Boundedness monitor over this block's columns (each thread reads the columns it
                // updated above); the new iterate is (x, w_k) with w_k as carried to the next x update
                const bool stage = !(err < A.tol_stop || it >= A.max_iter) && !first && kin == mstage;
                const double a_new = dsqrt(mu), ratio = A.w_rule == ACCSK_W_Y_CONTINUOUS ? a_new / alpha : 1.0;
                const CondCols cc{A.xg, A.wg, A.shat, A.bn, A.cond, A.cond + m, A.cond + 2 * m};
                const CondSums cv = cond_cols(cc, j0 + tid, j1, TT, 0, 0.0, 0.0, 0.0, alpha, first ? 0 : 1,
                                              stage ? 1 : 0, ratio, a_new);
                double s6[6] = {cv.lhs1, cv.lhs2, cv.vd, cv.K, cv.l1, cv.vd2};
                for (int q = 0; q < 6; q++) s6[q] = tblock_sum(s6[q], sred);
                if (tid == 0) {
                    double *cs = A.cscal + ((size_t)par * G + bid) * 8;
                    for (int q = 0; q < 6; q++) xstore(&cs[q], s6[q]);
                    if (bid == 0) {
                        cpend.fval = fval;
                        cpend.alpha = alpha;
                        cpend.mu = mu;
                        cpend.a_new = a_new;
                        cpend.mu_new = 0.5 * mu;
                        cpend.have = first ? 0 : 1;
                        cpend.stage = stage ? 1 : 0;
                        cpend.par = par;
                        cpend.valid = 1;
                    }
                }
            }
            if (err < A.tol_stop || it >= A.max_iter) stop = true;
            else {
                if (!first && kin == mstage) {
                    const double mu_new = mu / 2.0;
                    if (A.w_rule == ACCSK_W_Y_CONTINUOUS) {
                        const double ratio = dsqrt(2.0 * mu_new) / alpha;
                        for (long long j = j0 + tid; j < j1; j += TT) A.wg[j] *= ratio;
                    }
                    mu = mu_new;
                    alpha = dsqrt(2.0 * mu);
                    mstage = (long long)floor(1.4142135623730951 * (double)mstage) + 1;
                    kin = 0;
                }
                first = false;
                const double inv = 1.0 / (1.0 + alpha);
                for (long long j = j0 + tid; j < j1; j += TT) xstore(&A.xg[j], (A.wg[j] + (A.shat[j] - mean)) * inv);
            }
        }
        if (stop) break;
        if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) { status = ACCSK_HIP_ERROR; break; }
    }

    // ---------------- outputs ----------------
    if (status == ACCSK_OK || status == ACCSK_DIVERGED) {
        double ua = 0.0;
        for (long long i = r0 + tid; i < r1; i += TT) {
            const double u2 = A.rowU[i];
            ua += A.an[i] * u2;
            A.f_out[i] = A.eps * kLn2 * u2;
        }
        ua = tblock_sum(ua, sred);
        for (long long j = j0 + tid; j < j1; j += TT) A.g_out[j] = A.eps * kLn2 * A.xg[j];
        // <C, P> at the returned potentials: C in FP64 (recomputed from the points)
        double cst = 0.0;
        if (!(A.flags & ACCSK_FLAG_NO_COST)) {
            if constexpr (D == 0) {
                for (long long i = r0 + wid; i < r1; i += TW) {
                    const double u2 = A.rowU[i];
                    for (long long j = lane; j < m; j += 64) {
                        const double cij = (double)A.C[i * A.ldc + j];
                        const double t = A.xg[j] - kap2 * cij + u2;
                        cst += cij * (double)__builtin_amdgcn_exp2f((float)t);
                    }
                }
            } else {
                // 64 columns at a time in LDS (FP64, feature-major: lane c reads feature k of
                // its column at k * 64 + c), one column per lane; each wave takes four rows at
                // a time, so every LDS read feeds four FP64 FMAs
                constexpr int EC = 64, ER = 4;
                double *eyl = tl;              // [d][EC]
                double *exg = tl + d * EC;     // [EC] x_j
                double *eyn = exg + EC;        // [EC] |y_j|^2
                for (long long ja = 0; ja < m; ja += EC) {
                    __syncthreads();
                    for (long long q = tid; q < EC * d; q += TT) {
                        const long long c = q % EC, k = q / EC, j = std::min(ja + c, m - 1);
                        eyl[q] = (double)A.Y[j * d + k];
                    }
                    if (tid < EC) {
                        const long long j = std::min(ja + tid, m - 1);
                        exg[tid] = ja + tid < m ? A.xg[j] : -INFINITY;
                        eyn[tid] = A.ynrm[j];
                    }
                    __syncthreads();
                    for (long long i0 = r0 + (long long)wid * ER; i0 < r1; i0 += (long long)TW * ER) {
                        long long ir[ER];
                        double dot[ER];
#pragma unroll
                        for (int r = 0; r < ER; r++) {
                            ir[r] = std::min(i0 + r, r1 - 1);
                            dot[r] = 0.0;
                        }
                        for (long long k = 0; k < d; k++) {
                            const double y = eyl[k * EC + lane];
#pragma unroll
                            for (int r = 0; r < ER; r++) dot[r] = fma((double)A.X[ir[r] * d + k], y, dot[r]);
                        }
#pragma unroll
                        for (int r = 0; r < ER; r++) {
                            if (i0 + r >= r1) continue;
                            const double cij = (sq ? A.xnrm[ir[r]] + eyn[lane] - 2.0 * dot[r] : 1.0 - dot[r]) * A.inv_s;
                            const double t = exg[lane] - kap2 * cij + A.rowU[ir[r]];
                            if (t > -INFINITY) cst += cij * (double)__builtin_amdgcn_exp2f((float)t);
                        }
                    }
                }
            }
            cst = tblock_sum(cst, sred);
        }
        if (tid == 0) {
            xstore(&A.uapart[bid], ua);
            xstore(&A.costpart[bid], cst);
        }
        if (!grid_sync(A.bar, gen, &bflag, (unsigned)G)) status = ACCSK_HIP_ERROR;
        if (status != ACCSK_HIP_ERROR) cond_settle();  // the last iterate
        if (bid == 0 && tid == 0 && status != ACCSK_HIP_ERROR) {
            double ua2 = 0.0, c2 = 0.0;
            for (int b = 0; b < G; b++) {
                ua2 += A.uapart[b];
                c2 += A.costpart[b];
            }
            const double ua_ln = ua2 * kLn2, xb_ln = last_xb2 * kLn2;
            fval = 1.0 - ua_ln - xb_ln;
            eot = A.eps * (ua_ln + xb_ln - last_mass);
            if (!(A.flags & ACCSK_FLAG_NO_COST)) cost_total = c2;
        }
    }
    if (bid == 0 && tid == 0) {
        DevResult r;
        r.iters = it;
        r.steps = steps;
        r.fallback = fallbacks;
        r.incr = incr;
        r.restarts = restarts;
        r.err = err;
        r.eot = eot;
        r.fval = fval;
        r.cost = cost_total;
        r.converged = (status == ACCSK_OK && err < A.tol_stop) ? 1 : 0;
        r.status = status;
        r.cond1 = mon ? cpend.cs.n1 : -1;
        r.cond2 = mon ? cpend.cs.n2 : -1;
        r.lyap = mon ? cpend.cs.nl : -1;
        r.t0 = A.res->t0;
        r.t1 = dev_clock();
        *A.res = r;
    }
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

__global__ __launch_bounds__(64) void publish_tiled(const TiledArgs *__restrict__ pa, double tick_ms) {
    if (threadIdx.x == 0 && pa->pub) publish_record(pa->pub, *pa->res, tick_ms);
}

template <int D, bool TR, bool CD>
accsk_status tiled_launch(TiledArgs &A, const accsk_params *p, accsk_result *res, hipStream_t s) {
    int dev = 0, cu = 0, occ = 0;
    ACCSK_HIP_TRY(hipGetDevice(&dev));
    ACCSK_HIP_TRY(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t lds = tiled_lds_bytes<D>();
    ACCSK_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, tiled_solve<D, TR, CD>, TBlk<D>::TT, lds));
    if (occ < 1) return ACCSK_SHAPE;
    long long G = (long long)std::min(occ, 2) * cu;
    // matrix-core sweeps: 16-row tiles, one per wave and round, so about 128 rows per
    // block (each staged column chunk then serves 8 tiles)
    if (D == 3 || D >= 32)
        G = std::max<long long>(1, std::min<long long>(G, (A.n + TBlk<D>::ROWS - 1) / TBlk<D>::ROWS));
    const size_t n = A.n, m = A.m;
    size_t off = 0;
    const size_t o_args = off; off = align_up(off + sizeof(TiledArgs));
    const size_t o_res = off; off = align_up(off + sizeof(DevResult));
    const size_t o_small = off; off = align_up(off + 64 * 8);  // gscal, status
    const size_t o_bar = off; off = align_up(off + 256);
    const size_t o_n = off; off = align_up(off + 5 * n * 8);
    const size_t o_m = off; off = align_up(off + 7 * m * 8);
    const size_t o_pf = off; off = align_up(off + (size_t)G * m * 4);
    const size_t o_pe = off; off = align_up(off + 2 * (size_t)G * m * 8);
    const size_t o_bs = off; off = align_up(off + (2 * (size_t)G * kTNS + 2 * (size_t)G) * 8);
    const bool cond = (p->flags & ACCSK_FLAG_CONDITIONS) && p->method == ACCSK_ACC;
    const size_t o_cond = off; off = align_up(off + (cond ? (3 * m + 2 * (size_t)G * 8) * 8 : 0));
    constexpr int KC = D >= 32 ? D / 32 : 1;  // BF16 pieces of X and Y (matrix-core sweeps)
    const size_t xp_units = D >= 32 ? (n + 15) / 16 * KC * 3 * 64 : 0, yp_units = D >= 32 ? (m + 15) / 16 * KC * 3 * 64 : 0;
    const size_t o_xp = off; off = align_up(off + xp_units * sizeof(bf16x8));
    const size_t o_yp = off; off = align_up(off + yp_units * sizeof(bf16x8));
    char *base = nullptr;
    if (hipMallocAsync((void **)&base, off, s) != hipSuccess) return ACCSK_OOM;
    double *pn = (double *)(base + o_n), *pm = (double *)(base + o_m);
    A.an = pn;
    A.la2 = pn + n;
    A.xnrm = pn + 2 * n;
    A.rowL = pn + 3 * n;
    A.rowU = pn + 4 * n;
    A.bn = pm;
    A.lnb = pm + m;
    A.ynrm = pm + 2 * m;
    A.xg = pm + 3 * m;
    A.wg = pm + 4 * m;
    A.shat = pm + 5 * m;
    A.colL = pm + 6 * m;
    A.partf = (float *)(base + o_pf);
    A.part = (double *)(base + o_pe);
    A.partmax = A.part + (size_t)G * m;
    A.bscal = (double *)(base + o_bs);
    A.uapart = A.bscal + 2 * (size_t)G * kTNS;
    A.costpart = A.uapart + G;
    A.gscal = (double *)(base + o_small);
    A.status = (int *)(A.gscal + 8);
    A.bar = (unsigned long long *)(base + o_bar);
    A.res = (DevResult *)(base + o_res);
    A.cond = cond ? (double *)(base + o_cond) : nullptr;
    A.cscal = cond ? A.cond + 3 * m : nullptr;
    A.Xpk = D >= 32 ? (const bf16x8 *)(base + o_xp) : nullptr;
    A.Ypk = D >= 32 ? (const bf16x8 *)(base + o_yp) : nullptr;
    A.tol = p->tol;
    A.tol_stop = p->tol * (1.0 - 1.0 / 16.0);
    A.mu0 = p->mu0;
    A.max_iter = p->max_iter;
    A.m0 = p->m0;
    A.method = p->method;
    A.w_rule = p->w_rule;
    A.flags = p->flags;
    TiledArgs *d_args = (TiledArgs *)(base + o_args);
    const bool async = A.pub != nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (!async) {
        if (hipEventCreate(&ev0) != hipSuccess) ev0 = nullptr;
        if (hipEventCreate(&ev1) != hipSuccess) ev1 = nullptr;
    }
    // (tiled_setup also zeroes the barrier words)
    hipError_t e = async ? upload_args(d_args, &A, sizeof(TiledArgs), s)
                         : hipMemcpyAsync(d_args, &A, sizeof(TiledArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && D >= 32) {
        const long long ux = (long long)(n + 15) / 16 * KC * 64, uy = (long long)(m + 15) / 16 * KC * 64;
        hipLaunchKernelGGL(split_pieces, dim3((unsigned)((ux + 255) / 256)), dim3(256), 0, s, A.X, (long long)n, A.d,
                           KC, (bf16x8 *)A.Xpk, 0ll);
        hipLaunchKernelGGL(split_pieces, dim3((unsigned)((uy + 255) / 256)), dim3(256), 0, s, A.Y, (long long)m, A.d,
                           KC, (bf16x8 *)A.Ypk, 0ll);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(tiled_setup, dim3(1), dim3(1024), 0, s, (const TiledArgs *)d_args);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ev0) e = hipEventRecord(ev0, s);
    if (e == hipSuccess) {
        double *tr = TR ? p->err_trace : nullptr;
        long long tl = TR ? p->trace_len : 0;
        void *kargs[] = {&A, &tr, &tl};
        e = hipLaunchCooperativeKernel((const void *)tiled_solve<D, TR, CD>, dim3((unsigned)G), dim3(TBlk<D>::TT), kargs, lds, s);
    }
    if (e == hipSuccess && ev1) e = hipEventRecord(ev1, s);
    if (async) {
        if (e == hipSuccess) {
            hipLaunchKernelGGL(publish_tiled, dim3(1), dim3(64), 0, s, (const TiledArgs *)d_args, wall_tick_ms());
            e = hipGetLastError();
        }
        (void)hipFreeAsync(base, s);
        return e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
    }
    DevResult hr{};
    if (e == hipSuccess) e = hipMemcpyAsync(&hr, base + o_res, sizeof(DevResult), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float kms = -1.f;
    if (e == hipSuccess && ev0 && ev1 && hipEventElapsedTime(&kms, ev0, ev1) != hipSuccess) kms = -1.f;
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFreeAsync(base, s);
    if (e != hipSuccess) return ACCSK_HIP_ERROR;
    fill_result(*res, hr, (double)kms);
    return ACCSK_OK;
}

}  // namespace
}  // namespace accsk

using namespace accsk;

// Tiled solve of one problem (explicit C when X is null, else points with d <= 128:
// FP64 dot products up to d = 16, the matrix-core cross term of p->split pieces above).
// pub: null (results to *res, the call waits), or the device result record of
// the stream-ordered form (res unused, nothing waits).
accsk_status accsk_tiled_solve(const float *C, int64_t ldc, const float *X, const float *Y, int64_t d, int kind,
                               double cost_scale, int64_t n, int64_t m, const double *a, const double *b,
                               const accsk_params *p, double eps, double *f_out, double *g_out, accsk_result *res,
                               hipStream_t s, accsk_result *pub) {
    TiledArgs A{};
    A.C = C;
    A.ldc = ldc;
    A.X = X;
    A.Y = Y;
    A.d = X ? d : 0;
    A.kind = kind;
    A.inv_s = 1.0 / cost_scale;
    A.n = n;
    A.m = m;
    A.a_in = a;
    A.b_in = b;
    A.f_out = f_out;
    A.g_out = g_out;
    A.eps = eps;
    A.pub = pub;
    accsk_status st;
    const bool tr = p->err_trace && p->trace_len > 0;
    const bool cd = (p->flags & ACCSK_FLAG_CONDITIONS) && p->method == ACCSK_ACC;
    A.split = p->split == 2 ? 2 : 3;
    // diagnostic instantiations: the per-step trace; the boundedness monitor (with the trace code)
    auto launch = [&](auto dtag) {
        constexpr int DD = decltype(dtag)::value;
        if (cd) return tiled_launch<DD, true, true>(A, p, res, s);
        return tr ? tiled_launch<DD, true, false>(A, p, res, s) : tiled_launch<DD, false, false>(A, p, res, s);
    };
    if (!X) st = launch(std::integral_constant<int, 0>{});
    else if (d <= 3) st = launch(std::integral_constant<int, 3>{});
    else if (d <= 8) st = launch(std::integral_constant<int, 8>{});
    else if (d <= 16) st = launch(std::integral_constant<int, 16>{});
    else if (d <= 32) st = launch(std::integral_constant<int, 32>{});   // matrix-core cross term
    else if (d <= 64) st = launch(std::integral_constant<int, 64>{});
    else if (d <= 128) st = launch(std::integral_constant<int, 128>{});
    else st = ACCSK_SHAPE;
    if (st != ACCSK_OK || pub) return st;
    return (accsk_status)res->status;
}

// Upper bound of the workspace one tiled solve of an n x m problem allocates
// (at most two workgroups per CU).
size_t accsk_tiled_workspace_bound(int64_t n, int64_t m, int cu) {
    using namespace accsk;
    const size_t G = 2 * (size_t)cu;
    return align_up(sizeof(TiledArgs)) + align_up(sizeof(DevResult)) + align_up(64 * 8) + align_up(256) +
           align_up(5 * (size_t)n * 8) + align_up(7 * (size_t)m * 8) + align_up(G * (size_t)m * 4) +
           align_up(2 * G * (size_t)m * 8) + align_up((2 * G * kTNS + 2 * G) * 8) +
           align_up((3 * (size_t)m + 2 * G * 8) * 8) +
           align_up(((size_t)n + 15) / 16 * 4 * 3 * 64 * 16) + align_up(((size_t)m + 15) / 16 * 4 * 3 * 64 * 16);
}
