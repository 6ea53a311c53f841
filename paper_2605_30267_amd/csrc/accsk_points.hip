// Costs built from point clouds, point-cloud solves, and the backward pass.
//
// Costs (paper Sec. 5): squared Euclidean C_ij = ||x_i - y_j||^2 / s (colour
// transfer) and cosine C_ij = (1 - <x_i, y_j>) / s (word alignment).
//
// The cross term X Y^T is the only dense contraction of the method.  Two ways
// to form it:
//  * split = 0: FP64 dot products on the vector ALUs (exact up to the final
//    rounding of C to FP32);
//  * split = 2 or 3: BF16 matrix cores (v_mfma_f32_16x16x32_bf16) on a split
//    of each FP32 operand into 2 or 3 BF16 pieces, x = x_hi + x_mid (+ x_lo).
//    split 2 keeps hi*hi + hi*mid + mid*hi (pieces down to 2^-16 relative),
//    split 3 adds mid*mid, hi*lo, lo*hi (down to 2^-24).  Each product of
//    each 32-wide K chunk is accumulated separately in FP32 by the matrix core
//    and the partial sums are added in FP64, small terms first (cost_tiles.h).
// The cost error is amplified by 1/eps in the exponent, so the split depth is
// chosen by the caller and its error is measured by the tests.
//
// Backward (envelope theorem; the paper's primal map eq:P-from-dual gives
// dEOT/dC = P): with P_ij = exp((f_i + g_j - C_ij)/eps) recomputed tile by
// tile (never stored) as FP32 exponentials of FP64 arguments,
//   sq-Euclidean: dX_i = (2/s) (r_i x_i - sum_j P_ij y_j),
//                 dY_j = (2/s) (c_j y_j - sum_i P_ij x_i),
//   cosine:       dX_i = -(1/s) sum_j P_ij y_j,  dY_j = -(1/s) sum_i P_ij x_i,
//   da_i = (f_i - <f, a_hat>) / sum(a),  db_j = (g_j - <g, b_hat>) / sum(b),
// where r, c are the plan's row and column sums and a_hat = a / sum(a).

#include <limits.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "accsk_common.h"
#include "cost_tiles.h"

accsk_status accsk_tiled_solve(const float *C, int64_t ldc, const float *X, const float *Y, int64_t d, int kind,
                               double cost_scale, int64_t n, int64_t m, const double *a, const double *b,
                               const accsk_params *p, double eps, double *f_out, double *g_out, accsk_result *res,
                               hipStream_t s, accsk_result *pub);
accsk_status accsk_solve_batch_ws(const accsk_problem *probs, int64_t count, const accsk_params *p,
                                  accsk_result *res, void *stream, accsk::Workspace &ws, accsk_result *const *pub);

namespace accsk {
namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---------------------------------------------------------------------------
// Row norms ||x_i||^2 in FP64
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void row_norms(const float *__restrict__ X, long long rows, long long d,
                                                 double *__restrict__ out) {
    const long long i = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= rows) return;
    const double s = row_norm_wave(X + i * d, d, lane);
    if (lane == 0) out[i] = s;
}

// ---------------------------------------------------------------------------
// FP64 cost tile: block 16x16 outputs, X and Y rows staged in LDS.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(256) void cost_fp64(const float *__restrict__ X, const float *__restrict__ Y,
                                                 long long n, long long m, long long d, double inv_s,
                                                 float *__restrict__ C, long long ldc) {
    extern __shared__ float sm[];
    const long long ld = d + 1;  // padded row stride: rows start in different banks
    float *xs = sm;              // [16][d + 1]
    float *ys = sm + 16 * ld;    // [16][d + 1]
    const long long i0 = (long long)blockIdx.y * 16, j0 = (long long)blockIdx.x * 16;
    for (long long t = threadIdx.x; t < 16 * d; t += 256) {
        const long long r = t / d, k = t % d;
        xs[r * ld + k] = (i0 + r < n) ? X[(i0 + r) * d + k] : 0.f;
        ys[r * ld + k] = (j0 + r < m) ? Y[(j0 + r) * d + k] : 0.f;
    }
    __syncthreads();
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    const long long i = i0 + r, j = j0 + c;
    const double acc = cross_fp64<KIND>(xs + r * ld, ys + c * ld, d);
    if (i < n && j < m) C[i * ldc + j] = finish_fp64<KIND>(acc, inv_s);
}

// ---------------------------------------------------------------------------
// BF16-split matrix-core cost from pieces (split_pieces layout), for a batch of
// equal-shape problems (blockIdx.z).  Block tile 64 x 64: wave w owns the 16-row
// tile 4 blockIdx.y + w and the block's four 16-column tiles; for each 32-wide K
// chunk it loads its three A pieces once and applies them to the four column
// tiles.  The products and their FP64 sums are those of mfma_cross_tile (same
// pieces, same order), so the costs are the same as that per-lane form gives.
// ---------------------------------------------------------------------------
template <int SPLIT, int KIND>
__global__ __launch_bounds__(256) void cost_mfma(const bf16x8 *__restrict__ Xp, const bf16x8 *__restrict__ Yp,
                                                 const double *__restrict__ nx, const double *__restrict__ ny,
                                                 long long n, long long m, int KC, double inv_s,
                                                 float *__restrict__ C, long long ldc, long long xu, long long yu,
                                                 long long cstride) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long long b = blockIdx.z;
    Xp += b * xu;
    Yp += b * yu;
    nx += b * n;
    ny += b * m;
    C += b * cstride;
    const long long T = (long long)blockIdx.y * 4 + wid;  // row tile (pieces exist for every tile < ceil(n/16))
    const long long xt = (n + 15) / 16, yt = (m + 15) / 16;
    if (T >= xt) return;
    const long long U0 = (long long)blockIdx.x * 4;
    double g[4][4];
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
        for (int q = 0; q < 4; q++) g[c][q] = 0.0;
    const floatx4 z = {0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KC; kc++) {
        const bf16x8 *ap = Xp + ((T * KC + kc) * 3) * 64 + lane;
        const bf16x8 ah = ap[0], am = ap[64], al = ap[128];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const long long U = std::min(U0 + c, yt - 1);
            const bf16x8 *bp = Yp + ((U * KC + kc) * 3) * 64 + lane;
            const bf16x8 bh = bp[0], bm = bp[64], bl = bp[128];
            const floatx4 p_hl = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, SPLIT == 2 ? bm : bl, z, 0, 0, 0);
            const floatx4 p_lh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(SPLIT == 2 ? am : al, bh, z, 0, 0, 0);
            floatx4 p_mm = z, p_hm = z, p_mh = z;
            if (SPLIT == 3) {
                p_mm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, z, 0, 0, 0);
                p_hm = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, z, 0, 0, 0);
                p_mh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, z, 0, 0, 0);
            }
            const floatx4 p_hh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, z, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                double small = (double)p_hl[q] + (double)p_lh[q];
                if (SPLIT == 3) small += (double)p_mm[q] + ((double)p_hm[q] + (double)p_mh[q]);
                g[c][q] += small + (double)p_hh[q];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const long long j = (U0 + c) * 16 + (lane & 15);
        if (j >= m) continue;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const long long i = T * 16 + (lane >> 4) * 4 + q;
            if (i < n)
                C[i * ldc + j] = finish_mfma<KIND>(g[c][q], KIND == ACCSK_SQEUCLID ? nx[i] : 0.0,
                                                   KIND == ACCSK_SQEUCLID ? ny[j] : 0.0, inv_s);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward: one kernel per side.  A block owns 16 rows of one problem (rows
// side) and walks all columns in chunks of 64: P chunk (16 x 64) in LDS, then
// sum_j P_ij y_j for its 16 rows and d features, and the row sums r_i.
// The cost is recomputed in FP64 from the points.  The column side is the same
// with X and Y (and f and g) exchanged.
// ---------------------------------------------------------------------------
constexpr int kBR = 16, kBC = 64;

// 2^t for an FP64 argument: FP32 exponential of the fractional part, exact
// scaling by the integer part, so the FP32 rounding of a large |t| does not
// enter (relative error of a few FP32 ulps).
__device__ __forceinline__ float exp2_split(double t) {
    const double h = rint(fmax(t, -1000.0));
    return ldexpf(__builtin_amdgcn_exp2f((float)(t - h)), (int)h);
}

// MODE 0: gradient of the EOT value; MODE 1: barycentric projection
// T_i = sum_j P_ij y_j / sum_j P_ij (written to dX, gsc unused).
template <int KIND, int NQ, int MODE = 0>
__global__ __launch_bounds__(256) void grad_side(const float *__restrict__ X, const float *__restrict__ Y,
                                                 long long n, long long m, long long d, double inv_s,
                                                 double inv_eps, const double *__restrict__ f,
                                                 const double *__restrict__ g, const double *__restrict__ gsc,
                                                 float *__restrict__ dX, long long sX, long long sY,
                                                 long long sf, long long sg) {
    // batch index blockIdx.y; this block: rows [i0, i0+16) of X against all rows of Y
    extern __shared__ float sm[];
    const long long bidx = blockIdx.y;
    const double gscale = gsc ? gsc[bidx] : 1.0;
    X += bidx * sX;
    Y += bidx * sY;
    f += bidx * sf;
    g += bidx * sg;
    dX += bidx * sX;
    const long long ld = d + 1;           // padded row stride (bank spread)
    float *xs = sm;                       // [16][d + 1]
    float *ys = xs + kBR * ld;            // [64][d + 1]
    float *ps = ys + kBC * ld;            // [16][64]
    double *gk = reinterpret_cast<double *>(ps + kBR * kBC);  // [64] g_j log2(e) / eps
    const long long i0 = (long long)blockIdx.x * kBR;
    const int tid = threadIdx.x;
    const double k2 = inv_eps * kLog2e;   // log2 units: P_ij = 2^((f_i + g_j - C_ij) log2(e) / eps)
    for (long long t = tid; t < kBR * d; t += 256) {
        const long long r = t / d;
        xs[r * ld + (t % d)] = (i0 + r < n) ? X[(i0 + r) * d + (t % d)] : 0.f;
    }
    // each thread accumulates (row tr, features tk, tk+16, ...) of sum_j P_ij y_j
    const int tr = tid >> 4, tk = tid & 15;
    double acc[NQ];
    const int nk = (int)((d - tk + 15) / 16);  // features handled by this thread (<= NQ: d <= 16 NQ)
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;
    double rs = 0.0;
    for (long long j0 = 0; j0 < m; j0 += kBC) {
        __syncthreads();
        for (long long t = tid; t < kBC * d; t += 256) {
            const long long r = t / d;
            ys[r * ld + (t % d)] = (j0 + r < m) ? Y[(j0 + r) * d + (t % d)] : 0.f;
        }
        if (tid < kBC) gk[tid] = (j0 + tid < m) ? g[j0 + tid] * k2 : 0.0;
        __syncthreads();
        // P chunk: 16 x 64 = 1024 entries, 4 per thread (wave: one row, lanes: columns)
        for (int e = tid; e < kBR * kBC; e += 256) {
            const int r = e / kBC, c = e % kBC;
            const long long i = i0 + r, j = j0 + c;
            float pv = 0.f;
            if (i < n && j < m) {
                const double acc_c = cross_fp64<KIND>(xs + r * ld, ys + c * ld, d);
                const double cij = (KIND == ACCSK_SQEUCLID ? acc_c : 1.0 - acc_c) * inv_s;
                pv = exp2_split(fma(-cij, k2, f[i] * k2 + gk[c]));
            }
            ps[e] = pv;
        }
        __syncthreads();
        for (int c = 0; c < kBC; c++) {
            const double pv = ps[tr * kBC + c];
            if (tk == 0) rs += pv;
#pragma unroll
            for (int q = 0; q < NQ; q++)
                if (q < nk) acc[q] = fma(pv, (double)ys[c * ld + tk + 16 * q], acc[q]);
        }
    }
    const long long i = i0 + tr;
    // row sum r_i to every thread of the row
    __shared__ double rsh[kBR];
    if (tk == 0) rsh[tr] = rs;
    __syncthreads();
    if (i >= n) return;
    const double ri = rsh[tr];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        if (q >= nk) break;
        const long long k = tk + 16 * q;
        double v;
        if (MODE == 1) v = ri > 0.0 ? acc[q] / ri : NAN;
        else if (KIND == ACCSK_SQEUCLID) v = 2.0 * inv_s * (ri * (double)xs[tr * ld + k] - acc[q]);
        else v = -inv_s * acc[q];
        dX[i * d + k] = (float)(MODE == 1 ? v : gscale * v);
    }
}

// Backward of one side on the FP64 matrix cores (d <= 4 KK), gradient of the EOT
// value only.  A block owns 16 rows of X of one problem (blockIdx.y); its four
// waves take the 16-column tiles of Y in turn.  Per tile, v_mfma_f64_16x16x4f64
// forms C^T = Y X^T (A: Y rows, B: the block's X rows held in registers; lane
// group g supplies features g KK + kk at step kk), so that lane l holds
// P_ij for i = l % 16 and j = l / 16 + 4 q: exactly the A operand of the next
// product P Y at K step q (j = 4 q + l / 16).  P Y accumulates in FP64 registers
// per 16-feature tile; the waves' sums and row sums r_i are added in wave order
// through LDS.  Same quantities as grad_side (FP64 cost, FP32 exponential of the
// FP64 argument, FP64 sums), in a different order of FP64 additions.
template <int KIND, int KK>
__global__ __launch_bounds__(256) void grad_mfma(const float *__restrict__ X, const float *__restrict__ Y,
                                                 long long n, long long m, long long d, double inv_s,
                                                 double inv_eps, const double *__restrict__ f,
                                                 const double *__restrict__ g, const double *__restrict__ gsc,
                                                 float *__restrict__ dX, long long sX, long long sY,
                                                 long long sf, long long sg) {
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    constexpr int NFT = KK / 4;  // 16-feature tiles of the output (4 KK features)
    extern __shared__ double gm_red[];  // [4 waves][NFT][4][64] partial P Y, then [4][16] row sums
    const long long bidx = blockIdx.y;
    const double gscale = gsc ? gsc[bidx] : 1.0;
    X += bidx * sX;
    Y += bidx * sY;
    f += bidx * sf;
    g += bidx * sg;
    dX += bidx * sX;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int g4 = lane >> 4, r16 = lane & 15;
    const long long i0 = (long long)blockIdx.x * 16;
    const long long ib = i0 + r16;  // this lane's X row as a B operand and its P row
    const double k2 = inv_eps * kLog2e;
    double xb[KK];
    double xn = 0.0;
#pragma unroll
    for (int kk = 0; kk < KK; kk++) {
        const long long k = (long long)g4 * KK + kk;
        xb[kk] = (ib < n && k < d) ? (double)X[ib * d + k] : 0.0;
        xn = fma(xb[kk], xb[kk], xn);
    }
    xn += __shfl_xor(xn, 16, 64);
    xn += __shfl_xor(xn, 32, 64);  // |x_ib|^2
    const double fi2 = ib < n ? f[ib] * k2 : 0.0;
    f64x4 acc[NFT];
#pragma unroll
    for (int t = 0; t < NFT; t++) acc[t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    double rsum = 0.0;
    const long long ytiles = (m + 15) / 16;
    // this lane's Y values of a tile (FP32 as stored): its A-operand row and its P Y operands;
    // the next tile's are loaded while the current one is computed
    float yaf[KK], yvf[NFT][4];
    auto load_tile = [&](long long U, float (&ya_)[KK], float (&yv_)[NFT][4]) {
        const long long j0 = U * 16, ja = j0 + r16;
#pragma unroll
        for (int kk = 0; kk < KK; kk++) {
            const long long k = (long long)g4 * KK + kk;
            ya_[kk] = (ja < m && k < d) ? Y[ja * d + k] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < NFT; t++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const long long j = j0 + 4 * q + g4, ft = (long long)t * 16 + r16;
                yv_[t][q] = (j < m && ft < d) ? Y[j * d + ft] : 0.f;
            }
    };
    if (wid < ytiles) load_tile(wid, yaf, yvf);
    for (long long U = wid; U < ytiles; U += 4) {
        const long long j0 = U * 16;
        float nyaf[KK], nyvf[NFT][4];
        if (U + 4 < ytiles) load_tile(U + 4, nyaf, nyvf);
        double yn = 0.0;
#pragma unroll
        for (int kk = 0; kk < KK; kk++) yn = fma((double)yaf[kk], (double)yaf[kk], yn);
        yn += __shfl_xor(yn, 16, 64);
        yn += __shfl_xor(yn, 32, 64);  // |y_ja|^2 in every lane of row ja
        f64x4 cd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KK; kk++) cd = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yaf[kk], xb[kk], cd, 0, 0, 0);
        double pv[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int jr = g4 + 4 * q;  // row of the tile this value belongs to
            const long long j = j0 + jr;
            const double ynj = __shfl(yn, jr, 64);
            double cij = KIND == ACCSK_SQEUCLID ? xn + ynj - 2.0 * cd[q] : 1.0 - cd[q];
            cij *= inv_s;
            const double gj2 = g[std::min(j, m - 1)] * k2;
            pv[q] = (ib < n && j < m) ? (double)exp2_split(fma(-cij, k2, fi2 + gj2)) : 0.0;
            rsum += pv[q];
        }
#pragma unroll
        for (int t = 0; t < NFT; t++)
#pragma unroll
            for (int q = 0; q < 4; q++)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(pv[q], (double)yvf[t][q], acc[t], 0, 0, 0);
        if (U + 4 < ytiles) {
#pragma unroll
            for (int kk = 0; kk < KK; kk++) yaf[kk] = nyaf[kk];
#pragma unroll
            for (int t = 0; t < NFT; t++)
#pragma unroll
                for (int q = 0; q < 4; q++) yvf[t][q] = nyvf[t][q];
        }
    }
    // the waves' partial sums, added in wave order
    rsum += __shfl_xor(rsum, 16, 64);
    rsum += __shfl_xor(rsum, 32, 64);  // row ib over this wave's columns
    double *rr = gm_red + 4 * NFT * 4 * 64;  // [4][16]
#pragma unroll
    for (int t = 0; t < NFT; t++)
#pragma unroll
        for (int q = 0; q < 4; q++) gm_red[((wid * NFT + t) * 4 + q) * 64 + lane] = acc[t][q];
    if (lane < 16) rr[wid * 16 + lane] = rsum;
    __syncthreads();
    for (int t = wid; t < NFT; t += 4) {
        const long long ft = (long long)t * 16 + r16;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int ir = g4 + 4 * q;  // row of the output tile in this lane and register
            const long long i = i0 + ir;
            double v = 0.0, ri = 0.0;
            for (int w = 0; w < 4; w++) {
                v += gm_red[((w * NFT + t) * 4 + q) * 64 + lane];
                ri += rr[w * 16 + ir];
            }
            if (i < n && ft < d) {
                const double o = KIND == ACCSK_SQEUCLID ? 2.0 * inv_s * (ri * (double)X[i * d + ft] - v) : -inv_s * v;
                dX[i * d + ft] = (float)(gscale * o);
            }
        }
    }
}

__global__ __launch_bounds__(256) void grad_marginal(const double *__restrict__ pot, const double *__restrict__ w,
                                                     long long len, long long sp, long long sw,
                                                     const double *__restrict__ gsc, double *__restrict__ out) {
    const double gscale = gsc ? gsc[blockIdx.x] : 1.0;
    // out = gscale * (pot - <pot, w_hat>) / sum(w), one block per problem
    __shared__ double red[2][4];
    pot += blockIdx.x * sp;
    w += blockIdx.x * sw;
    out += blockIdx.x * sp;
    double s1 = 0.0, s2 = 0.0;
    for (long long i = threadIdx.x; i < len; i += 256) {
        s1 += pot[i] * w[i];
        s2 += w[i];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s1;
        red[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    const double pw = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double sw_ = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const double mean = pw / sw_;
    for (long long i = threadIdx.x; i < len; i += 256) out[i] = gscale * (pot[i] - mean) / sw_;
}

// dEOT/dC = gscale P for an explicit cost (envelope theorem, eq:P-from-dual):
// P_ij = exp((f_i + g_j - C_ij)/eps), FP64 argument and exponential, FP32
// output.  Block (x, y): columns 1024 x + [0, 1024), rows y, y + gridDim.y, ...;
// thread t takes columns t, t + 256, t + 512, t + 768 of its block (coalesced).
__global__ __launch_bounds__(256) void grad_cost_rows(const float *__restrict__ C, long long n, long long m,
                                                      long long ldc, double inv_eps, const double *__restrict__ f,
                                                      const double *__restrict__ g,
                                                      const double *__restrict__ gsc, float *__restrict__ dC,
                                                      long long ldd) {
    const double gs = gsc ? gsc[0] : 1.0;
    const long long j0 = (long long)blockIdx.x * 1024 + threadIdx.x;
    double gj[4];
#pragma unroll
    for (int k = 0; k < 4; k++) gj[k] = j0 + 256 * k < m ? g[j0 + 256 * k] : 0.0;
    for (long long i = blockIdx.y; i < n; i += gridDim.y) {
        const double fi = f[i];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const long long j = j0 + 256 * k;
            if (j < m) dC[i * ldd + j] = (float)(gs * exp((fi + gj[k] - (double)C[i * ldc + j]) * inv_eps));
        }
    }
}

// Plan rows from points (eq:P-from-dual): 16 x 16 tiles of
// P_ij = exp((f_i + g_j - C_ij) / eps), C_ij in FP64 as in cost_fp64, FP64
// exponential, FP32 output.  Tile row r covers plan row row0 + r.
template <int KIND>
__global__ __launch_bounds__(256) void plan_points_k(const float *__restrict__ X, const float *__restrict__ Y,
                                                     long long m, long long d, double inv_s, double inv_eps,
                                                     const double *__restrict__ f, const double *__restrict__ g,
                                                     long long row0, long long rows, float *__restrict__ P,
                                                     long long ldp) {
    extern __shared__ float sm[];
    const long long ld = d + 1;
    float *xs = sm, *ys = sm + 16 * ld;
    const long long r0 = (long long)blockIdx.y * 16, j0 = (long long)blockIdx.x * 16;
    for (long long t = threadIdx.x; t < 16 * d; t += 256) {
        const long long r = t / d, k = t % d;
        xs[r * ld + k] = (r0 + r < rows) ? X[(row0 + r0 + r) * d + k] : 0.f;
        ys[r * ld + k] = (j0 + r < m) ? Y[(j0 + r) * d + k] : 0.f;
    }
    __syncthreads();
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    const long long rr = r0 + r, j = j0 + c;
    if (rr >= rows || j >= m) return;
    const double acc = cross_fp64<KIND>(xs + r * ld, ys + c * ld, d);
    const double cij = (KIND == ACCSK_SQEUCLID ? acc : 1.0 - acc) * inv_s;
    P[rr * ldp + j] = (float)exp((f[row0 + rr] + g[j] - cij) * inv_eps);
}

// max over a 16-row x 256-column tile of the raw cost, FP64 entries as in cost_fp64
template <int KIND>
__global__ __launch_bounds__(256) void cost_max_part(const float *__restrict__ X, const float *__restrict__ Y,
                                                     long long n, long long m, long long d,
                                                     double *__restrict__ part) {
    extern __shared__ float xs[];  // [16][d]
    __shared__ double red[4];
    const long long i0 = (long long)blockIdx.y * 16;
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    for (long long t = threadIdx.x; t < 16 * d; t += 256) {
        const long long r = t / d;
        xs[t] = (i0 + r < n) ? X[(i0 + r) * d + (t % d)] : 0.f;
    }
    __syncthreads();
    double mx = -INFINITY;
    if (j < m) {
        const float *yr = Y + j * d;
        for (int r = 0; r < 16 && i0 + r < n; r++) {
            const double acc = cross_fp64<KIND>(xs + r * d, yr, d);
            mx = fmax(mx, KIND == ACCSK_SQEUCLID ? acc : 1.0 - acc);
        }
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0)
        part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(1024) void max_reduce(const double *__restrict__ part, long long cnt,
                                                   double *__restrict__ out) {
    __shared__ double red[16];
    double mx = -INFINITY;
    for (long long k = threadIdx.x; k < cnt; k += 1024) mx = fmax(mx, part[k]);
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = -INFINITY;
        for (int q = 0; q < 16; q++) v = fmax(v, red[q]);
        *out = v;
    }
}

// Row top-k of the plan: for row i the K columns with the largest
// P_ij = exp((f_i + g_j - C_ij)/eps), i.e. the largest g_j - C_ij, compared in
// FP64 (ties: lower column index first).  One wave per row; each lane keeps
// its K best in registers, then K rounds of a wave-wide maximum pick the
// result in order.
template <int KIND, int K>
__global__ __launch_bounds__(256) void topk_rows(const float *__restrict__ X, const float *__restrict__ Y, long long n,
                                                 long long m, long long d, double inv_s, double inv_eps,
                                                 const double *__restrict__ f, const double *__restrict__ g,
                                                 long long *__restrict__ idx_out, double *__restrict__ val_out) {
    extern __shared__ float xr_all[];  // [4][d]: the row of each wave
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long long i = (long long)blockIdx.x * 4 + wid;
    float *xr = xr_all + (size_t)wid * d;
    for (long long k = lane; k < d; k += 64) xr[k] = i < n ? X[i * d + k] : 0.f;
    __syncthreads();
    if (i >= n) return;
    double bv[K];
    long long bi[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        bv[q] = -INFINITY;
        bi[q] = -1;
    }
    for (long long j = lane; j < m; j += 64) {
        const double acc = cross_fp64<KIND>(xr, Y + j * d, d);
        const double v = g[j] - (KIND == ACCSK_SQEUCLID ? acc : 1.0 - acc) * inv_s;
        // insert (v, j) into the lane's sorted list (columns arrive in increasing j)
        if (v > bv[K - 1]) {
            double cv = v;
            long long ci = j;
#pragma unroll
            for (int q = 0; q < K; q++) {
                if (cv > bv[q]) {
                    const double tv = bv[q];
                    const long long ti = bi[q];
                    bv[q] = cv;
                    bi[q] = ci;
                    cv = tv;
                    ci = ti;
                }
            }
        }
    }
    int head = 0;  // next candidate of this lane
    for (int r = 0; r < K; r++) {
        double hv = -INFINITY;
        long long hi = LLONG_MAX;
#pragma unroll
        for (int q = 0; q < K; q++)
            if (q == head) {
                hv = bv[q];
                hi = bi[q] < 0 ? LLONG_MAX : bi[q];
            }
        // wave maximum of (value, -index)
        double mv = hv;
        long long mi = hi;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ov = __shfl_xor(mv, o, 64);
            const long long oi = __shfl_xor(mi, o, 64);
            if (ov > mv || (ov == mv && oi < mi)) {
                mv = ov;
                mi = oi;
            }
        }
        if (hv == mv && hi == mi) head++;
        if (lane == 0) {
            const bool ok = mi != LLONG_MAX;
            idx_out[i * K + r] = ok ? mi : -1;
            if (val_out) val_out[i * K + r] = ok ? exp((f[i] + mv) * inv_eps) : 0.0;
        }
    }
}

// Costs of `batch` equal-shape problems (X: batch x n x d, Y: batch x m x d, C:
// problem k at C + k cstride, leading dimension ldc).  split 0: FP64 dot
// products; split 2/3: BF16 pieces, one launch for the whole batch (pieces and
// norms in stream-ordered workspace).
accsk_status build_cost_batch(const float *X, const float *Y, long long batch, long long n, long long m,
                              long long d, int kind, double scale, int split, float *C, long long ldc,
                              long long cstride, hipStream_t s) {
    const double inv_s = 1.0 / scale;
    if (split == 0) {
        const size_t lds = 2 * 16 * (size_t)(d + 1) * sizeof(float);
        dim3 grid((unsigned)((m + 15) / 16), (unsigned)((n + 15) / 16));
        for (long long k = 0; k < batch; k++) {
            const float *Xk = X + k * n * d, *Yk = Y + k * m * d;
            float *Ck = C + k * cstride;
            if (kind == ACCSK_SQEUCLID)
                hipLaunchKernelGGL(cost_fp64<ACCSK_SQEUCLID>, grid, dim3(256), lds, s, Xk, Yk, n, m, d, inv_s, Ck, ldc);
            else
                hipLaunchKernelGGL(cost_fp64<ACCSK_COSINE>, grid, dim3(256), lds, s, Xk, Yk, n, m, d, inv_s, Ck, ldc);
        }
        return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
    }
    const int KC = (int)((d + 31) / 32);
    const long long xu = (n + 15) / 16 * KC * 3 * 64, yu = (m + 15) / 16 * KC * 3 * 64;  // piece units per problem
    const size_t pbytes = (size_t)batch * (xu + yu) * sizeof(bf16x8);
    const size_t nbytes = (size_t)batch * (n + m) * sizeof(double);
    char *ws = nullptr;
    if (hipMallocAsync((void **)&ws, pbytes + nbytes, s) != hipSuccess) return ACCSK_OOM;
    bf16x8 *Xp = (bf16x8 *)ws, *Yp = Xp + batch * xu;
    double *nx = (double *)(ws + pbytes), *ny = nx + batch * n;
    const long long ux = (n + 15) / 16 * KC * 64, uy = (m + 15) / 16 * KC * 64;
    hipLaunchKernelGGL(split_pieces, dim3((unsigned)((ux + 255) / 256), (unsigned)batch), dim3(256), 0, s, X, n, d, KC,
                       Xp, xu);
    hipLaunchKernelGGL(split_pieces, dim3((unsigned)((uy + 255) / 256), (unsigned)batch), dim3(256), 0, s, Y, m, d, KC,
                       Yp, yu);
    if (kind == ACCSK_SQEUCLID) {  // rows of consecutive problems are consecutive rows
        hipLaunchKernelGGL(row_norms, dim3((unsigned)((batch * n + 3) / 4)), dim3(256), 0, s, X, batch * n, d, nx);
        hipLaunchKernelGGL(row_norms, dim3((unsigned)((batch * m + 3) / 4)), dim3(256), 0, s, Y, batch * m, d, ny);
    }
    dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64), (unsigned)batch);
    if (kind == ACCSK_SQEUCLID) {
        if (split == 2)
            hipLaunchKernelGGL((cost_mfma<2, ACCSK_SQEUCLID>), grid, dim3(256), 0, s, Xp, Yp, nx, ny, n, m, KC, inv_s, C,
                               ldc, xu, yu, cstride);
        else
            hipLaunchKernelGGL((cost_mfma<3, ACCSK_SQEUCLID>), grid, dim3(256), 0, s, Xp, Yp, nx, ny, n, m, KC, inv_s, C,
                               ldc, xu, yu, cstride);
    } else {
        if (split == 2)
            hipLaunchKernelGGL((cost_mfma<2, ACCSK_COSINE>), grid, dim3(256), 0, s, Xp, Yp, nx, ny, n, m, KC, inv_s, C,
                               ldc, xu, yu, cstride);
        else
            hipLaunchKernelGGL((cost_mfma<3, ACCSK_COSINE>), grid, dim3(256), 0, s, Xp, Yp, nx, ny, n, m, KC, inv_s, C,
                               ldc, xu, yu, cstride);
    }
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ws, s);
    return e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

accsk_status build_cost(const float *X, const float *Y, long long n, long long m, long long d, int kind,
                        double scale, int split, float *C, long long ldc, hipStream_t s) {
    return build_cost_batch(X, Y, 1, n, m, d, kind, scale, split, C, ldc, 0, s);
}

accsk_status check_points(const float *X, const float *Y, long long n, long long m, long long d, int kind,
                          double scale, int split) {
    if (!X || !Y) return ACCSK_INVALID_ARG;
    if (kind != ACCSK_SQEUCLID && kind != ACCSK_COSINE) return ACCSK_INVALID_ARG;
    if (!finite_pos(scale)) return ACCSK_INVALID_ARG;
    if (split != 0 && split != 2 && split != 3) return ACCSK_INVALID_ARG;
    if (n < 1 || m < 1 || d < 1 || d > 512) return ACCSK_SHAPE;
    return ACCSK_OK;
}

}  // namespace
}  // namespace accsk

using namespace accsk;

extern "C" accsk_status accsk_cost_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                          double cost_scale, int split, float *C, int64_t ldc, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, split);
    if (st != ACCSK_OK) return st;
    if (!C || ldc < m) return C ? ACCSK_SHAPE : ACCSK_INVALID_ARG;
    return build_cost(X, Y, n, m, d, kind, cost_scale, split, C, ldc, (hipStream_t)stream);
}

extern "C" accsk_status accsk_cost_points_batched(const float *X, const float *Y, int64_t batch, int64_t n,
                                                  int64_t m, int64_t d, int kind, double cost_scale, int split,
                                                  float *C, int64_t ldc, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, split);
    if (st != ACCSK_OK) return st;
    if (!C || batch < 1) return ACCSK_INVALID_ARG;
    if (ldc < m || batch > 65535) return ACCSK_SHAPE;
    return build_cost_batch(X, Y, batch, n, m, d, kind, cost_scale, split, C, ldc, n * ldc, (hipStream_t)stream);
}

extern "C" accsk_status accsk_plan_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                          double cost_scale, double eps, const double *f, const double *g,
                                          int64_t row0, int64_t rows, float *P, int64_t ldp, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, 0);
    if (st != ACCSK_OK) return st;
    if (!f || !g || !P || !finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (ldp < m || row0 < 0 || rows < 0 || row0 + rows > n) return ACCSK_SHAPE;
    if (rows == 0) return ACCSK_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = 2 * 16 * (size_t)(d + 1) * sizeof(float);
    for (int64_t r = 0; r < rows; r += 16 * 65535) {  // grid.y limit
        const int64_t rc = std::min<int64_t>(16 * 65535, rows - r);
        dim3 grid((unsigned)((m + 15) / 16), (unsigned)((rc + 15) / 16));
        if (kind == ACCSK_SQEUCLID)
            hipLaunchKernelGGL(plan_points_k<ACCSK_SQEUCLID>, grid, dim3(256), lds, s, X, Y, m, d, 1.0 / cost_scale,
                               1.0 / eps, f, g, row0 + r, rc, P + r * ldp, ldp);
        else
            hipLaunchKernelGGL(plan_points_k<ACCSK_COSINE>, grid, dim3(256), lds, s, X, Y, m, d, 1.0 / cost_scale,
                               1.0 / eps, f, g, row0 + r, rc, P + r * ldp, ldp);
    }
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

extern "C" accsk_status accsk_barycentric_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d,
                                                 int kind, double cost_scale, double eps, const double *f,
                                                 const double *g, float *T, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, 0);
    if (st != ACCSK_OK) return st;
    if (!f || !g || !T || !finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (d > 448) return ACCSK_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = ((size_t)(kBR + kBC) * (d + 1) + kBR * kBC) * sizeof(float) + kBC * sizeof(double);
    dim3 grid((unsigned)((n + kBR - 1) / kBR), 1u);
    auto run = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, X, Y, n, m, d, 1.0 / cost_scale, 1.0 / eps, f, g,
                           (const double *)nullptr, T, n * d, m * d, n, m);
    };
    if (kind == ACCSK_SQEUCLID) {
        if (d <= 64) run(grad_side<ACCSK_SQEUCLID, 4, 1>);
        else if (d <= 128) run(grad_side<ACCSK_SQEUCLID, 8, 1>);
        else if (d <= 256) run(grad_side<ACCSK_SQEUCLID, 16, 1>);
        else run(grad_side<ACCSK_SQEUCLID, 28, 1>);
    } else {
        if (d <= 64) run(grad_side<ACCSK_COSINE, 4, 1>);
        else if (d <= 128) run(grad_side<ACCSK_COSINE, 8, 1>);
        else if (d <= 256) run(grad_side<ACCSK_COSINE, 16, 1>);
        else run(grad_side<ACCSK_COSINE, 28, 1>);
    }
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

extern "C" accsk_status accsk_topk_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                          double cost_scale, double eps, const double *f, const double *g, int k,
                                          int64_t *idx, double *val, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, 0);
    if (st != ACCSK_OK) return st;
    if (!f || !g || !idx || !finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (k < 1 || k > 8) return ACCSK_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    const size_t lds = 4 * (size_t)d * sizeof(float);
    const dim3 grid((unsigned)((n + 3) / 4));
    const double inv_s = 1.0 / cost_scale, inv_eps = 1.0 / eps;
    auto run = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, X, Y, n, m, d, inv_s, inv_eps, f, g, (long long *)idx, val);
    };
    const bool sq = kind == ACCSK_SQEUCLID;
    if (k == 1) sq ? run(topk_rows<ACCSK_SQEUCLID, 1>) : run(topk_rows<ACCSK_COSINE, 1>);
    else if (k <= 5) {
        if (k == 5) sq ? run(topk_rows<ACCSK_SQEUCLID, 5>) : run(topk_rows<ACCSK_COSINE, 5>);
        else return ACCSK_SHAPE;
    } else if (k == 8) sq ? run(topk_rows<ACCSK_SQEUCLID, 8>) : run(topk_rows<ACCSK_COSINE, 8>);
    else return ACCSK_SHAPE;
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

extern "C" accsk_status accsk_cost_max_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d,
                                              int kind, double *out, void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, 1.0, 0);
    if (st != ACCSK_OK) return st;
    if (!out) return ACCSK_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const long long gx = (m + 255) / 256, gy = (n + 15) / 16;
    if (gy > 65535) return ACCSK_SHAPE;
    double *buf = nullptr;
    if (hipMallocAsync((void **)&buf, (size_t)(gx * gy + 1) * 8, s) != hipSuccess) return ACCSK_OOM;
    const size_t lds = 16 * (size_t)d * sizeof(float);
    if (kind == ACCSK_SQEUCLID)
        hipLaunchKernelGGL(cost_max_part<ACCSK_SQEUCLID>, dim3((unsigned)gx, (unsigned)gy), dim3(256), lds, s, X, Y, n,
                           m, d, buf + 1);
    else
        hipLaunchKernelGGL(cost_max_part<ACCSK_COSINE>, dim3((unsigned)gx, (unsigned)gy), dim3(256), lds, s, X, Y, n,
                           m, d, buf + 1);
    hipLaunchKernelGGL(max_reduce, dim3(1), dim3(1024), 0, s, buf + 1, gx * gy, buf);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, buf, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(buf, s);
    return e == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

// Tiled solves of a batch of point-cloud problems, one after the other: costs on
// the fly (FP64 dot products for d <= 16, the matrix-core cross term for
// 16 < d <= 128 with split 2 or 3), else built explicitly one problem at a time.
// dres (device records, one per problem): the stream-ordered form, res unused.
static accsk_status solve_points_tiled(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                       int64_t d, int kind, double cost_scale, const double *a, const double *b,
                                       const accsk_params *p, double *f_out, double *g_out, accsk_result *res,
                                       accsk_result *dres, hipStream_t s) {
    float *C = nullptr;
    const long long ldc = (m + 3) / 4 * 4;
    const bool fly = d <= 16 || (d <= 128 && p->split != 0);
    if (!fly) {
        if (hipMallocAsync((void **)&C, (size_t)n * ldc * sizeof(float), s) != hipSuccess) return ACCSK_OOM;
    }
    accsk_status worst = ACCSK_OK;
    for (int64_t k = 0; k < batch; k++) {
        const float *Xk = X + k * n * d, *Yk = Y + k * m * d;
        accsk_status st;
        accsk_result *rk = res ? &res[k] : nullptr, *pk = dres ? dres + k : nullptr;
        if (fly) {
            st = accsk_tiled_solve(nullptr, 0, Xk, Yk, d, kind, cost_scale, n, m, a + k * n, b + k * m, p, p->eps,
                                   f_out + k * n, g_out + k * m, rk, s, pk);
        } else {
            st = build_cost(Xk, Yk, n, m, d, kind, cost_scale, p->split, C, ldc, s);
            if (st == ACCSK_OK)
                st = accsk_tiled_solve(C, ldc, nullptr, nullptr, 0, kind, 1.0, n, m, a + k * n, b + k * m, p, p->eps,
                                       f_out + k * n, g_out + k * m, rk, s, pk);
        }
        if (dres) {
            if (st != ACCSK_OK) {  // a call failure: later problems are not enqueued
                if (C) (void)hipFreeAsync(C, s);
                return st;
            }
            continue;
        }
        if (st != ACCSK_OK && st != ACCSK_NOT_CONVERGED && res[k].status == ACCSK_OK) res[k].status = st;
        if (st == ACCSK_OK) continue;
        if (worst == ACCSK_OK || (worst == ACCSK_NOT_CONVERGED && st != ACCSK_NOT_CONVERGED)) worst = st;
    }
    if (C) (void)hipFreeAsync(C, s);
    if (dres) return ACCSK_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return ACCSK_HIP_ERROR;
    return worst;
}

// Batch of point-cloud problems: host records (res, the call waits) or device
// records (dres, stream-ordered).
static accsk_status solve_points_batched(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                         int64_t d, int kind, double cost_scale, const double *a, const double *b,
                                         const accsk_params *p, double *f_out, double *g_out, accsk_result *res,
                                         accsk_result *dres, void *stream) {
    if (!p || !a || !b || !f_out || !g_out || !(res || dres) || batch < 1) return ACCSK_INVALID_ARG;
    if (p->err_trace && batch > 1) return ACCSK_INVALID_ARG;  // one trace buffer: one problem
    if (p->trace_len < 0 || (p->trace_len > 0 && !p->err_trace)) return ACCSK_INVALID_ARG;
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, p->split);
    if (st != ACCSK_OK) return st;
    if (!finite_pos(p->eps)) return ACCSK_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if ((p->flags & ACCSK_FLAG_ON_THE_FLY) || m > 8192) {
        if ((p->flags & ACCSK_FLAG_ON_THE_FLY) && d > 16 && (p->split == 0 || d > 128)) return ACCSK_SHAPE;
        return solve_points_tiled(X, Y, batch, n, m, d, kind, cost_scale, a, b, p, f_out, g_out, res, dres, s);
    }
    const long long ldc = (m + 3) / 4 * 4;
    const size_t cbytes = (size_t)batch * n * ldc * sizeof(float);
    char *ws = nullptr;
    if (hipMallocAsync((void **)&ws, cbytes, s) != hipSuccess) return ACCSK_OOM;
    float *C = (float *)ws;
    st = build_cost_batch(X, Y, batch, n, m, d, kind, cost_scale, p->split, C, ldc, n * ldc, s);
    if (st == ACCSK_OK) {
        std::vector<accsk_problem> probs((size_t)batch);
        for (int64_t k = 0; k < batch; k++)
            probs[(size_t)k] = accsk_problem{C + k * n * ldc, n, m, ldc, a + k * n, b + k * m,
                                             f_out + k * n, g_out + k * m, p->eps};
        Workspace bws;  // stream-ordered allocations
        if (dres) {
            std::vector<accsk_result *> pub((size_t)batch);
            for (int64_t k = 0; k < batch; k++) pub[(size_t)k] = dres + k;
            st = accsk_solve_batch_ws(probs.data(), batch, p, nullptr, stream, bws, pub.data());
        } else {
            st = accsk_solve_batch_ws(probs.data(), batch, p, res, stream, bws, nullptr);
        }
    }
    (void)hipFreeAsync(ws, s);
    if (dres) return st;
    if (hipStreamSynchronize(s) != hipSuccess) return ACCSK_HIP_ERROR;
    return st;
}

extern "C" accsk_status accsk_solve_points_batched(const float *X, const float *Y, int64_t batch, int64_t n,
                                                   int64_t m, int64_t d, int kind, double cost_scale,
                                                   const double *a, const double *b, const accsk_params *p,
                                                   double *f_out, double *g_out, accsk_result *res,
                                                   void *stream) {
    if (!res) return ACCSK_INVALID_ARG;
    return solve_points_batched(X, Y, batch, n, m, d, kind, cost_scale, a, b, p, f_out, g_out, res, nullptr,
                                stream);
}

extern "C" accsk_status accsk_solve_points_batched_async(const float *X, const float *Y, int64_t batch, int64_t n,
                                                         int64_t m, int64_t d, int kind, double cost_scale,
                                                         const double *a, const double *b, const accsk_params *p,
                                                         double *f_out, double *g_out, accsk_result *res,
                                                         void *stream) {
    if (!res) return ACCSK_INVALID_ARG;
    return solve_points_batched(X, Y, batch, n, m, d, kind, cost_scale, a, b, p, f_out, g_out, nullptr, res,
                                stream);
}

extern "C" accsk_status accsk_solve_points(const float *X, const float *Y, int64_t n, int64_t m, int64_t d, int kind,
                                           double cost_scale, const double *a, const double *b,
                                           const accsk_params *p, double *f_out, double *g_out, accsk_result *res,
                                           void *stream) {
    return accsk_solve_points_batched(X, Y, 1, n, m, d, kind, cost_scale, a, b, p, f_out, g_out, res, stream);
}

extern "C" accsk_status accsk_backward_points(const float *X, const float *Y, int64_t batch, int64_t n, int64_t m,
                                              int64_t d, int kind, double cost_scale, double eps, const double *a,
                                              const double *b, const double *f, const double *g,
                                              const double *grad_scale, float *dX, float *dY, double *da, double *db,
                                              void *stream) {
    accsk_status st = check_points(X, Y, n, m, d, kind, cost_scale, 0);
    if (st != ACCSK_OK) return st;
    if (!f || !g || !dX || !dY || batch < 1 || !finite_pos(eps))
        return ACCSK_INVALID_ARG;
    if (d > 448) return ACCSK_SHAPE;  // X, Y and P tiles staged in on-chip memory
    hipStream_t s = (hipStream_t)stream;
    const double inv_s = 1.0 / cost_scale, inv_eps = 1.0 / eps;
    const size_t lds = ((size_t)(kBR + kBC) * (d + 1) + kBR * kBC) * sizeof(float) + kBC * sizeof(double);
    dim3 gx((unsigned)((n + kBR - 1) / kBR), (unsigned)batch), gy((unsigned)((m + kBR - 1) / kBR), (unsigned)batch);
    auto sides = [&](auto kern) {
        hipLaunchKernelGGL(kern, gx, dim3(256), lds, s, X, Y, n, m, d, inv_s, inv_eps, f, g, grad_scale, dX, n * d,
                           m * d, n, m);
        hipLaunchKernelGGL(kern, gy, dim3(256), lds, s, Y, X, m, n, d, inv_s, inv_eps, g, f, grad_scale, dY, m * d,
                           n * d, m, n);
    };
    // d <= 128: the FP64 matrix-core form (one block per 16 rows of a problem)
    if (d <= 128) {
        auto msides = [&](auto kern, size_t glds) {
            hipLaunchKernelGGL(kern, dim3((unsigned)((n + 15) / 16), (unsigned)batch), dim3(256), glds, s, X, Y, n, m,
                               d, inv_s, inv_eps, f, g, grad_scale, dX, n * d, m * d, n, m);
            hipLaunchKernelGGL(kern, dim3((unsigned)((m + 15) / 16), (unsigned)batch), dim3(256), glds, s, Y, X, m, n,
                               d, inv_s, inv_eps, g, f, grad_scale, dY, m * d, n * d, m, n);
        };
        const size_t l16 = (4 * 4 * 4 * 64 + 64) * sizeof(double), l32 = (4 * 8 * 4 * 64 + 64) * sizeof(double);
        if (kind == ACCSK_SQEUCLID) {
            if (d <= 64) msides(grad_mfma<ACCSK_SQEUCLID, 16>, l16);
            else msides(grad_mfma<ACCSK_SQEUCLID, 32>, l32);
        } else {
            if (d <= 64) msides(grad_mfma<ACCSK_COSINE, 16>, l16);
            else msides(grad_mfma<ACCSK_COSINE, 32>, l32);
        }
    } else if (kind == ACCSK_SQEUCLID) {
        if (d <= 64) sides(grad_side<ACCSK_SQEUCLID, 4>);
        else if (d <= 128) sides(grad_side<ACCSK_SQEUCLID, 8>);
        else if (d <= 256) sides(grad_side<ACCSK_SQEUCLID, 16>);
        else sides(grad_side<ACCSK_SQEUCLID, 28>);
    } else {
        if (d <= 64) sides(grad_side<ACCSK_COSINE, 4>);
        else if (d <= 128) sides(grad_side<ACCSK_COSINE, 8>);
        else if (d <= 256) sides(grad_side<ACCSK_COSINE, 16>);
        else sides(grad_side<ACCSK_COSINE, 28>);
    }
    if (da && a) hipLaunchKernelGGL(grad_marginal, dim3((unsigned)batch), dim3(256), 0, s, f, a, n, n, n, grad_scale, da);
    if (db && b) hipLaunchKernelGGL(grad_marginal, dim3((unsigned)batch), dim3(256), 0, s, g, b, m, m, m, grad_scale, db);
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}

extern "C" accsk_status accsk_backward_dense(const float *C, int64_t n, int64_t m, int64_t ldc, double eps,
                                             const double *a, const double *b, const double *f, const double *g,
                                             const double *grad_scale, float *dC, int64_t lddc, double *da,
                                             double *db, void *stream) {
    if (!f || !g || (dC && !C) || (da && !a) || (db && !b) || !finite_pos(eps)) return ACCSK_INVALID_ARG;
    if (n < 1 || m < 1 || (dC && (ldc < m || lddc < m))) return ACCSK_SHAPE;
    hipStream_t s = (hipStream_t)stream;
    if (dC) {
        const dim3 grid((unsigned)((m + 1023) / 1024), (unsigned)std::min<int64_t>(n, 4096));
        hipLaunchKernelGGL(grad_cost_rows, grid, dim3(256), 0, s, C, (long long)n, (long long)m, (long long)ldc,
                           1.0 / eps, f, g, grad_scale, dC, (long long)lddc);
    }
    if (da) hipLaunchKernelGGL(grad_marginal, dim3(1), dim3(256), 0, s, f, a, n, n, n, grad_scale, da);
    if (db) hipLaunchKernelGGL(grad_marginal, dim3(1), dim3(256), 0, s, g, b, m, m, m, grad_scale, db);
    return hipGetLastError() == hipSuccess ? ACCSK_OK : ACCSK_HIP_ERROR;
}
