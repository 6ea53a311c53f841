// Cost entries from point clouds (paper Sec. 5: squared Euclidean and cosine
// costs), shared by the cost kernels and the serving loop so that both produce
// the same bits for the same points.
//
//  * FP64 path: the d-term sum accumulated in FP64 in the order k = 0..d-1,
//    one rounding to FP32 at the end.
//  * Matrix-core path: the cross term x . y on v_mfma_f32_16x16x32_bf16 over a
//    2- or 3-piece BF16 split of each FP32 operand.  One wave computes a 16x16
//    tile: lane l supplies A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16] and
//    receives D[4(l/16)+i][l%16], i = 0..3.  Each product of each 32-wide K
//    chunk is accumulated separately by the matrix core in FP32; the partial
//    sums are added in FP64, small terms first.  The squared Euclidean cost is
//    then |x|^2 + |y|^2 - 2 x.y with FP64 norms (clamped at 0).
#pragma once

#include "accsk_common.h"

namespace accsk {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// acc + sum_k (x_k - y_k)^2 (KIND = SQEUCLID) or acc + sum_k x_k y_k (COSINE),
// FP64, k in order; a sum split into consecutive chunks gives the same bits.
template <int KIND>
__device__ __forceinline__ double cross_fp64_acc(const float *xr, const float *yr, long long d, double acc) {
    for (long long k = 0; k < d; k++) {
        const double xv = xr[k], yv = yr[k];
        if (KIND == ACCSK_SQEUCLID) {
            const double t = xv - yv;
            acc = fma(t, t, acc);
        } else {
            acc = fma(xv, yv, acc);
        }
    }
    return acc;
}

template <int KIND>
__device__ __forceinline__ double cross_fp64(const float *xr, const float *yr, long long d) {
    return cross_fp64_acc<KIND>(xr, yr, d, 0.0);
}

template <int KIND>
__device__ __forceinline__ float finish_fp64(double acc, double inv_s) {
    return (float)((KIND == ACCSK_SQEUCLID ? acc : 1.0 - acc) * inv_s);
}

// |x|^2 of one row by one wave (lane-strided FP64 partial sums, xor butterfly);
// every lane gets the result.
__device__ __forceinline__ double row_norm_wave(const float *xr, long long d, int lane) {
    double s = 0.0;
    for (long long k = lane; k < d; k += 64) {
        const double v = xr[k];
        s = fma(v, v, s);
    }
    return wave_sum(s);
}

__device__ __forceinline__ void bf16_split3(float v, __bf16 &h, __bf16 &mi, __bf16 &lo) {
    h = (__bf16)v;
    const float r1 = v - (float)h;
    mi = (__bf16)r1;
    lo = (__bf16)(r1 - (float)mi);
}

// Cross term of the 16x16 tile whose lane-l operands are rows xrow (A side)
// and yrow (B side); g[q] receives x_i . y_j for i = 4(l/16)+q, j = l%16 of
// the tile.  SPLIT 2 keeps hi*hi + hi*mid + mid*hi (mid acting as the low
// piece), SPLIT 3 adds mid*mid, hi*lo and lo*hi.
template <int SPLIT>
__device__ __forceinline__ void mfma_cross_tile(const float *xrow, const float *yrow, long long d, int lane,
                                                double (&g)[4]) {
    const int kq = (lane >> 4) * 8;
#pragma unroll
    for (int q = 0; q < 4; q++) g[q] = 0.0;
    for (long long k0 = 0; k0 < d; k0 += 32) {
        bf16x8 ah, am, al, bh, bm, bl;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const long long k = k0 + kq + e;
            const float xv = k < d ? xrow[k] : 0.f;
            const float yv = k < d ? yrow[k] : 0.f;
            __bf16 h, mi, lo;
            bf16_split3(xv, h, mi, lo);
            ah[e] = h;
            am[e] = mi;
            al[e] = lo;
            bf16_split3(yv, h, mi, lo);
            bh[e] = h;
            bm[e] = mi;
            bl[e] = lo;
        }
        const floatx4 z = {0.f, 0.f, 0.f, 0.f};
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
            g[q] += small + (double)p_hh[q];
        }
    }
}

// Point rows split into BF16 pieces (bf16_split3) in the matrix-core operand
// layout: unit ((T KC + kc) 3 + piece) 64 + lane (16 B) holds features
// kc 32 + (lane / 16) 8 + [0, 8) of row 16 T + lane % 16, zeros past the rows and
// features.  One thread per (T, kc, lane); blockIdx.y = problem of a batch
// (rows x d points each, consecutive; out_stride units between problems).
__global__ __launch_bounds__(256) void split_pieces(const float *__restrict__ P, long long rows, long long d, int KC,
                                                    bf16x8 *__restrict__ out, long long out_stride = 0) {
    const long long u = (long long)blockIdx.x * 256 + threadIdx.x;
    if (u >= (rows + 15) / 16 * KC * 64) return;
    P += (long long)blockIdx.y * rows * d;
    out += (long long)blockIdx.y * out_stride;
    const int ln = (int)(u % 64);
    const long long tk = u / 64, T = tk / KC;
    const int kc = (int)(tk % KC);
    const long long p = T * 16 + (ln & 15), k0 = (long long)kc * 32 + (ln >> 4) * 8;
    bf16x8 h, mi, lo;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const float v = (p < rows && k0 + e < d) ? P[p * d + k0 + e] : 0.f;
        __bf16 bh, bm, bl;
        bf16_split3(v, bh, bm, bl);
        h[e] = bh;
        mi[e] = bm;
        lo[e] = bl;
    }
    bf16x8 *dst = out + ((T * KC + kc) * 3) * 64 + ln;
    dst[0] = h;
    dst[64] = mi;
    dst[128] = lo;
}

template <int KIND>
__device__ __forceinline__ float finish_mfma(double g, double nx, double ny, double inv_s) {
    const double v = KIND == ACCSK_SQEUCLID ? fmax(nx + ny - 2.0 * g, 0.0) : 1.0 - g;
    return (float)(v * inv_s);
}

}  // namespace
}  // namespace accsk
