// RBM S-build on the matrix cores (the precision form).  The centred log-derivatives
// O_c = O - <O> are formed in FP64 and each real and imaginary part is split into two BF16
// terms, x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (|x - hi - lo| <= 2^-17 |x|).
// S = O_c^H O_c / N_s (definitions after Eq. 8) is accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16 from the three leading products hi*hi + hi*lo + lo*hi of every real
// product (the dropped lo*lo term is below 2^-16 of the product):
//   Re S_kl = sum Re_k Re_l + Im_k Im_l,   Im S_kl = sum Re_k Im_l - Im_k Re_l,
// i.e. 12 MFMAs per 16x16 complex block and 32 samples.  Centring before the products keeps
// the FP32 sums free of the cancellation that <O^* O> - <O>^* <O> would suffer.
// Output: S + eps I, lower triangle, complex interleaved, as in the FP64 kernel.
#pragma once
#include "common.hpp"
#include "made.hpp"
#include "rbm.hpp"

namespace tvmc {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split_bf16(double x, uint16_t &hi, uint16_t &lo) {
    hi = f2bf((float)x);
    lo = f2bf((float)(x - (double)bf2f(hi)));
}

// P [T][4][Mp][N_s] BF16 planes: 0 Re hi, 1 Re lo, 2 Im hi, 3 Im lo; rows M..Mp-1 are zero.
// Grid (ceil(N_s / 256), Mp, T); a thread writes one sample of one row in all four planes.
__global__ __launch_bounds__(256) void k_rbm_split(Dev a) {
    const int t = blockIdx.z, r = blockIdx.y;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.ns) return;
    double re = 0.0, im = 0.0;
    if (r < a.m) {
        const size_t sidx = (size_t)t * a.ns + s;
        const double2 o = rbm_o(a, r, a.samples[sidx], a.tt + sidx * a.nh);
        const double2 ob = a.obarc[(size_t)t * a.m + r];
        re = o.x - ob.x;
        im = o.y - ob.y;
    }
    uint16_t rh, rl, ih, il;
    split_bf16(re, rh, rl);
    split_bf16(im, ih, il);
    const size_t plane = (size_t)a.mp * a.ns;
    uint16_t *p = a.rbmP + (size_t)t * 4 * plane + (size_t)r * a.ns + s;
    p[0] = rh;
    p[plane] = rl;
    p[2 * plane] = ih;
    p[3 * plane] = il;
}

__device__ __forceinline__ bf16x8_t neg_bf16x8(bf16x8_t v) {
    u32x4_t u = __builtin_bit_cast(u32x4_t, v);
    u ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8_t, u);
}

#define MFMA_BF16(A, B, C) __builtin_amdgcn_mfma_f32_16x16x32_bf16((A), (B), (C), 0, 0, 0)

// One workgroup (4 waves) per 128x128 complex tile of the lower triangle; wave (wr, wc) takes
// the 64x64 sub-tile, 4x4 blocks of 16x16 (128 FP32 accumulators).  Operand fragments come
// straight from P (16 bytes per lane: row lane & 15, samples 8 (lane >> 4) .. +7 of the
// 32-sample step; the Gram product only needs the row and column operands to use the same
// sample order): per step a wave loads 32 fragments and issues 192 MFMAs.
constexpr int RQ_T = 128;
constexpr int RQ_W = 64;
__global__ __launch_bounds__(256) void k_sbuild_rbm_bf16(Dev a) {
    const int t = blockIdx.y, tile = blockIdx.x;
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = w >> 1, wc = w & 1;
    if (bi == bj && wr < wc) return;            // strictly upper sub-tile of a diagonal tile
    const int r0 = bi * RQ_T + wr * RQ_W, c0 = bj * RQ_T + wc * RQ_W;
    const int m = a.m;
    if (r0 >= m || c0 >= m) return;
    const int rr = lane & 15, kg = lane >> 4;
    const size_t ns = (size_t)a.ns, plane = (size_t)a.mp * ns;
    const uint16_t *Pt = a.rbmP + (size_t)t * 4 * plane;
    const uint16_t *rowp = Pt + (size_t)(r0 + rr) * ns + 8 * kg;
    const uint16_t *colp = Pt + (size_t)(c0 + rr) * ns + 8 * kg;
    f32x4_t sre[4][4], sim[4][4];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            sre[u][v] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            sim[u][v] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
    // operands of step k0 + 32 are loaded while step k0 is multiplied (one wave per SIMD,
    // so the load latency is hidden by the wave's own MFMAs)
    bf16x8_t A[4][4], B[4][4], An[4][4], Bn[4][4];
    for (int u = 0; u < 4; ++u)
        for (int q = 0; q < 4; ++q) {
            An[u][q] = *(const bf16x8_t *)(rowp + (size_t)u * 16 * ns + q * plane);
            Bn[u][q] = *(const bf16x8_t *)(colp + (size_t)u * 16 * ns + q * plane);
        }
    for (size_t k0 = 0; k0 < ns; k0 += 32) {
        for (int u = 0; u < 4; ++u)
            for (int q = 0; q < 4; ++q) {
                A[u][q] = An[u][q];
                B[u][q] = Bn[u][q];
            }
        if (k0 + 32 < ns)
            for (int u = 0; u < 4; ++u)
                for (int q = 0; q < 4; ++q) {
                    An[u][q] = *(const bf16x8_t *)(rowp + (size_t)u * 16 * ns + q * plane + k0 + 32);
                    Bn[u][q] = *(const bf16x8_t *)(colp + (size_t)u * 16 * ns + q * plane + k0 + 32);
                }
        for (int u = 0; u < 4; ++u) {
            const bf16x8_t nih = neg_bf16x8(A[u][2]), nil = neg_bf16x8(A[u][3]);
            for (int v = 0; v < 4; ++v) {
                f32x4_t x = sre[u][v];
                x = MFMA_BF16(A[u][0], B[v][0], x);
                x = MFMA_BF16(A[u][0], B[v][1], x);
                x = MFMA_BF16(A[u][1], B[v][0], x);
                x = MFMA_BF16(A[u][2], B[v][2], x);
                x = MFMA_BF16(A[u][2], B[v][3], x);
                x = MFMA_BF16(A[u][3], B[v][2], x);
                sre[u][v] = x;
                f32x4_t y = sim[u][v];
                y = MFMA_BF16(A[u][0], B[v][2], y);
                y = MFMA_BF16(A[u][0], B[v][3], y);
                y = MFMA_BF16(A[u][1], B[v][2], y);
                y = MFMA_BF16(nih, B[v][0], y);
                y = MFMA_BF16(nih, B[v][1], y);
                y = MFMA_BF16(nil, B[v][0], y);
                sim[u][v] = y;
            }
        }
    }
    const double inv = 1.0 / (double)a.ns;
    double2 *S = (double2 *)a.S + (size_t)t * m * m;
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v)
            for (int e = 0; e < 4; ++e) {
                const int k = r0 + u * 16 + 4 * kg + e, l = c0 + v * 16 + rr;   // D[4 (lane >> 4) + e][lane & 15]
                if (k >= m || l >= m || l > k) continue;
                double re = (double)sre[u][v][e] * inv;
                const double im = (double)sim[u][v][e] * inv;
                if (k == l) re += a.eps;
                S[(size_t)k * m + l] = make_double2(re, k == l ? 0.0 : im);
            }
}

#undef MFMA_BF16

}  // namespace tvmc
