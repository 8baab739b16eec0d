// S + eps I for the Jastrow ansaetze on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// O_sk is +-1, or for a shared LJPHd distance an integer of magnitude <= N - 1 <= 127, so
// sum_s O_sk O_sl is computed exactly as an int32 dot product of int8 values.
// Samples are first transposed to site-major bit planes (bit s of plane i = spin i of sample
// s is up).  For a 64-sample chunk the sign bits of a parameter row are one XOR of two planes
// (two-body) or a complement (one-body); four sign bits expand to four +-1 bytes with one
// multiply; a shared-distance row takes one popcount per sample from the packed samples.  A
// 128x128 output tile per workgroup (four waves, 64x64 each, 4x4 MFMA blocks)
// amortises that expansion over 128 output columns.  The epilogue centres in FP64 exactly as
// the plain form does, so both forms give the same bits.
#pragma once
#include "common.hpp"
#include "sbuild.hpp"

namespace tvmc {

typedef int v4i __attribute__((ext_vector_type(4)));

// samples[t][s] (W words, bit i % 64 of word i / 64 = site i) -> sbits[t][i][s/32] (u32, bit
// s%32 = sample s); one thread per site
__global__ void k_transpose_bits(Dev a) {
    const int t = blockIdx.y, wd = blockIdx.x, i = threadIdx.x;
    if (i >= a.n) return;
    const int W = a.nw;
    const uint64_t *smp = a.samples + ((size_t)t * a.ns + (size_t)wd * 32) * W + (i >> 6);
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) v |= (uint32_t)((smp[(size_t)b * W] >> (i & 63)) & 1ull) << b;
    a.sbits[((size_t)t * a.n + i) * (a.ns / 32) + wd] = v;
}

constexpr int SB_TILE = 128;
constexpr int SB_ROWW = 20;   // u32 words per LDS row: 16 data + 4 padding

__device__ __forceinline__ uint32_t expand4(uint32_t nib) {
    const uint32_t spread = (nib * 0x00204081u) & 0x01010101u;   // bit j -> byte j
    return 0x01010101u ^ (spread * 0xFEu);                        // 0x01 (+1) or 0xFF (-1)
}

// four samples' O of a shared distance p (sum of s_j s_{j+p}) as four int8 bytes
template <int W>
__device__ __forceinline__ uint32_t dist_bytes4(const uint64_t *sp, int p, int n) {
    uint32_t w = 0;
    for (int b = 0; b < 4; ++b)
        w |= (uint32_t)(uint8_t)(int8_t)o_int<true>(cfg_load<W>(sp + (size_t)b * W), p, -2, n) << (8 * b);
    return w;
}

template <bool DIST, int W>
__global__ __launch_bounds__(256) void k_sbuild_i8(Dev a) {
    __shared__ uint32_t As[SB_TILE * SB_ROWW];
    __shared__ uint32_t Bs[SB_TILE * SB_ROWW];
    const int t = blockIdx.y;
    const int tile = blockIdx.x;
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = wave >> 1, wc = wave & 1;   // wave's 64x64 quadrant

    // generator role: row gr of the A and B tiles, half gh (32 samples) of each chunk
    const int gr = tid >> 1, gh = tid & 1;
    const int ka = bi * SB_TILE + gr, kb = bj * SB_TILE + gr;
    const bool va = ka < a.m, vb = kb < a.m;
    const int ap = va ? a.pa[ka] : 0, aq = va ? a.pb[ka] : -1;
    const int bp = vb ? a.pa[kb] : 0, bq = vb ? a.pb[kb] : -1;
    const int nw = a.ns / 32;
    const uint32_t *planes = a.sbits + (size_t)t * a.n * nw;

    v4i acc[4][4];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) acc[u][v] = (v4i){0, 0, 0, 0};

    for (int w0 = 0; w0 < nw; w0 += 2) {
        const int w = w0 + gh;
        const uint32_t pa_ = planes[(size_t)ap * nw + w];
        const uint32_t na = va ? (aq < 0 ? ~pa_ : (pa_ ^ planes[(size_t)aq * nw + w])) : 0u;
        const uint32_t pb_ = planes[(size_t)bp * nw + w];
        const uint32_t nb = vb ? (bq < 0 ? ~pb_ : (pb_ ^ planes[(size_t)bq * nw + w])) : 0u;
        __syncthreads();
        if (DIST) {
            const uint64_t *sp = a.samples + ((size_t)t * a.ns + (size_t)w * 32) * W;
            for (int q = 0; q < 8; ++q) {
                As[gr * SB_ROWW + gh * 8 + q] = !va ? 0u : aq == -2 ? dist_bytes4<W>(sp + 4 * q * W, ap, a.n)
                                                                   : expand4((na >> (4 * q)) & 0xFu);
                Bs[gr * SB_ROWW + gh * 8 + q] = !vb ? 0u : bq == -2 ? dist_bytes4<W>(sp + 4 * q * W, bp, a.n)
                                                                   : expand4((nb >> (4 * q)) & 0xFu);
            }
        } else {
            for (int q = 0; q < 8; ++q) {
                As[gr * SB_ROWW + gh * 8 + q] = va ? expand4((na >> (4 * q)) & 0xFu) : 0u;
                Bs[gr * SB_ROWW + gh * 8 + q] = vb ? expand4((nb >> (4 * q)) & 0xFu) : 0u;
            }
        }
        __syncthreads();
        v4i fa[4], fb[4];
        const int kq = (lane >> 4) * 4;   // 16-byte slice of the 64-sample chunk
        for (int u = 0; u < 4; ++u) {
            const uint32_t *pa4 = &As[(wr * 64 + u * 16 + (lane & 15)) * SB_ROWW + kq];
            const uint32_t *pb4 = &Bs[(wc * 64 + u * 16 + (lane & 15)) * SB_ROWW + kq];
            fa[u] = (v4i){(int)pa4[0], (int)pa4[1], (int)pa4[2], (int)pa4[3]};
            fb[u] = (v4i){(int)pb4[0], (int)pb4[1], (int)pb4[2], (int)pb4[3]};
        }
        for (int u = 0; u < 4; ++u)
            for (int v = 0; v < 4; ++v) acc[u][v] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[u], fb[v], acc[u][v], 0, 0, 0);
    }

    // epilogue: lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 block
    const double inv = 1.0 / (double)a.ns;
    const double *ob = a.obar + (size_t)t * a.m;
    double *S = a.S + (size_t)t * a.m * a.m;
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v)
            for (int r = 0; r < 4; ++r) {
                const int k = bi * SB_TILE + wr * 64 + u * 16 + 4 * (lane >> 4) + r;
                const int l = bj * SB_TILE + wc * 64 + v * 16 + (lane & 15);
                if (k >= a.m || l >= a.m || l > k) continue;
                double sv = centre((double)acc[u][v][r], inv, ob[k], ob[l]);
                if (k == l) sv = add_shift(sv, a.eps);
                S[(size_t)k * a.m + l] = sv;
            }
}

inline tvmc_status launch_transpose_bits(const Dev &d, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_bits, dim3(d.ns / 32, d.nt), dim3(64 * d.nw), 0, st, d);
    return hipGetLastError() == hipSuccess ? TVMC_OK : TVMC_E_DEVICE;
}

inline tvmc_status launch_sbuild_mfma(const Dev &d, hipStream_t st) {
    const int nt = (d.m + SB_TILE - 1) / SB_TILE;
    const dim3 grid(nt * (nt + 1) / 2, d.nt);
    if (d.kind == TVMC_ANSATZ_LJPH) {
        if (d.nw == 1) hipLaunchKernelGGL((k_sbuild_i8<true, 1>), grid, dim3(256), 0, st, d);
        else if (d.nw == 2) hipLaunchKernelGGL((k_sbuild_i8<true, 2>), grid, dim3(256), 0, st, d);
        else hipLaunchKernelGGL((k_sbuild_i8<true, 3>), grid, dim3(256), 0, st, d);
    } else {
        hipLaunchKernelGGL((k_sbuild_i8<false, 1>), grid, dim3(256), 0, st, d);   // the samples are not read
    }
    if (hipGetLastError() != hipSuccess) return TVMC_E_DEVICE;
    return TVMC_OK;
}

}  // namespace tvmc
