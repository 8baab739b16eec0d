// S + eps I for the Jastrow ansaetze on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// O_sk is +-1, or for a shared LJPHd distance D the sum over the len = N - D pairs at that
// distance of s_j s_{j+D}, an integer of len's parity with |O| <= len <= N - 1.  Up to N = 128
// (one or two configuration words) |O| <= 127 fits a byte.  With three words (N <= 192) such a
// row is fed as its half h = (O - (len & 1)) / 2, |h| <= 96, and with c = 2, p = len & 1 for
// those rows (c = 1, p = 0, h = O for the +-1 rows) the exact sum is rebuilt from the int32
// MFMA sum of h_k h_l and the row sums of h:
//   sum_s O_k O_l = c_k c_l sum h_k h_l + c_k p_l sum h_k + c_l p_k sum h_l + N_s p_k p_l.
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

// four samples' O of a shared distance p (O = sum of s_j s_{j+p} over the len = n - p pairs) as
// four int8 bytes, or with HALF their halves h = (O - (len & 1)) / 2, whose sum is added to hsum
template <int W, bool HALF>
__device__ __forceinline__ uint32_t dist_bytes4(const uint64_t *sp, int p, int n, int &hsum) {
    const int par = (n - p) & 1;
    uint32_t w = 0;
    for (int b = 0; b < 4; ++b) {
        int o = o_int<true>(cfg_load<W>(sp + (size_t)b * W), p, -2, n);
        if (HALF) {
            o = (o - par) >> 1;   // exact: O - par is even
            hsum += o;
        }
        w |= (uint32_t)(uint8_t)(int8_t)o << (8 * b);
    }
    return w;
}

template <bool DIST, int W>
__global__ __launch_bounds__(256) void k_sbuild_i8(Dev a) {
    constexpr bool HALF = DIST && W == 3;   // shared-distance rows fed as halves
    __shared__ uint32_t As[SB_TILE * SB_ROWW];
    __shared__ uint32_t Bs[SB_TILE * SB_ROWW];
    // HALF: per tile row of A and B, the two halves' sums of h, then c + 4 p and a scaled sum
    __shared__ int hs[HALF ? 2 * 2 * SB_TILE : 1];
    __shared__ int rw[HALF ? 2 * 2 * SB_TILE : 1];
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
    int hsa = 0, hsb = 0;   // HALF: this thread's share of the row sums of h

    for (int w0 = 0; w0 < nw; w0 += 2) {
        const int w = w0 + gh;
        const uint32_t pa_ = planes[(size_t)ap * nw + w];
        const uint32_t na = va ? (aq < 0 ? ~pa_ : (pa_ ^ planes[(size_t)aq * nw + w])) : 0u;
        const uint32_t pb_ = planes[(size_t)bp * nw + w];
        const uint32_t nb = vb ? (bq < 0 ? ~pb_ : (pb_ ^ planes[(size_t)bq * nw + w])) : 0u;
        __syncthreads();
        if (DIST) {
            const uint64_t *sp = a.samples + ((size_t)t * a.ns + (size_t)w * 32) * W;
            if (HALF) {   // a +-1 row's 32 values sum to 32 - 2 popcount (a set bit is -1)
                if (va && aq != -2) hsa += 32 - 2 * __popc(na);
                if (vb && bq != -2) hsb += 32 - 2 * __popc(nb);
            }
            for (int q = 0; q < 8; ++q) {
                As[gr * SB_ROWW + gh * 8 + q] = !va ? 0u : aq == -2 ? dist_bytes4<W, HALF>(sp + 4 * q * W, ap, a.n, hsa)
                                                                   : expand4((na >> (4 * q)) & 0xFu);
                Bs[gr * SB_ROWW + gh * 8 + q] = !vb ? 0u : bq == -2 ? dist_bytes4<W, HALF>(sp + 4 * q * W, bp, a.n, hsb)
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

    if (HALF) {
        // with x_k = c_k sum h_k for the rows k of A and y_l = c_l sum h_l + N_s p_l for the rows
        // l of B, sum_s O_k O_l = c_k c_l sum h_k h_l + p_l x_k + p_k y_l (p is 0 or 1); rw holds
        // [A / B][c + 4 p, x or y][row]
        hs[gh * SB_TILE + gr] = hsa;
        hs[(2 + gh) * SB_TILE + gr] = hsb;
        __syncthreads();
        if (gh == 0) {
            const int ca = aq == -2 ? 2 : 1, pa_ = aq == -2 ? (a.n - ap) & 1 : 0;
            const int cb = bq == -2 ? 2 : 1, pb_ = bq == -2 ? (a.n - bp) & 1 : 0;
            rw[gr] = ca + 4 * pa_;
            rw[SB_TILE + gr] = ca * (hs[gr] + hs[SB_TILE + gr]);
            rw[2 * SB_TILE + gr] = cb + 4 * pb_;
            rw[3 * SB_TILE + gr] = cb * (hs[2 * SB_TILE + gr] + hs[3 * SB_TILE + gr]) + a.ns * pb_;
        }
        __syncthreads();
    }
    // epilogue: lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 block
    const double inv = 1.0 / (double)a.ns;
    const double *ob = a.obar + (size_t)t * a.m;
    double *S = a.S + (size_t)t * a.m * a.m;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rk = wr * 64 + u * 16 + 4 * (lane >> 4) + r, rl = wc * 64 + v * 16 + (lane & 15);
                const int k = bi * SB_TILE + rk, l = bj * SB_TILE + rl;
                if (k >= a.m || l >= a.m || l > k) continue;
                double g = (double)acc[u][v][r];
                if (HALF) {   // every term an integer below 2^53: exact in FP64
                    const int fk = rw[rk], fl = rw[2 * SB_TILE + rl];
                    g = (double)((fk & 3) * (fl & 3)) * g + (double)((fl & 4) ? rw[SB_TILE + rk] : 0) +
                        (double)((fk & 4) ? rw[3 * SB_TILE + rl] : 0);
                }
                double sv = centre(g, inv, ob[k], ob[l]);
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
