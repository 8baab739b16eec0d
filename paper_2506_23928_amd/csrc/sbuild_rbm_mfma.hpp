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

// hi = bf16(float(x)), lo = bf16(float(x - hi)), each step rounded to nearest even.  The float is
// passed through an empty asm so that the compiler keeps the two hardware conversions
// (v_cvt_f32_f64, v_cvt_pk_bf16_f32) instead of fusing them into one longer double -> bfloat16
// sequence.
__device__ __forceinline__ uint16_t f64_to_bf(double x) {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return f2bf(f);
}
__device__ __forceinline__ void split_bf16(double x, uint16_t &hi, uint16_t &lo) {
    hi = f64_to_bf(x);
    lo = f64_to_bf(x - (double)bf2f(hi));
}

// P holds the four BF16 planes 0 Re hi, 1 Re lo, 2 Im hi, 3 Im lo in the order the S-build
// stages them: [T][Mp / 128 row blocks][N_s / 32 steps][4 planes][128 rows][32 samples], so
// that one step of one row block is a contiguous 32 KB chunk; rows M..Mp-1 are zero.
// Grid (N_s / 32, ceil(Mp / 512), T); a block takes SPL_R slices of 64 rows, thread tid row
// tid / 4 of each slice and the 8 samples 8 (tid % 4) .. +7 of the step, and writes 16 bytes
// per plane: a wavefront writes 16 rows x 64 bytes, one contiguous kilobyte of each plane.  The
// thread's rows differ by 64, so where N' divides 64 and the weights start on a multiple of 64
// they share the hidden unit j and its 8 tanh values are loaded once.
constexpr int RQ_CHUNK = 4 * 128 * 32;   // elements of one staged step of one row block
constexpr int SPL_R = 8;
typedef unsigned short u16x8_t __attribute__((ext_vector_type(8)));
template <int W>
__global__ __launch_bounds__(256) void k_rbm_split(Dev a) {
    const int t = blockIdx.z, st = blockIdx.x, n = a.n, nh = a.nh, wb = n + nh;
    const int s0 = st * 32 + 8 * (threadIdx.x & 3);
    const size_t sbase = (size_t)t * a.ns + s0;
    const double2 *tts = a.tt + sbase * nh;
    Cfg<W> mk[8];
    for (int e = 0; e < 8; ++e) mk[e] = cfg_load<W>(a.samples + (sbase + e) * W);
    double2 tv[8];
    int jc = -1;
    const int nst = a.ns / 32;
    for (int sl = 0; sl < SPL_R; ++sl) {
        const int r = (blockIdx.y * SPL_R + sl) * 64 + (threadIdx.x >> 2);
        if (r >= a.mp) break;     // whole slices: Mp is a multiple of 128
        double2 ob = make_double2(0.0, 0.0);
        int wi = -1;
        if (r < a.m) {
            ob = a.obarc[(size_t)t * a.m + r];
            if (r >= wb) {
                wi = (r - wb) / nh;
                const int j = (r - wb) % nh;
                if (j != jc) {
                    for (int e = 0; e < 8; ++e) tv[e] = tts[(size_t)e * nh + j];
                    jc = j;
                }
            }
        }
        u16x8_t rh, rl, ih, il;
        for (int e = 0; e < 8; ++e) {
            double re = 0.0, im = 0.0;
            if (r < a.m) {
                double2 o;
                if (wi >= 0) {
                    const double si = spin(mk[e], wi);
                    o = make_double2(si * tv[e].x, si * tv[e].y);
                } else {
                    o = rbm_o(a, r, mk[e], tts + (size_t)e * nh);
                }
                re = o.x - ob.x;
                im = o.y - ob.y;
            }
            uint16_t h, l;
            split_bf16(re, h, l);
            rh[e] = h;
            rl[e] = l;
            split_bf16(im, h, l);
            ih[e] = h;
            il[e] = l;
        }
        uint16_t *p = a.rbmP + ((size_t)(t * (a.mp / 128) + (r >> 7)) * nst + st) * RQ_CHUNK + (r & 127) * 32 +
                      8 * (threadIdx.x & 3);
        *(u16x8_t *)p = rh;
        *(u16x8_t *)(p + 128 * 32) = rl;
        *(u16x8_t *)(p + 2 * 128 * 32) = ih;
        *(u16x8_t *)(p + 3 * 128 * 32) = il;
    }
}

__device__ __forceinline__ bf16x8_t neg_bf16x8(bf16x8_t v) {
    u32x4_t u = __builtin_bit_cast(u32x4_t, v);
    u ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8_t, u);
}

#define MFMA_BF16(A, B, C) __builtin_amdgcn_mfma_f32_16x16x32_bf16((A), (B), (C), 0, 0, 0)

// One workgroup (8 waves) per 128x128 complex tile of the lower triangle; wave (wr, wc) =
// (w >> 2, w & 3) takes rows 64 wr .. +63 and columns 32 wc .. +31 of the tile, 4x2 blocks of
// 16x16 (64 FP32 accumulators), which keeps a wave under 256 registers so that two waves
// share each SIMD and hide each other's LDS and MFMA latencies.  Per step of 32 samples the
// workgroup copies the tile's row and column operands (4 planes x 128 rows x 32 samples each,
// 64 KB) from global memory straight into double-buffered LDS (global_load_lds, no register
// staging), with the fragments of the next step read while the products of the current one
// are issued (the pipeline is described at the main loop).  A fragment is 16 bytes per lane:
// row lane & 15, samples 8 (lane >> 4) .. +7 of the step (the Gram product only needs the row
// and column operands to use the same sample order).
constexpr int RQ_T = 128;
constexpr int RQ_K = 32;          // samples per step
constexpr int RQ_THREADS = 512;
constexpr int RQ_BAND = 4;        // tile rows per band of the work order
__global__ __launch_bounds__(RQ_THREADS) void k_sbuild_rbm_bf16(Dev a) {
    // [step parity][row / column operand][plane][128 rows][32 samples], 128 KB
    __shared__ __attribute__((aligned(1024))) uint16_t sbuf[2][2][4 * RQ_T * RQ_K];
    // Work order.  Workgroups are dealt round-robin to the 8 XCDs, so workgroup L runs on XCD
    // L % 8; XCD x takes the contiguous run of work items x * per .. x * per + per - 1 in
    // turn, and the items of a trajectory are ordered in bands of RQ_BAND tile rows, column by
    // column, so that the tiles resident on one XCD at a time share few operand panels in its
    // L2.  The grid is padded to a multiple of 8; padding workgroups exit at once.
    const int nt = a.mp / RQ_T, ntl = nt * (nt + 1) / 2;
    const int L = blockIdx.x, per = (int)gridDim.x / 8;
    const int g = (L & 7) * per + (L >> 3);
    if (g >= ntl * a.nt) return;
    const int t = g / ntl, wdx = g % ntl;
    int band = 0;
    while ((band + 1) * RQ_BAND * ((band + 1) * RQ_BAND + 1) / 2 <= wdx) ++band;
    const int b0 = band * RQ_BAND, bh = min(RQ_BAND, nt - b0);
    int rem = wdx - b0 * (b0 + 1) / 2, bi, bj;
    if (rem < b0 * bh) {          // full columns left of the band's diagonal block
        bj = rem / bh;
        bi = b0 + rem % bh;
    } else {                      // the band's triangular diagonal block, column by column
        rem -= b0 * bh;
        int col = 0;
        while (rem >= bh - col) rem -= bh - col++;
        bj = b0 + col;
        bi = bj + rem;
    }
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int wr = w >> 2, wc = w & 3;
    const int m = a.m;
    const int r0 = bi * RQ_T + wr * 64, c0 = bj * RQ_T + wc * 32;
    // sub-tiles strictly above the diagonal of a diagonal tile and padding rows do no MFMAs,
    // but their waves still stage operands and meet every barrier
    const bool active = !(bi == bj && c0 > r0 + 63) && r0 < m && c0 < m;
    const int rr = lane & 15, kg = lane >> 4;
    const size_t ns = (size_t)a.ns, nst = ns / RQ_K;
    const uint16_t *Pt = a.rbmP + (size_t)t * (a.mp / RQ_T) * nst * RQ_CHUNK;
    // LDS layout of a staged operand: [plane][128 rows][32 samples], rows of 64 bytes with the
    // four 16-byte pieces of row r permuted by c -> c ^ ((r >> 1) & 3), under which the 16-byte
    // fragment reads of 16 consecutive rows meet no bank conflict (measured with the LDS bank
    // conflict counter: the permutation by r >> 2 costs a second pass on every read).  The chunks are copied from
    // global memory straight into LDS: wave instruction i (of 32 per operand and step) fills
    // bytes 1024 i .. +1023, i.e. plane i / 8, rows 16 (i % 8) .. +15; lane L lands in row
    // 16 (i % 8) + L / 4 at piece L % 4, so it reads the logical piece (L % 4) ^ ((row >> 1) & 3)
    const uint16_t *gA = Pt + (size_t)bi * nst * RQ_CHUNK, *gB = Pt + (size_t)bj * nst * RQ_CHUNK;
    int gofs[4];                                   // element offset in the chunk, per instruction
    for (int j = 0; j < 4; ++j) {
        const int i = w * 4 + j, q = i >> 3, row = (i & 7) * 16 + (lane >> 2);
        gofs[j] = q * 4096 + row * 32 + (((lane & 3) ^ ((row >> 1) & 3)) * 8);
    }
    typedef __attribute__((address_space(1))) void gvoid_t;
    typedef __attribute__((address_space(3))) void lvoid_t;
#define RQ_STAGE(BUF, STEP)                                                                     \
    for (int j = 0; j < 4; ++j) {                                                               \
        const int i = w * 4 + j;                                                                \
        __builtin_amdgcn_global_load_lds((gvoid_t *)(gA + (size_t)(STEP) * RQ_CHUNK + gofs[j]),  \
                                         (lvoid_t *)(sbuf[BUF][0] + i * 512), 16, 0, 0);       \
        __builtin_amdgcn_global_load_lds((gvoid_t *)(gB + (size_t)(STEP) * RQ_CHUNK + gofs[j]),  \
                                         (lvoid_t *)(sbuf[BUF][1] + i * 512), 16, 0, 0);       \
    }
    f32x4_t sre[4][2], sim[4][2];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 2; ++v) {
            sre[u][v] = f32x4_t{0.f, 0.f, 0.f, 0.f};
            sim[u][v] = f32x4_t{0.f, 0.f, 0.f, 0.f};
        }
    const int arow = wr * 64 + rr, brow = wc * 32 + rr;
#define RQ_SW(row) ((((kg) ^ (((row) >> 1) & 3))) * 8)
#define RQ_LDA(BUF, Q) for (int u = 0; u < 4; ++u) A[u][Q] = *(const bf16x8_t *)(sbuf[BUF][0] + ((Q) * RQ_T + arow + 16 * u) * 32 + RQ_SW(arow + 16 * u));
#define RQ_LDB(BUF, Q) for (int v = 0; v < 2; ++v) B[v][Q] = *(const bf16x8_t *)(sbuf[BUF][1] + ((Q) * RQ_T + brow + 16 * v) * 32 + RQ_SW(brow + 16 * v));
#define RQ_TERM(ACC, AX, BX) for (int u = 0; u < 4; ++u) for (int v = 0; v < 2; ++v) ACC[u][v] = MFMA_BF16(AX, BX, ACC[u][v]);
    // Pipeline: at the start of step k the fragments of step k are in registers and LDS buffer
    // (k+1)&1 holds step k+1.  Step k copies step k+2 into buffer k&1 (whose step-k contents
    // were read into registers during step k-1) and issues its 12 products plane by plane,
    // reloading each fragment plane from buffer (k+1)&1 as soon as its last product of step k
    // has been issued; the copy is waited for and one barrier ends the step.
    RQ_STAGE(0, 0)
    if (1 < nst) RQ_STAGE(1, 1)
    bf16x8_t A[4][4], B[2][4];
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (active) {
        RQ_LDA(0, 0) RQ_LDA(0, 1) RQ_LDA(0, 2) RQ_LDA(0, 3)
        RQ_LDB(0, 0) RQ_LDB(0, 1) RQ_LDB(0, 2) RQ_LDB(0, 3)
    }
    __syncthreads();
    for (int k = 0; k < (int)nst; ++k) {
        const int wb = k & 1, rb = wb ^ 1;
        const bool more = k + 1 < (int)nst;
        if (k + 2 < (int)nst) RQ_STAGE(wb, k + 2)
        if (active) {
            //   Re += Ar.Br + Ai.Bi,  Im += Ar.Bi + Ai.(-Br), each as hi hi + hi lo + lo hi
            bf16x8_t NB[2][2];
            for (int v = 0; v < 2; ++v) {
                NB[v][0] = neg_bf16x8(B[v][0]);
                NB[v][1] = neg_bf16x8(B[v][1]);
            }
            RQ_TERM(sre, A[u][0], B[v][0])
            RQ_TERM(sim, A[u][0], B[v][2])
            RQ_TERM(sre, A[u][0], B[v][1])
            RQ_TERM(sim, A[u][0], B[v][3])
            if (more) { RQ_LDA(rb, 0) RQ_LDB(rb, 1) }
            RQ_TERM(sre, A[u][1], B[v][0])
            RQ_TERM(sim, A[u][1], B[v][2])
            if (more) { RQ_LDA(rb, 1) RQ_LDB(rb, 0) }
            RQ_TERM(sre, A[u][2], B[v][2])
            RQ_TERM(sim, A[u][2], NB[v][0])
            RQ_TERM(sre, A[u][2], B[v][3])
            RQ_TERM(sim, A[u][2], NB[v][1])
            if (more) { RQ_LDA(rb, 2) RQ_LDB(rb, 3) }
            RQ_TERM(sre, A[u][3], B[v][2])
            RQ_TERM(sim, A[u][3], NB[v][0])
            if (more) { RQ_LDA(rb, 3) RQ_LDB(rb, 2) }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
#undef RQ_STAGE
#undef RQ_SW
#undef RQ_LDA
#undef RQ_LDB
#undef RQ_TERM
    if (!active) return;
    const double inv = 1.0 / (double)a.ns;
    double2 *S = (double2 *)a.S + (size_t)t * m * m;
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 2; ++v)
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
