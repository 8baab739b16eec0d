// Regularised solve for a complex Hermitian S (RBM ansatz): (S + eps I) delta = D with
// S + eps I = L L^H, in FP64 on the matrix cores, several workgroups per trajectory.  The
// steps mirror the real solver (left-looking panels of CN = 64 columns, one launch per step):
//   k_zmw_update(j0):  for this chunk's rows below the current panel, the previous panel's
//                      TRSM L[rows, prev] = C Linv_prev^H, z[rows] -= L[rows, prev] y_prev; then
//                      C[rows, panel] = A[rows, panel] - L[rows, 0:j0] L[panel, 0:j0]^H
//                      Re C -= Lr Lr'^T + Li Li'^T,  Im C -= Li Lr'^T - Lr Li'^T   (4 real MFMA products)
//   k_zmw_diag(j0):    L_pp L_pp^H = C_pp in LDS, Linv = L_pp^-1, y_p = Linv z_p, and the TRSM of
//                      the next panel's rows (the next update reads them as its panel rows)
//   so a panel takes two launches on the chain of dependent launches instead of three.
//   k_zmw_update_lds is the same update with its operand slices copied straight into LDS; the
//   host takes it whenever a trajectory's matrix is under 4 GiB (32-bit byte offsets).
//   k_zmw_bwd(p):      L^H x = y by row panels: x_p = Linv^H w_p, w_c -= L[p, c]^H x_p (c < j0)
// Matrices are complex [T][M][M] (lower triangle), interleaved (re, im).
#pragma once
#include "cholesky.hpp"

namespace tvmc {

struct ZCholArgs {
    double2 *A;
    const double2 *rhs;
    double2 *x;
    double2 *linv;   // [T][panels][64 * 64]
    int *flags;
    int m;
};


__global__ __launch_bounds__(256) void k_zmw_init(ZCholArgs a) {
    const int t = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < a.m) a.x[(size_t)t * a.m + i] = a.rhs[(size_t)t * a.m + i];
}

constexpr int ZK = 16;          // k-slice staged through LDS
constexpr int ZKP = ZK + 1;
constexpr int ZT = 512;         // threads of k_zmw_update: 8 waves, 16 rows of the 128-row chunk each
constexpr int ZBUF = 2 * (CR + CN) * ZKP;   // one staging buffer: Ar, Ai [CR][ZKP], Br, Bi [CN][ZKP]

static_assert(2 * ZBUF >= 2 * CN * CSP + 2 * CN, "the staging buffers hold a block inverse and y");

// The TRSM of the previous panel pp for this chunk's rows below the current panel (the
// diagonal kernel did the current panel's own rows), then the update of the current panel:
//   X = C[rows, panel pp] Linv_pp^H written over C, z[rows] -= X y_pp;
//   C[rows, panel] = A[rows, panel] - L[rows, 0:j0] L[panel, 0:j0]^H.
// pp < 0: no previous panel (j0 = 0).  The TRSM's values are read back by the update loop from
// global memory after a workgroup barrier (same workgroup, so the barrier orders them).
__global__ __launch_bounds__(ZT) void k_zmw_update(ZCholArgs a, int j0, int pp, int nt) {
    __shared__ double stage[2 * ZBUF];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    int t, chunk;
    if (!chunk_item((M - j0 + CR - 1) / CR, nt, t, chunk)) return;
    const int r0 = j0 + chunk * CR;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    double2 *A = a.A + (size_t)t * M * M;
    if (pp >= 0) {
        const int jq = j0 - CN;   // the previous panel's columns (a full panel: another follows it)
        double *Lr = stage, *Li = stage + CN * CSP, *yr = stage + 2 * CN * CSP, *yi = yr + CN;
        double2 *z = a.x + (size_t)t * M;
        const double2 *lv = a.linv + ((size_t)t * chol_panels(M) + pp) * CN * CN;
        for (int e = tid; e < CN * CN; e += ZT) {
            const double2 l = lv[e];
            Lr[(e / CN) * CSP + e % CN] = l.x;
            Li[(e / CN) * CSP + e % CN] = l.y;
        }
        if (tid < CN) {
            const double2 y = z[jq + tid];
            yr[tid] = y.x;
            yi[tid] = y.y;
        }
        __syncthreads();
        // rows j0 .. j0 + CN - 1 belong to the diagonal kernel; a wave's 16 rows lie on one side
        const int wrow = r0 + wave * 16;
        if (wrow >= j0 + CN && wrow < M) {
            double2 cf[CN / 4];   // C[row wrow + li][4 ks + lk]
            {
                const int row = wrow + li;
                for (int ks = 0; ks < CN / 4; ++ks)
                    cf[ks] = row < M ? A[(size_t)row * M + jq + ks * 4 + lk] : make_double2(0.0, 0.0);
            }
            v4d xr[4], xi[4];
            for (int v = 0; v < 4; ++v) {
                xr[v] = (v4d){0.0, 0.0, 0.0, 0.0};
                xi[v] = (v4d){0.0, 0.0, 0.0, 0.0};
            }
            // Linv is lower triangular: column block v of Linv^H is zero in the k-steps ks >= 4 v + 4
            for (int ks = 0; ks < CN / 4; ++ks) {
                double fbr[4], fbi[4];
                for (int v = 0; v < 4; ++v) {
                    if (v < (ks >> 2)) continue;
                    fbr[v] = Lr[(v * 16 + li) * CSP + ks * 4 + lk];
                    fbi[v] = Li[(v * 16 + li) * CSP + ks * 4 + lk];
                }
                const double fcr = cf[ks].x, fci = cf[ks].y;
                for (int v = 0; v < 4; ++v) {
                    if (v < (ks >> 2)) continue;
                    xr[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fcr, fbr[v], xr[v], 0, 0, 0);
                    xr[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fci, fbi[v], xr[v], 0, 0, 0);
                    xi[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fci, fbr[v], xi[v], 0, 0, 0);
                    xi[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fcr, -fbi[v], xi[v], 0, 0, 0);
                }
            }
            for (int r = 0; r < 4; ++r) {
                const int row = wrow + lk + 4 * r;
                double sr = 0.0, si = 0.0;
                for (int v = 0; v < 4; ++v) {
                    const int col = v * 16 + li;
                    const double a_ = xr[v][r], b_ = xi[v][r];
                    if (row < M) A[(size_t)row * M + jq + col] = make_double2(a_, b_);
                    sr += a_ * yr[col] - b_ * yi[col];
                    si += a_ * yi[col] + b_ * yr[col];
                }
                for (int o = 1; o < 16; o <<= 1) {
                    sr += __shfl_xor(sr, o, 64);
                    si += __shfl_xor(si, o, 64);
                }
                if (li == 0 && row < M) {
                    const double2 zr = z[row];
                    z[row] = make_double2(zr.x - sr, zr.y - si);
                }
            }
        }
        __syncthreads();   // the staging buffers are free again; this chunk's X is visible to every wave
    }
    v4d cre[4], cim[4];
    for (int v = 0; v < 4; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            const double2 c = (r0 + row < M && col < jb) ? A[(size_t)(r0 + row) * M + j0 + col] : make_double2(0.0, 0.0);
            cre[v][r] = c.x;
            cim[v][r] = c.y;
        }
    if (j0 > 0) {
        double2 pa[CR * ZK / ZT], pb[CN * ZK / ZT];
        auto fetch = [&](int kc) {
            for (int q = 0; q < CR * ZK / ZT; ++q) {
                const int e = tid + ZT * q, rr = e / ZK, kk = e % ZK;
                pa[q] = (r0 + rr < M) ? A[(size_t)(r0 + rr) * M + kc + kk] : make_double2(0.0, 0.0);
            }
            for (int q = 0; q < CN * ZK / ZT; ++q) {
                const int e = tid + ZT * q, cc = e / ZK, kk = e % ZK;
                pb[q] = (cc < jb) ? A[(size_t)(j0 + cc) * M + kc + kk] : make_double2(0.0, 0.0);
            }
        };
        auto stash = [&](int buf) {
            double *Ar = stage + buf * ZBUF, *Ai = Ar + CR * ZKP, *Br = Ai + CR * ZKP, *Bi = Br + CN * ZKP;
            for (int q = 0; q < CR * ZK / ZT; ++q) {
                const int e = tid + ZT * q;
                Ar[(e / ZK) * ZKP + e % ZK] = -pa[q].x;
                Ai[(e / ZK) * ZKP + e % ZK] = -pa[q].y;
            }
            for (int q = 0; q < CN * ZK / ZT; ++q) {
                const int e = tid + ZT * q;
                Br[(e / ZK) * ZKP + e % ZK] = pb[q].x;
                Bi[(e / ZK) * ZKP + e % ZK] = pb[q].y;
            }
        };
        // double-buffered: slice k+1 is fetched before and staged after the products of slice
        // k, into the buffer whose last readers passed the previous barrier
        fetch(0);
        stash(0);
        __syncthreads();
        for (int kc = 0, buf = 0; kc < j0; kc += ZK, buf ^= 1) {
            const bool more = kc + ZK < j0;
            if (more) fetch(kc + ZK);
            const double *Ar = stage + buf * ZBUF, *Ai = Ar + CR * ZKP, *Br = Ai + CR * ZKP, *Bi = Br + CN * ZKP;
            for (int ks = 0; ks < ZK / 4; ++ks) {
                double fbr[4], fbi[4];
                const double far_ = Ar[(wave * 16 + li) * ZKP + ks * 4 + lk];   // -Lr (rows)
                const double fai = Ai[(wave * 16 + li) * ZKP + ks * 4 + lk];    // -Li (rows)
                for (int v = 0; v < 4; ++v) {
                    fbr[v] = Br[(v * 16 + li) * ZKP + ks * 4 + lk];                // Lr' (panel rows)
                    fbi[v] = Bi[(v * 16 + li) * ZKP + ks * 4 + lk];                // Li'
                }
                for (int v = 0; v < 4; ++v) {
                    cre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(far_, fbr[v], cre[v], 0, 0, 0);
                    cre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fai, fbi[v], cre[v], 0, 0, 0);
                    cim[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fai, fbr[v], cim[v], 0, 0, 0);
                    cim[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(far_, -fbi[v], cim[v], 0, 0, 0);
                }
            }
            if (more) stash(buf ^ 1);
            __syncthreads();
        }
    }
    for (int v = 0; v < 4; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            if (r0 + row < M && col < jb)
                A[(size_t)(r0 + row) * M + j0 + col] = make_double2(cre[v][r], cim[v][r]);
        }
}

// The same update with the operand slices copied from global memory straight into LDS
// (global_load_lds, no register staging) through three buffers, so that the copies run up to
// two slices ahead of the products and a slice costs one barrier and one partial wait.  A slice is
// ZK complex columns: CR chunk rows and CN panel rows of 256 bytes each, the 16-byte pieces of
// row r stored at position piece ^ (r & 15), which puts the 16 rows of a fragment read on
// distinct banks.  Each fragment is one 16-byte read of (re, im).  The product P = L[rows, 0:j0]
// L[panel, 0:j0]^H accumulates from zero as Re P (two products per block), Im P's two halves
// Li Lr'^T and Lr Li'^T separately (no negated operands), and C = A - P at the end.
constexpr int ZU_STAGES = 3;
constexpr int ZU_ROWS = CR + CN;                       // rows of one staged slice
constexpr int ZU_SLICE = ZU_ROWS * ZK;                 // double2 elements of one staged slice
static_assert(ZK == 16 && ZT == 512, "one slice is 48 wave copies of 1 KB: six per wave");
__global__ __launch_bounds__(ZT) void k_zmw_update_lds(ZCholArgs a, int j0, int pp, int nt) {
    __shared__ __attribute__((aligned(1024))) double2 sl[ZU_STAGES * ZU_SLICE];   // 144 KB
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    int t, chunk;
    if (!chunk_item((M - j0 + CR - 1) / CR, nt, t, chunk)) return;
    const int r0 = j0 + chunk * CR;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    double2 *A = a.A + (size_t)t * M * M;
    if (pp >= 0) {   // the previous panel's TRSM of this chunk's rows below the current panel
        const int jq = j0 - CN;
        double *Lr = (double *)sl, *Li = Lr + CN * CSP, *yr = Lr + 2 * CN * CSP, *yi = yr + CN;
        double2 *z = a.x + (size_t)t * M;
        const double2 *lv = a.linv + ((size_t)t * chol_panels(M) + pp) * CN * CN;
        for (int e = tid; e < CN * CN; e += ZT) {
            const double2 l = lv[e];
            Lr[(e / CN) * CSP + e % CN] = l.x;
            Li[(e / CN) * CSP + e % CN] = l.y;
        }
        if (tid < CN) {
            const double2 y = z[jq + tid];
            yr[tid] = y.x;
            yi[tid] = y.y;
        }
        __syncthreads();
        const int wrow = r0 + wave * 16;
        if (wrow >= j0 + CN && wrow < M) {
            double2 cf[CN / 4];
            {
                const int row = wrow + li;
                for (int ks = 0; ks < CN / 4; ++ks)
                    cf[ks] = row < M ? A[(size_t)row * M + jq + ks * 4 + lk] : make_double2(0.0, 0.0);
            }
            v4d xr[4], xi[4];
            for (int v = 0; v < 4; ++v) {
                xr[v] = (v4d){0.0, 0.0, 0.0, 0.0};
                xi[v] = (v4d){0.0, 0.0, 0.0, 0.0};
            }
            // Linv is lower triangular: column block v of Linv^H is zero in the k-steps ks >= 4 v + 4
            for (int ks = 0; ks < CN / 4; ++ks) {
                double fbr[4], fbi[4];
                for (int v = 0; v < 4; ++v) {
                    if (v < (ks >> 2)) continue;
                    fbr[v] = Lr[(v * 16 + li) * CSP + ks * 4 + lk];
                    fbi[v] = Li[(v * 16 + li) * CSP + ks * 4 + lk];
                }
                const double fcr = cf[ks].x, fci = cf[ks].y;
                for (int v = 0; v < 4; ++v) {
                    if (v < (ks >> 2)) continue;
                    xr[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fcr, fbr[v], xr[v], 0, 0, 0);
                    xr[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fci, fbi[v], xr[v], 0, 0, 0);
                    xi[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fci, fbr[v], xi[v], 0, 0, 0);
                    xi[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fcr, -fbi[v], xi[v], 0, 0, 0);
                }
            }
            for (int r = 0; r < 4; ++r) {
                const int row = wrow + lk + 4 * r;
                double sr = 0.0, si = 0.0;
                for (int v = 0; v < 4; ++v) {
                    const int col = v * 16 + li;
                    const double a_ = xr[v][r], b_ = xi[v][r];
                    if (row < M) A[(size_t)row * M + jq + col] = make_double2(a_, b_);
                    sr += a_ * yr[col] - b_ * yi[col];
                    si += a_ * yi[col] + b_ * yr[col];
                }
                for (int o = 1; o < 16; o <<= 1) {
                    sr += __shfl_xor(sr, o, 64);
                    si += __shfl_xor(si, o, 64);
                }
                if (li == 0 && row < M) {
                    const double2 zr = z[row];
                    z[row] = make_double2(zr.x - sr, zr.y - si);
                }
            }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // X is stored before the copies read it
        __syncthreads();
    }
    v4d pre[4], pia[4], pib[4];
    for (int v = 0; v < 4; ++v) {
        pre[v] = (v4d){0.0, 0.0, 0.0, 0.0};
        pia[v] = (v4d){0.0, 0.0, 0.0, 0.0};
        pib[v] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    if (j0 > 0) {
        // copy instruction c (0..5) of this wave: 1 KB = slice rows 4 (6 wave + c) .. +3; lane L
        // takes row 4 (6 wave + c) + L / 16 at LDS piece position L % 16, i.e. the logical piece
        // (L % 16) ^ (row % 16) of that row; slice rows < CR are chunk rows, the rest panel rows
        // (rows past M are read from row M - 1: they only feed outputs that are not stored)
        unsigned voff[6];   // byte offset of this lane's piece within the trajectory's matrix
        for (int c = 0; c < 6; ++c) {
            const int srow = 4 * (6 * wave + c) + (lane >> 4);
            const int grow0 = srow < CR ? r0 + srow : j0 + (srow - CR);
            const int grow = grow0 < M ? grow0 : M - 1;
            voff[c] = (unsigned)(((size_t)grow * M + ((lane & 15) ^ (srow & 15))) * sizeof(double2));
        }
        // The copies are issued from inline assembly (scalar base: the slice's first column,
        // vector offsets fixed for the launch): the compiler then keeps no record of them, and
        // the waits above each slice are the explicit partial ones below (a copy the compiler
        // knew of would make it wait for every outstanding copy before the first LDS read of a
        // slice, which is the whole look-ahead).  M0 holds the wave's LDS destination.
        typedef __attribute__((address_space(3))) void lvoid_t;
#define ZU_COPY(BUF, KC)                                                                          \
        for (int c = 0; c < 6; ++c) {                                                             \
            const unsigned dst = __builtin_amdgcn_readfirstlane(                                  \
                (unsigned)(size_t)(lvoid_t *)(sl + (BUF) * ZU_SLICE + 64 * (6 * wave + c)));      \
            asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"                      \
                         :: "v"(voff[c]), "s"(A + (KC)), "s"(dst) : "memory", "m0");              \
        }
        const int nk = j0 / ZK;
        ZU_COPY(0, 0)
        if (nk > 1) ZU_COPY(1, ZK)
        const int arow = wave * 16 + li;
        for (int k = 0; k < nk; ++k) {
            // this wave's part of slice k has landed once at most the six copies of slice k + 1
            // are outstanding; the barrier then makes every wave's part visible, and also
            // certifies that every wave has finished reading slice k - 1, whose buffer the copy
            // of slice k + 2 refills
            if (k + 1 < nk)
                asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (k + 2 < nk) ZU_COPY((k + 2) % ZU_STAGES, (k + 2) * ZK)
            const double2 *Sb = sl + (k % ZU_STAGES) * ZU_SLICE;
            for (int ks = 0; ks < ZK / 4; ++ks) {
                const int p = ks * 4 + lk;
                const double2 fa = Sb[arow * ZK + (p ^ (arow & 15))];
                double2 fb[4];
                for (int v = 0; v < 4; ++v) {
                    const int brow = CR + v * 16 + li;
                    fb[v] = Sb[brow * ZK + (p ^ (brow & 15))];
                }
                for (int v = 0; v < 4; ++v) {
                    pre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x, fb[v].x, pre[v], 0, 0, 0);
                    pia[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.y, fb[v].x, pia[v], 0, 0, 0);
                }
                for (int v = 0; v < 4; ++v) {
                    pre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.y, fb[v].y, pre[v], 0, 0, 0);
                    pib[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x, fb[v].y, pib[v], 0, 0, 0);
                }
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // this wave's reads of slice k are done
        }
#undef ZU_COPY
    }
    double2 cv[4][4];   // every load of C issued before the first subtraction waits for one
    for (int v = 0; v < 4; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            cv[v][r] = (r0 + row < M && col < jb) ? A[(size_t)(r0 + row) * M + j0 + col] : make_double2(0.0, 0.0);
        }
    for (int v = 0; v < 4; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            if (r0 + row < M && col < jb)
                A[(size_t)(r0 + row) * M + j0 + col] =
                    make_double2(cv[v][r].x - pre[v][r], cv[v][r].y - (pia[v][r] - pib[v][r]));
        }
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {   // a conj(b)
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// One workgroup of ZD threads per trajectory factors the 64 x 64 diagonal block in blocks of
// ZDB = 16 columns (right-looking): one wavefront factors a 16 x 16 diagonal block in registers,
// the rows below it solve for their part of the block column (one lane per row, forward
// substitution), and the workgroup applies the trailing update.  Then the inverse: the four
// diagonal blocks at once (a wavefront each), the off-diagonal blocks by block rows,
// Linv_ij = -Linv_ii sum_{j <= k < i} L_ik Linv_kj.  About twenty workgroup barriers in all,
// against one per column for a column-by-column factor; the serial chain is the 16 steps of
// each diagonal block and the substitution below it.
constexpr int ZD = 1024;
constexpr int ZDB = 16;

__device__ __forceinline__ double2 zshfl(double2 v, int src) {
    return make_double2(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}

// v from lane SEL of each quad of lanes, to all four
template <int SEL>
__device__ __forceinline__ double2 zquad_bcast_t(double2 v) {
    return make_double2(dpp_d<SEL * 0x55, 0xF>(v.x, v.x), dpp_d<SEL * 0x55, 0xF>(v.y, v.y));
}
__device__ __forceinline__ double2 zquad_bcast(double2 v, int sel) {
    switch (sel) {
    case 0: return zquad_bcast_t<0>(v);
    case 1: return zquad_bcast_t<1>(v);
    case 2: return zquad_bcast_t<2>(v);
    default: return zquad_bcast_t<3>(v);
    }
}

// The 16 x 16 diagonal block at (o, o) of Cs (already updated by the blocks to its left),
// factored by one wavefront: lane (r, q) = (lane / 4, lane % 4) holds columns q, q + 4, q + 8,
// q + 12 of row r.  Step c scales column c by 1 / sqrt(C_cc) (the hardware's reciprocal square
// root and two Newton steps) and subtracts L_rc conj(L_kc) from the columns k > c: L_rc comes
// from the lane's own quad, L_kc from lane (k, c % 4).  Column c + 1, which holds the next
// pivot, is updated first from the one value L_{c+1,c} it needs, so the next step's chain does
// not wait for the moves of the other columns.  L goes over the block's lower triangle in Cs,
// the reciprocals of its diagonal into dinv.  Returns true on lanes that saw a pivot that is not
// positive.
__device__ __forceinline__ bool zdiag_block16(double2 *Cs, double *dinv, int o, int lane) {
    asm volatile("" : "+v"(lane));   // keeps the lane masks of the unrolled steps inside the caller's loop
    const int r = lane >> 2, q = lane & 3;
    double2 a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = q + 4 * s;
        a[s] = c <= r ? Cs[(o + r) * CSP + o + c] : make_double2(0.0, 0.0);
    }
    bool bad = false;
#pragma unroll
    for (int c = 0; c < ZDB; ++c) {
        const double piv = readlane_d(a[c >> 2].x, c * 4 + (c & 3));
        bad |= !(piv > 0.0);
        double y = __builtin_amdgcn_rsq(piv);
        y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
        y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
        const double d = piv * y;
        if (lane == 0) dinv[o + c] = y;
        const double2 lc = make_double2(a[c >> 2].x * y, a[c >> 2].y * y);   // L_rc on lanes q == c % 4
        const double2 lrc = zquad_bcast(lc, c & 3);
        if (c + 1 < ZDB) {
            const int l1 = 4 * (c + 1) + (c & 3);
            const double2 lk = make_double2(readlane_d(lc.x, l1), readlane_d(lc.y, l1));   // L_{c+1,c}
            if (q == ((c + 1) & 3) && r > c) {
                a[(c + 1) >> 2].x -= lrc.x * lk.x + lrc.y * lk.y;
                a[(c + 1) >> 2].y -= lrc.y * lk.x - lrc.x * lk.y;
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {   // C_rk -= L_rc conj(L_kc), c + 1 < k <= r
            const int k = q + 4 * s;
            const double2 lkc = zshfl(lc, k * 4 + (c & 3));
            if (k > c + 1 && k <= r) {
                a[s].x -= lrc.x * lkc.x + lrc.y * lkc.y;
                a[s].y -= lrc.y * lkc.x - lrc.x * lkc.y;
            }
        }
        if (q == (c & 3)) a[c >> 2] = r > c ? lc : (r == c ? make_double2(d, 0.0) : make_double2(0.0, 0.0));
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = q + 4 * s;
        if (c <= r) Cs[(o + r) * CSP + o + c] = a[s];
    }
    return bad;
}

// L^-1 of the factored 16 x 16 diagonal block at (o, o) into the same block of Ls (zeros above
// the diagonal), by one wavefront: lane c < 16 solves L x = e_c down the rows (x_k = 0 above row
// c), x in registers.
__device__ __forceinline__ void zdiag_inv16(const double2 *Cs, double2 *Ls, const double *dinv, int o, int lane) {
    asm volatile("" : "+v"(lane));
    if (lane < ZDB) {
        const int c = lane;
        double2 x[ZDB];
#pragma unroll
        for (int rr = 0; rr < ZDB; ++rr) {
            double sr = rr == c ? 1.0 : 0.0, si = 0.0;
#pragma unroll
            for (int k = 0; k < rr; ++k) {
                const double2 l = Cs[(o + rr) * CSP + o + k];
                sr -= l.x * x[k].x - l.y * x[k].y;
                si -= l.x * x[k].y + l.y * x[k].x;
            }
            const double il = dinv[o + rr];
            x[rr] = make_double2(sr * il, si * il);
            Ls[(o + rr) * CSP + o + c] = x[rr];
        }
    }
}

__global__ __launch_bounds__(ZD) void k_zmw_diag(ZCholArgs a, int j0, int p) {
    __shared__ double2 Cs[CN * CSP];
    __shared__ double2 Ls[CN * CSP];
    __shared__ double2 Ws[(CN / ZDB - 1) * ZDB * ZDB];
    __shared__ double2 ys[CN], zs[CN];
    __shared__ double dinv[CN];
    __shared__ int bad;
    const int t = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int M = a.m;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    const int nblk = (jb + ZDB - 1) / ZDB;
    double2 *A = a.A + (size_t)t * M * M;
    double2 *z = a.x + (size_t)t * M;
    if (tid == 0) bad = 0;
    // rows and columns past jb (the last, ragged panel) are padded with the identity
    for (int e = tid; e < CN * CN; e += ZD) {
        const int r = e / CN, c = e % CN;
        Cs[r * CSP + c] = (r < jb && c <= r) ? A[(size_t)(j0 + r) * M + j0 + c]
                        : make_double2(r == c ? 1.0 : 0.0, 0.0);
        if (c / ZDB > r / ZDB) Ls[r * CSP + c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
        const int o = b * ZDB;
        if (wave == 0 && zdiag_block16(Cs, dinv, o, lane)) bad = 1;
        __syncthreads();
        const int n = CN - o - ZDB;   // rows below the block (padding included)
        if (b + 1 == nblk || n <= 0) break;
        // L[r, block] L_bb^H = C[r, block]: forward substitution along the row, one lane per row
        for (int e = tid; e < n; e += ZD) {
            const int r = o + ZDB + e;
            double2 x[ZDB];
#pragma unroll
            for (int c = 0; c < ZDB; ++c) {
                double2 v = Cs[r * CSP + o + c];
#pragma unroll
                for (int k = 0; k < c; ++k) {   // v -= x_k conj(L_ck)
                    const double2 l = Cs[(o + c) * CSP + o + k];
                    v.x -= x[k].x * l.x + x[k].y * l.y;
                    v.y -= x[k].y * l.x - x[k].x * l.y;
                }
                const double il = dinv[o + c];
                x[c] = make_double2(v.x * il, v.y * il);
            }
#pragma unroll
            for (int c = 0; c < ZDB; ++c) Cs[r * CSP + o + c] = x[c];
        }
        __syncthreads();
        // trailing update C[r, k] -= L[r, block] L[k, block]^H, o + 16 <= k <= r
        for (int e = tid; e < n * n; e += ZD) {
            const int rr = e / n, kk = e % n;
            if (kk > rr) continue;
            const int r = o + ZDB + rr, k = o + ZDB + kk;
            double sr = 0.0, si = 0.0;
#pragma unroll 4
            for (int m = 0; m < ZDB; ++m) {
                const double2 u = Cs[r * CSP + o + m], v = Cs[k * CSP + o + m];
                sr += u.x * v.x + u.y * v.y;
                si += u.y * v.x - u.x * v.y;
            }
            const double2 cv = Cs[r * CSP + k];
            Cs[r * CSP + k] = make_double2(cv.x - sr, cv.y - si);
        }
        __syncthreads();
    }
    if (tid == 0 && bad) a.flags[t] = 1;
    for (int e = tid; e < jb * jb; e += ZD) {
        const int r = e / jb, c = e % jb;
        if (c <= r) A[(size_t)(j0 + r) * M + j0 + c] = Cs[r * CSP + c];
    }
    // the diagonal blocks of Linv, one wavefront each, then the off-diagonal blocks by block rows
    if (wave < nblk) zdiag_inv16(Cs, Ls, dinv, wave * ZDB, lane);
    __syncthreads();
    for (int i = 1; i < nblk; ++i) {
        for (int e = tid; e < i * ZDB * ZDB; e += ZD) {   // W_ij = sum_{j <= k < i} L_ik Linv_kj
            const int j = e / (ZDB * ZDB), c = (e / ZDB) % ZDB, r = e % ZDB;
            double sr = 0.0, si = 0.0;
#pragma unroll 8
            for (int m = j * ZDB; m < i * ZDB; ++m) {
                const double2 l = Cs[(i * ZDB + r) * CSP + m], v = Ls[m * CSP + j * ZDB + c];
                sr += l.x * v.x - l.y * v.y;
                si += l.x * v.y + l.y * v.x;
            }
            Ws[(j * ZDB + r) * ZDB + c] = make_double2(sr, si);
        }
        __syncthreads();
        for (int e = tid; e < i * ZDB * ZDB; e += ZD) {   // Linv_ij = -Linv_ii W_ij
            const int j = e / (ZDB * ZDB), c = (e / ZDB) % ZDB, r = e % ZDB;
            double sr = 0.0, si = 0.0;
#pragma unroll 4
            for (int m = 0; m < ZDB; ++m) {
                const double2 l = Ls[(i * ZDB + r) * CSP + i * ZDB + m], w = Ws[(j * ZDB + m) * ZDB + c];
                sr += l.x * w.x - l.y * w.y;
                si += l.x * w.y + l.y * w.x;
            }
            Ls[(i * ZDB + r) * CSP + j * ZDB + c] = make_double2(-sr, -si);
        }
        __syncthreads();
    }
    if (tid < jb) zs[tid] = z[j0 + tid];
    __syncthreads();
    if (tid < jb) {   // y = Linv z_panel
        double sr = 0.0, si = 0.0;
#pragma unroll 8
        for (int k = 0; k <= tid; ++k) {
            const double2 pr = zmul(Ls[tid * CSP + k], zs[k]);
            sr += pr.x;
            si += pr.y;
        }
        ys[tid] = make_double2(sr, si);
    }
    double2 *lv = a.linv + ((size_t)t * chol_panels(M) + p) * CN * CN;
    for (int e = tid; e < CN * CN; e += ZD) {
        const int r = e / CN, c = e % CN;
        lv[e] = (r < jb && c < jb) ? Ls[r * CSP + c] : make_double2(0.0, 0.0);
    }
    // the next panel's rows (the first CN rows below the block): L[r, panel] = C[r, panel]
    // Linv^H over C and z[r] -= L[r, panel] y; the update kernel of the next panel does the
    // TRSM of the rows below those.  Thread (fr, fs): row fr, columns fs, fs + 16, fs + 32, fs + 48
    // (Linv is zero above its diagonal, so column block q needs the k blocks up to q).
    const int nr0 = j0 + jb, nrb = (M - nr0) < CN ? (M - nr0) : CN;
    if (nrb > 0) {
        for (int e = tid; e < nrb * CN; e += ZD) {
            const int r = e / CN, c = e % CN;
            Cs[r * CSP + c] = A[(size_t)(nr0 + r) * M + j0 + c];
        }
        __syncthreads();
        const int fr = tid >> 4, fs = tid & 15;
        double sr = 0.0, si = 0.0;
        if (fr < nrb) {
            double2 x[CN / ZDB];
#pragma unroll
            for (int q = 0; q < CN / ZDB; ++q) x[q] = make_double2(0.0, 0.0);
#pragma unroll
            for (int kb = 0; kb < CN / ZDB; ++kb)
#pragma unroll 4
                for (int k = kb * ZDB; k < kb * ZDB + ZDB; ++k) {
                    const double2 cv = Cs[fr * CSP + k];
#pragma unroll
                    for (int q = kb; q < CN / ZDB; ++q) {   // sum_k C_rk conj(Linv_ck)
                        const double2 l = Ls[(fs + ZDB * q) * CSP + k];
                        x[q].x += cv.x * l.x + cv.y * l.y;
                        x[q].y += cv.y * l.x - cv.x * l.y;
                    }
                }
#pragma unroll
            for (int q = 0; q < CN / ZDB; ++q) {
                const int c = fs + ZDB * q;
                A[(size_t)(nr0 + fr) * M + j0 + c] = x[q];
                const double2 xy = zmul(x[q], ys[c]);
                sr += xy.x;
                si += xy.y;
            }
        }
        for (int o = 1; o < 16; o <<= 1) {
            sr += __shfl_xor(sr, o, 64);
            si += __shfl_xor(si, o, 64);
        }
        if (fs == 0 && fr < nrb) {
            const double2 zr = z[nr0 + fr];
            z[nr0 + fr] = make_double2(zr.x - sr, zr.y - si);
        }
    }
    __syncthreads();
    if (tid < jb) z[j0 + tid] = ys[tid];
}

// L^H x = y by row panels, last panel first, one launch per panel p (then a closing launch
// p = -1).  w starts as y (in x) and, once every panel below p has been applied, w_p = y_p -
// sum_{r below} conj(L_rp) x_r, so x_p = Linv_p^H w_p.  Launch p: every workgroup forms x_p
// and subtracts conj(L[rows of p][c]) x_p from w_c for its chunk of ZB_COLS columns c < j0 (one
// column per thread, the panel's rows read row by row, coalesced); workgroup 0 also writes
// x_{p+1} over w_{p+1}, which no workgroup of launch p reads.  The closing launch writes x_0
// and flags non-finite solutions.
constexpr int ZB_COLS = 256;
// x = Linv^H w for one panel, by the whole workgroup: thread (c, g) = (tid % 64, tid / 64) sums
// conj(Linv_kc) w_k over the rows k = g, g + 4, ... of the stored inverse (zero above its
// diagonal; a row is 64 contiguous entries, so each step is one coalesced read per wavefront),
// and the four partial sums meet in LDS.  w in LDS (ws); x into xs.
__device__ __forceinline__ void zbwd_x(const double2 *__restrict__ lv, const double2 *ws, double2 *part, double2 *xs,
                                       int jb, int tid) {
    const int c = tid & (CN - 1), g = tid >> 6;
    double xr = 0.0, xi = 0.0;
#pragma unroll 4
    for (int k = g; k < jb; k += ZB_COLS / CN) {
        const double2 l = lv[k * CN + c], w = ws[k];
        xr += l.x * w.x + l.y * w.y;
        xi += l.x * w.y - l.y * w.x;
    }
    part[tid] = make_double2(xr, xi);
    __syncthreads();
    if (tid < jb) {
        double2 s = part[tid];
        for (int q = 1; q < ZB_COLS / CN; ++q) {
            s.x += part[tid + q * CN].x;
            s.y += part[tid + q * CN].y;
        }
        xs[tid] = s;
    }
}

__global__ __launch_bounds__(ZB_COLS) void k_zmw_bwd(ZCholArgs a, int p) {
    __shared__ double2 ws[CN], xs[CN], part[ZB_COLS];
    const int t = blockIdx.y, tid = threadIdx.x;
    const int M = a.m, np = chol_panels(M);
    const double2 *A = a.A + (size_t)t * M * M;
    const double2 *linv = a.linv + (size_t)t * np * CN * CN;
    double2 *z = a.x + (size_t)t * M;
    if (blockIdx.x == 0 && p + 1 < np) {   // x_{p+1} over w_{p+1}
        const int j1 = (p + 1) * CN, jb1 = min(CN, M - j1);
        if (tid < jb1) ws[tid] = z[j1 + tid];
        __syncthreads();
        zbwd_x(linv + (size_t)(p + 1) * CN * CN, ws, part, xs, jb1, tid);
        __syncthreads();
        if (tid < jb1) z[j1 + tid] = xs[tid];
        __syncthreads();
    }
    if (p < 0) {   // every thread scans a share of the solution for non-finite entries
        int nf = 0;
        for (int i = tid; i < M; i += ZB_COLS) nf |= !isfinite(z[i].x) || !isfinite(z[i].y);
        nf = __syncthreads_or(nf);
        if (tid == 0 && nf) a.flags[t] = 1;
        return;
    }
    const int j0 = p * CN, jb = min(CN, M - j0);
    if (tid < jb) ws[tid] = z[j0 + tid];
    __syncthreads();
    zbwd_x(linv + (size_t)p * CN * CN, ws, part, xs, jb, tid);
    __syncthreads();
    const int c = blockIdx.x * ZB_COLS + tid;
    if (c < j0) {
        double sr = 0.0, si = 0.0;
        const double2 *col = A + (size_t)j0 * M + c;
#pragma unroll 16
        for (int r = 0; r < jb; ++r) {
            const double2 l = col[(size_t)r * M], x = xs[r];
            sr += l.x * x.x + l.y * x.y;   // conj(l) x
            si += l.x * x.y - l.y * x.x;
        }
        z[c] = make_double2(z[c].x - sr, z[c].y - si);
    }
}

}  // namespace tvmc
