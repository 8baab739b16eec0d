// Regularised solve (S + eps I) delta = D in FP64 with several workgroups per trajectory, for
// batches too small to fill the device with one workgroup per trajectory.  The factorisation
// is the same left-looking panel algorithm as k_chol_solve, split into one launch per step so
// that the row chunks of a panel run on different compute units:
//   k_cmw_update(j0):  C[rows, panel] = A[rows, panel] - L[rows, 0:j0] L[panel, 0:j0]^T
//                      (every chunk of CR rows at or below the panel; FP64 MFMA)
//   k_cmw_diag(j0):    factor the diagonal block, invert it (Linv), forward substitution of
//                      the panel's part of the right-hand side (one workgroup per trajectory)
//   k_cmw_trsm(j0):    L[rows, panel] = C Linv^T for the chunks below, and the right-hand side
//                      update z[rows] -= L[rows, panel] y_panel
//   k_cmw_backward:    backward substitution L^T x = y with the stored block inverses.
// k_cmw_update_lds and k_cmw_diag(.., next > 0) are the form the host takes when a trajectory's
// matrix is under 4 GiB: the update copies its operand slices straight into LDS and first does
// the previous panel's TRSM of its rows below those the diagonal kernel did, and the diagonal
// kernel does the TRSM of the next CN or 2 CN rows, so k_cmw_trsm drops out; panels go in
// pairs (one 128-column update over [0, j0), one 64-column update over the first panel).
#pragma once
#include "cholesky.hpp"

namespace tvmc {

__global__ __launch_bounds__(256) void k_cmw_init(CholArgs a) {
    const int t = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < a.m) a.x[(size_t)t * a.m + i] = a.rhs[(size_t)t * a.m + i];
}

__global__ __launch_bounds__(256) void k_cmw_update(CholArgs a, int j0) {
    __shared__ double As[CR * CKP];
    __shared__ double Bs[CN * CKP];
    const int t = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    const int r0 = j0 + blockIdx.x * CR;
    if (r0 >= M) return;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    double *A = a.A + (size_t)t * M * M;
    v4d acc[2][4];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 4; ++v)
            for (int r = 0; r < 4; ++r) {
                const int row = wave * 32 + u * 16 + lk + 4 * r, col = v * 16 + li;
                acc[u][v][r] = (r0 + row < M && col < jb) ? A[(size_t)(r0 + row) * M + j0 + col] : 0.0;
            }
    double pa[CR * CK / 256], pb[CN * CK / 256];
    auto fetch = [&](int kc) {
        for (int q = 0; q < CR * CK / 256; ++q) {
            const int e = tid + 256 * q, rr = e / CK, kk = e % CK;
            pa[q] = (r0 + rr < M) ? A[(size_t)(r0 + rr) * M + kc + kk] : 0.0;
        }
        for (int q = 0; q < CN * CK / 256; ++q) {
            const int e = tid + 256 * q, cc = e / CK, kk = e % CK;
            pb[q] = (cc < jb) ? A[(size_t)(j0 + cc) * M + kc + kk] : 0.0;
        }
    };
    fetch(0);
    for (int kc = 0; kc < j0; kc += CK) {
        __syncthreads();
        for (int q = 0; q < CR * CK / 256; ++q) {
            const int e = tid + 256 * q;
            As[(e / CK) * CKP + e % CK] = -pa[q];
        }
        for (int q = 0; q < CN * CK / 256; ++q) {
            const int e = tid + 256 * q;
            Bs[(e / CK) * CKP + e % CK] = pb[q];
        }
        __syncthreads();
        if (kc + CK < j0) fetch(kc + CK);
        for (int ks = 0; ks < CK / 4; ++ks) {
            double fa[2], fb[4];
            for (int u = 0; u < 2; ++u) fa[u] = As[(wave * 32 + u * 16 + li) * CKP + ks * 4 + lk];
            for (int v = 0; v < 4; ++v) fb[v] = Bs[(v * 16 + li) * CKP + ks * 4 + lk];
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 4; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[v], acc[u][v], 0, 0, 0);
        }
    }
    // every read of the panel columns above happened before the last barrier of the k loop
    // or belongs to this workgroup's own rows; chunks of other workgroups are disjoint
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 4; ++v)
            for (int r = 0; r < 4; ++r) {
                const int row = wave * 32 + u * 16 + lk + 4 * r, col = v * 16 + li;
                if (r0 + row < M && col < jb) A[(size_t)(r0 + row) * M + j0 + col] = acc[u][v][r];
            }
}

// The update with the operand slices copied from global memory straight into LDS, with partial
// waits and one barrier per slice (as the complex k_zmw_update_lds), for NC = 64 or 128 output
// columns j0 .. j0 + NC - 1 and the k range [k0, j0):
//   C[rows, cols] = A[rows, cols] - L[rows, k0:j0] L[cols, k0:j0]^T.
// A slice is CW = 32 columns of k, CR chunk rows and NC panel rows of 256 bytes, the 16-byte
// pieces of row r at position piece ^ (r & 15); three slices deep for NC = 64, two for NC = 128
// (a slice of 64 KB: the products of one cover the copy of the next).  Lane (li, lk) reads the
// pieces lk, lk + 4, lk + 8, lk + 12 of its row (16 bytes each, the same bank-conflict-free
// pattern as the complex update) and feeds their 8 columns to 8 products: the k order of a slice
// is permuted the same way for both operands, which the sum does not see.  Before the update,
// the previous panel pp's TRSM of this chunk's rows from j0 + skip on: X = C Linv_pp^T over C,
// z[rows] -= X y_pp (the diagonal kernel of panel pp did the rows before; skip = CN or 2 CN).
// The product accumulates from zero and C = A - P at the end.  NC = 128 halves the reads of
// L[rows, 0:j0] per column factored: the host pairs panels, one wide update over [0, j0) and a
// narrow one of the second panel over the first panel's columns.
constexpr int CW = 32;
constexpr int CUT = 512;   // 8 waves, 16 rows of the chunk each
static_assert(CW * 8 == 256 && CUT == 512, "a slice row is 16 pieces of 16 bytes");
template <int NC>
__global__ __launch_bounds__(CUT) void k_cmw_update_lds(CholArgs a, int j0, int pp, int k0, int skip, int nt) {
    constexpr int STAGES = NC == 64 ? 3 : 2;
    constexpr int SLICE = (CR + NC) * CW;               // doubles of one staged slice
    constexpr int COPIES = (CR + NC) * CW * 8 / 8192;   // 1 KB wave copies per wave and slice
    constexpr int NV = NC / 16;                          // 16 x 16 output blocks per wave
    static_assert(STAGES * SLICE * 8 <= 160 * 1024 && STAGES * SLICE >= CN * CSP + 2 * CN, "LDS budget");
    __shared__ __attribute__((aligned(1024))) double sl[STAGES * SLICE];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    int t, chunk;
    if (!chunk_item((M - j0 + CR - 1) / CR, nt, t, chunk)) return;
    const int r0 = j0 + chunk * CR;
    const int jb = (M - j0) < NC ? (M - j0) : NC;
    double *A = a.A + (size_t)t * M * M;
    if (pp >= 0) {
        const int jq = j0 - CN;   // the previous panel's columns (a full panel: another follows it)
        double *Ls = sl, *yr = sl + CN * CSP, *yi = yr + CN;
        double2 *z = a.x + (size_t)t * M;
        const double *lv = a.linv + ((size_t)t * chol_panels(M) + pp) * CN * CN;
        for (int e = tid; e < CN * CN; e += CUT) Ls[(e / CN) * CSP + e % CN] = lv[e];
        if (tid < CN) {
            const double2 y = z[jq + tid];
            yr[tid] = y.x;
            yi[tid] = y.y;
        }
        __syncthreads();
        const int wrow = r0 + wave * 16;
        if (wrow >= j0 + skip && wrow < M) {
            double cf[CN / 4];   // C[row wrow + li][4 ks + lk]
            {
                const int row = wrow + li;
                for (int ks = 0; ks < CN / 4; ++ks) cf[ks] = row < M ? A[(size_t)row * M + jq + ks * 4 + lk] : 0.0;
            }
            v4d x[4];
            for (int v = 0; v < 4; ++v) x[v] = (v4d){0.0, 0.0, 0.0, 0.0};
            for (int ks = 0; ks < CN / 4; ++ks) {
                double fb[4];
                for (int v = 0; v < 4; ++v) fb[v] = v >= (ks >> 2) ? Ls[(v * 16 + li) * CSP + ks * 4 + lk] : 0.0;
                for (int v = 0; v < 4; ++v)   // Linv^T is zero in the k-steps past 4 v + 3
                    if (v >= (ks >> 2)) x[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[ks], fb[v], x[v], 0, 0, 0);
            }
            for (int r = 0; r < 4; ++r) {
                const int row = wrow + lk + 4 * r;
                double sr = 0.0, si = 0.0;
                for (int v = 0; v < 4; ++v) {
                    const int col = v * 16 + li;
                    const double xv = x[v][r];
                    if (row < M) A[(size_t)row * M + jq + col] = xv;
                    sr += xv * yr[col];
                    si += xv * yi[col];
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
    v4d acc[NV];
    for (int v = 0; v < NV; ++v) acc[v] = (v4d){0.0, 0.0, 0.0, 0.0};
    const int nk = (j0 - k0) / CW;
    if (nk > 0) {
        // copy instruction c of this wave: 1 KB = slice rows 4 (COPIES wave + c) .. +3; lane L
        // takes row 4 (COPIES wave + c) + L / 16 at LDS piece position L % 16, i.e. the logical
        // piece (L % 16) ^ (row % 16) of that row; rows < CR are chunk rows, the rest panel rows
        // (rows past M are read from row M - 1: they only feed outputs that are not stored)
        unsigned voff[COPIES];   // byte offset of this lane's piece within the trajectory's matrix
        for (int c = 0; c < COPIES; ++c) {
            const int srow = 4 * (COPIES * wave + c) + (lane >> 4);
            const int grow0 = srow < CR ? r0 + srow : j0 + (srow - CR);
            const int grow = grow0 < M ? grow0 : M - 1;
            voff[c] = (unsigned)(((size_t)grow * M + 2 * ((lane & 15) ^ (srow & 15))) * sizeof(double));
        }
        // issued from inline assembly, so that the compiler keeps no record of the copies and the
        // waits are the explicit partial ones below; M0 holds the wave's LDS destination
        typedef __attribute__((address_space(3))) void lvoid_t;
#define CU_COPY(BUF, KC)                                                                          \
        for (int c = 0; c < COPIES; ++c) {                                                        \
            const unsigned dst = __builtin_amdgcn_readfirstlane(                                  \
                (unsigned)(size_t)(lvoid_t *)(sl + (BUF) * SLICE + 128 * (COPIES * wave + c)));   \
            asm volatile("s_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %0, %1"                      \
                         :: "v"(voff[c]), "s"(A + (KC)), "s"(dst) : "memory", "m0");              \
        }
        for (int k = 0; k < STAGES - 1 && k < nk; ++k) CU_COPY(k, k0 + k * CW)
        const int arow = wave * 16 + li;
        for (int k = 0; k < nk; ++k) {
            // this wave's part of slice k has landed once at most the copies of the slices after
            // it are outstanding; the barrier then makes every wave's part visible, and also
            // certifies that every wave has finished reading slice k - 1, whose buffer the copy
            // of slice k + STAGES - 1 refills
            if (STAGES == 3 && k + 1 < nk)
                asm volatile("s_waitcnt vmcnt(%0)" :: "n"(COPIES) : "memory");
            else
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            if (k + STAGES - 1 < nk) CU_COPY((k + STAGES - 1) % STAGES, k0 + (k + STAGES - 1) * CW)
            const double2 *Sb = (const double2 *)(sl + (k % STAGES) * SLICE);
            for (int h = 0; h < 2; ++h) {   // pieces 4 (2 h + j) + lk, j = 0, 1: steps 4 h .. 4 h + 3
                double2 fa[2], fb[NV][2];
                for (int j = 0; j < 2; ++j) {
                    const int q = 4 * (2 * h + j) + lk;
                    fa[j] = Sb[arow * 16 + (q ^ (arow & 15))];
                    for (int v = 0; v < NV; ++v) {
                        const int brow = CR + v * 16 + li;
                        fb[v][j] = Sb[brow * 16 + (q ^ (brow & 15))];
                    }
                }
                for (int j = 0; j < 2; ++j) {
                    for (int v = 0; v < NV; ++v)
                        acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[j].x, fb[v][j].x, acc[v], 0, 0, 0);
                    for (int v = 0; v < NV; ++v)
                        acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[j].y, fb[v][j].y, acc[v], 0, 0, 0);
                }
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // this wave's reads of slice k are done
        }
#undef CU_COPY
    }
    double cv[NV][4];   // every load of C issued before the first subtraction waits for one
    for (int v = 0; v < NV; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            cv[v][r] = (r0 + row < M && col < jb) ? A[(size_t)(r0 + row) * M + j0 + col] : 0.0;
        }
    for (int v = 0; v < NV; ++v)
        for (int r = 0; r < 4; ++r) {
            const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
            if (r0 + row < M && col < jb) A[(size_t)(r0 + row) * M + j0 + col] = cv[v][r] - acc[v][r];
        }
}

// The 64 x 64 diagonal block in blocks of RDB = 16 columns, as the complex kernel does it: one
// wavefront factors each 16 x 16 diagonal block in registers (lane (r, q) = (lane / 4, lane % 4)
// holds columns q, q + 4, q + 8, q + 12 of row r; the pivot by readlane, the row's column value
// by a quad broadcast, 1 / sqrt by the hardware reciprocal square root and two Newton steps,
// the next pivot's column updated first), the rows below solve for their block column by
// forward substitution (a lane per row), the workgroup applies the trailing update; then the
// inverse: the diagonal blocks at once (a wavefront each), the off-diagonal blocks by block rows,
// Linv_ij = -Linv_ii sum_{j <= k < i} L_ik Linv_kj.
__global__ __launch_bounds__(256) void k_cmw_diag(CholArgs a, int j0, int p, int next) {
    __shared__ double Cs[CN * CSP];
    __shared__ double Ls[CN * CSP];
    __shared__ double Ws[(CN / RDB - 1) * RDB * RDB];
    __shared__ double yre[CN], yim[CN], dinv[CN];
    __shared__ double2 zs[CN];
    __shared__ int bad;
    const int t = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int M = a.m;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    const int nblk = (jb + RDB - 1) / RDB;
    double *A = a.A + (size_t)t * M * M;
    double2 *z = a.x + (size_t)t * M;
    if (tid == 0) bad = 0;
    // rows and columns past jb (the last, ragged panel) are padded with the identity
    for (int e = tid; e < CN * CN; e += 256) {
        const int r = e / CN, c = e % CN;
        Cs[r * CSP + c] = (r < jb && c <= r) ? A[(size_t)(j0 + r) * M + j0 + c] : (r == c ? 1.0 : 0.0);
        if (c / RDB > r / RDB) Ls[r * CSP + c] = 0.0;
    }
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
        const int o = b * RDB;
        if (wave == 0 && rdiag_block16(Cs, dinv, o, lane)) bad = 1;
        __syncthreads();
        const int n = CN - o - RDB;   // rows below the block (padding included)
        if (b + 1 == nblk || n <= 0) break;
        // L[r, block] L_bb^T = C[r, block]: forward substitution along the row, a lane per row
        for (int e = tid; e < n; e += 256) {
            const int r = o + RDB + e;
            double x[RDB];
#pragma unroll
            for (int c = 0; c < RDB; ++c) {
                double v = Cs[r * CSP + o + c];
#pragma unroll
                for (int k = 0; k < c; ++k) v -= x[k] * Cs[(o + c) * CSP + o + k];
                x[c] = v * dinv[o + c];
            }
#pragma unroll
            for (int c = 0; c < RDB; ++c) Cs[r * CSP + o + c] = x[c];
        }
        __syncthreads();
        // trailing update C[r, k] -= L[r, block] L[k, block]^T, o + 16 <= k <= r: thread
        // (row rr, phase kq) takes the columns kk = kq, kq + 4, ... of its row
        {
            const int rr = tid >> 2, kq = tid & 3;
            if (rr < n) {
                const int r = o + RDB + rr;
                double acc[(CN - RDB) / 4];
#pragma unroll
                for (int j = 0; j < (CN - RDB) / 4; ++j) acc[j] = 0.0;
#pragma unroll 4
                for (int m = 0; m < RDB; ++m) {
                    const double u = Cs[r * CSP + o + m];
#pragma unroll
                    for (int j = 0; j < (CN - RDB) / 4; ++j) {
                        const int kk = kq + 4 * j;
                        if (kk <= rr) acc[j] += u * Cs[(o + RDB + kk) * CSP + o + m];
                    }
                }
#pragma unroll
                for (int j = 0; j < (CN - RDB) / 4; ++j) {
                    const int kk = kq + 4 * j;
                    if (kk <= rr) Cs[r * CSP + o + RDB + kk] -= acc[j];
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < jb * jb; e += 256) {
        const int r = e / jb, c = e % jb;
        if (c <= r) A[(size_t)(j0 + r) * M + j0 + c] = Cs[r * CSP + c];
    }
    // the diagonal blocks of Linv, a wavefront each, then the off-diagonal blocks by block rows
    if (wave < nblk) rdiag_inv16(Cs, Ls, dinv, wave * RDB, lane);
    __syncthreads();
    for (int i = 1; i < nblk; ++i) {
        for (int e = tid; e < i * RDB * RDB; e += 256) {   // W_ij = sum_{j <= k < i} L_ik Linv_kj
            const int j = e / (RDB * RDB), c = (e / RDB) % RDB, r = e % RDB;
            double s = 0.0;
#pragma unroll 8
            for (int m = j * RDB; m < i * RDB; ++m) s += Cs[(i * RDB + r) * CSP + m] * Ls[m * CSP + j * RDB + c];
            Ws[(j * RDB + r) * RDB + c] = s;
        }
        __syncthreads();
        for (int e = tid; e < i * RDB * RDB; e += 256) {   // Linv_ij = -Linv_ii W_ij
            const int j = e / (RDB * RDB), c = (e / RDB) % RDB, r = e % RDB;
            double s = 0.0;
#pragma unroll 4
            for (int m = 0; m < RDB; ++m) s += Ls[(i * RDB + r) * CSP + i * RDB + m] * Ws[(j * RDB + m) * RDB + c];
            Ls[(i * RDB + r) * CSP + j * RDB + c] = -s;
        }
        __syncthreads();
    }
    if (tid < jb) zs[tid] = z[j0 + tid];
    __syncthreads();
    if (tid < jb) {   // y = Linv z_panel
        double sr = 0.0, si = 0.0;
#pragma unroll 8
        for (int k = 0; k <= tid; ++k) {
            const double l = Ls[tid * CSP + k];
            sr += l * zs[k].x;
            si += l * zs[k].y;
        }
        yre[tid] = sr;
        yim[tid] = si;
    }
    double *lv = a.linv + ((size_t)t * chol_panels(M) + p) * CN * CN;
    for (int e = tid; e < CN * CN; e += 256) {
        const int r = e / CN, c = e % CN;
        lv[e] = (r < jb && c < jb) ? Ls[r * CSP + c] : 0.0;
    }
    if (tid >= jb && tid < CN) {
        yre[tid] = 0.0;
        yim[tid] = 0.0;
    }
    __syncthreads();
    for (int nr0 = j0 + jb; nr0 < j0 + jb + next; nr0 += CN) {
        // the following rows (the first `next` rows below the block, CN at a time): X = C Linv^T
        // over C and z[rows] -= X y; wave w takes rows 16 w .. +15 (the next update does the
        // TRSM of the rows below those)
        const int li = lane & 15, lk = lane >> 4;
        v4d x[4];
        for (int v = 0; v < 4; ++v) x[v] = (v4d){0.0, 0.0, 0.0, 0.0};
        for (int ks = 0; ks < CN / 4; ++ks) {
            double fb[4];
            const int row = nr0 + wave * 16 + li, col = ks * 4 + lk;
            const double fa = (row < M && col < jb) ? A[(size_t)row * M + j0 + col] : 0.0;
            for (int v = 0; v < 4; ++v) fb[v] = v >= (ks >> 2) ? Ls[(v * 16 + li) * CSP + ks * 4 + lk] : 0.0;
            for (int v = 0; v < 4; ++v)   // Linv^T is zero in the k-steps past 4 v + 3
                    if (v >= (ks >> 2)) x[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb[v], x[v], 0, 0, 0);
        }
        __syncthreads();   // every lane has read its C before any lane overwrites it
        for (int r = 0; r < 4; ++r) {
            const int row = nr0 + wave * 16 + lk + 4 * r;
            double sr = 0.0, si = 0.0;
            for (int v = 0; v < 4; ++v) {
                const int col = v * 16 + li;
                const double xv = x[v][r];
                if (row < M && col < jb) A[(size_t)row * M + j0 + col] = xv;
                sr += xv * yre[col];
                si += xv * yim[col];
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
    if (tid < jb) z[j0 + tid] = make_double2(yre[tid], yim[tid]);
    if (tid == 0 && bad) a.flags[t] = 1;
}

// rows below the diagonal block: X = C Linv^T (B[k][j] = Linv[j][k]) and z[rows] -= X y
__global__ __launch_bounds__(256) void k_cmw_trsm(CholArgs a, int j0, int p) {
    __shared__ double Ls[CN * CSP];
    __shared__ double yre[CN], yim[CN];
    const int t = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    const int jb = (M - j0) < CN ? (M - j0) : CN;
    const int r0 = j0 + jb + blockIdx.x * CR;
    if (r0 >= M) return;
    double *A = a.A + (size_t)t * M * M;
    double2 *z = a.x + (size_t)t * M;
    const double *lv = a.linv + ((size_t)t * chol_panels(M) + p) * CN * CN;
    for (int e = tid; e < CN * CN; e += 256) Ls[(e / CN) * CSP + e % CN] = lv[e];
    if (tid < CN) {
        const double2 y = tid < jb ? z[j0 + tid] : make_double2(0.0, 0.0);
        yre[tid] = y.x;
        yim[tid] = y.y;
    }
    __syncthreads();
    v4d x[2][4];
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 4; ++v) x[u][v] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < CN / 4; ++ks) {
        double fa[2], fb[4];
        for (int u = 0; u < 2; ++u) {
            const int row = r0 + wave * 32 + u * 16 + li, col = ks * 4 + lk;
            fa[u] = (row < M && col < jb) ? A[(size_t)row * M + j0 + col] : 0.0;
        }
        for (int v = 0; v < 4; ++v) fb[v] = v >= (ks >> 2) ? Ls[(v * 16 + li) * CSP + ks * 4 + lk] : 0.0;
        for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 4; ++v)   // Linv^T is zero in the k-steps past 4 v + 3
                if (v >= (ks >> 2)) x[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[v], x[u][v], 0, 0, 0);
    }
    // every lane has finished reading C before any lane overwrites it
    __syncthreads();
    for (int u = 0; u < 2; ++u)
        for (int r = 0; r < 4; ++r) {
            const int row = r0 + wave * 32 + u * 16 + lk + 4 * r;
            double sr = 0.0, si = 0.0;
            for (int v = 0; v < 4; ++v) {
                const int col = v * 16 + li;
                const double xv = x[u][v][r];
                if (row < M && col < jb) A[(size_t)row * M + j0 + col] = xv;
                sr += xv * yre[col];
                si += xv * yim[col];
            }
            // sum over the 16 lanes li that hold this row
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

// backward substitution L^T x = y, last panel first; wave w owns 16 panel columns.  Per panel:
// the block inverse is copied to LDS (its loads in flight during the row loop), w_p = y_p -
// sum over the rows below of L[r, panel]^T x_r (each lane walks rows 64 apart, four rows per
// pass), then x_p = Linv_p^T w_p by all 256 threads: thread (c, g) sums the rows k = g, g + 4,
// ... of the inverse (zero above its diagonal) and the four partial sums meet in LDS.
__global__ __launch_bounds__(256) void k_cmw_backward(CholArgs a) {
    __shared__ double yre[CN], yim[CN];
    __shared__ double lvs[CN * CN];
    __shared__ double2 part[256];
    const int t = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int M = a.m;
    const double *A = a.A + (size_t)t * M * M;
    const double *linv = a.linv + (size_t)t * chol_panels(M) * CN * CN;
    double2 *z = a.x + (size_t)t * M;
    for (int p = chol_panels(M) - 1; p >= 0; --p) {
        const int j0 = p * CN, jb = (M - j0) < CN ? (M - j0) : CN;
        {
            const double *lv = linv + (size_t)p * CN * CN;
            double lq[CN * CN / 256];
#pragma unroll
            for (int q = 0; q < CN * CN / 256; ++q) lq[q] = lv[tid + 256 * q];
#pragma unroll
            for (int q = 0; q < CN * CN / 256; ++q) lvs[tid + 256 * q] = lq[q];
        }
        double sr[16], si[16];
        for (int q = 0; q < 16; ++q) sr[q] = si[q] = 0.0;
#pragma unroll 4
        for (int r = j0 + jb + lane; r < M; r += 64) {
            const double2 xr = z[r];
            const double *row = A + (size_t)r * M + j0 + wave * 16;
            for (int q = 0; q < 16; ++q) {
                const double l = (wave * 16 + q < jb) ? row[q] : 0.0;
                sr[q] += l * xr.x;
                si[q] += l * xr.y;
            }
        }
        for (int q = 0; q < 16; ++q) {
            const double tr = wave_sum(sr[q]), ti = wave_sum(si[q]);
            if (lane == 0) {
                const int c = wave * 16 + q;
                yre[c] = c < jb ? z[j0 + c].x - tr : 0.0;
                yim[c] = c < jb ? z[j0 + c].y - ti : 0.0;
            }
        }
        __syncthreads();
        {
            const int c = tid & (CN - 1), g = tid >> 6;
            double xr = 0.0, xi = 0.0;
#pragma unroll 4
            for (int k = g; k < jb; k += 4) {
                const double l = lvs[k * CN + c];
                xr += l * yre[k];
                xi += l * yim[k];
            }
            part[tid] = make_double2(xr, xi);
        }
        __syncthreads();
        if (tid < jb) {
            double2 x = part[tid];
            for (int g = 1; g < 4; ++g) {
                x.x += part[tid + CN * g].x;
                x.y += part[tid + CN * g].y;
            }
            z[j0 + tid] = x;
        }
        __syncthreads();
    }
    int nf = 0;   // a non-finite entry of the solution
    for (int i = tid; i < M; i += 256) nf |= !isfinite(z[i].x) || !isfinite(z[i].y);
    nf = __syncthreads_or(nf);
    if (tid == 0 && nf) a.flags[t] = 1;
}

}  // namespace tvmc
