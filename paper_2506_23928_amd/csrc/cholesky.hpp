// Regularised solve (S + eps I) delta = D in FP64 (the solve of the paragraph after Eq. 9).
//
// One workgroup (8 waves) per trajectory factors its own matrix, left-looking, in panels of
// CN = 64 columns, on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
//   for each panel j and each chunk of CR = 128 rows at or below it:
//     C = A[rows, panel] - L[rows, 0:j] L[panel, 0:j]^T       (MFMA, k-slices of the operands
//                                                              double-buffered through LDS)
//     first chunk: factor the 64x64 diagonal block in LDS and invert it (Linv);
//     rows below:  L[rows, panel] = C Linv^T                  (MFMA)
// The forward substitution L y = D rides along panel by panel; the backward substitution
// L^T x = y afterwards reads L once more and reuses the stored block inverses.
// The real factor of the Jastrow S is applied to the real and imaginary parts of D (the
// complex Hermitian S of the RBM has its own solver, cholesky_z.hpp).
#pragma once
#include "common.hpp"

namespace tvmc {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int CN = 64;        // panel width
constexpr int CR = 128;       // rows per chunk (8 waves x 16 rows)
constexpr int CK = 32;        // k-slice staged through LDS
constexpr int CSP = CN + 1;   // padded LDS row of Cs / Ls
constexpr int CKP = CK + 1;   // padded LDS row of As / Bs
constexpr int CKBUF = (CR + CN) * CKP;   // one k-slice staging buffer: As [CR][CKP] then Bs [CN][CKP]
constexpr int CT1 = 512;      // threads of the one-workgroup solver: 8 waves, 16 rows of a chunk each

// Work item of a panel-update workgroup on a one-dimensional grid padded to a multiple of 8:
// the items (trajectory, row chunk) are numbered trajectory by trajectory; workgroup L runs on
// XCD L % 8 and XCD x takes the items x * per .. x * per + per - 1, so the row chunks of a
// trajectory run on one XCD and share its L2 copy of the panel rows and of the previous panel's
// block inverse.  False for a padding workgroup.
__device__ __forceinline__ bool chunk_item(int nchunk, int nt, int &t, int &chunk) {
    const int per = (int)gridDim.x / 8;
    const int g = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (g >= nchunk * nt) return false;
    t = g / nchunk;
    chunk = g % nchunk;
    return true;
}
static_assert(CN % (2 * CK) == 0, "the update loop takes k-slices in pairs");

__host__ __device__ inline int chol_panels(int m) { return (m + CN - 1) / CN; }

// The 64 x 64 diagonal block of a panel is factored in blocks of RDB = 16 columns (the
// kernels below and the several-workgroup k_cmw_diag): one wavefront per 16 x 16 block.
constexpr int RDB = 16;

template <int SEL>
__device__ __forceinline__ double rquad_bcast_t(double v) { return dpp_d<SEL * 0x55, 0xF>(v, v); }
__device__ __forceinline__ double rquad_bcast(double v, int sel) {
    switch (sel) {
    case 0: return rquad_bcast_t<0>(v);
    case 1: return rquad_bcast_t<1>(v);
    case 2: return rquad_bcast_t<2>(v);
    default: return rquad_bcast_t<3>(v);
    }
}

// L of the 16 x 16 diagonal block at (o, o) of Cs over its lower triangle, the reciprocals of
// its diagonal into dinv; true on lanes that saw a pivot that is not positive.
__device__ __forceinline__ bool rdiag_block16(double *Cs, double *dinv, int o, int lane) {
    asm volatile("" : "+v"(lane));   // keeps the lane masks of the unrolled steps inside the caller's loop
    const int r = lane >> 2, q = lane & 3;
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = q + 4 * s;
        a[s] = c <= r ? Cs[(o + r) * CSP + o + c] : 0.0;
    }
    bool bad = false;
#pragma unroll
    for (int c = 0; c < RDB; ++c) {
        const double piv = readlane_d(a[c >> 2], c * 4 + (c & 3));
        bad |= !(piv > 0.0);
        double y = __builtin_amdgcn_rsq(piv);
        y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
        y = fma(0.5 * y, fma(-piv * y, y, 1.0), y);
        const double d = piv * y;
        if (lane == 0) dinv[o + c] = y;
        const double lc = a[c >> 2] * y;   // L_rc on lanes q == c % 4
        const double lrc = rquad_bcast(lc, c & 3);
        if (c + 1 < RDB) {
            const double lk = readlane_d(lc, 4 * (c + 1) + (c & 3));   // L_{c+1,c}
            if (q == ((c + 1) & 3) && r > c) a[(c + 1) >> 2] -= lrc * lk;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {   // C_rk -= L_rc L_kc, c + 1 < k <= r
            const int k = q + 4 * s;
            const double lkc = __shfl(lc, k * 4 + (c & 3), 64);
            if (k > c + 1 && k <= r) a[s] -= lrc * lkc;
        }
        if (q == (c & 3)) a[c >> 2] = r > c ? lc : (r == c ? d : 0.0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int c = q + 4 * s;
        if (c <= r) Cs[(o + r) * CSP + o + c] = a[s];
    }
    return bad;
}

// L^-1 of the factored 16 x 16 diagonal block at (o, o) into the same block of Ls (zeros above
// the diagonal): lane c < 16 solves L x = e_c down the rows, x in registers.
__device__ __forceinline__ void rdiag_inv16(const double *Cs, double *Ls, const double *dinv, int o, int lane) {
    asm volatile("" : "+v"(lane));
    if (lane < RDB) {
        const int c = lane;
        double x[RDB];
#pragma unroll
        for (int rr = 0; rr < RDB; ++rr) {
            double s = rr == c ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < rr; ++k) s -= Cs[(o + rr) * CSP + o + k] * x[k];
            x[rr] = s * dinv[o + rr];
            Ls[(o + rr) * CSP + o + c] = x[rr];
        }
    }
}

// One real symmetric positive-definite system per trajectory: A [T][M][M] (lower triangle,
// overwritten by L), right-hand sides rhs [T][M] (two real columns packed as double2),
// solution x [T][M], block inverses linv [T][panels][64*64], failure flags [T].
struct CholArgs {
    double *A;
    const double2 *rhs;
    double2 *x;
    double *linv;
    int *flags;
    int m;
};

__global__ __launch_bounds__(CT1) void k_chol_solve(CholArgs a) {
    // the two k-slice staging buffers (As | Bs) and the chunk tile Cs are never live at once
    __shared__ double smem[2 * CKBUF > CR * CSP ? 2 * CKBUF : CR * CSP];
    __shared__ double Ls[CN * CSP];
    __shared__ double yre[CN], yim[CN], dinv[CN];
    __shared__ double Ws[(CN / RDB - 1) * RDB * RDB];
    double *Cs = smem;
    __shared__ int bad;
    const int t = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int M = a.m;
    double *A = a.A + (size_t)t * M * M;
    double *linv = a.linv + (size_t)t * chol_panels(M) * CN * CN;
    double2 *z = a.x + (size_t)t * M;
    const double2 *Dv = a.rhs + (size_t)t * M;
    if (tid == 0) bad = 0;
    for (int i = tid; i < M; i += CT1) z[i] = Dv[i];
    __syncthreads();

    for (int j0 = 0, p = 0; j0 < M; j0 += CN, ++p) {
        const int jb = (M - j0) < CN ? (M - j0) : CN;
        for (int r0 = j0; r0 < M; r0 += CR) {
            // ---- C = A - L[rows, 0:j0] L[panel, 0:j0]^T: the accumulators start from A (FP64
            // accumulator layout: register r of lane (lk, li) holds row lk + 4r, column li) and
            // the row operand is staged negated
            v4d acc[4];
            for (int v = 0; v < 4; ++v)
                for (int r = 0; r < 4; ++r) {
                    const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
                    acc[v][r] = (r0 + row < M && col < jb) ? A[(size_t)(r0 + row) * M + j0 + col] : 0.0;
                }
            if (j0 > 0) {
                // one k-slice in registers: CR*CK/CT1 doubles of the chunk rows, CN*CK/CT1 of
                // the panel rows
                constexpr int QA = CR * CK / CT1, QB = CN * CK / CT1;
                double ra[QA + QB], rb[QA + QB];
                auto fetch = [&](double (&p)[QA + QB], int kc) {
                    for (int q = 0; q < QA; ++q) {
                        const int e = tid + CT1 * q, rr = e / CK, kk = e % CK;
                        p[q] = (r0 + rr < M) ? A[(size_t)(r0 + rr) * M + kc + kk] : 0.0;
                    }
                    for (int q = 0; q < QB; ++q) {
                        const int e = tid + CT1 * q, cc = e / CK, kk = e % CK;
                        p[QA + q] = (cc < jb) ? A[(size_t)(j0 + cc) * M + kc + kk] : 0.0;
                    }
                };
                auto stash = [&](const double (&p)[QA + QB], int buf) {
                    double *As = smem + buf * CKBUF, *Bs = As + CR * CKP;
                    for (int q = 0; q < QA; ++q) {
                        const int e = tid + CT1 * q;
                        As[(e / CK) * CKP + e % CK] = -p[q];
                    }
                    for (int q = 0; q < QB; ++q) {
                        const int e = tid + CT1 * q;
                        Bs[(e / CK) * CKP + e % CK] = p[QA + q];
                    }
                };
                // Slice kc sits in LDS buffer buf and slice kc+CK in `cur` (in flight); slice
                // kc+2CK is fetched into `nxt` before the MFMAs of slice kc, and `cur` is staged
                // after them into the other buffer, whose last readers passed the previous
                // barrier.  Two slices of global loads stay in flight behind the matrix cores.
                auto step = [&](double (&cur)[QA + QB], double (&nxt)[QA + QB], int kc, int buf) {
                    if (kc + 2 * CK < j0) fetch(nxt, kc + 2 * CK);
                    const double *As = smem + buf * CKBUF, *Bs = As + CR * CKP;
                    for (int ks = 0; ks < CK / 4; ++ks) {
                        double fb[4];
                        const double fa = As[(wave * 16 + li) * CKP + ks * 4 + lk];
                        for (int v = 0; v < 4; ++v) fb[v] = Bs[(v * 16 + li) * CKP + ks * 4 + lk];
                        for (int v = 0; v < 4; ++v)
                            acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb[v], acc[v], 0, 0, 0);
                    }
                    if (kc + CK < j0) stash(cur, buf ^ 1);
                    __syncthreads();
                };
                fetch(ra, 0);
                stash(ra, 0);
                fetch(ra, CK);          // j0 is a multiple of CN = 2 CK: the slice count is even
                __syncthreads();
                for (int kc = 0; kc < j0; kc += 2 * CK) {
                    step(ra, rb, kc, 0);
                    step(rb, ra, kc + CK, 1);
                }
            }
            __syncthreads();
            for (int v = 0; v < 4; ++v)
                for (int r = 0; r < 4; ++r) {
                    const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
                    Cs[row * CSP + col] = acc[v][r];
                }
            __syncthreads();
            int rstart = 0;
            if (r0 == j0) {
                // ---- factor the diagonal block in LDS in blocks of 16 columns (rows and columns
                // past jb, the last panel's, padded with the identity): a wavefront factors each
                // 16 x 16 block, the rows below solve for their block column (a lane per row),
                // the workgroup applies the trailing update
                const int nblk = (jb + RDB - 1) / RDB;
                for (int e = tid; e < CN * CN; e += CT1) {
                    const int r = e / CN, c = e % CN;
                    if (r >= jb && c <= r) Cs[r * CSP + c] = r == c ? 1.0 : 0.0;
                    if (c / RDB > r / RDB) Ls[r * CSP + c] = 0.0;
                }
                __syncthreads();
                for (int b = 0; b < nblk; ++b) {
                    const int o = b * RDB;
                    if (wave == 0 && rdiag_block16(Cs, dinv, o, lane)) bad = 1;
                    __syncthreads();
                    const int n = CN - o - RDB;
                    if (b + 1 == nblk || n <= 0) break;
                    for (int e = tid; e < n; e += CT1) {   // L[r, block] L_bb^T = C[r, block]
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
                    {   // C[r, k] -= L[r, block] L[k, block]^T: thread (row rr, phase kq), columns kq + 8 j
                        const int rr = tid >> 3, kq = tid & 7;
                        if (rr < n) {
                            const int r = o + RDB + rr;
                            double acc[(CN - RDB) / 8];
#pragma unroll
                            for (int j = 0; j < (CN - RDB) / 8; ++j) acc[j] = 0.0;
#pragma unroll 4
                            for (int m = 0; m < RDB; ++m) {
                                const double u = Cs[r * CSP + o + m];
#pragma unroll
                                for (int j = 0; j < (CN - RDB) / 8; ++j) {
                                    const int kk = kq + 8 * j;
                                    if (kk <= rr) acc[j] += u * Cs[(o + RDB + kk) * CSP + o + m];
                                }
                            }
#pragma unroll
                            for (int j = 0; j < (CN - RDB) / 8; ++j) {
                                const int kk = kq + 8 * j;
                                if (kk <= rr) Cs[r * CSP + o + RDB + kk] -= acc[j];
                            }
                        }
                    }
                    __syncthreads();
                }
                for (int e = tid; e < jb * jb; e += CT1) {
                    const int r = e / jb, c = e % jb;
                    if (c <= r) A[(size_t)(j0 + r) * M + j0 + c] = Cs[r * CSP + c];
                }
                // ---- Linv: the diagonal blocks at once (a wavefront each), then the
                // off-diagonal blocks by block rows, Linv_ij = -Linv_ii sum_{j <= k < i} L_ik Linv_kj
                if (wave < nblk) rdiag_inv16(Cs, Ls, dinv, wave * RDB, lane);
                __syncthreads();
                for (int i = 1; i < nblk; ++i) {
                    for (int e = tid; e < i * RDB * RDB; e += CT1) {
                        const int j = e / (RDB * RDB), c = (e / RDB) % RDB, r = e % RDB;
                        double sm = 0.0;
#pragma unroll 8
                        for (int m = j * RDB; m < i * RDB; ++m) sm += Cs[(i * RDB + r) * CSP + m] * Ls[m * CSP + j * RDB + c];
                        Ws[(j * RDB + r) * RDB + c] = sm;
                    }
                    __syncthreads();
                    for (int e = tid; e < i * RDB * RDB; e += CT1) {
                        const int j = e / (RDB * RDB), c = (e / RDB) % RDB, r = e % RDB;
                        double sm = 0.0;
#pragma unroll 4
                        for (int m = 0; m < RDB; ++m) sm += Ls[(i * RDB + r) * CSP + i * RDB + m] * Ws[(j * RDB + m) * RDB + c];
                        Ls[(i * RDB + r) * CSP + j * RDB + c] = -sm;
                    }
                    __syncthreads();
                }
                for (int e = tid; e < CN * CN; e += CT1) {   // padding rows and columns of Linv are zero
                    const int r = e / CN, c = e % CN;
                    if (r >= jb || c >= jb) Ls[r * CSP + c] = 0.0;
                }
                __syncthreads();
                // ---- forward substitution of this panel: y = Linv z_panel
                if (tid < jb) {
                    double sr = 0.0, si = 0.0;
                    for (int k = 0; k <= tid; ++k) {
                        const double l = Ls[tid * CSP + k];
                        const double2 zk = z[j0 + k];
                        sr += l * zk.x;
                        si += l * zk.y;
                    }
                    yre[tid] = sr;
                    yim[tid] = si;
                } else if (tid < CN) {
                    yre[tid] = 0.0;
                    yim[tid] = 0.0;
                }
                for (int e = tid; e < CN * CN; e += CT1) linv[(size_t)p * CN * CN + e] = Ls[(e / CN) * CSP + e % CN];
                __syncthreads();
                if (tid < jb) z[j0 + tid] = make_double2(yre[tid], yim[tid]);
                rstart = CN;
            }
            // ---- rows below the diagonal block: X = C Linv^T (B[k][j] = Linv[j][k])
            v4d x[4];
            for (int v = 0; v < 4; ++v) x[v] = (v4d){0.0, 0.0, 0.0, 0.0};
            for (int ks = 0; ks < CN / 4; ++ks) {
                double fb[4];
                const double fa = Cs[(wave * 16 + li) * CSP + ks * 4 + lk];
                for (int v = 0; v < 4; ++v) fb[v] = v >= (ks >> 2) ? Ls[(v * 16 + li) * CSP + ks * 4 + lk] : 0.0;
                for (int v = 0; v < 4; ++v)   // Linv^T is zero in the k-steps past 4 v + 3
                    if (v >= (ks >> 2)) x[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb[v], x[v], 0, 0, 0);
            }
            __syncthreads();
            for (int v = 0; v < 4; ++v)
                for (int r = 0; r < 4; ++r) {
                    const int row = wave * 16 + lk + 4 * r, col = v * 16 + li;
                    if (row >= rstart) Cs[row * CSP + col] = x[v][r];
                }
            __syncthreads();
            const int nrows = (M - r0) < CR ? (M - r0) : CR;
            for (int e = tid; e < (nrows - rstart) * jb; e += CT1) {
                const int rr = rstart + e / jb, c = e % jb;
                A[(size_t)(r0 + rr) * M + j0 + c] = Cs[rr * CSP + c];
            }
            for (int rr = rstart + tid; rr < nrows; rr += CT1) {
                double2 zr = z[r0 + rr];
                for (int c = 0; c < jb; ++c) {
                    const double xv = Cs[rr * CSP + c];
                    zr.x -= xv * yre[c];
                    zr.y -= xv * yim[c];
                }
                z[r0 + rr] = zr;
            }
            __syncthreads();
        }
    }

    // ---- backward substitution L^T x = y, last panel first; wave w owns 8 panel columns
    for (int p = chol_panels(M) - 1; p >= 0; --p) {
        const int j0 = p * CN, jb = (M - j0) < CN ? (M - j0) : CN;
        double sr[8], si[8];
        for (int q = 0; q < 8; ++q) sr[q] = si[q] = 0.0;
        for (int r = j0 + jb + lane; r < M; r += 64) {
            const double2 xr = z[r];
            const double *row = A + (size_t)r * M + j0 + wave * 8;
            for (int q = 0; q < 8; ++q) {
                const double l = (wave * 8 + q < jb) ? row[q] : 0.0;
                sr[q] += l * xr.x;
                si[q] += l * xr.y;
            }
        }
        for (int q = 0; q < 8; ++q) {
            const double tr = wave_sum(sr[q]), ti = wave_sum(si[q]);
            if (lane == 0) {
                const int c = wave * 8 + q;
                yre[c] = c < jb ? z[j0 + c].x - tr : 0.0;
                yim[c] = c < jb ? z[j0 + c].y - ti : 0.0;
            }
        }
        // the block inverse to LDS (the staging space is free after the factorization)
        for (int e = tid; e < jb * CN; e += CT1) smem[e] = linv[(size_t)p * CN * CN + e];
        __syncthreads();
        if (tid < jb) {   // x_c = sum_{k >= c} Linv[k][c] w_k
            double xr = 0.0, xi = 0.0;
            for (int k = tid; k < jb; ++k) {
                const double l = smem[k * CN + tid];
                xr += l * yre[k];
                xi += l * yim[k];
            }
            z[j0 + tid] = make_double2(xr, xi);
        }
        __syncthreads();
    }
    int nf = 0;   // a non-finite entry of the solution
    for (int i = tid; i < M; i += CT1) nf |= !isfinite(z[i].x) || !isfinite(z[i].y);
    nf = __syncthreads_or(nf);
    if (tid == 0 && (nf || bad)) a.flags[t] = 1;
}

}  // namespace tvmc
