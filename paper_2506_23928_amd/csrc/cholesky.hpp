// Regularised solve (S + eps I) delta = D in FP64 (the solve of the paragraph after Eq. 9).
//
// One workgroup per trajectory factors its own matrix: left-looking blocked Cholesky with
// NB-column panels.  Panel j is first updated with the already-factored columns (a GEMM
// staged through LDS), then its diagonal block is factored in LDS and the rows below are
// solved against it.  The forward substitution L y = D runs panel by panel alongside the
// factorisation (column-oriented), the backward substitution L^T x = y afterwards.
// The real factor of the Jastrow S is applied to the real and imaginary parts of D.
#pragma once
#include "common.hpp"

namespace tvmc {

constexpr int CH_NB = 32;

__global__ __launch_bounds__(256) void k_chol_solve(Dev a, int which) {
    __shared__ double As[64][CH_NB + 1];
    __shared__ double Bs[CH_NB][CH_NB + 1];
    __shared__ double Ld[CH_NB][CH_NB + 1];
    __shared__ double yre[CH_NB], yim[CH_NB];
    __shared__ double red[32][2 * CH_NB + 1];
    __shared__ int bad;
    const int t = blockIdx.x, tid = threadIdx.x;
    const int M = a.m;
    double *A = a.S + (size_t)t * M * M;
    double2 *z = (which ? a.d1 : a.d0) + (size_t)t * M;
    const double2 *Dv = a.D + (size_t)t * M;
    if (tid == 0) bad = 0;
    for (int i = tid; i < M; i += 256) z[i] = Dv[i];
    __syncthreads();

    for (int j0 = 0; j0 < M; j0 += CH_NB) {
        const int jb = (M - j0) < CH_NB ? (M - j0) : CH_NB;
        // 1. panel update: A[j0:M, j0:j0+jb] -= L[j0:M, 0:j0] L[j0:j0+jb, 0:j0]^T
        if (j0 > 0) {
            const int ty = tid >> 3, tx = tid & 7;
            for (int r0 = j0; r0 < M; r0 += 64) {
                double acc[2][4] = {};
                for (int k0 = 0; k0 < j0; k0 += CH_NB) {
                    for (int e = tid; e < 64 * CH_NB; e += 256) {
                        const int rr = e / CH_NB, kk = e % CH_NB;
                        As[rr][kk] = (r0 + rr < M) ? A[(size_t)(r0 + rr) * M + k0 + kk] : 0.0;
                    }
                    for (int e = tid; e < CH_NB * CH_NB; e += 256) {
                        const int cc = e / CH_NB, kk = e % CH_NB;
                        Bs[cc][kk] = (cc < jb) ? A[(size_t)(j0 + cc) * M + k0 + kk] : 0.0;
                    }
                    __syncthreads();
                    for (int kk = 0; kk < CH_NB; ++kk) {
                        const double a0 = As[2 * ty][kk], a1 = As[2 * ty + 1][kk];
                        for (int q = 0; q < 4; ++q) {
                            const double b = Bs[4 * tx + q][kk];
                            acc[0][q] += a0 * b;
                            acc[1][q] += a1 * b;
                        }
                    }
                    __syncthreads();
                }
                for (int u = 0; u < 2; ++u) {
                    const int r = r0 + 2 * ty + u;
                    if (r >= M) continue;
                    for (int q = 0; q < 4; ++q) {
                        const int cc = 4 * tx + q;
                        if (cc < jb) A[(size_t)r * M + j0 + cc] -= acc[u][q];
                    }
                }
            }
            __syncthreads();
        }
        // 2. factor the diagonal block in LDS
        for (int e = tid; e < CH_NB * CH_NB; e += 256) {
            const int r = e / CH_NB, cc = e % CH_NB;
            Ld[r][cc] = (r < jb && cc <= r) ? A[(size_t)(j0 + r) * M + j0 + cc] : 0.0;
        }
        __syncthreads();
        for (int cc = 0; cc < jb; ++cc) {
            if (tid == 0) {
                const double d = Ld[cc][cc];
                if (!(d > 0.0)) bad = 1;
                Ld[cc][cc] = sqrt(d);
            }
            __syncthreads();
            for (int r = cc + 1 + tid; r < jb; r += 256) Ld[r][cc] /= Ld[cc][cc];
            __syncthreads();
            for (int e = tid; e < CH_NB * CH_NB; e += 256) {
                const int r = e / CH_NB, k = e % CH_NB;
                if (k > cc && r >= k && r < jb) Ld[r][k] -= Ld[r][cc] * Ld[k][cc];
            }
            __syncthreads();
        }
        for (int e = tid; e < CH_NB * CH_NB; e += 256) {
            const int r = e / CH_NB, cc = e % CH_NB;
            if (r < jb && cc <= r) A[(size_t)(j0 + r) * M + j0 + cc] = Ld[r][cc];
        }
        // forward substitution for this block: y_j = L_jj^{-1} z_j
        if (tid == 0) {
            for (int r = 0; r < jb; ++r) {
                double vr = z[j0 + r].x, vi = z[j0 + r].y;
                for (int k = 0; k < r; ++k) {
                    vr -= Ld[r][k] * yre[k];
                    vi -= Ld[r][k] * yim[k];
                }
                yre[r] = vr / Ld[r][r];
                yim[r] = vi / Ld[r][r];
                z[j0 + r] = make_double2(yre[r], yim[r]);
            }
        }
        __syncthreads();
        // 3. rows below: L[r, panel] = A[r, panel] L_jj^{-T}; z_r -= L[r, panel] y_j
        for (int r = j0 + jb + tid; r < M; r += 256) {
            double x[CH_NB];
            for (int cc = 0; cc < jb; ++cc) x[cc] = A[(size_t)r * M + j0 + cc];
            double zr = z[r].x, zi = z[r].y;
            for (int cc = 0; cc < jb; ++cc) {
                double v = x[cc];
                for (int k = 0; k < cc; ++k) v -= x[k] * Ld[cc][k];
                x[cc] = v / Ld[cc][cc];
                A[(size_t)r * M + j0 + cc] = x[cc];
                zr -= x[cc] * yre[cc];
                zi -= x[cc] * yim[cc];
            }
            z[r] = make_double2(zr, zi);
        }
        __syncthreads();
    }

    // backward substitution L^T x = y (z holds y; overwritten by x from the last block up)
    const int nblk = (M + CH_NB - 1) / CH_NB;
    for (int b = nblk - 1; b >= 0; --b) {
        const int j0 = b * CH_NB;
        const int jb = (M - j0) < CH_NB ? (M - j0) : CH_NB;
        const int cg = tid & 7, rl = tid >> 3;   // 8 column groups of 4, 32 row lanes
        double pr[4] = {}, pi[4] = {};
        for (int r = j0 + jb + rl; r < M; r += 32) {
            const double2 xr = z[r];
            for (int q = 0; q < 4; ++q) {
                const int cc = 4 * cg + q;
                if (cc < jb) {
                    const double l = A[(size_t)r * M + j0 + cc];
                    pr[q] += l * xr.x;
                    pi[q] += l * xr.y;
                }
            }
        }
        for (int q = 0; q < 4; ++q) {
            red[rl][2 * (4 * cg + q)] = pr[q];
            red[rl][2 * (4 * cg + q) + 1] = pi[q];
        }
        for (int e = tid; e < CH_NB * CH_NB; e += 256) {
            const int r = e / CH_NB, cc = e % CH_NB;
            Ld[r][cc] = (r < jb && cc <= r) ? A[(size_t)(j0 + r) * M + j0 + cc] : 0.0;
        }
        __syncthreads();
        if (tid < jb) {
            double sr = 0.0, si = 0.0;
            for (int l = 0; l < 32; ++l) {
                sr += red[l][2 * tid];
                si += red[l][2 * tid + 1];
            }
            yre[tid] = z[j0 + tid].x - sr;
            yim[tid] = z[j0 + tid].y - si;
        }
        __syncthreads();
        if (tid == 0) {
            for (int cc = jb - 1; cc >= 0; --cc) {
                double vr = yre[cc], vi = yim[cc];
                for (int k = cc + 1; k < jb; ++k) {
                    vr -= Ld[k][cc] * yre[k];
                    vi -= Ld[k][cc] * yim[k];
                }
                yre[cc] = vr / Ld[cc][cc];
                yim[cc] = vi / Ld[cc][cc];
                z[j0 + cc] = make_double2(yre[cc], yim[cc]);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        int nf = bad;
        for (int i = 0; i < M && !nf; ++i)
            if (!isfinite(z[i].x) || !isfinite(z[i].y)) nf = 1;
        if (nf) a.flags[t] = 1;
    }
}

}  // namespace tvmc
