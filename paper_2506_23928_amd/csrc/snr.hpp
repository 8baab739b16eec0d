// SNR-regularised solve (the regulariser named in the text after Eq. 9) for a real symmetric S
// (the Jastrow ansaetze; the complex Hermitian S of the RBM at the end of this file): D is written in the eigenbasis of S + eps I and each component
// rho_k = (V^T D)_k is kept with weight 1 / (1 + (tau / SNR_k)^6), the smooth cutoff of Schmitt
// and Heyl's scheme, where SNR_k = |rho_k| sqrt(N_s) / sqrt(<|q_k|^2> - |rho_k|^2) is computed
// from the per-sample contributions q_k(x) = u_k(x) (G(x) - <G>), u_k(x) = sum_l V_lk
// (O_l(x) - <O_l>), whose mean is rho_k.  delta = sum_k V_k keep_k rho_k / lam_k; eigenvalues
// below 1e-14 of the largest are dropped.
//
// Eigen-decomposition: parallel two-sided Jacobi, one workgroup per trajectory, in place on the
// trajectory's S (global memory, L2 / Infinity-Cache resident).  A sweep is M' - 1 rounds of
// M'/2 disjoint rotations (round-robin pairing, M' = M rounded up to even, the odd index out
// paired with a dummy); a round computes every rotation from the current matrix, then applies
// all of them to the rows (A <- J^T A, and to V^T), then to the columns (A <- A J).  Sweeps
// continue until the off-diagonal mass is below 1e-30 of the total.
#pragma once
#include "common.hpp"
#include "cholesky.hpp"   // v4d, the FP64 matrix-core accumulator

namespace tvmc {

constexpr int JAC_THREADS = 1024;
constexpr int JAC_MAXP = 1088;       // rotation pairs per round: M <= 2176
constexpr int JAC_MAX_SWEEPS = 40;

// S + eps I (lower triangle) -> full symmetric matrix; V^T = I
__global__ void k_snr_init(Dev a) {
    const int t = blockIdx.y;
    const size_t mm = (size_t)a.m * a.m;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= mm) return;
    const int i = (int)(idx / a.m), j = (int)(idx % a.m);
    double *S = a.S + (size_t)t * mm;
    if (j > i) S[idx] = S[(size_t)j * a.m + i];
    a.snrV[(size_t)t * mm + idx] = (i == j) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(JAC_THREADS) void k_jacobi(Dev a) {
    __shared__ int sp[JAC_MAXP], sq[JAC_MAXP];
    __shared__ double sc[JAC_MAXP], ss[JAC_MAXP];
    __shared__ double red[JAC_THREADS / 64][2];
    __shared__ int done;
    const int t = blockIdx.x, m = a.m;
    const int mp = m + (m & 1), K = mp - 1, np = mp / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *A = a.S + (size_t)t * m * m;
    double *Vt = a.snrV + (size_t)t * m * m;
    for (int sweep = 0;; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < m * m; e += JAC_THREADS) {
            const double v = A[e];
            tot += v * v;
            if (e / m != e % m) off += v * v;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if (lane == 0) {
            red[wave][0] = off;
            red[wave][1] = tot;
        }
        __syncthreads();
        if (tid == 0) {
            double o = 0.0, s = 0.0;
            for (int w = 0; w < JAC_THREADS / 64; ++w) {
                o += red[w][0];
                s += red[w][1];
            }
            done = (o <= 1e-30 * s) ? 1 : (sweep == JAC_MAX_SWEEPS ? -1 : 0);
        }
        __syncthreads();
        if (done != 0) break;
        for (int r = 0; r < K; ++r) {
            for (int i = tid; i < np; i += JAC_THREADS) {
                int p = i == 0 ? r : (r + i) % K;
                int q = i == 0 ? K : (r - i + K) % K;
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double apq = A[(size_t)p * m + q];
                    if (apq != 0.0) {
                        const double theta = (A[(size_t)q * m + q] - A[(size_t)p * m + p]) / (2.0 * apq);
                        const double tn = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tn * tn + 1.0);
                        s = tn * c;
                    }
                }
                sp[i] = p;
                sq[i] = q;
                sc[i] = c;
                ss[i] = s;
            }
            __syncthreads();
            for (int e = tid; e < np * m; e += JAC_THREADS) {   // rows p, q of A and of V^T
                const int i = e / m, j = e % m, p = sp[i], q = sq[i];
                if (q >= m) continue;
                const double c = sc[i], s = ss[i];
                const double apj = A[(size_t)p * m + j], aqj = A[(size_t)q * m + j];
                A[(size_t)p * m + j] = c * apj - s * aqj;
                A[(size_t)q * m + j] = s * apj + c * aqj;
                const double vpj = Vt[(size_t)p * m + j], vqj = Vt[(size_t)q * m + j];
                Vt[(size_t)p * m + j] = c * vpj - s * vqj;
                Vt[(size_t)q * m + j] = s * vpj + c * vqj;
            }
            __syncthreads();
            for (int e = tid; e < np * m; e += JAC_THREADS) {   // columns p, q of A
                const int i = e % np, k = e / np, p = sp[i], q = sq[i];
                if (q >= m) continue;
                const double c = sc[i], s = ss[i];
                const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                A[(size_t)k * m + p] = c * akp - s * akq;
                A[(size_t)k * m + q] = s * akp + c * akq;
            }
            __syncthreads();
        }
    }
    if (tid == 0 && done < 0) a.flags[t] = 1;
}

// The same Jacobi with S held in LDS (packed lower triangle) when M <= JL_MAXM: a round is one
// pass over the 2 x 2 blocks of every pair of rotation pairs (A <- J^T A J in one step, each
// entry touched once; the diagonal blocks by the stable update A_pp - t A_pq, A_qq + t A_pq,
// A_pq = 0).  The rotations (c, s) of every round are written out instead of being applied to
// V^T at once; k_jacobi_apply_v applies them afterwards to column tiles of V^T = I held in LDS
// (the pairs follow from the round index), so V^T crosses global memory once, not once per
// round.  S is written back at the end.
constexpr int JL_MAXM = 196;
constexpr int JL_NA = JL_MAXM * (JL_MAXM + 1) / 2;
constexpr int JL_MAXP = JL_MAXM / 2;

__device__ __forceinline__ int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

__global__ __launch_bounds__(JAC_THREADS) void k_jacobi_lds(Dev a) {
    __shared__ double As[JL_NA];
    __shared__ double sc[JL_MAXP], ss[JL_MAXP], stn[JL_MAXP];
    __shared__ int sp[JL_MAXP], sq[JL_MAXP];
    __shared__ double red[JAC_THREADS / 64][2];
    __shared__ int done;
    const int t = blockIdx.x, m = a.m;
    const int mp = m + (m & 1), K = mp - 1, np = mp / 2, nb = np * (np + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *S = a.S + (size_t)t * m * m;
    double2 *rot = a.snrRot + (size_t)t * JAC_MAX_SWEEPS * K * np;
    int nsweep = 0;
    for (int e = tid; e < m * m; e += JAC_THREADS) {
        const int i = e / m, j = e % m;
        if (j <= i) As[tri(i, j)] = S[e];
    }
    // this thread's blocks b = tid + k JAC_THREADS, as pairs (i1 >= i2) of rotation pairs with
    // b = i1 (i1 + 1) / 2 + i2: the same in every round
    constexpr int JL_ITEMS = (JL_MAXP * (JL_MAXP + 1) / 2 + JAC_THREADS - 1) / JAC_THREADS;
    int bi1[JL_ITEMS], bi2[JL_ITEMS];
    for (int k = 0; k < JL_ITEMS; ++k) {
        const int b = tid + k * JAC_THREADS;
        int i1 = 0;
        if (b < nb) {
            i1 = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
            while ((i1 + 1) * (i1 + 2) / 2 <= b) ++i1;
            while (i1 * (i1 + 1) / 2 > b) --i1;
        }
        bi1[k] = i1;
        bi2[k] = b - i1 * (i1 + 1) / 2;
    }
    __syncthreads();
    for (int sweep = 0;; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < m * m; e += JAC_THREADS) {
            const int i = e / m, j = e % m;
            if (j > i) continue;
            const double v = As[tri(i, j)];
            tot += (i == j ? 1.0 : 2.0) * v * v;
            if (i != j) off += 2.0 * v * v;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if (lane == 0) {
            red[wave][0] = off;
            red[wave][1] = tot;
        }
        __syncthreads();
        if (tid == 0) {
            double o = 0.0, s = 0.0;
            for (int w = 0; w < JAC_THREADS / 64; ++w) {
                o += red[w][0];
                s += red[w][1];
            }
            done = (o <= 1e-30 * s) ? 1 : (sweep == JAC_MAX_SWEEPS ? -1 : 0);
        }
        __syncthreads();
        if (done != 0) break;
        for (int r = 0; r < K; ++r) {
            if (tid < np) {
                const int i = tid;
                int p = i == 0 ? r : (r + i) % K;
                int q = i == 0 ? K : (r - i + K) % K;
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, s = 0.0, tn = 0.0;
                if (q < m) {
                    const double apq = As[tri(q, p)];
                    if (apq != 0.0) {
                        const double theta = (As[tri(q, q)] - As[tri(p, p)]) / (2.0 * apq);
                        tn = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tn * tn + 1.0);
                        s = tn * c;
                    }
                }
                sp[i] = p;
                sq[i] = q;
                sc[i] = c;
                ss[i] = s;
                stn[i] = tn;
                rot[((size_t)nsweep * K + r) * np + i] = make_double2(c, s);
            }
            __syncthreads();
            for (int k = 0; k < JL_ITEMS; ++k) {
                if (tid + k * JAC_THREADS >= nb) continue;
                const int i1 = bi1[k], i2 = bi2[k];
                const int p1 = sp[i1], q1 = sq[i1], p2 = sp[i2], q2 = sq[i2];
                const bool h1 = q1 < m, h2 = q2 < m;
                if (i1 == i2) {
                    if (!h1) continue;
                    const double apq = As[tri(q1, p1)], tn = stn[i1];
                    As[tri(p1, p1)] -= tn * apq;
                    As[tri(q1, q1)] += tn * apq;
                    As[tri(q1, p1)] = 0.0;
                    continue;
                }
                const double c1 = sc[i1], s1 = ss[i1], c2 = sc[i2], s2 = ss[i2];
                const double x00 = As[tri(p1, p2)];
                const double x01 = h2 ? As[tri(p1, q2)] : 0.0;
                const double x10 = h1 ? As[tri(q1, p2)] : 0.0;
                const double x11 = (h1 && h2) ? As[tri(q1, q2)] : 0.0;
                const double y00 = c1 * x00 - s1 * x10, y10 = s1 * x00 + c1 * x10;
                const double y01 = c1 * x01 - s1 * x11, y11 = s1 * x01 + c1 * x11;
                As[tri(p1, p2)] = c2 * y00 - s2 * y01;
                if (h2) As[tri(p1, q2)] = s2 * y00 + c2 * y01;
                if (h1) As[tri(q1, p2)] = c2 * y10 - s2 * y11;
                if (h1 && h2) As[tri(q1, q2)] = s2 * y10 + c2 * y11;
            }
            __syncthreads();
        }
        ++nsweep;
    }
    for (int e = tid; e < m * m; e += JAC_THREADS) S[e] = As[tri(e / m, e % m)];
    if (tid == 0) {
        a.snrSweeps[t] = nsweep;
        if (done < 0) a.flags[t] = 1;
    }
}

// V^T = (product of the recorded rotations) applied to I, a tile of JV_COLS columns per
// workgroup held in LDS: for every recorded round in order, rows p, q of the tile are rotated
// (the pairs of round r follow from r as in k_jacobi_lds).  Tiles of 32 columns (48 KB) let
// three workgroups share a compute unit, so one's per-round barrier overlaps the others' work.
constexpr int JV_COLS = 32;
constexpr int JV_THREADS = 512;
__global__ __launch_bounds__(JV_THREADS, 6) void k_jacobi_apply_v(Dev a) {   // 6 waves per SIMD: three workgroups per CU
    __shared__ double Vs[JL_MAXM * JV_COLS];
    const int t = blockIdx.y, j0 = blockIdx.x * JV_COLS, m = a.m;
    const int mp = m + (m & 1), K = mp - 1, np = mp / 2;
    const int tid = threadIdx.x;
    const int cols = (m - j0) < JV_COLS ? (m - j0) : JV_COLS;
    for (int e = tid; e < m * JV_COLS; e += JV_THREADS) {
        const int i = e / JV_COLS, j = e % JV_COLS;
        Vs[e] = (i == j0 + j) ? 1.0 : 0.0;
    }
    __syncthreads();
    const double2 *rot = a.snrRot + (size_t)t * JAC_MAX_SWEEPS * K * np;
    const int rounds = a.snrSweeps[t] * K;
    // a thread's items (pair i, column j) are the same every round; the other workgroups on the
    // compute unit cover the latency of loading each round's rotations at its start
    constexpr int JV_ITEMS = (JL_MAXP * JV_COLS + JV_THREADS - 1) / JV_THREADS;
    double2 cur[JV_ITEMS];
    for (int rr = 0, r = 0; rr < rounds; ++rr, r = (r + 1 == K ? 0 : r + 1)) {
        for (int k = 0; k < JV_ITEMS; ++k) {
            const int i = (tid + k * JV_THREADS) / JV_COLS;
            cur[k] = i < np ? rot[(size_t)rr * np + i] : make_double2(1.0, 0.0);
        }
        for (int k = 0; k < JV_ITEMS; ++k) {
            const int e = tid + k * JV_THREADS, i = e / JV_COLS, j = e % JV_COLS;
            if (i >= np) continue;
            // pair i of round r: (r + i) mod K and (r - i) mod K, both arguments in [0, 2K)
            int p = i == 0 ? r : (r + i >= K ? r + i - K : r + i);
            int q = i == 0 ? K : (r - i < 0 ? r - i + K : r - i);
            if (p > q) {
                const int x = p;
                p = q;
                q = x;
            }
            if (q >= m || j >= cols) continue;
            const double2 cs = cur[k];
            const double vp = Vs[p * JV_COLS + j], vq = Vs[q * JV_COLS + j];
            Vs[p * JV_COLS + j] = cs.x * vp - cs.y * vq;
            Vs[q * JV_COLS + j] = cs.y * vp + cs.x * vq;
        }
        __syncthreads();
    }
    double *Vt = a.snrV + (size_t)t * m * m;
    for (int e = tid; e < m * JV_COLS; e += JV_THREADS) {
        const int i = e / JV_COLS, j = e % JV_COLS;
        if (j < cols) Vt[(size_t)i * m + j0 + j] = Vs[e];
    }
}

// rho_k = sum_l V_lk D_l
__global__ void k_snr_rho(Dev a) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const double *v = a.snrV + ((size_t)t * a.m + k) * a.m;
    const double2 *D = a.D + (size_t)t * a.m;
    double re = 0.0, im = 0.0;
    for (int l = 0; l < a.m; ++l) {
        re += v[l] * D[l].x;
        im += v[l] * D[l].y;
    }
    a.snrRho[(size_t)t * a.m + k] = make_double2(re, im);
}

// Partial sums over 64-sample blocks of u_k(x)^2 |G(x) - <G>|^2: a 64 x 64 (eigenvector x
// sample) tile per workgroup, u = V^T (O - <O>) accumulated over 32-row slabs staged in LDS
// (O_l(x) recomputed from the packed samples) on the FP64 matrix cores: wave w takes
// eigenvectors 16 w .. +15 against the 64 samples, four 16 x 16 accumulators (register r of
// lane (lk, li) holds row lk + 4 r, column li).
constexpr int SV_K = 64, SV_X = 64, SV_L = 32;
__global__ __launch_bounds__(256) void k_snr_var(Dev a) {
    __shared__ double vs[SV_K][SV_L + 1];
    __shared__ double os[SV_L][SV_X + 1];
    const int t = blockIdx.z, k0 = blockIdx.x * SV_K, x0 = blockIdx.y * SV_X;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int m = a.m, ns = a.ns;
    const double *Vt = a.snrV + (size_t)t * m * m;
    const uint64_t *smp = a.samples + (size_t)t * ns;
    const double *ob = a.obar + (size_t)t * m;
    v4d u[4];
    for (int v = 0; v < 4; ++v) u[v] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < m; l0 += SV_L) {
        __syncthreads();
        for (int e = tid; e < SV_K * SV_L; e += 256) {
            const int kk = e / SV_L, ll = e % SV_L, k = k0 + kk, l = l0 + ll;
            vs[kk][ll] = (k < m && l < m) ? Vt[(size_t)k * m + l] : 0.0;
        }
        for (int e = tid; e < SV_L * SV_X; e += 256) {
            const int ll = e / SV_X, xx = e % SV_X, l = l0 + ll, x = x0 + xx;
            os[ll][xx] = (l < m && x < ns) ? (double)o_int(smp[x], a.pa[l], a.pb[l], a.n) - ob[l] : 0.0;
        }
        __syncthreads();
        for (int ks = 0; ks < SV_L / 4; ++ks) {
            const double fa = vs[wave * 16 + li][ks * 4 + lk];
            for (int v = 0; v < 4; ++v)
                u[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, os[ks * 4 + lk][v * 16 + li], u[v], 0, 0, 0);
        }
    }
    const double2 gb = a.gbar[t];
    double g2[4];
    for (int v = 0; v < 4; ++v) {
        const int x = x0 + v * 16 + li;
        g2[v] = 0.0;
        if (x < ns) {
            const double2 g = a.G[(size_t)t * ns + x];
            const double dr = g.x - gb.x, di = g.y - gb.y;
            g2[v] = dr * dr + di * di;
        }
    }
    for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        for (int v = 0; v < 4; ++v) s += u[v][r] * u[v][r] * g2[v];
        for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o, 64);
        const int k = k0 + wave * 16 + lk + 4 * r;
        if (li == 0 && k < m) a.snrPart[((size_t)t * a.snr_nxb + blockIdx.y) * m + k] = s;
    }
}

// SNR_k, the kept weight and w_k = keep_k rho_k / lam_k; (lam_k, SNR_k) kept for inspection
__global__ __launch_bounds__(256) void k_snr_finish(Dev a) {
    __shared__ double red[4];
    const int t = blockIdx.x, m = a.m, tid = threadIdx.x;
    const double *A = a.S + (size_t)t * m * m;
    double lmax = 0.0;
    for (int k = tid; k < m; k += 256) lmax = fmax(lmax, A[(size_t)k * m + k]);
    for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o));
    if ((tid & 63) == 0) red[tid >> 6] = lmax;
    __syncthreads();
    lmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    for (int k = tid; k < m; k += 256) {
        double q2 = 0.0;
        for (int b = 0; b < a.snr_nxb; ++b) q2 += a.snrPart[((size_t)t * a.snr_nxb + b) * m + k];
        const double2 r = a.snrRho[(size_t)t * m + k];
        const double ar = sqrt(r.x * r.x + r.y * r.y);
        const double var = q2 / (double)a.ns - (r.x * r.x + r.y * r.y);
        const double snr = var > 0.0 ? ar * sqrt((double)a.ns) / sqrt(var) : INFINITY;
        const double lam = A[(size_t)k * m + k];
        const double keep = (lam > 1e-14 * lmax && ar > 0.0) ? 1.0 / (1.0 + pow(a.snr_tau / snr, 6.0)) : 0.0;
        a.snrW[(size_t)t * m + k] = keep > 0.0 ? make_double2(keep * r.x / lam, keep * r.y / lam) : make_double2(0.0, 0.0);
        a.snrEig[((size_t)t * m + k) * 2] = lam;
        a.snrEig[((size_t)t * m + k) * 2 + 1] = snr;
    }
}

// delta_l = sum_k V_lk w_k
__global__ void k_snr_back(Dev a, int stage) {
    const int t = blockIdx.y;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.m) return;
    const double *Vt = a.snrV + (size_t)t * a.m * a.m;
    const double2 *w = a.snrW + (size_t)t * a.m;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < a.m; ++k) {
        const double v = Vt[(size_t)k * a.m + l];
        re += v * w[k].x;
        im += v * w[k].y;
    }
    double2 *out = stage ? a.d1 : a.d0;
    const double2 dl = make_double2(re, im);
    out[(size_t)t * a.m + l] = dl;
    if (!isfinite(re) || !isfinite(im)) a.flags[t] = 1;
}

// ---------------------------------------------------------------- complex Hermitian S (RBM)
// The same steps with W = V^H kept as rows.  The rotation of a pair (p, q) folds the phase
// e^{i phi} = A_pq / |A_pq| into the real rotation of |A_pq|: A <- U^H A U with U_pp = c,
// U_pq = s, U_qp = -s e^{-i phi}, U_qq = c e^{-i phi}, and W <- U^H W.  rho = W D,
// u_k(x) = sum_l conj(W_kl) (O_l(x) - <O_l>), q_k = conj(u_k) (G - <G>), delta = W^H w.

__device__ __forceinline__ double2 zmul_(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj_(double2 a) { return make_double2(a.x, -a.y); }
// c a - s (ph b), s a + c (ph b)
__device__ __forceinline__ void zrot(double2 &a, double2 &b, double c, double s, double2 ph) {
    const double2 pb = zmul_(ph, b);
    const double2 na = make_double2(c * a.x - s * pb.x, c * a.y - s * pb.y);
    const double2 nb = make_double2(s * a.x + c * pb.x, s * a.y + c * pb.y);
    a = na;
    b = nb;
}

// S + eps I (lower triangle) -> full Hermitian matrix; W = I
__global__ void k_zsnr_init(Dev a) {
    const int t = blockIdx.y;
    const size_t mm = (size_t)a.m * a.m;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= mm) return;
    const int i = (int)(idx / a.m), j = (int)(idx % a.m);
    double2 *S = (double2 *)a.S + (size_t)t * mm;
    if (j > i) S[idx] = zconj_(S[(size_t)j * a.m + i]);
    ((double2 *)a.snrV)[(size_t)t * mm + idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

__global__ __launch_bounds__(JAC_THREADS) void k_zjacobi(Dev a) {
    __shared__ int sp[JAC_MAXP], sq[JAC_MAXP];
    __shared__ double sc[JAC_MAXP], ss[JAC_MAXP];
    __shared__ double2 sph[JAC_MAXP];
    __shared__ double red[JAC_THREADS / 64][2];
    __shared__ int done;
    const int t = blockIdx.x, m = a.m;
    const int mp = m + (m & 1), K = mp - 1, np = mp / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double2 *A = (double2 *)a.S + (size_t)t * m * m;
    double2 *W = (double2 *)a.snrV + (size_t)t * m * m;
    for (int sweep = 0;; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < m * m; e += JAC_THREADS) {
            const double2 v = A[e];
            const double v2 = v.x * v.x + v.y * v.y;
            tot += v2;
            if (e / m != e % m) off += v2;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if (lane == 0) {
            red[wave][0] = off;
            red[wave][1] = tot;
        }
        __syncthreads();
        if (tid == 0) {
            double o = 0.0, s = 0.0;
            for (int w = 0; w < JAC_THREADS / 64; ++w) {
                o += red[w][0];
                s += red[w][1];
            }
            done = (o <= 1e-30 * s) ? 1 : (sweep == JAC_MAX_SWEEPS ? -1 : 0);
        }
        __syncthreads();
        if (done != 0) break;
        for (int r = 0; r < K; ++r) {
            for (int i = tid; i < np; i += JAC_THREADS) {
                int p = i == 0 ? r : (r + i) % K;
                int q = i == 0 ? K : (r - i + K) % K;
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, s = 0.0;
                double2 ph = make_double2(1.0, 0.0);
                if (q < m) {
                    const double2 apq = A[(size_t)p * m + q];
                    const double aa = sqrt(apq.x * apq.x + apq.y * apq.y);
                    if (aa != 0.0) {
                        ph = make_double2(apq.x / aa, apq.y / aa);
                        const double theta = (A[(size_t)q * m + q].x - A[(size_t)p * m + p].x) / (2.0 * aa);
                        const double tn = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tn * tn + 1.0);
                        s = tn * c;
                    }
                }
                sp[i] = p;
                sq[i] = q;
                sc[i] = c;
                ss[i] = s;
                sph[i] = ph;
            }
            __syncthreads();
            for (int e = tid; e < np * m; e += JAC_THREADS) {   // rows p, q of A and of W: U^H .
                const int i = e / m, j = e % m, p = sp[i], q = sq[i];
                if (q >= m) continue;
                double2 x = A[(size_t)p * m + j], y = A[(size_t)q * m + j];
                zrot(x, y, sc[i], ss[i], sph[i]);
                A[(size_t)p * m + j] = x;
                A[(size_t)q * m + j] = y;
                double2 u = W[(size_t)p * m + j], v = W[(size_t)q * m + j];
                zrot(u, v, sc[i], ss[i], sph[i]);
                W[(size_t)p * m + j] = u;
                W[(size_t)q * m + j] = v;
            }
            __syncthreads();
            for (int e = tid; e < np * m; e += JAC_THREADS) {   // columns p, q of A: . U
                const int i = e % np, k = e / np, p = sp[i], q = sq[i];
                if (q >= m) continue;
                double2 x = A[(size_t)k * m + p], y = A[(size_t)k * m + q];
                zrot(x, y, sc[i], ss[i], zconj_(sph[i]));
                A[(size_t)k * m + p] = x;
                A[(size_t)k * m + q] = y;
            }
            __syncthreads();
        }
    }
    if (tid == 0 && done < 0) a.flags[t] = 1;
}

// rho_k = sum_l W_kl D_l
__global__ void k_zsnr_rho(Dev a) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const double2 *w = (const double2 *)a.snrV + ((size_t)t * a.m + k) * a.m;
    const double2 *D = a.D + (size_t)t * a.m;
    double re = 0.0, im = 0.0;
    for (int l = 0; l < a.m; ++l) {
        const double2 v = zmul_(w[l], D[l]);
        re += v.x;
        im += v.y;
    }
    a.snrRho[(size_t)t * a.m + k] = make_double2(re, im);
}

// centred RBM log-derivative O_l(x) - <O_l>: s_l, tanh g_j, s_i tanh g_j
__device__ __forceinline__ double2 rbm_dO(const Dev &a, int t, int l, int x) {
    const uint64_t mk = a.samples[(size_t)t * a.ns + x];
    double2 o;
    if (l < a.n) {
        o = make_double2(((mk >> l) & 1ull) ? 1.0 : -1.0, 0.0);
    } else if (l < a.n + a.nh) {
        o = a.tt[((size_t)t * a.ns + x) * a.nh + (l - a.n)];
    } else {
        const int i = (l - a.n - a.nh) / a.nh, j = (l - a.n - a.nh) % a.nh;
        const double si = ((mk >> i) & 1ull) ? 1.0 : -1.0;
        const double2 th = a.tt[((size_t)t * a.ns + x) * a.nh + j];
        o = make_double2(si * th.x, si * th.y);
    }
    const double2 ob = a.obarc[(size_t)t * a.m + l];
    return make_double2(o.x - ob.x, o.y - ob.y);
}

// Partial sums over 64-sample blocks of |u_k(x)|^2 |G(x) - <G>|^2 (as k_snr_var, complex)
__global__ __launch_bounds__(256) void k_zsnr_var(Dev a) {
    __shared__ double2 vs[SV_K][SV_L + 1];
    __shared__ double2 os[SV_L][SV_X + 1];
    __shared__ double red[16][SV_K];
    const int t = blockIdx.z, k0 = blockIdx.x * SV_K, x0 = blockIdx.y * SV_X;
    const int tid = threadIdx.x, tk = tid >> 4, tx = tid & 15;
    const int m = a.m, ns = a.ns;
    const double2 *W = (const double2 *)a.snrV + (size_t)t * m * m;
    double ur[4][4] = {}, ui[4][4] = {};
    for (int l0 = 0; l0 < m; l0 += SV_L) {
        __syncthreads();
        for (int e = tid; e < SV_K * SV_L; e += 256) {
            const int kk = e / SV_L, ll = e % SV_L, k = k0 + kk, l = l0 + ll;
            vs[kk][ll] = (k < m && l < m) ? zconj_(W[(size_t)k * m + l]) : make_double2(0.0, 0.0);
        }
        for (int e = tid; e < SV_L * SV_X; e += 256) {
            const int ll = e / SV_X, xx = e % SV_X, l = l0 + ll, x = x0 + xx;
            os[ll][xx] = (l < m && x < ns) ? rbm_dO(a, t, l, x) : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int ll = 0; ll < SV_L; ++ll) {
            double2 v[4], o[4];
            for (int i = 0; i < 4; ++i) v[i] = vs[tk * 4 + i][ll];
            for (int j = 0; j < 4; ++j) o[j] = os[ll][tx * 4 + j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    ur[i][j] += v[i].x * o[j].x - v[i].y * o[j].y;
                    ui[i][j] += v[i].x * o[j].y + v[i].y * o[j].x;
                }
        }
    }
    const double2 gb = a.gbar[t];
    double g2[4];
    for (int j = 0; j < 4; ++j) {
        const int x = x0 + tx * 4 + j;
        g2[j] = 0.0;
        if (x < ns) {
            const double2 g = a.G[(size_t)t * ns + x];
            const double dr = g.x - gb.x, di = g.y - gb.y;
            g2[j] = dr * dr + di * di;
        }
    }
    for (int i = 0; i < 4; ++i) {
        double s = 0.0;
        for (int j = 0; j < 4; ++j) s += (ur[i][j] * ur[i][j] + ui[i][j] * ui[i][j]) * g2[j];
        red[tx][tk * 4 + i] = s;
    }
    __syncthreads();
    if (tid < SV_K && k0 + tid < m) {
        double s = 0.0;
        for (int q = 0; q < 16; ++q) s += red[q][tid];
        a.snrPart[((size_t)t * a.snr_nxb + blockIdx.y) * m + k0 + tid] = s;
    }
}

// SNR_k, keep_k and w_k (lam_k from the real diagonal)
__global__ __launch_bounds__(256) void k_zsnr_finish(Dev a) {
    __shared__ double red[4];
    const int t = blockIdx.x, m = a.m, tid = threadIdx.x;
    const double2 *A = (const double2 *)a.S + (size_t)t * m * m;
    double lmax = 0.0;
    for (int k = tid; k < m; k += 256) lmax = fmax(lmax, A[(size_t)k * m + k].x);
    for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o));
    if ((tid & 63) == 0) red[tid >> 6] = lmax;
    __syncthreads();
    lmax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    for (int k = tid; k < m; k += 256) {
        double q2 = 0.0;
        for (int b = 0; b < a.snr_nxb; ++b) q2 += a.snrPart[((size_t)t * a.snr_nxb + b) * m + k];
        const double2 r = a.snrRho[(size_t)t * m + k];
        const double ar = sqrt(r.x * r.x + r.y * r.y);
        const double var = q2 / (double)a.ns - (r.x * r.x + r.y * r.y);
        const double snr = var > 0.0 ? ar * sqrt((double)a.ns) / sqrt(var) : INFINITY;
        const double lam = A[(size_t)k * m + k].x;
        const double keep = (lam > 1e-14 * lmax && ar > 0.0) ? 1.0 / (1.0 + pow(a.snr_tau / snr, 6.0)) : 0.0;
        a.snrW[(size_t)t * m + k] = keep > 0.0 ? make_double2(keep * r.x / lam, keep * r.y / lam) : make_double2(0.0, 0.0);
        a.snrEig[((size_t)t * m + k) * 2] = lam;
        a.snrEig[((size_t)t * m + k) * 2 + 1] = snr;
    }
}

// delta_l = sum_k conj(W_kl) w_k
__global__ void k_zsnr_back(Dev a, int stage) {
    const int t = blockIdx.y;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.m) return;
    const double2 *W = (const double2 *)a.snrV + (size_t)t * a.m * a.m;
    const double2 *w = a.snrW + (size_t)t * a.m;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < a.m; ++k) {
        const double2 v = zmul_(zconj_(W[(size_t)k * a.m + l]), w[k]);
        re += v.x;
        im += v.y;
    }
    double2 *out = stage ? a.d1 : a.d0;
    out[(size_t)t * a.m + l] = make_double2(re, im);
    if (!isfinite(re) || !isfinite(im)) a.flags[t] = 1;
}

}  // namespace tvmc
