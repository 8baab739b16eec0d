// Sample-space solve (for M > N_s).  With A[x][k] = (O_k(x) - <O_k>) / sqrt(N_s) and
// g[x] = (G(x) - <G>) / sqrt(N_s) one has S = A^H A and D = A^H g (definitions after Eq. 8),
// and the push-through identity (A^H A + eps I)^-1 A^H = A^H (A A^H + eps I)^-1 gives
//   delta = (1 / N_s) sum_x (O_k(x) - <O_k>)^* u_x,   (T + eps I) u = G - <G>,
//   T = A A^H = H K H / N_s,  K_xy = sum_k O_k(x) O_k(y)^*,  H = I - 1 1^T / N_s,
// exactly the parameter-space increment, through an N_s x N_s system.  The uncentred kernel
// has closed forms in q = s(x).s(y):
//   Jastrow (O = s_i, s_j s_k):      K = q + (q^2 - N) / 2            (integers, exact)
//   RBM (O = s_i, t_j, s_i t_j):     K = (1 + q)(1 + g) - 1,  g = sum_j t_j(x) t_j(y)^*
// so T costs N_s^2 popcounts (plus an N_s^2 N' complex product for the RBM) instead of the
// N_s^2 M of the defining sum.  K is written in full, its row means r_x = (1/N_s) sum_y K_xy
// and their mean rbar are formed, then T_xy = (K_xy - r_x - r_y^* + rbar) / N_s (+ eps on the
// diagonal) replaces the lower triangle in place.
#pragma once
#include "common.hpp"
#include "cholesky.hpp"
#include "rbm.hpp"

namespace tvmc {

template <int W>
__device__ __forceinline__ int spin_overlap(const uint64_t *x, const uint64_t *y, int n) {
    return n - 2 * cfg_diff(cfg_load<W>(x), cfg_load<W>(y));   // bits at and above n are zero in both
}

// Jastrow K (real) into the S buffer, full matrix.  Grid (ceil(N_s/256), N_s, T).
template <int W>
__global__ __launch_bounds__(256) void k_tk_jastrow(Dev a) {
    const int t = blockIdx.z, x = blockIdx.y;
    const int y = blockIdx.x * 256 + threadIdx.x;
    if (y >= a.ns) return;
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double q = (double)spin_overlap<W>(smp + (size_t)x * W, smp + (size_t)y * W, a.n);
    a.S[((size_t)t * a.ns + x) * a.ns + y] = q + 0.5 * (q * q - (double)a.n);
}

// RBM K (complex) into the S buffer, full matrix, on the FP64 matrix cores.  K is Hermitian, so
// one workgroup forms one 64 x 64 tile of the lower block triangle (bi >= bj) and writes it and,
// off the diagonal, its conjugate transpose (through LDS, so that both stores are row-contiguous).
// g = t(x) t(y)^H accumulates over the hidden units in chunks of 16 staged through LDS: rows of
// 256 bytes, the 16-byte piece j of row r at position j ^ (r & 15), which puts the 16-byte
// fragment reads of 16 rows on distinct banks.  Wave w takes rows 16 w .. +15 of the tile and all
// 64 columns (four 16 x 16 blocks); per block and step of 4 hidden units
//   Re g += tr tr'^T + ti ti'^T,   Im g = ti tr'^T - tr ti'^T   (the two halves kept apart).
// Grid (tiles nb (nb + 1) / 2, T), 256 threads; LDS 65 KB (the transpose buffer; staging takes
// its first 32 KB).
constexpr int TK_T = 64;
constexpr int TK_J = 16;
constexpr int TK_TP = TK_T + 1;   // row stride of the transpose buffer (16-byte slots)
template <int W>
__global__ __launch_bounds__(256) void k_tk_rbm(Dev a) {
    __shared__ __attribute__((aligned(16))) double2 sm[TK_T * TK_TP];
    const int t = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int x0 = bi * TK_T, y0 = bj * TK_T, ns = a.ns, nh = a.nh;
    const int wave = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const double2 *tt = a.tt + (size_t)t * ns * nh;
    double2 *tx = sm, *ty = sm + TK_T * TK_J;
    v4d gre[4], gia[4], gib[4];
    for (int v = 0; v < 4; ++v) {
        gre[v] = (v4d){0.0, 0.0, 0.0, 0.0};
        gia[v] = (v4d){0.0, 0.0, 0.0, 0.0};
        gib[v] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    const int ar = wave * 16 + li;
    for (int j0 = 0; j0 < nh; j0 += TK_J) {
        __syncthreads();
        for (int e = tid; e < TK_T * TK_J; e += 256) {
            const int r = e / TK_J, j = e % TK_J, pos = r * TK_J + (j ^ (r & 15));
            const bool okj = j0 + j < nh;
            tx[pos] = (okj && x0 + r < ns) ? tt[(size_t)(x0 + r) * nh + j0 + j] : make_double2(0.0, 0.0);
            ty[pos] = (okj && y0 + r < ns) ? tt[(size_t)(y0 + r) * nh + j0 + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int ks = 0; ks < TK_J / 4; ++ks) {
            const int p = ks * 4 + lk;
            const double2 fa = tx[ar * TK_J + (p ^ (ar & 15))];
            double2 fb[4];
            for (int v = 0; v < 4; ++v) {
                const int br = v * 16 + li;
                fb[v] = ty[br * TK_J + (p ^ (br & 15))];
            }
            for (int v = 0; v < 4; ++v) {
                gre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x, fb[v].x, gre[v], 0, 0, 0);
                gre[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.y, fb[v].y, gre[v], 0, 0, 0);
                gia[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.y, fb[v].x, gia[v], 0, 0, 0);
                gib[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x, fb[v].y, gib[v], 0, 0, 0);
            }
        }
    }
    __syncthreads();   // the staging buffers become the transpose buffer
    const uint64_t *smp = a.samples + (size_t)t * ns * W;
    double2 *K = (double2 *)a.S + (size_t)t * ns * ns;
    for (int r = 0; r < 4; ++r) {
        const int row = wave * 16 + lk + 4 * r, x = x0 + row;
        for (int v = 0; v < 4; ++v) {
            const int col = v * 16 + li, y = y0 + col;
            if (x >= ns || y >= ns) continue;
            const double q1 = 1.0 + (double)spin_overlap<W>(smp + (size_t)x * W, smp + (size_t)y * W, a.n);
            const double2 k = make_double2(q1 * (1.0 + gre[v][r]) - 1.0, q1 * (gia[v][r] - gib[v][r]));
            K[(size_t)x * ns + y] = k;
            sm[row * TK_TP + col] = k;
        }
    }
    if (bi == bj) return;   // the diagonal tile was formed whole
    __syncthreads();
    for (int e = tid; e < TK_T * TK_T; e += 256) {   // K[y][x] = K[x][y]^*
        const int yr = e / TK_T, xc = e % TK_T;
        if (y0 + yr < ns && x0 + xc < ns) {
            const double2 k = sm[xc * TK_TP + yr];
            K[(size_t)(y0 + yr) * ns + x0 + xc] = make_double2(k.x, -k.y);
        }
    }
}

// row means r_x = (1/N_s) sum_y K_xy (fixed-order tree).  Grid (N_s, T).
__global__ __launch_bounds__(256) void k_tk_rowmean(Dev a) {
    __shared__ double sre[256], sim[256];
    const int t = blockIdx.y, x = blockIdx.x;
    const bool cplx = a.kind == 1;
    double re = 0.0, im = 0.0;
    if (cplx) {
        const double2 *row = (const double2 *)a.S + ((size_t)t * a.ns + x) * a.ns;
        for (int y = threadIdx.x; y < a.ns; y += 256) {
            re += row[y].x;
            im += row[y].y;
        }
    } else {
        const double *row = a.S + ((size_t)t * a.ns + x) * a.ns;
        for (int y = threadIdx.x; y < a.ns; y += 256) re += row[y];
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sre[threadIdx.x] += sre[threadIdx.x + o];
            sim[threadIdx.x] += sim[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ssrow[(size_t)t * a.ns + x] = make_double2(sre[0] / (double)a.ns, sim[0] / (double)a.ns);
}

// rbar = (1/N_s) sum_x r_x and the centred right-hand side G - <G>.  Grid (T).
__global__ __launch_bounds__(256) void k_tk_rbar(Dev a) {
    __shared__ double sre[256];
    const int t = blockIdx.x;
    double re = 0.0;
    for (int x = threadIdx.x; x < a.ns; x += 256) re += a.ssrow[(size_t)t * a.ns + x].x;
    sre[threadIdx.x] = re;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sre[threadIdx.x] += sre[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ssbar[t] = sre[0] / (double)a.ns;   // real: sum_xy K_xy is real
    const double2 gb = a.gbar[t];
    for (int x = threadIdx.x; x < a.ns; x += 256) {
        const double2 g = a.G[(size_t)t * a.ns + x];
        a.ssrhs[(size_t)t * a.ns + x] = make_double2(g.x - gb.x, g.y - gb.y);
    }
}

// T = (K - r_x - r_y^* + rbar) / N_s + eps I, lower triangle in place.  Grid (ceil(N_s/256), N_s, T).
__global__ __launch_bounds__(256) void k_tk_centre(Dev a) {
    const int t = blockIdx.z, x = blockIdx.y;
    const int y = blockIdx.x * 256 + threadIdx.x;
    if (y > x || y >= a.ns) return;
    const double inv = 1.0 / (double)a.ns;
    const double2 rx = a.ssrow[(size_t)t * a.ns + x], ry = a.ssrow[(size_t)t * a.ns + y];
    const double rb = a.ssbar[t];
    const size_t e = ((size_t)t * a.ns + x) * a.ns + y;
    if (a.kind == 1) {
        double2 *K = (double2 *)a.S;
        const double2 k = K[e];
        double re = ((k.x - rx.x) - ry.x + rb) * inv;
        double im = ((k.y - rx.y) + ry.y) * inv;
        if (x == y) {
            re += a.eps;
            im = 0.0;
        }
        K[e] = make_double2(re, im);
    } else {
        double v = ((a.S[e] - rx.x) - ry.x + rb) * inv;
        if (x == y) v += a.eps;
        a.S[e] = v;
    }
}

// delta_k = (1/N_s) [sum_x O_k(x)^* u_x - <O_k>^* sum_x u_x].  Grid (ceil(M/256), T).
template <int W>
__global__ __launch_bounds__(256) void k_pushback(Dev a, int which) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double2 *u = a.ssu + (size_t)t * a.ns;
    double re = 0.0, im = 0.0, ur = 0.0, ui = 0.0;
    double2 ob;
    if (a.kind == 1) {
        const double2 *tt = a.tt + (size_t)t * a.ns * a.nh;
        for (int x = 0; x < a.ns; ++x) {
            const double2 o = rbm_o(a, k, cfg_load<W>(smp + (size_t)x * W), tt + (size_t)x * a.nh);
            const double2 v = u[x];
            re += o.x * v.x + o.y * v.y;   // conj(o) u
            im += o.x * v.y - o.y * v.x;
            ur += v.x;
            ui += v.y;
        }
        ob = a.obarc[(size_t)t * a.m + k];
    } else {
        const int p = a.pa[k], q = a.pb[k];
        for (int x = 0; x < a.ns; ++x) {
            const Cfg<W> mk = cfg_load<W>(smp + (size_t)x * W);
            const bool plus = (q < 0) ? cfg_up(mk, p) : (cfg_up(mk, p) == cfg_up(mk, q));
            const double2 v = u[x];
            re += plus ? v.x : -v.x;
            im += plus ? v.y : -v.y;
            ur += v.x;
            ui += v.y;
        }
        ob = make_double2(a.obar[(size_t)t * a.m + k], 0.0);
    }
    const double inv = 1.0 / (double)a.ns;
    // conj(<O_k>) sum u
    const double cr = ob.x * ur + ob.y * ui, ci = ob.x * ui - ob.y * ur;
    double2 *d = (which ? a.d1 : a.d0) + (size_t)t * a.m;
    d[k] = make_double2((re - cr) * inv, (im - ci) * inv);
}

}  // namespace tvmc
