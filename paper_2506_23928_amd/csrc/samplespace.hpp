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

// RBM K (complex) into the S buffer, full matrix: a 64 x 64 tile per workgroup, 4 x 4 outputs
// per thread, tanh rows staged 16 hidden units at a time through LDS.  Grid (tiles^2, T).
constexpr int TK_T = 64;
constexpr int TK_J = 16;
template <int W>
__global__ __launch_bounds__(256) void k_tk_rbm(Dev a) {
    __shared__ double2 tx[TK_T][TK_J + 1], ty[TK_T][TK_J + 1];
    const int t = blockIdx.y;
    const int nb = (a.ns + TK_T - 1) / TK_T;
    const int x0 = (blockIdx.x / nb) * TK_T, y0 = (blockIdx.x % nb) * TK_T;
    const int ix = threadIdx.x >> 4, iy = threadIdx.x & 15;   // rows x0 + ix + 16 u, cols y0 + iy + 16 v
    const int nh = a.nh;
    const double2 *tt = a.tt + (size_t)t * a.ns * nh;
    double gr[4][4], gi[4][4];
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) gr[u][v] = gi[u][v] = 0.0;
    for (int j0 = 0; j0 < nh; j0 += TK_J) {
        __syncthreads();
        for (int e = threadIdx.x; e < TK_T * TK_J; e += 256) {
            const int r = e / TK_J, j = e % TK_J;
            const bool okj = j0 + j < nh;
            tx[r][j] = (okj && x0 + r < a.ns) ? tt[(size_t)(x0 + r) * nh + j0 + j] : make_double2(0.0, 0.0);
            ty[r][j] = (okj && y0 + r < a.ns) ? tt[(size_t)(y0 + r) * nh + j0 + j] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int j = 0; j < TK_J; ++j) {
            double2 xv[4], yv[4];
            for (int u = 0; u < 4; ++u) xv[u] = tx[ix + 16 * u][j];
            for (int v = 0; v < 4; ++v) yv[v] = ty[iy + 16 * v][j];
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) {   // t(x) t(y)^*
                    gr[u][v] += xv[u].x * yv[v].x + xv[u].y * yv[v].y;
                    gi[u][v] += xv[u].y * yv[v].x - xv[u].x * yv[v].y;
                }
        }
    }
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    double2 *K = (double2 *)a.S + (size_t)t * a.ns * a.ns;
    for (int u = 0; u < 4; ++u) {
        const int x = x0 + ix + 16 * u;
        if (x >= a.ns) continue;
        for (int v = 0; v < 4; ++v) {
            const int y = y0 + iy + 16 * v;
            if (y >= a.ns) continue;
            const double q1 = 1.0 + (double)spin_overlap<W>(smp + (size_t)x * W, smp + (size_t)y * W, a.n);
            K[(size_t)x * a.ns + y] = make_double2(q1 * (1.0 + gr[u][v]) - 1.0, q1 * gi[u][v]);
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
