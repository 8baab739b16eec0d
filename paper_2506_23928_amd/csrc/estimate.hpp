// Local estimators and Monte Carlo means (definitions after Eq. 8).
//
//   B^n(x)  = (L_n psi)(x)/psi(x):  sigma^- on site i -> sqrt(g) [s_i=-1] R_i,
//                                    sigma^+ -> sqrt(g) [s_i=+1] R_i,  sigma^z -> sqrt(g) s_i
//   (L^+L)_loc + (L^2)_loc:          sigma^- -> g [s_i=+1], sigma^+ -> g [s_i=-1], sigma^z -> 2g
//   E_eff(x) = E_H(x) - (i/2) sum_n [ (L^+L)_loc - 2 <L+L^+> B^n + (L^2)_loc ]    (Eq. 5)
// with <L+L^+> = 2 Re <B^n> estimated from the same samples, the c-number terms of Eq. 5
// dropped (they cancel in every covariance).  The linear SSE (App. B) drops the drive term:
// E_eff^lin(x) = E_H(x) - (i/2) sum_n [ (L^+L)_loc + (L^2)_loc ], which has no c-number terms,
// so <G> = -i dt <E_eff^lin> + sum_n <B^n> dW_n and 2 Re <G> is the increment of log Q.  The increment vector of the regularised solve
// is D = -i F dt + sum_n N^n dW_n = cov(O*, G) with G(x) = -i dt E_eff(x) + sum_n B^n(x) dW_n,
// so one covariance replaces F and every N^n.
#pragma once
#include "common.hpp"

namespace tvmc {

template <int W>
__device__ __forceinline__ double2 jump_local(int kind, int site, double sq, const Cfg<W> &mask, const double2 *Rrow) {
    const bool up = cfg_up(mask, site);
    if (kind == 0) return up ? make_double2(0.0, 0.0) : make_double2(sq * Rrow[site].x, sq * Rrow[site].y);
    if (kind == 1) return up ? make_double2(sq * Rrow[site].x, sq * Rrow[site].y) : make_double2(0.0, 0.0);
    return make_double2(sq * (up ? 1.0 : -1.0), 0.0);
}

template <int W>
__device__ __forceinline__ double jump_ll(int kind, int site, double g, const Cfg<W> &mask) {
    const bool up = cfg_up(mask, site);
    if (kind == 0) return up ? g : 0.0;
    if (kind == 1) return up ? 0.0 : g;
    return g + g;
}

// <B^n> per channel.  A workgroup takes CM_CH channels of one trajectory; each thread sums a
// strided subset of the samples, then the block reduces in a fixed order (reproducible).
constexpr int CM_CH = 8;
template <int W>
__global__ __launch_bounds__(256) void k_channel_means(Dev a) {
    __shared__ double red[4][2 * CM_CH];
    const int t = blockIdx.y, c0 = blockIdx.x * CM_CH;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double2 *R = a.R + (size_t)t * a.ns * a.n;
    int kind[CM_CH], st[CM_CH];
    double sq[CM_CH], re[CM_CH], im[CM_CH];
    for (int q = 0; q < CM_CH; ++q) {
        const int ch = c0 + q < a.nch ? c0 + q : a.nch - 1;
        kind[q] = a.jkind[ch];
        st[q] = a.jsite[ch];
        sq[q] = sqrt(a.jrate[t * a.r_stride + ch]);
        re[q] = im[q] = 0.0;
    }
    for (int s = threadIdx.x; s < a.ns; s += blockDim.x) {
        const Cfg<W> mk = cfg_load<W>(smp + (size_t)s * W);
        const double2 *Rrow = R + (size_t)s * a.n;
        for (int q = 0; q < CM_CH; ++q) {
            const double2 b = jump_local(kind[q], st[q], sq[q], mk, Rrow);
            re[q] += b.x;
            im[q] += b.y;
        }
    }
    for (int q = 0; q < CM_CH; ++q) {
        const double r = wave_sum(re[q]), i = wave_sum(im[q]);
        if (lane == 0) {
            red[wave][2 * q] = r;
            red[wave][2 * q + 1] = i;
        }
    }
    __syncthreads();
    if (threadIdx.x < CM_CH && c0 + (int)threadIdx.x < a.nch) {
        const int q = threadIdx.x;
        const double r = (red[0][2 * q] + red[1][2 * q]) + (red[2][2 * q] + red[3][2 * q]);
        const double i = (red[0][2 * q + 1] + red[1][2 * q + 1]) + (red[2][2 * q + 1] + red[3][2 * q + 1]);
        const double norm = 1.0 / (double)a.ns;
        a.bmean[(size_t)t * a.nch + c0 + q] = make_double2(r * norm, i * norm);
    }
}

// G(x) per sample.
template <int W>
__global__ __launch_bounds__(256) void k_build_G(Dev a) {
    __shared__ int skind[256], ssite[256];
    __shared__ double srate[256], ssq[256], sdw[256], sc[256];
    const int t = blockIdx.y;
    for (int ch = threadIdx.x; ch < a.nch; ch += blockDim.x) {
        skind[ch] = a.jkind[ch];
        ssite[ch] = a.jsite[ch];
        srate[ch] = a.jrate[t * a.r_stride + ch];
        ssq[ch] = sqrt(a.jrate[t * a.r_stride + ch]);
        sdw[ch] = a.dw[(size_t)t * a.nch + ch];
        sc[ch] = a.linear ? 0.0 : 2.0 * (2.0 * a.bmean[(size_t)t * a.nch + ch].x);
    }
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.ns) return;
    const size_t sidx = (size_t)t * a.ns + s;
    const Cfg<W> mask = cfg_load<W>(a.samples + sidx * W);
    const double2 *Rrow = a.R + sidx * a.n;
    double dre = 0.0, dim = 0.0, ll = 0.0, nre = 0.0, nim = 0.0;
    for (int ch = 0; ch < a.nch; ++ch) {
        const double2 b = jump_local(skind[ch], ssite[ch], ssq[ch], mask, Rrow);
        dre += sc[ch] * b.x;
        dim += sc[ch] * b.y;
        ll += jump_ll(skind[ch], ssite[ch], srate[ch], mask);
        nre += b.x * sdw[ch];
        nim += b.y * sdw[ch];
    }
    const double2 e = a.eloc[sidx];
    const double eeff_re = e.x - 0.5 * dim;          // E_H - (i/2)(ll - drive)
    const double eeff_im = e.y - 0.5 * (ll - dre);
    a.G[sidx] = make_double2(a.dt * eeff_im + nre, -a.dt * eeff_re + nim);
}

// mean of G over the samples (fixed-order tree: reproducible).
__global__ __launch_bounds__(256) void k_gbar(Dev a) {
    __shared__ double sre[256], sim[256];
    const int t = blockIdx.x;
    const double2 *G = a.G + (size_t)t * a.ns;
    double re = 0.0, im = 0.0;
    for (int s = threadIdx.x; s < a.ns; s += blockDim.x) {
        re += G[s].x;
        im += G[s].y;
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
    if (threadIdx.x == 0) a.gbar[t] = make_double2(sre[0] / (double)a.ns, sim[0] / (double)a.ns);
}

// <O_k> and D_k = <O_k G> - <O_k><G> for the Jastrow ansaetze (O_k = s_i, s_j s_k, or an
// LJPHd distance sum when DIST: real integers; o G is exact for o = +-1, so the sums are the
// same for either instance).
template <bool DIST, int W>
__global__ __launch_bounds__(256) void k_obar_D(Dev a) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.m) return;
    const int p = a.pa[k], q = a.pb[k];
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double2 *G = a.G + (size_t)t * a.ns;
    int64_t cnt = 0;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < a.ns; ++s) {
        const int o = o_int<DIST>(cfg_load<W>(smp + (size_t)s * W), p, q, a.n);
        const double2 g = G[s];
        const double od = (double)o;
        cnt += o;
        re += od * g.x;
        im += od * g.y;
    }
    const double inv = 1.0 / (double)a.ns;
    const double ob = (double)cnt * inv;
    const double2 gb = a.gbar[t];
    a.obar[(size_t)t * a.m + k] = ob;
    a.D[(size_t)t * a.m + k] = make_double2(re * inv - ob * gb.x, im * inv - ob * gb.y);
}

}  // namespace tvmc
