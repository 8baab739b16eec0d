// Metropolis sampling of |psi_theta|^2 for the two-body Jastrow ansatz (Eq. 12) and the
// local quantities the estimators need (text after Eq. 9; definitions after Eq. 8).
//
// One wavefront per Markov chain; lane i owns spin i (N <= 64; two spins per lane up to N = 128
// in k_sample_jastrow_wn).  The configuration lives in a wave-uniform 64-bit mask.  Lane i keeps the complex field f_i = a_i + sum_{k!=i} eta_ik s_k,
// so the flip log-ratio of site i is -2 s_i f_i (O(1)); an accepted flip of site i updates
// every lane's field with one row of eta, read from LDS (the dense symmetric eta of the
// trajectory, staged once per workgroup and shared by its CPB chains).  Random numbers for
// 64 consecutive proposals are drawn at once, one Philox block per lane, and read back with
// readlane, so the sequential part of a proposal is a readlane, a compare and (on accept)
// one LDS row.
#pragma once
#include "common.hpp"
#include "made.hpp"

namespace tvmc {

// theta (or theta_eval) -> dense symmetric eta, split into real / imaginary planes (for LJPHd
// every pair at a shared distance reads that distance's parameter).
__global__ void k_prepare_jastrow(Dev a, const double2 *__restrict__ src) {
    const int t = blockIdx.y;
    const int n = a.n, nn = n * n;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    const int i = idx / n, k = idx % n;
    double re = 0.0, im = 0.0;
    if (i != k) {
        const double2 v = src[(size_t)t * a.m + a.pidx[idx]];
        re = v.x;
        im = v.y;
    }
    a.eta_re[(size_t)t * nn + idx] = re;
    a.eta_im[(size_t)t * nn + idx] = im;
}

// Uniformly random initial configurations (an exact sample of |psi|^2 at the +x state).
__global__ void k_init_chains(Dev a) {
    const int t = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nc) return;
    // blocks of 128 random bits, block b from the counter (b, chain, 0, 3 << 24 | trajectory):
    // its sites 0..63 from words 0, 1 of the draw and 64..127 from words 2, 3
    for (int q = 0; q < a.nw; ++q) {
        uint32_t r[4];
        philox4x32_10((uint32_t)(q >> 1), (uint32_t)c, 0u, (3u << 24) | (uint32_t)(a.traj0 + t), a.key0, a.key1, r);
        const int h = 2 * (q & 1);
        uint64_t m = (uint64_t)r[h] | ((uint64_t)r[h + 1] << 32);
        const int bits = a.n - 64 * q;
        if (bits < 64) m &= (1ull << bits) - 1ull;
        a.chains[((size_t)t * a.nc + c) * a.nw + q] = m;
    }
}

// the step index read by the samplers and k_draw_dw
__global__ void k_set_step(Dev a, int step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) a.dstep[0] = step;
}

// theta_eval = theta (the predictor's evaluation point)
__global__ void k_copy_theta(Dev a) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)a.nt * a.m) a.theta_eval[i] = a.theta[i];
}

// Real Gaussian Wiener increments dW ~ N(0, dt), Box-Muller on two 53-bit uniforms.
__global__ void k_draw_dw(Dev a) {
    const int t = blockIdx.x;
    const int step = a.dstep[0];
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = threadIdx.x; 2 * q < a.nch; q += blockDim.x) {
        uint32_t r[4];
        philox4x32_10((uint32_t)q, 0u, (uint32_t)step, (2u << 24) | (uint32_t)(a.traj0 + t), a.key0, a.key1, r);
        const double u1 = u53(r[0], r[1]), u2 = u53(r[2], r[3]);
        const double rad = sqrt(-2.0 * log(1.0 - u1));
        double sn, cs;
        sincos(two_pi * u2, &sn, &cs);
        a.dw[(size_t)t * a.nch + 2 * q] = sqrt(a.dt) * (rad * cs);
        if (2 * q + 1 < a.nch) a.dw[(size_t)t * a.nch + 2 * q + 1] = sqrt(a.dt) * (rad * sn);
    }
}

template <int CPB, bool AR>
__global__ __launch_bounds__(64 * CPB) void k_sample_jastrow(Dev a, int stage, int burn) {
    const int step = a.dstep[0];
    __shared__ double lre[64 * 64];
    __shared__ double lim[64 * 64];
    __shared__ uint16_t arw_s[AR ? 2 * AR_LDS_W : 1];
    __shared__ float arb_s[AR ? 256 + 64 : 1];
    const int n = a.n;
    const int t = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x * CPB + w;
    {
        const double *er = a.eta_re + (size_t)t * n * n;
        const double *ei = a.eta_im + (size_t)t * n * n;
        for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
            lre[i] = er[i];
            lim[i] = ei[i];
        }
    }
    ArNet net{};
    if (AR) net = ar_net(a, t, arw_s, arw_s + AR_LDS_W, arb_s, arb_s + 256);
    __syncthreads();
    const bool act = lane < n;
    const double2 *th = a.theta_eval + (size_t)t * a.m;
    uint64_t mask = a.chains[(size_t)t * a.nc + c];

    // fields in the order a_i, then k = 0..N-1 (each term is exact: s_k = +-1)
    double fre = 0.0, fim = 0.0;
    if (act) {
        fre = th[lane].x;
        fim = th[lane].y;
        for (int k = 0; k < n; ++k) {
            if (k == lane) continue;
            const double sk = spin(mask, k);
            fre += lre[k * n + lane] * sk;
            fim += lim[k * n + lane] * sk;
        }
    }

    const uint32_t ctr1 = ((uint32_t)stage << 31) | (uint32_t)c;
    const uint32_t ctr3 = (1u << 24) | (uint32_t)(a.traj0 + t);
    // proposal counts fit in 31 bits (checked on the host)
    const int total = (burn + a.per * a.thin) * n;
    const int rec_stride = a.thin * n;
    int next_rec = burn * n + rec_stride - 1;   // proposal after which the next sample is taken
    int rec = 0;
    uint32_t nacc = 0;
    const size_t tbase = (size_t)t * a.ns;
    // learned proposal: one independent proposal at the start of every sweep
    int next_ar = 0;
    uint32_t ar_idx = 0, ar_nacc = 0;
    float lq_cur = 0.f;
    bool lq_valid = false;

    for (int base = 0; base < total; base += 64) {
        uint32_t r[4];
        philox4x32_10((uint32_t)(base + lane), ctr1, (uint32_t)step, ctr3, a.key0, a.key1, r);
        const int site_l = (int)(((uint64_t)r[0] * (uint64_t)n) >> 32);
        const double logu_l = log(u53(r[1], r[2]));
        const int cnt = (total - base) < 64 ? (total - base) : 64;
        for (int j = 0; j < cnt; ++j) {
            if (AR && base + j == next_ar) {
                next_ar += n;
                if (!lq_valid) {
                    lq_cur = ar_logq(a, net, mask, lane);
                    lq_valid = true;
                }
                float lqn;
                double uacc;
                const uint64_t mnew = ar_draw(a, net, t, ctr1, step, ar_idx++, lane, lqn, uacc);
                // fields of s' and Re log psi of both configurations
                double nre = 0.0, nim = 0.0, lpc = 0.0, lpn = 0.0;
                if (act) {
                    nre = th[lane].x;
                    nim = th[lane].y;
                    for (int k = 0; k < n; ++k) {
                        if (k == lane) continue;
                        const double sk = spin(mnew, k);
                        nre += lre[k * n + lane] * sk;
                        nim += lim[k * n + lane] * sk;
                    }
                    lpc = 0.5 * spin(mask, lane) * (fre + th[lane].x);
                    lpn = 0.5 * spin(mnew, lane) * (nre + th[lane].x);
                }
                const double dlog = 2.0 * (wave_sum(lpn) - wave_sum(lpc)) + ((double)lq_cur - (double)lqn);
                if (log(uacc) < dlog) {
                    mask = mnew;
                    fre = nre;
                    fim = nim;
                    lq_cur = lqn;
                    ++ar_nacc;
                }
            }
            const int i = __builtin_amdgcn_readlane(site_l, j);
            const double lu = readlane_d(logu_l, j);
            const double fi = readlane_d(fre, i);
            const double si = spin(mask, i);
            const double dre = -2.0 * si * fi;
            if (lu < 2.0 * dre) {
                mask ^= (1ull << i);
                const double c2 = -2.0 * si;
                if (act) {
                    fre += c2 * lre[i * n + lane];
                    fim += c2 * lim[i * n + lane];
                }
                ++nacc;
                lq_valid = false;
            }
            if (base + j == next_rec) {
                const size_t sidx = tbase + (size_t)c * a.per + rec;
                ++rec;
                next_rec += rec_stride;
                double ere = 0.0, eim = 0.0;
                if (act) {
                    const double sl = spin(mask, lane);
                    const double dr = -2.0 * sl * fre, di = -2.0 * sl * fim;
                    const double ex = exp(dr);
                    double sn, cs;
                    sincos(di, &sn, &cs);
                    const double2 R = make_double2(ex * cs, ex * sn);
                    a.R[sidx * n + lane] = R;
                    double hj = 0.0;
                    for (int k = 0; k < n; ++k) hj += a.J[t * a.j_stride + k * n + lane] * spin(mask, k);
                    ere = 0.5 * sl * hj + a.hx * R.x;
                    eim = a.hx * R.y;
                }
                ere = wave_sum(ere);
                eim = wave_sum(eim);
                if (lane == 0) {
                    a.samples[sidx] = mask;
                    a.eloc[sidx] = make_double2(ere, eim);
                }
            }
        }
    }
    if (lane == 0) {
        a.chains[(size_t)t * a.nc + c] = mask;
        a.acc[(size_t)t * a.nc + c] = nacc;
        if (AR) a.aracc[(size_t)t * a.nc + c] = ar_nacc;
    }
}

// The same chain for 64 < N <= 192 (W = 2 or 3 configuration words).  Lane l owns sites l,
// l + 64, l + 128 and keeps their real fields, their imaginary fields and their Ising fields
// h_l = sum_k J_kl s_k; the real eta plane is staged in LDS where it fits (N <= 128: at most
// 128 KB) and read from global memory otherwise (a row of it is contiguous over the lanes'
// sites), and an accepted flip of site i adds -2 s_i times row i of each of the three planes
// (the imaginary eta plane and J from global memory), so a recorded sample reads its flip
// ratios and diagonal energy off the lanes' fields.  No learned proposal.
template <int CPB, int W>
__global__ __launch_bounds__(64 * CPB, W == 3 ? 4 : 1) void k_sample_jastrow_wn(Dev a, int stage, int burn) {
    static_assert(W == 2 || W == 3, "two or three configuration words");
    constexpr bool ETA_LDS = W == 2;
    const int step = a.dstep[0];
    __shared__ double lre_s[ETA_LDS ? 128 * 128 : 1];
    const int n = a.n;
    // Workgroup L runs on XCD L % 8; XCD x takes work items x * per .. x * per + per - 1, so
    // the N_c / CPB workgroups of a trajectory share one XCD's L2 (the rows of its eta planes
    // and of J that accepted flips read).  The grid is padded to a multiple of 8; padding
    // workgroups exit at once.
    const int nb = a.nc / CPB, per = (int)gridDim.x / 8;
    const int g = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (g >= nb * a.nt) return;
    const int t = g / nb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = (g % nb) * CPB + w;
    const double *er = a.eta_re + (size_t)t * n * n;
    if (ETA_LDS) {
        for (int i = threadIdx.x; i < n * n; i += blockDim.x) lre_s[i] = er[i];
        __syncthreads();
    }
    const double *lre = ETA_LDS ? lre_s : er;
    const double *eim_g = a.eta_im + (size_t)t * n * n;
    const double2 *th = a.theta_eval + (size_t)t * a.m;
    Cfg<W> cfg = cfg_load<W>(a.chains + ((size_t)t * a.nc + c) * W);

    const double *Jt = a.J + t * a.j_stride;
    double fre[W], fim[W], fh[W];
    for (int q = 0; q < W; ++q) {
        fre[q] = fim[q] = fh[q] = 0.0;
        const int site = lane + 64 * q;
        if (site >= n) continue;
        double f = th[site].x, g = th[site].y, h = 0.0;
        for (int k = 0; k < n; ++k) {
            const double sk = spin(cfg, k);
            h += Jt[k * n + site] * sk;
            if (k == site) continue;
            f += lre[k * n + site] * sk;
            g += eim_g[k * n + site] * sk;
        }
        fre[q] = f;
        fim[q] = g;
        fh[q] = h;
    }

    const uint32_t ctr1 = ((uint32_t)stage << 31) | (uint32_t)c;
    const uint32_t ctr3 = (1u << 24) | (uint32_t)(a.traj0 + t);
    const int total = (burn + a.per * a.thin) * n;
    const int rec_stride = a.thin * n;
    int next_rec = burn * n + rec_stride - 1;
    int rec = 0;
    uint32_t nacc = 0;
    const size_t tbase = (size_t)t * a.ns;

    for (int base = 0; base < total; base += 64) {
        uint32_t r[4];
        philox4x32_10((uint32_t)(base + lane), ctr1, (uint32_t)step, ctr3, a.key0, a.key1, r);
        const int site_l = (int)(((uint64_t)r[0] * (uint64_t)n) >> 32);
        const double logu_l = log(u53(r[1], r[2]));
        const int cnt = (total - base) < 64 ? (total - base) : 64;
        for (int j = 0; j < cnt; ++j) {
            const int i = __builtin_amdgcn_readlane(site_l, j);
            const double lu = readlane_d(logu_l, j);
            const int iq = i >> 6;
            double fsel = fre[0];
#pragma unroll
            for (int q = 1; q < W; ++q)
                if (iq == q) fsel = fre[q];
            const double fi = readlane_d(fsel, i & 63);
            const double si = spin(cfg, i);
            const double dre = -2.0 * si * fi;
            if (lu < 2.0 * dre) {
                cfg_flip(cfg, i);
                const double c2 = -2.0 * si;
                for (int q = 0; q < W; ++q) {
                    const int site = lane + 64 * q;
                    if (site < n) {   // eta_ii = 0; J_ii s_i is in h_i, as in the fresh sum
                        fre[q] += c2 * lre[i * n + site];
                        fim[q] += c2 * eim_g[i * n + site];
                        fh[q] += c2 * Jt[i * n + site];
                    }
                }
                ++nacc;
            }
            if (base + j == next_rec) {
                const size_t sidx = tbase + (size_t)c * a.per + rec;
                ++rec;
                next_rec += rec_stride;
                double ere = 0.0, eim = 0.0;
                for (int q = 0; q < W; ++q) {
                    const int site = lane + 64 * q;
                    if (site >= n) continue;
                    const double sl = spin(cfg, site);
                    const double hj = fh[q];
                    const double dr = -2.0 * sl * fre[q], di = -2.0 * sl * fim[q];
                    const double ex = exp(dr);
                    double sn, cs;
                    sincos(di, &sn, &cs);
                    const double2 R = make_double2(ex * cs, ex * sn);
                    a.R[sidx * n + site] = R;
                    ere += 0.5 * sl * hj + a.hx * R.x;
                    eim += a.hx * R.y;
                }
                ere = wave_sum(ere);
                eim = wave_sum(eim);
                if (lane == 0) {
                    cfg_store(a.samples + sidx * W, cfg);
                    a.eloc[sidx] = make_double2(ere, eim);
                }
            }
        }
    }
    if (lane == 0) {
        cfg_store(a.chains + ((size_t)t * a.nc + c) * W, cfg);
        a.acc[(size_t)t * a.nc + c] = nacc;
    }
}

}  // namespace tvmc
