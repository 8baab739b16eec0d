// Restricted-Boltzmann-machine ansatz (Eq. 11):
//   log psi(s) = sum_i a_i s_i + sum_j log 2cosh(g_j),   g_j = b_j + sum_i w_ij s_i,
//   O = (s_i ; tanh g_j ; s_i tanh g_j),  M = N + N' + N N' complex parameters.
// Sampling: one wavefront per chain, lane j owns hidden units j, j+64, ...; it keeps g_j and
// t_j = tanh g_j.  Flipping spin i multiplies psi by exp(-2 s_i a_i) prod_j cosh(g_j - 2 s_i
// w_ij) / cosh g_j, and each factor is cosh 2w_ij - s_i t_j sinh 2w_ij: with cosh 2w and
// sinh 2w tabulated once per evaluation, the accept test is a product of |.|^2 over the lanes
// (mantissas multiplied, exponents summed) compared with the uniform.  A learned proposal
// (a whole new configuration) compares log|cosh| sums.  The N single-flip ratios of a recorded
// sample (local energy) use the same factors, N N' complex multiply-adds per sample.
// The complex Hermitian S (lower triangle) is solved by the complex FP64 Cholesky.
#pragma once
#include "common.hpp"
#include "made.hpp"

namespace tvmc {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// log|cosh(x + i y)| = |x| - log 2 + log((1 + e)^2 - 4 e sin^2 y) / 2 with e = exp(-2|x|).
// The learned proposal's acceptance test takes its log-cosh differences as (|x'| - |x|) plus
// the differences of the last term (at most log 2), all in FP64, so the acceptance
// is the Metropolis-Hastings ratio for |psi|^2 itself up to double rounding.
__device__ __forceinline__ double log_cosh_rest(double x, double y) {
    const double e = exp(-2.0 * fabs(x)), sy = sin(y);
    return 0.5 * log((1.0 + e) * (1.0 + e) - 4.0 * e * sy * sy);
}

// tanh(x + i y) = (sinh 2x + i sin 2y) / (cosh 2x + cos 2y), written with e = exp(-2|x|)
__device__ __forceinline__ double2 ctanh_(double x, double y) {
    const double ax = fabs(x), e = exp(-2.0 * ax), e2 = e * e;
    double s2, c2;
    sincos(2.0 * y, &s2, &c2);
    // multiply numerator and denominator by 2 e^{-2|x|}
    const double den = 1.0 + e2 + 2.0 * e * c2;
    const double re = (1.0 - e2) / den, im = 2.0 * e * s2 / den;
    return make_double2(x < 0.0 ? -re : re, im);
}

// theta -> w planes [T][N][N'] and the tables cosh 2w, sinh 2w transposed [T][N'][N]
__global__ void k_prepare_rbm(Dev a, const double2 *__restrict__ src) {
    const int t = blockIdx.y;
    const int n = a.n, nh = a.nh;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nh) return;
    const int i = idx / nh, j = idx % nh;
    const double2 w = src[(size_t)t * a.m + n + nh + idx];
    a.w_re[(size_t)t * n * nh + idx] = w.x;
    a.w_im[(size_t)t * n * nh + idx] = w.y;
    const double x = 2.0 * w.x, y = 2.0 * w.y;
    double sy, cy;
    sincos(y, &sy, &cy);
    const double ch = cosh(x), sh = sinh(x);
    const double2 cw = make_double2(ch * cy, sh * sy), sw = make_double2(sh * cy, ch * sy);
    a.cT[((size_t)t * nh + j) * n + i] = cw;
    a.sT[((size_t)t * nh + j) * n + i] = sw;
    a.cW[(size_t)t * n * nh + idx] = cw;
    a.sW[(size_t)t * n * nh + idx] = sw;
}

// W_LDS: the weights fit in LDS (N N' <= 4096) and are read from there; a template flag, so
// that every weight read compiles to an LDS or a global instruction rather than a generic one.
// W: 64-bit words per configuration (W = 2: lane l owns the visible sites l and l + 64 for the
// single-flip factors and the recorded ratios; no learned proposal).
template <int CPB, int QH, bool AR, bool W_LDS, int W = 1>
__global__ __launch_bounds__(64 * CPB) void k_sample_rbm(Dev a, int stage, int burn) {
    static_assert(!AR || W == 1, "the learned proposal works on one configuration word");
    const int step = a.dstep[0];
    __shared__ double lwr[W_LDS ? 64 * 64 : 1];
    __shared__ double lwi[W_LDS ? 64 * 64 : 1];
    __shared__ double2 tl[CPB][64 * QH];
    __shared__ uint16_t arw_s[AR ? 2 * AR_LDS_W : 1];
    __shared__ float arb_s[AR ? 256 + 64 : 1];
    const int n = a.n, nh = a.nh;
    // Workgroup L runs on XCD L % 8; XCD x takes work items x * per .. x * per + per - 1, so
    // the N_c / CPB workgroups of a trajectory share one XCD's L2 (its cosh/sinh tables and
    // weights).  The grid is padded to a multiple of 8; padding workgroups exit at once.
    const int nb = a.nc / CPB, per = (int)gridDim.x / 8;
    const int g = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (g >= nb * a.nt) return;
    const int t = g / nb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = (g % nb) * CPB + w;
    const bool in_lds = W_LDS;
    const double *gwr = a.w_re + (size_t)t * n * nh, *gwi = a.w_im + (size_t)t * n * nh;
    if (in_lds) {
        for (int i = threadIdx.x; i < n * nh; i += blockDim.x) {
            lwr[i] = gwr[i];
            lwi[i] = gwi[i];
        }
    }
    ArNet net{};
    if (AR) net = ar_net(a, t, arw_s, arw_s + AR_LDS_W, arb_s, arb_s + 256);
    __syncthreads();
    const double *wr = W_LDS ? lwr : gwr;
    const double *wi = W_LDS ? lwi : gwi;
    const double2 *th = a.theta_eval + (size_t)t * a.m;
    Cfg<W> mask = cfg_load<W>(a.chains + ((size_t)t * a.nc + c) * W);

    // per hidden unit j (lane j, j + 64, ...): theta_j = b_j + sum_i w_ij s_i (updated in place)
    // and t_j = tanh theta_j
    double gre[QH], gim[QH], tr[QH], ti[QH];
    for (int q = 0; q < QH; ++q) {
        const int j = lane + 64 * q;
        gre[q] = gim[q] = tr[q] = ti[q] = 0.0;
        if (j < nh) {
            double xr = th[n + j].x, xi = th[n + j].y;   // b_j + sum_i w_ij s_i, i in order
            for (int i = 0; i < n; ++i) {
                const double si = spin(mask, i);
                xr += wr[i * nh + j] * si;
                xi += wi[i * nh + j] * si;
            }
            gre[q] = xr;
            gim[q] = xi;
            const double2 tj = ctanh_(xr, xi);
            tr[q] = tj.x;
            ti[q] = tj.y;
        }
    }
    // lane l, site l + 64 q: |exp(a (s' - s))|^2 for s = +1 (ev_dn) and s = -1 (ev_up)
    double ev_dn[W], ev_up[W];
    for (int q = 0; q < W; ++q) {
        ev_dn[q] = ev_up[q] = 1.0;
        if (lane + 64 * q < n) {
            ev_dn[q] = exp(-4.0 * th[lane + 64 * q].x);
            ev_up[q] = exp(4.0 * th[lane + 64 * q].x);
        }
    }

    const uint32_t ctr1 = ((uint32_t)stage << 31) | (uint32_t)c;
    const uint32_t ctr3 = (1u << 24) | (uint32_t)(a.traj0 + t);
    const int total = (burn + a.per * a.thin) * n;
    const int rec_stride = a.thin * n;
    int next_rec = burn * n + rec_stride - 1;
    int rec = 0;
    uint32_t nacc = 0;
    const size_t tbase = (size_t)t * a.ns;
    const double2 *cT = a.cT + (size_t)t * nh * n, *sT = a.sT + (size_t)t * nh * n;
    const double2 *cW = a.cW + (size_t)t * n * nh, *sW = a.sW + (size_t)t * n * nh;

    // learned proposal: one independent proposal at the start of every sweep
    int next_ar = 0;
    uint32_t ar_idx = 0, ar_nacc = 0;
    float lq_cur = 0.f;
    bool lq_valid = false;

    for (int base = 0; base < total; base += 64) {
        uint32_t r[4];
        philox4x32_10((uint32_t)(base + lane), ctr1, (uint32_t)step, ctr3, a.key0, a.key1, r);
        const int site_l = (int)(((uint64_t)r[0] * (uint64_t)n) >> 32);
        const double u_l = u53(r[1], r[2]);
        const int cnt = (total - base) < 64 ? (total - base) : 64;
        // cosh 2w_ij, sinh 2w_ij of the next flip's site, loaded one flip ahead
        double2 nc[QH], nsw[QH];
        {
            const int i0 = __builtin_amdgcn_readlane(site_l, 0);
            for (int q = 0; q < QH; ++q) {
                const int j = lane + 64 * q;
                nc[q] = nsw[q] = make_double2(0.0, 0.0);
                if (j < nh) {
                    nc[q] = cW[i0 * nh + j];
                    nsw[q] = sW[i0 * nh + j];
                }
            }
        }
        for (int jj = 0; jj < cnt; ++jj) {
            if (AR && base + jj == next_ar) {
                next_ar += n;
                if (!lq_valid) {
                    lq_cur = ar_logq(a, net, mask.w[0], lane);
                    lq_valid = true;
                }
                float lqn;
                double uacc;
                const uint64_t mnew = ar_draw(a, net, t, ctr1, step, ar_idx++, lane, lqn, uacc);
                // hidden pre-activations of s' (same summation order as at the start) and
                // Re log psi(s') - Re log psi(s)
                double ngr[QH], ngi[QH], dsum = 0.0;
                for (int q = 0; q < QH; ++q) {
                    const int j = lane + 64 * q;
                    ngr[q] = ngi[q] = 0.0;
                    if (j < nh) {
                        double xr = th[n + j].x, xi = th[n + j].y;
                        for (int i = 0; i < n; ++i) {
                            const double si = spin(mnew, i);
                            xr += wr[i * nh + j] * si;
                            xi += wi[i * nh + j] * si;
                        }
                        ngr[q] = xr;
                        ngi[q] = xi;
                        dsum += (fabs(xr) - fabs(gre[q])) +
                                (log_cosh_rest(xr, xi) - log_cosh_rest(gre[q], gim[q]));
                    }
                }
                if (lane < n) dsum += th[lane].x * (spin(mnew, lane) - spin(mask, lane));
                const double dlog = 2.0 * wave_sum(dsum) + ((double)lq_cur - (double)lqn);
                if (log(uacc) < dlog) {
                    mask.w[0] = mnew;
                    for (int q = 0; q < QH; ++q) {
                        const int j = lane + 64 * q;
                        gre[q] = ngr[q];
                        gim[q] = ngi[q];
                        if (j < nh) {
                            const double2 tj = ctanh_(ngr[q], ngi[q]);
                            tr[q] = tj.x;
                            ti[q] = tj.y;
                        }
                    }
                    lq_cur = lqn;
                    ++ar_nacc;
                }
            }
            const int i = __builtin_amdgcn_readlane(site_l, jj);
            const double u = readlane_d(u_l, jj);
            const double si = spin(mask, i);
            double2 cw[QH], sw[QH];
            for (int q = 0; q < QH; ++q) {
                cw[q] = nc[q];
                sw[q] = nsw[q];
            }
            if (jj + 1 < cnt) {
                const int i1 = __builtin_amdgcn_readlane(site_l, jj + 1);
                for (int q = 0; q < QH; ++q) {
                    const int j = lane + 64 * q;
                    if (j < nh) {
                        nc[q] = cW[i1 * nh + j];
                        nsw[q] = sW[i1 * nh + j];
                    }
                }
            }
            // cosh(theta_j - 2 s_i w_ij) / cosh(theta_j) = cosh 2w_ij - s_i t_j sinh 2w_ij; the
            // ratio |psi(s')/psi(s)|^2 is the product of |.|^2 over j times the visible factor,
            // formed as (product of frexp mantissas) * 2^(sum of exponents)
            double fr[QH], fi[QH], pm = 1.0;
            int pe = 0;
            for (int q = 0; q < QH; ++q) {
                const int j = lane + 64 * q;
                fr[q] = 1.0;
                fi[q] = 0.0;
                if (j < nh) {
                    const double tsr = tr[q] * sw[q].x - ti[q] * sw[q].y, tsi = tr[q] * sw[q].y + ti[q] * sw[q].x;
                    fr[q] = cw[q].x - si * tsr;
                    fi[q] = cw[q].y - si * tsi;
                    int e;
                    pm *= frexp(fr[q] * fr[q] + fi[q] * fi[q], &e);
                    pe += e;
                }
            }
            pm = wave_prod(pm);
            pe = wave_sum_i(pe);
            int ev;
            const int iq = W == 1 ? 0 : (i >> 6);
            const double mv = frexp(si > 0.0 ? readlane_d(ev_dn[iq], i & 63) : readlane_d(ev_up[iq], i & 63), &ev);
            if (u < ldexp(pm * mv, pe + ev)) {
                cfg_flip(mask, i);
                for (int q = 0; q < QH; ++q) {
                    const int j = lane + 64 * q;
                    if (j < nh) {
                        gre[q] -= 2.0 * si * wr[i * nh + j];
                        gim[q] -= 2.0 * si * wi[i * nh + j];
                        // tanh(theta - b) = (t cosh b - sinh b) / (cosh b - t sinh b)
                        const double gr = tr[q] * cw[q].x - ti[q] * cw[q].y - si * sw[q].x;
                        const double gi = tr[q] * cw[q].y + ti[q] * cw[q].x - si * sw[q].y;
                        const double inv = 1.0 / (fr[q] * fr[q] + fi[q] * fi[q]);
                        tr[q] = (gr * fr[q] + gi * fi[q]) * inv;
                        ti[q] = (gi * fr[q] - gr * fi[q]) * inv;
                    }
                }
                ++nacc;
                lq_valid = false;
            }
            if (base + jj == next_rec) {
                const size_t sidx = tbase + (size_t)c * a.per + rec;
                ++rec;
                next_rec += rec_stride;
                for (int q = 0; q < QH; ++q) {
                    const int j = lane + 64 * q;
                    if (j < nh) {
                        const double2 tj = ctanh_(gre[q], gim[q]);
                        tl[w][j] = tj;
                        a.tt[sidx * nh + j] = tj;
                        tr[q] = tj.x;
                        ti[q] = tj.y;
                    }
                }
                double ere = 0.0, eim = 0.0;
                for (int q = 0; q < W; ++q) {
                    const int site = lane + 64 * q;
                    if (site >= n) continue;
                    const double sl = spin(mask, site);
                    // prod_j (cosh 2w_lj - s_l t_j sinh 2w_lj), rescaled by a power of two every
                    // 16 factors (exponents summed in pe)
                    double pr = 1.0, pi = 0.0;
                    int pe = 0;
                    for (int j = 0; j < nh; ++j) {
                        const double2 ch = cT[(size_t)j * n + site], sh = sT[(size_t)j * n + site];
                        const double2 ts = cmul(tl[w][j], sh);
                        const double fr = ch.x - sl * ts.x, fi = ch.y - sl * ts.y;
                        const double nr = pr * fr - pi * fi, ni = pr * fi + pi * fr;
                        pr = nr;
                        pi = ni;
                        if ((j & 15) == 15) {
                            int e;
                            frexp(fmax(fabs(pr), fabs(pi)), &e);
                            pr = ldexp(pr, -e);
                            pi = ldexp(pi, -e);
                            pe += e;
                        }
                    }
                    const double er = -2.0 * sl * th[site].x, ei = -2.0 * sl * th[site].y;
                    const double ex = exp(er);
                    double sn, cs;
                    sincos(ei, &sn, &cs);
                    const double2 Rm = cmul(make_double2(pr, pi), make_double2(ex * cs, ex * sn));
                    const double2 R = make_double2(ldexp(Rm.x, pe), ldexp(Rm.y, pe));
                    a.R[sidx * n + site] = R;
                    double hj = 0.0;
                    for (int k = 0; k < n; ++k) hj += a.J[t * a.j_stride + k * n + site] * spin(mask, k);
                    ere += 0.5 * sl * hj + a.hx * R.x;
                    eim += a.hx * R.y;
                }
                ere = wave_sum(ere);
                eim = wave_sum(eim);
                if (lane == 0) {
                    cfg_store(a.samples + sidx * W, mask);
                    a.eloc[sidx] = make_double2(ere, eim);
                }
            }
        }
    }
    if (lane == 0) {
        cfg_store(a.chains + ((size_t)t * a.nc + c) * W, mask);
        a.acc[(size_t)t * a.nc + c] = nacc;
        if (AR) a.aracc[(size_t)t * a.nc + c] = ar_nacc;
    }
}

// O_k of sample s (complex): one-body s_i, hidden tanh g_j, weights s_i tanh g_j
template <typename C>
__device__ __forceinline__ double2 rbm_o(const Dev &a, int k, const C &mk, const double2 *tts) {
    if (k < a.n) return make_double2(spin(mk, k), 0.0);
    if (k < a.n + a.nh) return tts[k - a.n];
    const int idx = k - a.n - a.nh, i = idx / a.nh, j = idx % a.nh;
    const double si = spin(mk, i);
    const double2 tj = tts[j];
    return make_double2(si * tj.x, si * tj.y);
}

// <O_k> and D_k = <O_k^* G> - <O_k>^* <G>
// Lane l of the workgroup's 4 waves takes the 8 parameters k_c = 512 b + 64 c + l (b: the
// workgroup's block of its trajectory's parameters)
// (c < 8); wave w sums the samples of quarter w of the batch, and the four partial sums are
// added in wave order.  Weight rows k_c with the same hidden unit j (all 8 of them when N'
// divides 64 and the weights start on a multiple of 64) share one load of tanh g_j per sample.
constexpr int OD_R = 8;
template <int W>
__global__ __launch_bounds__(256) void k_obar_D_rbm(Dev a) {
    // waves 1..3 leave their partial sums here; wave 0 keeps its own in registers (48 KB, three
    // workgroups per compute unit)
    __shared__ double part[3][OD_R][4][64];
    // Workgroup L runs on XCD L % 8; XCD x takes work items x * per .. x * per + per - 1, so
    // the workgroups of a trajectory share one XCD's L2 copy of its samples, G and tanh rows.
    // The grid is padded to a multiple of 8; padding workgroups exit at once.
    const int nb = (a.m + 64 * OD_R - 1) / (64 * OD_R), per = (int)gridDim.x / 8;
    const int g = ((int)blockIdx.x & 7) * per + ((int)blockIdx.x >> 3);
    if (g >= nb * a.nt) return;
    const int t = g / nb, bx = g % nb;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, nh = a.nh, wb = n + nh;
    int ki[OD_R], kj[OD_R];
    int jl = -1;
    for (int c = 0; c < OD_R; ++c) {
        const int k = bx * 64 * OD_R + 64 * c + lane;
        ki[c] = kj[c] = -1;
        if (k >= wb && k < a.m) {
            ki[c] = (k - wb) / nh;
            kj[c] = (k - wb) % nh;
            if (jl < 0) jl = kj[c];
        }
    }
    double acc[OD_R][4];
    for (int c = 0; c < OD_R; ++c) acc[c][0] = acc[c][1] = acc[c][2] = acc[c][3] = 0.0;
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double2 *G = a.G + (size_t)t * a.ns;
    const double2 *tt = a.tt + (size_t)t * a.ns * nh;
    const int q = (a.ns + 3) / 4, s1 = min(a.ns, (w + 1) * q);
    for (int s = w * q; s < s1; ++s) {
        const Cfg<W> mk = cfg_load<W>(smp + (size_t)s * W);
        const double2 g = G[s];
        const double2 *tts = tt + (size_t)s * nh;
        const double2 tv = jl >= 0 ? tts[jl] : make_double2(0.0, 0.0);
        for (int c = 0; c < OD_R; ++c) {
            const int k = bx * 64 * OD_R + 64 * c + lane;
            if (k >= a.m) continue;
            double2 o;
            if (ki[c] >= 0 && kj[c] == jl) {
                const double si = spin(mk, ki[c]);
                o = make_double2(si * tv.x, si * tv.y);
            } else {
                o = rbm_o(a, k, mk, tts);
            }
            acc[c][0] += o.x;
            acc[c][1] += o.y;
            acc[c][2] += o.x * g.x + o.y * g.y;   // conj(o) g
            acc[c][3] += o.x * g.y - o.y * g.x;
        }
    }
    if (w > 0)
        for (int c = 0; c < OD_R; ++c)
            for (int v = 0; v < 4; ++v) part[w - 1][c][v][lane] = acc[c][v];
    __syncthreads();
    if (w != 0) return;
    const double inv = 1.0 / (double)a.ns;
    const double2 gb = a.gbar[t];
    for (int c = 0; c < OD_R; ++c) {
        const int k = bx * 64 * OD_R + 64 * c + lane;
        if (k >= a.m) continue;
        double sum[4];
        for (int v = 0; v < 4; ++v) sum[v] = acc[c][v] + part[0][c][v][lane] + part[1][c][v][lane] + part[2][c][v][lane];
        const double obr = sum[0] * inv, obi = sum[1] * inv;
        a.obarc[(size_t)t * a.m + k] = make_double2(obr, obi);
        a.D[(size_t)t * a.m + k] =
            make_double2(sum[2] * inv - (obr * gb.x + obi * gb.y), sum[3] * inv - (obr * gb.y - obi * gb.x));
    }
}

// Complex S + eps I (lower triangle, interleaved re/im), plain FP64:
// 32x32 complex tile per workgroup, 2x2 complex register tile per thread, samples staged 8 at
// a time (configuration word and tanh g row) through LDS.
constexpr int RB_T = 32;
constexpr int RB_S = 8;
template <int W>
__global__ __launch_bounds__(256) void k_sbuild_rbm_f64(Dev a) {
    __shared__ Cfg<W> smask[RB_S];
    __shared__ double2 stt[RB_S][256];
    const int t = blockIdx.y;
    const int tile = blockIdx.x;
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m = a.m, nh = a.nh;
    double2 acc[2][2] = {};
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    const double2 *tt = a.tt + (size_t)t * a.ns * nh;
    for (int s0 = 0; s0 < a.ns; s0 += RB_S) {
        const int cnt = (a.ns - s0) < RB_S ? (a.ns - s0) : RB_S;
        __syncthreads();
        if (threadIdx.x < cnt) smask[threadIdx.x] = cfg_load<W>(smp + (size_t)(s0 + threadIdx.x) * W);
        for (int e = threadIdx.x; e < cnt * nh; e += blockDim.x) stt[e / nh][e % nh] = tt[(size_t)(s0 + e / nh) * nh + e % nh];
        __syncthreads();
        for (int s = 0; s < cnt; ++s) {
            double2 ov[2], cv[2];
            for (int u = 0; u < 2; ++u) {
                const int k = bi * RB_T + ty * 2 + u, l = bj * RB_T + tx * 2 + u;
                ov[u] = k < m ? rbm_o(a, k, smask[s], stt[s]) : make_double2(0.0, 0.0);
                cv[u] = l < m ? rbm_o(a, l, smask[s], stt[s]) : make_double2(0.0, 0.0);
            }
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) {   // conj(o_k) o_l
                    acc[u][v].x += ov[u].x * cv[v].x + ov[u].y * cv[v].y;
                    acc[u][v].y += ov[u].x * cv[v].y - ov[u].y * cv[v].x;
                }
        }
    }
    const double inv = 1.0 / (double)a.ns;
    const double2 *ob = a.obarc + (size_t)t * m;
    double2 *S = (double2 *)a.S + (size_t)t * m * m;
    for (int u = 0; u < 2; ++u) {
        const int k = bi * RB_T + ty * 2 + u;
        if (k >= m) continue;
        for (int v = 0; v < 2; ++v) {
            const int l = bj * RB_T + tx * 2 + v;
            if (l >= m || l > k) continue;
            // S_kl = <O_k^* O_l> - <O_k>^* <O_l>
            double re = acc[u][v].x * inv - (ob[k].x * ob[l].x + ob[k].y * ob[l].y);
            const double im = acc[u][v].y * inv - (ob[k].x * ob[l].y - ob[k].y * ob[l].x);
            if (k == l) re += a.eps;
            S[(size_t)k * m + l] = make_double2(re, k == l ? 0.0 : im);
        }
    }
}

// Moments for the RBM, factored form (N N' <= 4096): with u = 2 s_a w_aj, v = 2 s_b w_bj and
// f_j(a) = cosh u - t_j sinh u (t_j = tanh g_j), the two-flip factor is
//   cosh(u + v) - t_j sinh(u + v) = f_j(a) f_j(b) + (1 - t_j^2) sinh u sinh v,
// so psi(s^(ab))/psi(s) = R_a R_b prod_j (1 + beta_j(a) alpha_j(b)) with alpha_j(a) =
// sinh u / f_j(a), beta_j(a) = (1 - t_j^2) alpha_j(a) and R_a the single-flip ratio.  A
// workgroup takes one sample at a time: alpha and beta for all (j, a) in LDS, then every
// unordered pair a < b (pairs spread over the 8 waves, a on the lanes, RMF_PB values of b per
// pass: that many independent product chains per lane, with two waves per SIMD, to cover the
// multiply latency) multiplies N' factors 1 + beta alpha, rescaled by a power of two every 16
// (exact).  The pair terms are symmetric except s_b Im R_ab, which enters as (s_a + s_b) Im R_ab.
constexpr int RMF_WAVES = 8;
constexpr int RMF_PB = 8;
__global__ __launch_bounds__(64 * RMF_WAVES) void k_moments_rbm_f(Dev a) {
    __shared__ double2 al[64 * 64], be[64 * 64];      // [j][a]
    __shared__ double2 tl[64];
    __shared__ double part[RMF_WAVES][9];
    const int t = blockIdx.y;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int n = a.n, nh = a.nh;
    const double N = (double)n;
    double acc[9] = {};
    const double2 *cT = a.cT + (size_t)t * nh * n, *sT = a.sT + (size_t)t * nh * n;
    for (int s = blockIdx.x; s < a.ns; s += gridDim.x) {
        const size_t sidx = (size_t)t * a.ns + s;
        const uint64_t mk = a.samples[sidx];
        __syncthreads();   // the previous sample's tables are no longer read
        for (int j = tid; j < nh; j += blockDim.x) tl[j] = a.tt[sidx * nh + j];
        __syncthreads();
        for (int e = tid; e < n * nh; e += blockDim.x) {
            const int j = e / n, i = e % n;
            const double si = spin(mk, i);
            const double2 ch = cT[e], sh = sT[e], tj = tl[j];
            const double2 sh_s = make_double2(si * sh.x, si * sh.y);            // sinh u
            const double2 ts = cmul(tj, sh_s);
            const double2 f = make_double2(ch.x - ts.x, ch.y - ts.y);           // f_j(i)
            const double fi = 1.0 / (f.x * f.x + f.y * f.y);
            const double2 alpha = make_double2((sh_s.x * f.x + sh_s.y * f.y) * fi, (sh_s.y * f.x - sh_s.x * f.y) * fi);
            const double2 t2 = cmul(tj, tj);
            al[e] = alpha;
            be[e] = cmul(make_double2(1.0 - t2.x, -t2.y), alpha);
        }
        __syncthreads();
        const bool act = lane < n;
        const double sa = spin(mk, lane);
        const double2 Ra = act ? a.R[sidx * n + lane] : make_double2(0.0, 0.0);
        double v[9] = {};
        if (w == 0 && act) {
            // single-flip terms and the pair sums that need only R_a
            int up = 0;
            for (int b = 0; b < n; ++b) up += (int)((mk >> b) & 1ull);
            const double ssum = (double)(2 * up - n) - sa;        // sum_{b != a} s_b
            v[0] = Ra.x;
            v[1] = sa * Ra.y;
            v[2] = sa;
            v[5] = sa * ssum;
            v[7] = ssum * Ra.x;
            v[8] = sa * ssum * Ra.y;
        }
        // wave w takes b = 1 + w + RMF_WAVES c; RMF_PB values of b at a time (b0 + RMF_WAVES k)
        // give RMF_PB independent product chains per lane
        const int li = act ? lane : 0;
        for (int b0 = 1 + w; b0 < n; b0 += RMF_PB * RMF_WAVES) {
            double pr[RMF_PB], pi[RMF_PB];
            int ex2[RMF_PB], bk[RMF_PB];   // products kept as (pr + i pi) 2^ex2, rescaled by powers of two
            for (int k = 0; k < RMF_PB; ++k) {
                pr[k] = 1.0;
                pi[k] = 0.0;
                ex2[k] = 0;
                bk[k] = b0 + RMF_WAVES * k < n ? b0 + RMF_WAVES * k : n - 1;
            }
            int blast = b0;
            for (int k = 1; k < RMF_PB; ++k)
                if (b0 + RMF_WAVES * k < n) blast = b0 + RMF_WAVES * k;
            if (!(act && lane < blast)) continue;   // pairs a < b of the group
            for (int j = 0; j < nh; ++j) {
                const double2 x = be[j * n + li];
                for (int k = 0; k < RMF_PB; ++k) {
                    const double2 y = al[j * n + bk[k]];
                    const double fr = 1.0 + (x.x * y.x - x.y * y.y), fi = x.x * y.y + x.y * y.x;
                    const double nr = pr[k] * fr - pi[k] * fi, ni = pr[k] * fi + pi[k] * fr;
                    pr[k] = nr;
                    pi[k] = ni;
                }
                if ((j & 15) == 15)
                    for (int k = 0; k < RMF_PB; ++k) {
                        int e;
                        frexp(fabs(pr[k]) + fabs(pi[k]), &e);
                        pr[k] = ldexp(pr[k], -e);
                        pi[k] = ldexp(pi[k], -e);
                        ex2[k] += e;
                    }
            }
            for (int k = 0; k < RMF_PB; ++k) {
                const int b = b0 + RMF_WAVES * k;
                if (b >= n) break;
                if (lane >= b) continue;
                const double sb = spin(mk, b), ss = sa * sb;
                const double2 Rb = a.R[sidx * n + b];
                const double2 Rab = cmul(cmul(Ra, Rb), make_double2(ldexp(pr[k], ex2[k]), ldexp(pi[k], ex2[k])));
                v[3] += 2.0 * Rab.x;
                v[4] += -2.0 * ss * Rab.x;
                v[6] += (sa + sb) * Rab.y;
            }
        }
        for (int q = 0; q < 9; ++q) acc[q] += v[q];
    }
    // per-sample normalisation as in the direct kernel: m = v / N, s = (N + v) / N^2 summed
    // over samples; the N / N^2 constants are added once per sample below
    for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0)
        for (int q = 0; q < 9; ++q) part[w][q] = acc[q];
    __syncthreads();
    if (tid < 9) {
        double v = 0.0;
        for (int ww = 0; ww < RMF_WAVES; ++ww) v += part[ww][tid];
        int cnt = 0;   // samples this workgroup took
        for (int s = blockIdx.x; s < a.ns; s += gridDim.x) ++cnt;
        double r;
        if (tid < 3) r = v / N;
        else if (tid < 6) r = (N * cnt + v) / (N * N);
        else r = v / (N * N);
        a.mom_part[((size_t)t * a.mom_blocks + blockIdx.x) * 9 + tid] = r;
    }
}

// Moments for the RBM, factored form with the tables in global memory (N > 64 or N N' > 4096,
// where alpha and beta do not fit LDS): the same pair products as k_moments_rbm_f, each
// workgroup writing alpha and beta of its current sample to its own slice of the workspace
// (2 N N' complex, read back from L2), lanes a = lane + 64 q over the configuration's words.
template <int W>
__global__ __launch_bounds__(64 * RMF_WAVES) void k_moments_rbm_g(Dev a) {
    __shared__ double2 tl[256];
    __shared__ double part[RMF_WAVES][9];
    const int t = blockIdx.y;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int n = a.n, nh = a.nh;
    const double N = (double)n;
    double acc[9] = {};
    const double2 *cT = a.cT + (size_t)t * nh * n, *sT = a.sT + (size_t)t * nh * n;
    double2 *al = a.momtab + ((size_t)t * a.mom_blocks + blockIdx.x) * 2 * (size_t)n * nh;   // [j][a]
    double2 *be = al + (size_t)n * nh;
    for (int s = blockIdx.x; s < a.ns; s += gridDim.x) {
        const size_t sidx = (size_t)t * a.ns + s;
        const Cfg<W> mk = cfg_load<W>(a.samples + sidx * W);
        __syncthreads();   // the previous sample's tables are no longer read
        for (int j = tid; j < nh; j += blockDim.x) tl[j] = a.tt[sidx * nh + j];
        __syncthreads();
        for (int e = tid; e < n * nh; e += blockDim.x) {
            const int j = e / n, i = e % n;
            const double si = spin(mk, i);
            const double2 ch = cT[e], sh = sT[e], tj = tl[j];
            const double2 sh_s = make_double2(si * sh.x, si * sh.y);            // sinh u
            const double2 ts = cmul(tj, sh_s);
            const double2 f = make_double2(ch.x - ts.x, ch.y - ts.y);           // f_j(i)
            const double fi = 1.0 / (f.x * f.x + f.y * f.y);
            const double2 alpha = make_double2((sh_s.x * f.x + sh_s.y * f.y) * fi, (sh_s.y * f.x - sh_s.x * f.y) * fi);
            const double2 t2 = cmul(tj, tj);
            al[e] = alpha;
            be[e] = cmul(make_double2(1.0 - t2.x, -t2.y), alpha);
        }
        __syncthreads();   // the tables are written before any wave reads them
        double v[9] = {};
        int up = 0;
        for (int q = 0; q < W; ++q) up += __popcll(mk.w[q]);
        for (int q = 0; q < W; ++q) {
            const int ai = lane + 64 * q;
            const bool act = ai < n;
            const double sa = act ? spin(mk, ai) : 1.0;
            const double2 Ra = act ? a.R[sidx * n + ai] : make_double2(0.0, 0.0);
            if (w == 0 && act) {
                // single-flip terms and the pair sums that need only R_a
                const double ssum = (double)(2 * up - n) - sa;   // sum_{b != a} s_b
                v[0] += Ra.x;
                v[1] += sa * Ra.y;
                v[2] += sa;
                v[5] += sa * ssum;
                v[7] += ssum * Ra.x;
                v[8] += sa * ssum * Ra.y;
            }
            const int li = act ? ai : 0;
            for (int b0 = 1 + w; b0 < n; b0 += RMF_PB * RMF_WAVES) {
                double pr[RMF_PB], pi[RMF_PB];
                int ex2[RMF_PB], bk[RMF_PB];
                for (int k = 0; k < RMF_PB; ++k) {
                    pr[k] = 1.0;
                    pi[k] = 0.0;
                    ex2[k] = 0;
                    bk[k] = b0 + RMF_WAVES * k < n ? b0 + RMF_WAVES * k : n - 1;
                }
                int blast = b0;
                for (int k = 1; k < RMF_PB; ++k)
                    if (b0 + RMF_WAVES * k < n) blast = b0 + RMF_WAVES * k;
                if (!(act && ai < blast)) continue;   // pairs a < b of the group
                for (int j = 0; j < nh; ++j) {
                    const double2 x = be[(size_t)j * n + li];
                    for (int k = 0; k < RMF_PB; ++k) {
                        const double2 y = al[(size_t)j * n + bk[k]];
                        const double fr = 1.0 + (x.x * y.x - x.y * y.y), fi = x.x * y.y + x.y * y.x;
                        const double nr = pr[k] * fr - pi[k] * fi, ni = pr[k] * fi + pi[k] * fr;
                        pr[k] = nr;
                        pi[k] = ni;
                    }
                    if ((j & 15) == 15)
                        for (int k = 0; k < RMF_PB; ++k) {
                            int e;
                            frexp(fabs(pr[k]) + fabs(pi[k]), &e);
                            pr[k] = ldexp(pr[k], -e);
                            pi[k] = ldexp(pi[k], -e);
                            ex2[k] += e;
                        }
                }
                for (int k = 0; k < RMF_PB; ++k) {
                    const int b = b0 + RMF_WAVES * k;
                    if (b >= n) break;
                    if (ai >= b) continue;
                    const double sb = spin(mk, b), ss = sa * sb;
                    const double2 Rb = a.R[sidx * n + b];
                    const double2 Rab = cmul(cmul(Ra, Rb), make_double2(ldexp(pr[k], ex2[k]), ldexp(pi[k], ex2[k])));
                    v[3] += 2.0 * Rab.x;
                    v[4] += -2.0 * ss * Rab.x;
                    v[6] += (sa + sb) * Rab.y;
                }
            }
        }
        for (int q = 0; q < 9; ++q) acc[q] += v[q];
    }
    for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
    if (lane == 0)
        for (int q = 0; q < 9; ++q) part[w][q] = acc[q];
    __syncthreads();
    if (tid < 9) {
        double v = 0.0;
        for (int ww = 0; ww < RMF_WAVES; ++ww) v += part[ww][tid];
        int cnt = 0;   // samples this workgroup took
        for (int s = blockIdx.x; s < a.ns; s += gridDim.x) ++cnt;
        double r;
        if (tid < 3) r = v / N;
        else if (tid < 6) r = (N * cnt + v) / (N * N);
        else r = v / (N * N);
        a.mom_part[((size_t)t * a.mom_blocks + blockIdx.x) * 9 + tid] = r;
    }
}

}  // namespace tvmc
