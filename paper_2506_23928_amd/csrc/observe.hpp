// Predictor-corrector updates (App. C) and the observables of the LITF section:
// magnetisation M_a = <(1/N) sum_i sigma^a_i>, moments s_ab = (1/2)<{M_a, M_b}>, the
// trajectory average of Eq. 3, C_ab = avg s_ab - M_a M_b and Wineland's xi^2.
#pragma once
#include "common.hpp"

namespace tvmc {

// stage 0: theta_eval = theta + d0 (Heun) or theta + d0/2 (midpoint)
// stage 1: theta = theta + (d0 + d1)/2 (Heun) or theta + d1 (midpoint)
// Linear SSE: log Q by the same scheme, its increment at an evaluation point being 2 Re <G>
// (the norm SDE of App. B in Stratonovich form, so the chain rule holds for log Q).
__global__ void k_update(Dev a, int stage) {
    const int t = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (a.linear && k == 0) {
        const double q = 2.0 * a.gbar[t].x;
        if (stage == 0) a.dq0[t] = q;
        else a.lognorm[t] += a.scheme == 0 ? 0.5 * (a.dq0[t] + q) : q;
    }
    if (k >= a.m) return;
    const size_t i = (size_t)t * a.m + k;
    const double2 th = a.theta[i], d0 = a.d0[i];
    if (stage == 0) {
        a.theta_eval[i] = a.scheme == 0 ? make_double2(th.x + d0.x, th.y + d0.y)
                                        : make_double2(th.x + 0.5 * d0.x, th.y + 0.5 * d0.y);
    } else {
        const double2 d1 = a.d1[i];
        a.theta[i] = a.scheme == 0 ? make_double2(th.x + 0.5 * (d0.x + d1.x), th.y + 0.5 * (d0.y + d1.y))
                                   : make_double2(th.x + d1.x, th.y + d1.y);
    }
}

// exp(+4 eta_ab) and exp(-4 eta_ab): the pair factor of a two-flip ratio,
// psi(s^(ab))/psi(s) = R_a R_b exp(4 s_a s_b eta_ab).
__global__ void k_prepare_pairs(Dev a) {
    const int t = blockIdx.y;
    const int nn = a.n * a.n;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nn) return;
    const double re = a.eta_re[(size_t)t * nn + idx], im = a.eta_im[(size_t)t * nn + idx];
    double sn, cs;
    sincos(4.0 * im, &sn, &cs);
    const double ep = exp(4.0 * re), em = exp(-4.0 * re);
    a.epair[(size_t)t * 2 * nn + idx] = make_double2(ep * cs, ep * sn);
    a.epair[(size_t)t * 2 * nn + nn + idx] = make_double2(em * cs, -em * sn);
}

// One wavefront per sample, lane a = site a (and a + 64 for two-word configurations);
// per-block partial sums of the 9 moments.
constexpr int MOM_WAVES = 4;
template <int W>
__global__ __launch_bounds__(64 * MOM_WAVES) void k_moments(Dev a) {
    __shared__ double part[MOM_WAVES][9];
    const int t = blockIdx.y;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, nn = n * n;
    const double N = (double)n;
    double acc[9] = {};
    const double2 *ep = a.epair + (size_t)t * 2 * nn;
    for (int s = blockIdx.x * MOM_WAVES + w; s < a.ns; s += gridDim.x * MOM_WAVES) {
        const size_t sidx = (size_t)t * a.ns + s;
        const Cfg<W> mk = cfg_load<W>(a.samples + sidx * W);
        double sa[W];
        double2 Ra[W];
        bool act[W];
        double v[9] = {};
        for (int q = 0; q < W; ++q) {
            const int ai = lane + 64 * q;
            act[q] = ai < n;
            sa[q] = spin(mk, ai < n ? ai : 0);
            Ra[q] = act[q] ? a.R[sidx * n + ai] : make_double2(0.0, 0.0);
            if (act[q]) {
                v[0] += Ra[q].x;
                v[1] += sa[q] * Ra[q].y;
                v[2] += sa[q];
            }
        }
        for (int b = 0; b < n; ++b) {
            const int bq = W == 1 ? 0 : (b >> 6);
            const double rbx = readlane_d(Ra[bq].x, b & 63), rby = readlane_d(Ra[bq].y, b & 63);
            const double sb = spin(mk, b);
            for (int q = 0; q < W; ++q) {
                const int ai = lane + 64 * q;
                if (!act[q] || b == ai) continue;
                const double ss = sa[q] * sb;
                const double2 e = ep[(ss > 0.0 ? 0 : nn) + b * n + ai];
                const double px = Ra[q].x * rbx - Ra[q].y * rby, py = Ra[q].x * rby + Ra[q].y * rbx;
                const double rx = px * e.x - py * e.y, ry = px * e.y + py * e.x;
                v[3] += rx;
                v[4] += -ss * rx;
                v[5] += ss;
                v[6] += sb * ry;
                v[7] += sb * Ra[q].x;
                v[8] += ss * Ra[q].y;
            }
        }
        for (int q = 0; q < 9; ++q) v[q] = wave_sum(v[q]);
        acc[0] += v[0] / N;
        acc[1] += v[1] / N;
        acc[2] += v[2] / N;
        acc[3] += (N + v[3]) / (N * N);
        acc[4] += (N + v[4]) / (N * N);
        acc[5] += (N + v[5]) / (N * N);
        acc[6] += v[6] / (N * N);
        acc[7] += v[7] / (N * N);
        acc[8] += v[8] / (N * N);
    }
    if (lane == 0)
        for (int q = 0; q < 9; ++q) part[w][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 9) {
        double s = 0.0;
        for (int ww = 0; ww < MOM_WAVES; ++ww) s += part[ww][threadIdx.x];
        a.mom_part[((size_t)t * a.mom_blocks + blockIdx.x) * 9 + threadIdx.x] = s;
    }
}

// per-trajectory mean over the sample blocks, optionally stored into the history slot
__global__ void k_moments_reduce(Dev a, int slot) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.nt) return;
    for (int q = 0; q < 9; ++q) {
        double s = 0.0;
        for (int b = 0; b < a.mom_blocks; ++b) s += a.mom_part[((size_t)t * a.mom_blocks + b) * 9 + q];
        s /= (double)a.ns;
        a.mom[(size_t)t * 9 + q] = s;
        if (slot >= 0) a.hist[((size_t)slot * a.nt + t) * 9 + q] = s;
    }
    a.momlq[t] = a.lognorm[t];
    if (slot >= 0) a.qhist[(size_t)slot * a.nt + t] = a.lognorm[t];
}

// Trajectory average (Eq. 3) -> M, C, xi^2 = N lambda_min(C restricted to the plane
// orthogonal to M) / |M|^2.  Linear SSE: each trajectory's moments weighted by its Q (App. B),
// still divided by N_T.  slot < 0: the last moments; otherwise history record `slot`.  Block b
// of the launch leaves out trajectory b - 1 (block 0 leaves out none) and writes its 13 values
// to out[16 b ..]: the leave-one-out ensembles of a jackknife over the trajectories.
__global__ void k_ensemble(Dev a, int slot, double *out) {
    __shared__ double avg[9];
    const int skip = (int)blockIdx.x - 1;
    const double *mom = slot < 0 ? a.mom : a.hist + (size_t)slot * a.nt * 9;
    const double *lq = slot < 0 ? a.momlq : a.qhist + (size_t)slot * a.nt;
    const int cnt = skip < 0 ? a.nt : a.nt - 1;
    if (threadIdx.x < 9) {
        double s = 0.0;
        for (int t = 0; t < a.nt; ++t) {
            if (t == skip) continue;
            const double v = mom[(size_t)t * 9 + threadIdx.x];
            s += a.linear ? v * exp(lq[t]) : v;
        }
        avg[threadIdx.x] = s / (double)cnt;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double M[3] = {avg[0], avg[1], avg[2]};
    double C[3][3];
    C[0][0] = avg[3] - M[0] * M[0];
    C[1][1] = avg[4] - M[1] * M[1];
    C[2][2] = avg[5] - M[2] * M[2];
    C[0][1] = C[1][0] = avg[6] - M[0] * M[1];
    C[0][2] = C[2][0] = avg[7] - M[0] * M[2];
    C[1][2] = C[2][1] = avg[8] - M[1] * M[2];
    const double nm = sqrt(M[0] * M[0] + M[1] * M[1] + M[2] * M[2]);
    const double u[3] = {M[0] / nm, M[1] / nm, M[2] / nm};
    int am = 0;
    for (int i = 1; i < 3; ++i)
        if (fabs(u[i]) < fabs(u[am])) am = i;
    double e1[3] = {0.0, 0.0, 0.0};
    e1[am] = 1.0;
    const double ue = u[am];
    for (int i = 0; i < 3; ++i) e1[i] -= u[i] * ue;
    const double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int i = 0; i < 3; ++i) e1[i] /= n1;
    const double e2[3] = {u[1] * e1[2] - u[2] * e1[1], u[2] * e1[0] - u[0] * e1[2], u[0] * e1[1] - u[1] * e1[0]};
    double c11 = 0.0, c22 = 0.0, c12 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            c11 += e1[i] * C[i][j] * e1[j];
            c22 += e2[i] * C[i][j] * e2[j];
            c12 += e1[i] * C[i][j] * e2[j];
        }
    const double lmin = 0.5 * (c11 + c22) - sqrt(0.25 * (c11 - c22) * (c11 - c22) + c12 * c12);
    double *o = out + 16 * (size_t)blockIdx.x;
    for (int i = 0; i < 3; ++i) o[i] = M[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o[3 + 3 * i + j] = C[i][j];
    o[12] = (double)a.n * lmin / (nm * nm);
}

}  // namespace tvmc
