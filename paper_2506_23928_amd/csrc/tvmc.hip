// C ABI of the otVMC library (declarations and contracts in include/tvmc.h).
// Host side: argument checks, the workspace layout, the stage machine of one SDE step, and
// kernel launches on the caller's stream.  No device allocation happens here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tvmc.h"
#include "cholesky.hpp"
#include "cholesky_mw.hpp"
#include "cholesky_z.hpp"
#include "samplespace.hpp"
#include "common.hpp"
#include "estimate.hpp"
#include "observe.hpp"
#include "rbm.hpp"
#include "sampler.hpp"
#include "snr.hpp"
#include "sbuild.hpp"
#include "sbuild_mfma.hpp"
#include "sbuild_rbm_mfma.hpp"

using namespace tvmc;

namespace {

struct Timer {
    std::vector<hipEvent_t> start, stop;
    size_t used = 0;
};

}  // namespace

constexpr int NSIDE = 2;   // side streams of the several-workgroup solves

struct tvmc_ctx {
    Dev d{};
    hipStream_t stream = nullptr;
    // NSIDE side streams (default priority) for the several-workgroup solves: each takes an
    // equal share of the trajectories, so one share's small diagonal and TRSM launches overlap
    // the others' panel updates; forked from and joined back into `stream` with events
    hipStream_t side[NSIDE] = {};
    hipEvent_t fork = nullptr, join[NSIDE] = {};
    tvmc_config cfg{};
    int step = 0, stage = 0, phase = 0, nobs = 0, adam_t = 0;
    int cpb = 1;
    // a plain step (no moments, no training, no timing) captured once and replayed
    bool capturing = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    char err[512] = {0};
    int static_dev = -1;   // device whose static workspace this context uses (tvmc_init_static), or -1
    bool timing = false;
    std::vector<std::string> groups;
    std::vector<Timer> timers;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t J, jk, js, jr, pa, pb, pidx, theta, theta_eval, d0, d1, eta_re, eta_im, epair, chains, samples, sbits, R, eloc, acc, dw,
        bmean, G, gbar, obar, obarc, w_re, w_im, cT, sT, cW, sW, tt, D, S, linv, mom_part, momtab, mom, hist, ens, flags, lognorm, qhist, snrV, snrRho, snrW, snrEig, snrPart, snrRot, snrSweeps, arP, arG, arM, arV, arW1Tb, arW2Tb, arh, arda,
        arg, arlogq, arlogqb, arloss, aracc, rbmP, ssrow, ssrhs, ssu, ssbar, dstep, total;
};

int mom_blocks_for(int ns) {
    int b = (ns + MOM_WAVES - 1) / MOM_WAVES;
    return b < 64 ? b : 64;
}

// LJPHd: pairs within distance d that keep their own eta
int ljph_own_pairs(int n, int d) { return d * (2 * n - d - 1) / 2; }
int n_params(const tvmc_ansatz *a, int n) {
    if (a->kind == TVMC_ANSATZ_RBM) return n + a->n_hidden + n * a->n_hidden;
    if (a->kind == TVMC_ANSATZ_LJPH) return n + ljph_own_pairs(n, a->range) + (n - 1 - a->range);
    return n + n * (n - 1) / 2;
}
// theta index of the parameter that multiplies s_j s_k (j != k)
int eta_param(const tvmc_ansatz *a, int n, int j, int k) {
    if (j > k) std::swap(j, k);
    if (a->kind != TVMC_ANSATZ_LJPH) return pair_index(n, j, k);
    const int d = a->range, dist = k - j;
    if (dist > d) return n + ljph_own_pairs(n, d) + (dist - d - 1);
    int at = n;
    for (int r = 0; r < j; ++r) at += std::min(d, n - 1 - r);
    return at + dist - 1;
}
// whether the solve runs in sample space (N_s x N_s) rather than parameter space (M x M)
int use_sample_space(const tvmc_config *c, const tvmc_ansatz *a, int m) {
    if (a->kind == TVMC_ANSATZ_LJPH || c->regulariser == TVMC_REG_SNR) return 0;
    return c->solver == TVMC_SOLVER_SAMPLE_SPACE || (c->solver == TVMC_SOLVER_AUTO && m > c->n_samples);
}

// S + eps I per trajectory: real symmetric M x M (Jastrow) or complex Hermitian M x M (RBM)
size_t s_doubles(int kind, int m) { return (kind == TVMC_ANSATZ_RBM ? 2 : 1) * (size_t)m * m; }

Layout layout(int kind, int n, int nh, int m, int nch, int T, int ns, int nc, int nobs, int ar, int ah, int nprob, int prec, int ss,
              int snr) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + (bytes ? bytes : 1));
        return at;
    };
    const size_t tt = (size_t)T;
    L.J = take(sizeof(double) * n * n * (size_t)nprob);
    L.jk = take(sizeof(int) * (nch + 1));
    L.js = take(sizeof(int) * (nch + 1));
    L.jr = take(sizeof(double) * (nch + 1) * (size_t)nprob);
    L.pa = take(sizeof(int) * m);
    L.pb = take(sizeof(int) * m);
    L.pidx = take(sizeof(int) * n * n);
    L.theta = take(sizeof(double2) * tt * m);
    L.theta_eval = take(sizeof(double2) * tt * m);
    L.d0 = take(sizeof(double2) * tt * m);
    L.d1 = take(sizeof(double2) * tt * m);
    L.eta_re = take(sizeof(double) * tt * n * n);
    L.eta_im = take(sizeof(double) * tt * n * n);
    L.epair = take(sizeof(double2) * tt * 2 * n * n);
    const size_t nw = (size_t)(n + 63) / 64;   // words per configuration
    L.chains = take(sizeof(uint64_t) * tt * nc * nw);
    L.samples = take(sizeof(uint64_t) * tt * ns * nw);
    L.sbits = take(sizeof(uint32_t) * tt * n * ((ns + 31) / 32));
    L.R = take(sizeof(double2) * tt * ns * n);
    L.eloc = take(sizeof(double2) * tt * ns);
    L.acc = take(sizeof(uint32_t) * tt * nc);
    L.dw = take(sizeof(double) * tt * (nch + 1));
    L.bmean = take(sizeof(double2) * tt * (nch + 1));
    L.G = take(sizeof(double2) * tt * ns);
    L.gbar = take(sizeof(double2) * tt);
    const bool rbm = kind == TVMC_ANSATZ_RBM;
    L.obar = take(sizeof(double) * tt * m);
    L.obarc = take(rbm ? sizeof(double2) * tt * m : 0);
    L.w_re = take(rbm ? sizeof(double) * tt * n * nh : 0);
    L.w_im = take(rbm ? sizeof(double) * tt * n * nh : 0);
    L.cT = take(rbm ? sizeof(double2) * tt * n * nh : 0);
    L.sT = take(rbm ? sizeof(double2) * tt * n * nh : 0);
    L.cW = take(rbm ? sizeof(double2) * tt * n * nh : 0);
    L.sW = take(rbm ? sizeof(double2) * tt * n * nh : 0);
    L.tt = take(rbm ? sizeof(double2) * tt * ns * nh : 0);
    L.D = take(sizeof(double2) * tt * m);
    const int dim = ss ? ns : m;   // dimension of the system solved
    L.S = take(sizeof(double) * tt * s_doubles(kind, dim));
    L.linv = take((rbm ? sizeof(double2) : sizeof(double)) * tt * chol_panels(dim) * CN * CN);
    L.ssrow = take(ss ? sizeof(double2) * tt * ns : 0);
    L.ssrhs = take(ss ? sizeof(double2) * tt * ns : 0);
    L.ssu = take(ss ? sizeof(double2) * tt * ns : 0);
    L.ssbar = take(ss ? sizeof(double) * tt : 0);
    L.mom_part = take(sizeof(double) * tt * mom_blocks_for(ns) * 9);
    L.momtab = take(rbm && (nw > 1 || (size_t)n * nh > 64 * 64) ? sizeof(double2) * tt * mom_blocks_for(ns) * 2 * n * nh : 0);
    L.mom = take(sizeof(double) * tt * 9);
    L.hist = take(sizeof(double) * (size_t)(nobs > 0 ? nobs : 1) * tt * 9);
    L.ens = take(sizeof(double) * 16 * (tt + 1));
    L.flags = take(sizeof(int) * tt);
    L.dstep = take(sizeof(int));
    L.lognorm = take(sizeof(double) * tt * 3);
    L.qhist = take(sizeof(double) * (size_t)(nobs > 0 ? nobs : 1) * tt);
    const size_t nxb = (size_t)(ns + 63) / 64;
    L.snrV = take(snr ? (rbm ? sizeof(double2) : sizeof(double)) * tt * m * m : 0);
    L.snrRho = take(snr ? sizeof(double2) * tt * m : 0);
    L.snrW = take(snr ? sizeof(double2) * tt * m : 0);
    L.snrEig = take(snr ? sizeof(double) * tt * m * 2 : 0);
    L.snrPart = take(snr ? sizeof(double) * tt * nxb * m : 0);
    const bool jl = snr && !rbm && m <= JL_MAXM;   // the LDS Jacobi records its rotations
    const size_t mpe = (size_t)(m + (m & 1));
    L.snrRot = take(jl ? sizeof(double2) * tt * JAC_MAX_SWEEPS * (mpe - 1) * (mpe / 2) : 0);
    L.snrSweeps = take(jl ? sizeof(int) * tt : 0);
    const size_t np = ar ? ar_params(n, ah) : 0;
    L.arP = take(sizeof(float) * tt * np);
    L.arG = take(sizeof(float) * tt * np);
    L.arM = take(sizeof(float) * tt * np);
    L.arV = take(sizeof(float) * tt * np);
    L.arW1Tb = take(ar ? sizeof(uint16_t) * tt * ah * n : 0);
    L.arW2Tb = take(ar ? sizeof(uint16_t) * tt * ah * n : 0);
    L.arh = take(ar ? sizeof(float) * tt * ns * ah : 0);
    L.arda = take(ar ? sizeof(float) * tt * ns * ah : 0);
    L.arg = take(ar ? sizeof(float) * tt * ns * n : 0);
    L.arlogq = take(ar ? sizeof(float) * tt * ns : 0);
    L.arlogqb = take(ar ? sizeof(float) * tt * ns : 0);
    L.arloss = take(sizeof(double) * tt);
    L.aracc = take(sizeof(uint32_t) * tt * nc);
    const size_t mp = ((size_t)m + RQ_T - 1) / RQ_T * RQ_T;
    L.rbmP = take(rbm && prec == TVMC_PREC_MFMA && !ss ? sizeof(uint16_t) * tt * 4 * mp * ns : 0);
    L.total = o;
    return L;
}

void set_err(tvmc_ctx *c, const char *fmt, ...) {
    if (!c) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
}

thread_local char g_err[512];

tvmc_status check_args(const tvmc_problem *p, const tvmc_ansatz *a, const tvmc_config *c, char *msg, size_t len) {
    if (!p || !a || !c) return snprintf(msg, len, "null argument"), TVMC_E_INVAL;
    if (p->n_sites < 1 || p->n_sites > 64 * MAX_WORDS)
        return snprintf(msg, len, "n_sites must be in [1, %d]", 64 * MAX_WORDS), TVMC_E_INVAL;
    if (!p->J) return snprintf(msg, len, "J is null"), TVMC_E_INVAL;
    if (p->n_jumps < 0 || p->n_jumps > 256) return snprintf(msg, len, "n_jumps must be in [0, 256]"), TVMC_E_INVAL;
    if (p->n_jumps > 0 && (!p->jump_kind || !p->jump_site || !p->jump_rate))
        return snprintf(msg, len, "jump arrays are null"), TVMC_E_INVAL;
    for (int i = 0; i < p->n_jumps; ++i) {
        if (p->jump_kind[i] < 0 || p->jump_kind[i] > 2) return snprintf(msg, len, "bad jump kind"), TVMC_E_INVAL;
        if (p->jump_site[i] < 0 || p->jump_site[i] >= p->n_sites) return snprintf(msg, len, "bad jump site"), TVMC_E_INVAL;
        if (!(p->jump_rate[i] >= 0.0) || !std::isfinite(p->jump_rate[i]))
            return snprintf(msg, len, "bad jump rate"), TVMC_E_INVAL;
    }
    for (int i = 0; i < p->n_sites * p->n_sites; ++i)
        if (!std::isfinite(p->J[i])) return snprintf(msg, len, "J not finite"), TVMC_E_INVAL;
    for (int i = 0; i < p->n_sites; ++i) {
        if (p->J[i * p->n_sites + i] != 0.0) return snprintf(msg, len, "J diagonal must be zero"), TVMC_E_INVAL;
        for (int j = 0; j < i; ++j)
            if (p->J[i * p->n_sites + j] != p->J[j * p->n_sites + i])
                return snprintf(msg, len, "J must be symmetric"), TVMC_E_INVAL;
    }
    if (a->kind != TVMC_ANSATZ_JASTROW && a->kind != TVMC_ANSATZ_RBM && a->kind != TVMC_ANSATZ_LJPH)
        return snprintf(msg, len, "bad ansatz"), TVMC_E_INVAL;
    if (a->kind == TVMC_ANSATZ_RBM && (a->n_hidden < 1 || a->n_hidden > 256))
        return snprintf(msg, len, "RBM hidden units must be in [1, 256]"), TVMC_E_INVAL;
    if (a->kind == TVMC_ANSATZ_LJPH) {
        if (a->range < 0 || a->range > p->n_sites - 1)
            return snprintf(msg, len, "LJPHd range d must be in [0, N-1]"), TVMC_E_INVAL;
        // the int8 S-build feeds a shared distance D > d (O = sum over the len = N - D pairs at that
        // distance of s_j s_{j+D}, |O| <= N - d - 1) as O itself up to N = 128 and as its half
        // h = (O - (len & 1)) / 2, |h| <= (N - d) / 2, beyond; the int32 sums of products of
        // these operands stay exact below 2^31
        const int64_t nd = p->n_sites - a->range;
        const int64_t omax = std::max<int64_t>(1, p->n_sites <= 128 ? nd - 1 : nd / 2);
        if (c->precision == TVMC_PREC_MFMA && (int64_t)c->n_samples * omax * omax >= ((int64_t)1 << 31))
            return snprintf(msg, len, "LJPHd int8 S-build: n_samples times the squared largest operand (N-d-1, or "
                                      "(N-d)/2 beyond N = 128) must stay below 2^31"), TVMC_E_INVAL;
        if (c->solver == TVMC_SOLVER_SAMPLE_SPACE)
            return snprintf(msg, len, "LJPHd solves in parameter space"), TVMC_E_INVAL;
    }
    if (c->n_traj < 1 || (int64_t)c->traj_offset + c->n_traj > (1 << 24) || c->traj_offset < 0)
        return snprintf(msg, len, "trajectory ids must lie in [0, 2^24)"), TVMC_E_INVAL;
    if (c->n_chains < 1 || c->n_samples < 1 || c->n_samples % c->n_chains)
        return snprintf(msg, len, "n_samples must be a positive multiple of n_chains"), TVMC_E_INVAL;
    if (c->n_chains >= 8 && c->n_chains % 8) return snprintf(msg, len, "n_chains must be < 8 or a multiple of 8"), TVMC_E_INVAL;
    if (c->burn_sweeps < 0 || c->thin_sweeps < 1 || c->init_sweeps < 0)
        return snprintf(msg, len, "bad sweep counts"), TVMC_E_INVAL;
    if ((int64_t)(c->burn_sweeps + c->init_sweeps + (int64_t)(c->n_samples / c->n_chains) * c->thin_sweeps) * p->n_sites >=
        ((int64_t)1 << 31))
        return snprintf(msg, len, "too many proposals per evaluation"), TVMC_E_INVAL;
    if (!(c->dt > 0.0) || !(c->diag_shift >= 0.0)) return snprintf(msg, len, "bad dt or diag_shift"), TVMC_E_INVAL;
    if (c->scheme != 0 && c->scheme != 1) return snprintf(msg, len, "bad scheme"), TVMC_E_INVAL;
    if (c->precision != 0 && c->precision != 1) return snprintf(msg, len, "bad precision"), TVMC_E_INVAL;
    if (c->precision == TVMC_PREC_MFMA && c->n_samples % 64)
        return snprintf(msg, len, "the MFMA S-build needs n_samples to be a multiple of 64"), TVMC_E_INVAL;
    if (c->obs_every < 0 || c->n_obs_max < 0) return snprintf(msg, len, "bad observation settings"), TVMC_E_INVAL;
    if (c->proposal != TVMC_PROPOSAL_FLIP && c->proposal != TVMC_PROPOSAL_LEARNED)
        return snprintf(msg, len, "bad proposal"), TVMC_E_INVAL;
    if (c->proposal == TVMC_PROPOSAL_LEARNED) {
        if (p->n_sites > 64) return snprintf(msg, len, "the learned proposal takes at most 64 sites"), TVMC_E_INVAL;
        if (c->ar_hidden < 1 || c->ar_hidden > 256 || c->ar_hidden * p->n_sites > AR_LDS_W)
            return snprintf(msg, len, "ar_hidden must be in [1, 256] with ar_hidden * n_sites <= %d", AR_LDS_W), TVMC_E_INVAL;
        if (c->ar_train_every < 0 || c->ar_train_iters < 0 || !(c->ar_lr > 0.0))
            return snprintf(msg, len, "bad training settings"), TVMC_E_INVAL;
    }
    if (c->solver < TVMC_SOLVER_AUTO || c->solver > TVMC_SOLVER_SAMPLE_SPACE)
        return snprintf(msg, len, "bad solver"), TVMC_E_INVAL;
    if (c->unravelling != TVMC_SSE_NONLINEAR && c->unravelling != TVMC_SSE_LINEAR)
        return snprintf(msg, len, "bad unravelling"), TVMC_E_INVAL;
    if (c->regulariser != TVMC_REG_SHIFT && c->regulariser != TVMC_REG_SNR)
        return snprintf(msg, len, "bad regulariser"), TVMC_E_INVAL;
    if (c->use_graph != 0 && c->use_graph != 1) return snprintf(msg, len, "bad use_graph"), TVMC_E_INVAL;
    if (c->sampler_chains != 0) {
        const int sc = c->sampler_chains;
        const bool rbm16 = a->kind == TVMC_ANSATZ_RBM && a->n_hidden <= 128;
        if (!(sc == 1 || sc == 2 || sc == 4 || sc == 8 || (sc == 16 && rbm16)) || c->n_chains % sc)
            return snprintf(msg, len, "sampler_chains must be 1, 2, 4, 8 (or 16 for the RBM with N' <= 128) and "
                            "divide n_chains"), TVMC_E_INVAL;
    }
    if (c->regulariser == TVMC_REG_SNR) {
        if (p->n_sites > 64) return snprintf(msg, len, "the SNR solve takes at most 64 sites"), TVMC_E_INVAL;
        if (c->solver == TVMC_SOLVER_SAMPLE_SPACE)
            return snprintf(msg, len, "the SNR solve works in parameter space"), TVMC_E_INVAL;
        if (n_params(a, p->n_sites) > 2 * JAC_MAXP)
            return snprintf(msg, len, "the SNR solve takes at most %d parameters", 2 * JAC_MAXP), TVMC_E_INVAL;
        if (!(c->snr_tau >= 0.0) || !std::isfinite(c->snr_tau))
            return snprintf(msg, len, "bad snr_tau"), TVMC_E_INVAL;
    }
    if (use_sample_space(c, a, n_params(a, p->n_sites)) && c->n_samples > 65535)
        return snprintf(msg, len, "the sample-space solve takes at most 65535 samples"), TVMC_E_INVAL;
    return TVMC_OK;
}

tvmc_status check_batch(const tvmc_problem *p, int np, const tvmc_ansatz *a, const tvmc_config *c, char *msg,
                        size_t len) {
    if (!p || np < 1) return snprintf(msg, len, "no problems"), TVMC_E_INVAL;
    if (!c || (np != 1 && np != c->n_traj))
        return snprintf(msg, len, "n_problems must be 1 or n_traj"), TVMC_E_INVAL;
    for (int q = 0; q < np; ++q) {
        tvmc_status st = check_args(p + q, a, c, msg, len);
        if (st != TVMC_OK) return st;
        if (p[q].n_sites != p[0].n_sites || p[q].n_jumps != p[0].n_jumps || p[q].hx != p[0].hx)
            return snprintf(msg, len, "problems of one batch must share N, hx and the jump channels"), TVMC_E_INVAL;
        for (int i = 0; i < p[0].n_jumps; ++i)
            if (p[q].jump_kind[i] != p[0].jump_kind[i] || p[q].jump_site[i] != p[0].jump_site[i])
                return snprintf(msg, len, "problems of one batch must share the jump channels"), TVMC_E_INVAL;
    }
    return TVMC_OK;
}

#define HIPCHECK(ctx, call)                                                              \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            set_err(ctx, "%s failed: %s", #call, hipGetErrorString(e_));                 \
            return TVMC_E_DEVICE;                                                        \
        }                                                                                \
    } while (0)

#define LAUNCHCHECK(ctx, name)                                                           \
    do {                                                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) {                                                          \
            set_err(ctx, "launch of %s failed: %s", name, hipGetErrorString(e_));        \
            return TVMC_E_DEVICE;                                                        \
        }                                                                                \
    } while (0)

// Launch a kernel template instantiated for the context's configuration words (W_ = 1 or 2).
#define BY_WORDS(d, LAUNCH)              \
    do {                                 \
        if ((d).nw == 1) {               \
            constexpr int W_ = 1;        \
            LAUNCH;                      \
        } else if ((d).nw == 2) {        \
            constexpr int W_ = 2;        \
            LAUNCH;                      \
        } else {                         \
            constexpr int W_ = 3;        \
            LAUNCH;                      \
        }                                \
    } while (0)

struct Scope {
    tvmc_ctx *c;
    int g = -1;
    Scope(tvmc_ctx *ctx, const char *group) : c(ctx) {
        if (!c->timing) return;
        for (size_t i = 0; i < c->groups.size(); ++i)
            if (c->groups[i] == group) g = (int)i;
        if (g < 0) {
            c->groups.push_back(group);
            c->timers.emplace_back();
            g = (int)c->groups.size() - 1;
        }
        Timer &tm = c->timers[g];
        if (tm.used == tm.start.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                g = -1;
                return;
            }
            tm.start.push_back(a);
            tm.stop.push_back(b);
        }
        (void)hipEventRecord(tm.start[tm.used], c->stream);
    }
    ~Scope() {
        if (g < 0) return;
        Timer &tm = c->timers[g];
        (void)hipEventRecord(tm.stop[tm.used], c->stream);
        ++tm.used;
    }
};

tvmc_status run_sample(tvmc_ctx *c) {
    Dev &d = c->d;
    const int T = d.nt;
    if (c->stage == 0) {
        // a captured step graph leaves the step index out: it is set before every replay
        if (!c->capturing) {
            hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, c->stream, d, c->step);
            LAUNCHCHECK(c, "k_set_step");
        }
        hipLaunchKernelGGL(k_draw_dw, dim3(T), dim3(64), 0, c->stream, d);
        LAUNCHCHECK(c, "k_draw_dw");
        hipLaunchKernelGGL(k_copy_theta, dim3((unsigned)(((size_t)T * d.m + 255) / 256)), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_copy_theta");
    }
    const int nn = d.n * d.n;
    const int burn = d.burn + ((c->step == 0 && c->stage == 0) ? d.init_sweeps : 0);
    if (d.kind == TVMC_ANSATZ_RBM) {
        hipLaunchKernelGGL(k_prepare_rbm, dim3((d.n * d.nh + 255) / 256, T), dim3(256), 0, c->stream, d,
                           (const double2 *)d.theta_eval);
        LAUNCHCHECK(c, "k_prepare_rbm");
        Scope sc(c, "sample");
        const int qh = (d.nh + 63) / 64;
        // 16 chains per workgroup (4 waves per SIMD, every chain resident at once) where the
        // chain count allows and the per-chain LDS rows fit (N' <= 128)
        const int cpb = c->cfg.sampler_chains > 0 ? c->cpb : (c->cpb == 8 && d.nc % 16 == 0 && qh <= 2) ? 16 : c->cpb;
        dim3 grid((d.nc / cpb * T + 7) / 8 * 8);
#define RBM_LAUNCH(CPB, QH, AR, WL, WD) hipLaunchKernelGGL((k_sample_rbm<CPB, QH, AR, WL, WD>), grid, dim3(64 * CPB), 0, c->stream, d, c->stage, burn)
#define RBM_CPB(QH, AR, WL, WD)                         \
    switch (cpb) {                                      \
    case 16: if constexpr (QH <= 2) { RBM_LAUNCH(16, QH, AR, WL, WD); } break; \
    case 8: RBM_LAUNCH(8, QH, AR, WL, WD); break;       \
    case 4: RBM_LAUNCH(4, QH, AR, WL, WD); break;       \
    case 2: RBM_LAUNCH(2, QH, AR, WL, WD); break;       \
    default: RBM_LAUNCH(1, QH, AR, WL, WD); break;      \
    }
        // N' <= 64 fits in LDS with N <= 64; other layers fit when N N' <= 4096
        const bool wl = d.n * d.nh <= 64 * 64;
        if (d.ar) {   // one configuration word (checked at initialisation)
            if (qh == 1) { RBM_CPB(1, true, true, 1) }
            else if (qh == 2) { if (wl) { RBM_CPB(2, true, true, 1) } else { RBM_CPB(2, true, false, 1) } }
            else { if (wl) { RBM_CPB(4, true, true, 1) } else { RBM_CPB(4, true, false, 1) } }
        } else if (d.nw == 1) {
            if (qh == 1) { RBM_CPB(1, false, true, 1) }
            else if (qh == 2) { if (wl) { RBM_CPB(2, false, true, 1) } else { RBM_CPB(2, false, false, 1) } }
            else { if (wl) { RBM_CPB(4, false, true, 1) } else { RBM_CPB(4, false, false, 1) } }
        } else if (d.nw == 2) {
            if (qh == 1) { if (wl) { RBM_CPB(1, false, true, 2) } else { RBM_CPB(1, false, false, 2) } }
            else if (qh == 2) { if (wl) { RBM_CPB(2, false, true, 2) } else { RBM_CPB(2, false, false, 2) } }
            else { if (wl) { RBM_CPB(4, false, true, 2) } else { RBM_CPB(4, false, false, 2) } }
        } else {
            if (qh == 1) { if (wl) { RBM_CPB(1, false, true, 3) } else { RBM_CPB(1, false, false, 3) } }
            else if (qh == 2) { if (wl) { RBM_CPB(2, false, true, 3) } else { RBM_CPB(2, false, false, 3) } }
            else { if (wl) { RBM_CPB(4, false, true, 3) } else { RBM_CPB(4, false, false, 3) } }
        }
#undef RBM_CPB
#undef RBM_LAUNCH
        LAUNCHCHECK(c, "k_sample_rbm");
        c->phase = 1;
        return TVMC_OK;
    }
    hipLaunchKernelGGL(k_prepare_jastrow, dim3((nn + 255) / 256, T), dim3(256), 0, c->stream, d,
                       (const double2 *)d.theta_eval);
    LAUNCHCHECK(c, "k_prepare_jastrow");
    {
        Scope sc(c, "sample");
        dim3 grid(d.nc / c->cpb, T);
        // several words: 16 chains per workgroup (4 waves per SIMD, every chain resident at once:
        // the eta plane in LDS allows one workgroup per compute unit) where the chain count
        // allows, on a grid padded to a multiple of 8 for the XCD-aware placement
        const int cpbw = c->cfg.sampler_chains > 0 ? c->cpb : (c->cpb == 8 && d.nc % 16 == 0) ? 16 : c->cpb;
        const dim3 gridw((d.nc / cpbw * T + 7) / 8 * 8);
#define JAS_LAUNCH(CPB, AR) hipLaunchKernelGGL((k_sample_jastrow<CPB, AR>), grid, dim3(64 * CPB), 0, c->stream, d, c->stage, burn)
#define JASW_LAUNCH(CPB, W) hipLaunchKernelGGL((k_sample_jastrow_wn<CPB, W>), gridw, dim3(64 * CPB), 0, c->stream, d, c->stage, burn)
        if (d.nw == 2) {
            switch (cpbw) {
            case 16: JASW_LAUNCH(16, 2); break;
            case 8: JASW_LAUNCH(8, 2); break;
            case 4: JASW_LAUNCH(4, 2); break;
            case 2: JASW_LAUNCH(2, 2); break;
            default: JASW_LAUNCH(1, 2); break;
            }
        } else if (d.nw == 3) {
            switch (cpbw) {
            case 16: JASW_LAUNCH(16, 3); break;
            case 8: JASW_LAUNCH(8, 3); break;
            case 4: JASW_LAUNCH(4, 3); break;
            case 2: JASW_LAUNCH(2, 3); break;
            default: JASW_LAUNCH(1, 3); break;
            }
        } else if (d.ar) {
            switch (c->cpb) {
            case 8: JAS_LAUNCH(8, true); break;
            case 4: JAS_LAUNCH(4, true); break;
            case 2: JAS_LAUNCH(2, true); break;
            default: JAS_LAUNCH(1, true); break;
            }
        } else {
            switch (c->cpb) {
            case 8: JAS_LAUNCH(8, false); break;
            case 4: JAS_LAUNCH(4, false); break;
            case 2: JAS_LAUNCH(2, false); break;
            default: JAS_LAUNCH(1, false); break;
            }
        }
#undef JAS_LAUNCH
#undef JASW_LAUNCH
        LAUNCHCHECK(c, "k_sample_jastrow");
    }
    c->phase = 1;
    return TVMC_OK;
}

tvmc_status run_estimate(tvmc_ctx *c) {
    Dev &d = c->d;
    const int T = d.nt;
    {
        Scope sc(c, "estimate");
        if (d.nch > 0) {
            BY_WORDS(d, hipLaunchKernelGGL((k_channel_means<W_>), dim3((d.nch + CM_CH - 1) / CM_CH, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_channel_means");
        }
        BY_WORDS(d, hipLaunchKernelGGL((k_build_G<W_>), dim3((d.ns + 255) / 256, T), dim3(256), 0, c->stream, d));
        LAUNCHCHECK(c, "k_build_G");
        hipLaunchKernelGGL(k_gbar, dim3(T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_gbar");
        if (d.kind == TVMC_ANSATZ_RBM) {
            BY_WORDS(d, hipLaunchKernelGGL((k_obar_D_rbm<W_>), dim3(((d.m + 64 * OD_R - 1) / (64 * OD_R) * T + 7) / 8 * 8),
                                           dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_obar_D_rbm");
        } else {
            if (d.kind == TVMC_ANSATZ_LJPH)
                BY_WORDS(d, hipLaunchKernelGGL((k_obar_D<true, W_>), dim3((d.m + 255) / 256, T), dim3(256), 0, c->stream, d));
            else
                BY_WORDS(d, hipLaunchKernelGGL((k_obar_D<false, W_>), dim3((d.m + 255) / 256, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_obar_D");
        }
    }
    if (d.ss) {
        Scope sc(c, "sbuild");
        if (d.kind == TVMC_ANSATZ_RBM) {
            const int nb = (d.ns + TK_T - 1) / TK_T;
            BY_WORDS(d, hipLaunchKernelGGL((k_tk_rbm<W_>), dim3(nb * (nb + 1) / 2, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_tk_rbm");
        } else {
            BY_WORDS(d, hipLaunchKernelGGL((k_tk_jastrow<W_>), dim3((d.ns + 255) / 256, d.ns, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_tk_jastrow");
        }
        hipLaunchKernelGGL(k_tk_rowmean, dim3(d.ns, T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_tk_rowmean");
        hipLaunchKernelGGL(k_tk_rbar, dim3(T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_tk_rbar");
        hipLaunchKernelGGL(k_tk_centre, dim3((d.ns + 255) / 256, d.ns, T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_tk_centre");
        c->phase = 2;
        return TVMC_OK;
    }
    if (d.kind == TVMC_ANSATZ_RBM) {
        if (c->cfg.precision == TVMC_PREC_MFMA) {
            {
                Scope sc(c, "transpose");
                BY_WORDS(d, hipLaunchKernelGGL((k_rbm_split<W_>), dim3(d.ns / 32, (d.mp + 64 * SPL_R - 1) / (64 * SPL_R), T), dim3(256), 0, c->stream, d));
                LAUNCHCHECK(c, "k_rbm_split");
            }
            Scope sc(c, "sbuild");
            const int nt = d.mp / RQ_T;
            hipLaunchKernelGGL(k_sbuild_rbm_bf16, dim3((nt * (nt + 1) / 2 * T + 7) / 8 * 8), dim3(RQ_THREADS), 0, c->stream, d);
            LAUNCHCHECK(c, "k_sbuild_rbm_bf16");
        } else {
            Scope sc(c, "sbuild");
            const int nt = (d.m + RB_T - 1) / RB_T;
            BY_WORDS(d, hipLaunchKernelGGL((k_sbuild_rbm_f64<W_>), dim3(nt * (nt + 1) / 2, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_sbuild_rbm_f64");
        }
        c->phase = 2;
        return TVMC_OK;
    }
    if (c->cfg.precision == TVMC_PREC_MFMA) {
        Scope sc(c, "transpose");
        if (launch_transpose_bits(d, c->stream) != TVMC_OK) {
            set_err(c, "launch of k_transpose_bits failed");
            return TVMC_E_DEVICE;
        }
    }
    {
        Scope sc(c, "sbuild");
        if (c->cfg.precision == TVMC_PREC_MFMA) {
            tvmc_status st = launch_sbuild_mfma(d, c->stream);
            if (st != TVMC_OK) {
                set_err(c, "launch of the int8 MFMA S-build failed");
                return st;
            }
        } else {
            const int nt = (d.m + 63) / 64;
            BY_WORDS(d, hipLaunchKernelGGL((k_sbuild_f64<W_>), dim3(nt * (nt + 1) / 2, T), dim3(256), 0, c->stream, d));
            LAUNCHCHECK(c, "k_sbuild_f64");
        }
    }
    c->phase = 2;
    return TVMC_OK;
}

// The FP64 Cholesky solve: one workgroup per trajectory, or several per trajectory when the
// batch alone would leave most compute units idle.
// The several-workgroup solve of trajectories [0, T) of the arguments on stream st: one launch
// per panel step (update, diagonal block, TRSM), then the backward substitution.
template <typename Args, bool CPLX>
tvmc_status solve_sequence(tvmc_ctx *c, const Args &x, int T, hipStream_t st) {
    if constexpr (CPLX) {
        hipLaunchKernelGGL(k_zmw_init, dim3((x.m + 255) / 256, T), dim3(256), 0, st, x);
    } else {
        hipLaunchKernelGGL(k_cmw_init, dim3((x.m + 255) / 256, T), dim3(256), 0, st, x);
    }
    LAUNCHCHECK(c, "solver init");
    // real: the direct-to-LDS updates (32-bit byte offsets into a trajectory's matrix) carry the
    // previous panel's TRSM of their rows below those the diagonal kernel did, and the diagonal
    // kernel the following rows; panels go in pairs: one 128-column update over [0, j0), the
    // first panel's diagonal step (TRSM of the second panel's rows), the second panel's update
    // over the first panel's columns, its diagonal step (TRSM of the next pair's 2 CN rows)
    const bool real_lds = !CPLX && (size_t)x.m * x.m * sizeof(double) <= 0xffffffffull;
    if constexpr (!CPLX) {
        if (real_lds) {
            for (int j0 = 0, p = 0; j0 < x.m; j0 += 2 * CN, p += 2) {
                const bool second = j0 + CN < x.m;
                if (j0 > 0) {
                    hipLaunchKernelGGL(k_cmw_update_lds<2 * CN>, dim3(((x.m - j0 + CR - 1) / CR * T + 7) / 8 * 8), dim3(CUT),
                                       0, st, x, j0, p - 1, 0, 2 * CN, T);
                    LAUNCHCHECK(c, "panel-pair update");
                }
                hipLaunchKernelGGL(k_cmw_diag, dim3(T), dim3(256), 0, st, x, j0, p, second ? CN : 0);
                LAUNCHCHECK(c, "diagonal block");
                if (second) {
                    const int j1 = j0 + CN;
                    hipLaunchKernelGGL(k_cmw_update_lds<CN>, dim3(((x.m - j1 + CR - 1) / CR * T + 7) / 8 * 8), dim3(CUT), 0,
                                       st, x, j1, p, j0, CN, T);
                    LAUNCHCHECK(c, "panel update");
                    hipLaunchKernelGGL(k_cmw_diag, dim3(T), dim3(256), 0, st, x, j1, p + 1,
                                       j1 + CN < x.m ? 2 * CN : 0);
                    LAUNCHCHECK(c, "diagonal block");
                }
            }
            hipLaunchKernelGGL(k_cmw_backward, dim3(T), dim3(256), 0, st, x);
            LAUNCHCHECK(c, "backward substitution");
            return TVMC_OK;
        }
    }
    for (int j0 = 0, p = 0; j0 < x.m; j0 += CN, ++p) {
        if (j0 > 0) {
            // complex: the previous panel's TRSM of the rows below this panel rides in the update;
            // the direct-to-LDS form addresses a trajectory's matrix by 32-bit byte offsets
            if constexpr (CPLX) {
                // one-dimensional grid of (trajectory, row chunk) items, padded to a multiple of 8
                // (XCD-aware placement, chunk_item)
                const dim3 grid(((x.m - j0 + CR - 1) / CR * T + 7) / 8 * 8);
                if ((size_t)x.m * x.m * sizeof(double2) <= 0xffffffffull)
                    hipLaunchKernelGGL(k_zmw_update_lds, grid, dim3(ZT), 0, st, x, j0, p - 1, T);
                else
                    hipLaunchKernelGGL(k_zmw_update, grid, dim3(ZT), 0, st, x, j0, p - 1, T);
            } else {
                hipLaunchKernelGGL(k_cmw_update, dim3((x.m - j0 + CR - 1) / CR, T), dim3(256), 0, st, x, j0);
            }
            LAUNCHCHECK(c, "panel update");
        }
        if constexpr (CPLX)
            hipLaunchKernelGGL(k_zmw_diag, dim3(T), dim3(ZD), 0, st, x, j0, p);
        else
            hipLaunchKernelGGL(k_cmw_diag, dim3(T), dim3(256), 0, st, x, j0, p, 0);
        LAUNCHCHECK(c, "diagonal block");
        const int below = x.m - j0 - CN;
        if constexpr (!CPLX) {
            if (below > 0) {
                hipLaunchKernelGGL(k_cmw_trsm, dim3((below + CR - 1) / CR, T), dim3(256), 0, st, x, j0, p);
                LAUNCHCHECK(c, "panel TRSM");
            }
        }
    }
    if constexpr (CPLX) {
        for (int p = chol_panels(x.m) - 1; p >= -1; --p) {
            const int cols = p > 0 ? p * CN : 0;
            hipLaunchKernelGGL(k_zmw_bwd, dim3(cols > 0 ? (cols + ZB_COLS - 1) / ZB_COLS : 1, T), dim3(ZB_COLS), 0, st,
                               x, p);
        }
    } else {
        hipLaunchKernelGGL(k_cmw_backward, dim3(T), dim3(256), 0, st, x);
    }
    LAUNCHCHECK(c, "backward substitution");
    return TVMC_OK;
}

// Arguments of trajectories [t0, t0 + n) of a batch (every array is trajectory-major).
CholArgs sub_args(const CholArgs &a, int t0) {
    const size_t m = (size_t)a.m;
    return CholArgs{a.A + (size_t)t0 * m * m, a.rhs + (size_t)t0 * m, a.x + (size_t)t0 * m,
                    a.linv + (size_t)t0 * chol_panels(a.m) * CN * CN, a.flags + t0, a.m};
}
ZCholArgs sub_args(const ZCholArgs &a, int t0) {
    const size_t m = (size_t)a.m;
    return ZCholArgs{a.A + (size_t)t0 * m * m, a.rhs + (size_t)t0 * m, a.x + (size_t)t0 * m,
                     a.linv + (size_t)t0 * chol_panels(a.m) * CN * CN, a.flags + t0, a.m};
}

// The batch in min(T, NSIDE) contiguous shares on the side streams, joined back into the
// context's stream.
template <typename Args, bool CPLX>
tvmc_status solve_split(tvmc_ctx *c, const Args &x) {
    const int T = c->d.nt;
    const int parts = T < NSIDE ? T : NSIDE;
    if (parts < 2 || !c->side[0]) return solve_sequence<Args, CPLX>(c, x, T, c->stream);
    HIPCHECK(c, hipEventRecord(c->fork, c->stream));
    for (int g = 0; g < parts; ++g) {
        HIPCHECK(c, hipStreamWaitEvent(c->side[g], c->fork, 0));
        const int t0 = T * g / parts, t1 = T * (g + 1) / parts;
        tvmc_status st = solve_sequence<Args, CPLX>(c, sub_args(x, t0), t1 - t0, c->side[g]);
        if (st != TVMC_OK) return st;
        HIPCHECK(c, hipEventRecord(c->join[g], c->side[g]));
    }
    for (int g = 0; g < parts; ++g) HIPCHECK(c, hipStreamWaitEvent(c->stream, c->join[g], 0));
    return TVMC_OK;
}

// The FP64 Cholesky solve: one workgroup per trajectory, or several per trajectory when the
// batch alone would leave most compute units idle.
tvmc_status launch_chol(tvmc_ctx *c, const CholArgs &ca) {
    const int T = c->d.nt;
    const bool multi = c->cfg.solver == TVMC_SOLVER_MULTI_GROUP ||
                       (c->cfg.solver != TVMC_SOLVER_ONE_GROUP && T < 192);
    if (!multi) {
        hipLaunchKernelGGL(k_chol_solve, dim3(T), dim3(CT1), 0, c->stream, ca);
        LAUNCHCHECK(c, "k_chol_solve");
        return TVMC_OK;
    }
    return solve_split<CholArgs, false>(c, ca);
}

// The complex Hermitian solve (always several workgroups per trajectory).
tvmc_status launch_zchol(tvmc_ctx *c, const ZCholArgs &za) { return solve_split<ZCholArgs, true>(c, za); }

tvmc_status run_solve(tvmc_ctx *c) {
    Dev &d = c->d;
    {
        Scope sc(c, "solve");
        if (d.ss) {
            tvmc_status st;
            if (d.kind == TVMC_ANSATZ_RBM) {
                ZCholArgs za{(double2 *)d.S, d.ssrhs, d.ssu, (double2 *)d.linv, d.flags, d.ns};
                st = launch_zchol(c, za);
            } else {
                CholArgs ca{d.S, d.ssrhs, d.ssu, d.linv, d.flags, d.ns};
                st = launch_chol(c, ca);
            }
            if (st != TVMC_OK) return st;
            BY_WORDS(d, hipLaunchKernelGGL((k_pushback<W_>), dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d, c->stage));
            LAUNCHCHECK(c, "k_pushback");
        } else if (d.reg == TVMC_REG_SNR && d.kind == TVMC_ANSATZ_RBM) {
            const size_t mm = (size_t)d.m * d.m;
            hipLaunchKernelGGL(k_zsnr_init, dim3((unsigned)((mm + 255) / 256), d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_zsnr_init");
            hipLaunchKernelGGL(k_zjacobi, dim3(d.nt), dim3(JAC_THREADS), 0, c->stream, d);
            LAUNCHCHECK(c, "k_zjacobi");
            hipLaunchKernelGGL(k_zsnr_rho, dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_zsnr_rho");
            hipLaunchKernelGGL(k_zsnr_var, dim3((d.m + SV_K - 1) / SV_K, d.snr_nxb, d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_zsnr_var");
            hipLaunchKernelGGL(k_zsnr_finish, dim3(d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_zsnr_finish");
            hipLaunchKernelGGL(k_zsnr_back, dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d, c->stage);
            LAUNCHCHECK(c, "k_zsnr_back");
        } else if (d.reg == TVMC_REG_SNR) {
            const size_t mm = (size_t)d.m * d.m;
            hipLaunchKernelGGL(k_snr_init, dim3((unsigned)((mm + 255) / 256), d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_snr_init");
            if (d.m <= JL_MAXM) {
                hipLaunchKernelGGL(k_jacobi_lds, dim3(d.nt), dim3(JAC_THREADS), 0, c->stream, d);
                LAUNCHCHECK(c, "k_jacobi_lds");
                hipLaunchKernelGGL(k_jacobi_apply_v, dim3((d.m + JV_COLS - 1) / JV_COLS, d.nt), dim3(JV_THREADS), 0,
                                   c->stream, d);
                LAUNCHCHECK(c, "k_jacobi_apply_v");
            } else {
                hipLaunchKernelGGL(k_jacobi, dim3(d.nt), dim3(JAC_THREADS), 0, c->stream, d);
                LAUNCHCHECK(c, "k_jacobi");
            }
            hipLaunchKernelGGL(k_snr_rho, dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_snr_rho");
            hipLaunchKernelGGL(k_snr_var, dim3((d.m + SV_K - 1) / SV_K, d.snr_nxb, d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_snr_var");
            hipLaunchKernelGGL(k_snr_finish, dim3(d.nt), dim3(256), 0, c->stream, d);
            LAUNCHCHECK(c, "k_snr_finish");
            hipLaunchKernelGGL(k_snr_back, dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d, c->stage);
            LAUNCHCHECK(c, "k_snr_back");
        } else if (d.kind == TVMC_ANSATZ_RBM) {
            ZCholArgs za{(double2 *)d.S, d.D, c->stage ? d.d1 : d.d0, (double2 *)d.linv, d.flags, d.m};
            tvmc_status st = launch_zchol(c, za);
            if (st != TVMC_OK) return st;
        } else {
            CholArgs ca{d.S, d.D, c->stage ? d.d1 : d.d0, d.linv, d.flags, d.m};
            tvmc_status st = launch_chol(c, ca);
            if (st != TVMC_OK) return st;
        }
    }
    c->phase = 3;
    return TVMC_OK;
}

tvmc_status run_update(tvmc_ctx *c) {
    Dev &d = c->d;
    {
        Scope sc(c, "update");
        hipLaunchKernelGGL(k_update, dim3((d.m + 255) / 256, d.nt), dim3(256), 0, c->stream, d, c->stage);
        LAUNCHCHECK(c, "k_update");
    }
    if (c->stage == 0) {
        c->stage = 1;
    } else {
        c->stage = 0;
        ++c->step;
    }
    c->phase = 0;
    return TVMC_OK;
}

tvmc_status run_train(tvmc_ctx *c, int iters) {
    Dev &d = c->d;
    const int T = d.nt;
    Scope sc(c, "train");
    const int tiles = ((d.ah + 31) / 32) * ((d.n + 31) / 32);
    for (int it = 0; it <= iters; ++it) {
        hipLaunchKernelGGL(k_ar_forward, dim3((d.ns + AR_SAMPLES - 1) / AR_SAMPLES, T), dim3(64 * AR_WAVES), 0, c->stream, d,
                           1);
        LAUNCHCHECK(c, "k_ar_forward");
        hipLaunchKernelGGL(k_ar_grad, dim3(tiles, 2, T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_ar_grad");
        hipLaunchKernelGGL(k_ar_loss, dim3(T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_ar_loss");
        if (it == iters) break;
        ++c->adam_t;
        hipLaunchKernelGGL(k_ar_adam, dim3((unsigned)((d.arnp + 255) / 256), T), dim3(256), 0, c->stream, d,
                           (float)c->cfg.ar_lr, c->adam_t);
        LAUNCHCHECK(c, "k_ar_adam");
        hipLaunchKernelGGL(k_ar_copy, dim3((d.ah * d.n + 255) / 256, T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_ar_copy");
    }
    return TVMC_OK;
}

tvmc_status run_moments(tvmc_ctx *c, int slot) {
    Dev &d = c->d;
    const int T = d.nt, nn = d.n * d.n;
    Scope sc(c, "observe");
    if (d.kind == TVMC_ANSATZ_RBM && d.nw == 1 && d.n * d.nh <= 64 * 64) {
        hipLaunchKernelGGL(k_moments_rbm_f, dim3(d.mom_blocks, T), dim3(64 * RMF_WAVES), 0, c->stream, d);
        LAUNCHCHECK(c, "k_moments_rbm_f");
    } else if (d.kind == TVMC_ANSATZ_RBM) {
        BY_WORDS(d, hipLaunchKernelGGL((k_moments_rbm_g<W_>), dim3(d.mom_blocks, T), dim3(64 * RMF_WAVES), 0, c->stream, d));
        LAUNCHCHECK(c, "k_moments_rbm_g");
    } else {
        hipLaunchKernelGGL(k_prepare_pairs, dim3((nn + 255) / 256, T), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_prepare_pairs");
        BY_WORDS(d, hipLaunchKernelGGL((k_moments<W_>), dim3(d.mom_blocks, T), dim3(64 * MOM_WAVES), 0, c->stream, d));
        LAUNCHCHECK(c, "k_moments");
    }
    hipLaunchKernelGGL(k_moments_reduce, dim3((T + 127) / 128), dim3(128), 0, c->stream, d, slot);
    LAUNCHCHECK(c, "k_moments_reduce");
    return TVMC_OK;
}

size_t q_bytes(const tvmc_ctx *c, int what) {
    const Dev &d = c->d;
    switch (what) {
    case TVMC_Q_THETA: case TVMC_Q_THETA_EVAL: case TVMC_Q_DELTA0: case TVMC_Q_DELTA1: case TVMC_Q_D:
        return sizeof(double2) * d.m;
    case TVMC_Q_SAMPLES: return sizeof(uint64_t) * d.ns * d.nw;
    case TVMC_Q_ELOC: return sizeof(double2) * d.ns;
    case TVMC_Q_S: return sizeof(double) * s_doubles(d.kind, d.ss ? d.ns : d.m);
    case TVMC_Q_OBAR: return (d.kind == TVMC_ANSATZ_RBM ? sizeof(double2) : sizeof(double)) * d.m;
    case TVMC_Q_BMEAN: return sizeof(double2) * d.nch;
    case TVMC_Q_DW: return sizeof(double) * d.nch;
    case TVMC_Q_ACCEPTS: return sizeof(uint32_t) * d.nc;
    case TVMC_Q_CHAINS: return sizeof(uint64_t) * d.nc * d.nw;
    case TVMC_Q_MOMENTS: return sizeof(double) * 9;
    case TVMC_Q_OBS_HIST: return sizeof(double) * 9 * (size_t)d.nobs;
    case TVMC_Q_AR_PARAMS: case TVMC_Q_AR_GRAD: return d.ar ? sizeof(float) * d.arnp : 0;
    case TVMC_Q_AR_LOGQ: case TVMC_Q_AR_LOGQ_BF16: return d.ar ? sizeof(float) * d.ns : 0;
    case TVMC_Q_AR_LOSS: return d.ar ? sizeof(double) : 0;
    case TVMC_Q_AR_ACCEPTS: return d.ar ? sizeof(uint32_t) * d.nc : 0;
    case TVMC_Q_LOGNORM: return sizeof(double);
    case TVMC_Q_LOGNORM_HIST: return sizeof(double) * (size_t)d.nobs;
    case TVMC_Q_EIG: return d.reg == TVMC_REG_SNR ? sizeof(double) * 2 * d.m : 0;
    default: return 0;
    }
}

}  // namespace

extern "C" {

tvmc_status tvmc_workspace_size_batch(const tvmc_problem *p, int32_t np, const tvmc_ansatz *a, const tvmc_config *c,
                                      size_t *bytes) {
    tvmc_status st = check_batch(p, np, a, c, g_err, sizeof(g_err));
    if (st != TVMC_OK) return st;
    if (!bytes) return TVMC_E_INVAL;
    const int n = p->n_sites, m = n_params(a, n);
    *bytes = layout(a->kind, n, a->n_hidden, m, p->n_jumps, c->n_traj, c->n_samples, c->n_chains, c->n_obs_max,
                    c->proposal, c->ar_hidden, np, c->precision, use_sample_space(c, a, m),
                    c->regulariser == TVMC_REG_SNR).total;
    return TVMC_OK;
}

tvmc_status tvmc_workspace_size(const tvmc_problem *p, const tvmc_ansatz *a, const tvmc_config *c, size_t *bytes) {
    return tvmc_workspace_size_batch(p, 1, a, c, bytes);
}

}  // extern "C"

namespace {

// Context creation shared by tvmc_init_batch and tvmc_init_static; side_streams = false keeps
// every solve on the caller's stream (no stream or event is created).
tvmc_status init_impl(const tvmc_problem *pbs, int32_t np, const tvmc_ansatz *a, const tvmc_config *c,
                      const double *theta0, void *ws, size_t ws_bytes, void *stream, bool side_streams,
                      tvmc_ctx **out) {
    if (!out) return TVMC_E_INVAL;
    *out = nullptr;
    tvmc_status st = check_batch(pbs, np, a, c, g_err, sizeof(g_err));
    if (st != TVMC_OK) return st;
    const tvmc_problem *p = pbs;
    const int n = p->n_sites, m = n_params(a, n), nch = p->n_jumps, T = c->n_traj;
    const int nh = a->kind == TVMC_ANSATZ_RBM ? a->n_hidden : 0;
    const Layout L = layout(a->kind, n, nh, m, nch, T, c->n_samples, c->n_chains, c->n_obs_max, c->proposal,
                            c->ar_hidden, np, c->precision, use_sample_space(c, a, m), c->regulariser == TVMC_REG_SNR);
    if (!ws) return snprintf(g_err, sizeof(g_err), "workspace is null"), TVMC_E_INVAL;
    if (ws_bytes < L.total) return snprintf(g_err, sizeof(g_err), "workspace too small: %zu < %zu", ws_bytes, L.total), TVMC_E_NOMEM;
    if ((uintptr_t)ws % 256) return snprintf(g_err, sizeof(g_err), "workspace must be 256-byte aligned"), TVMC_E_INVAL;
    if (c->use_graph && !stream)   // the default stream cannot be captured
        return snprintf(g_err, sizeof(g_err), "use_graph needs a stream other than the default one"), TVMC_E_INVAL;

    tvmc_ctx *ctx = new (std::nothrow) tvmc_ctx();
    if (!ctx) return TVMC_E_NOMEM;
    ctx->stream = (hipStream_t)stream;
    ctx->cfg = *c;
    ctx->cpb = c->sampler_chains > 0 ? c->sampler_chains
                                     : (c->n_chains % 8 == 0 ? 8 : (c->n_chains % 4 == 0 ? 4 : (c->n_chains % 2 == 0 ? 2 : 1)));
    char *base = (char *)ws;
    Dev &d = ctx->d;
    d.n = n;
    d.nw = (n + 63) / 64;
    d.m = m;
    d.kind = a->kind;
    d.nh = nh;
    d.nch = nch;
    d.ns = c->n_samples;
    d.nc = c->n_chains;
    d.per = c->n_samples / c->n_chains;
    d.nt = T;
    d.nobs = c->n_obs_max;
    d.burn = c->burn_sweeps;
    d.thin = c->thin_sweeps;
    d.init_sweeps = c->init_sweeps;
    d.scheme = c->scheme;
    d.traj0 = c->traj_offset;
    d.key0 = (uint32_t)c->seed;
    d.key1 = (uint32_t)(c->seed >> 32);
    d.hx = p->hx;
    d.dt = c->dt;
    d.eps = c->diag_shift;
    d.mom_blocks = mom_blocks_for(c->n_samples);
    d.J = (const double *)(base + L.J);
    d.j_stride = np > 1 ? (size_t)n * n : 0;
    d.r_stride = np > 1 ? (size_t)nch : 0;
    d.jkind = (const int *)(base + L.jk);
    d.jsite = (const int *)(base + L.js);
    d.jrate = (const double *)(base + L.jr);
    d.pa = (const int *)(base + L.pa);
    d.pb = (const int *)(base + L.pb);
    d.pidx = (const int *)(base + L.pidx);
    d.theta = (double2 *)(base + L.theta);
    d.theta_eval = (double2 *)(base + L.theta_eval);
    d.d0 = (double2 *)(base + L.d0);
    d.d1 = (double2 *)(base + L.d1);
    d.eta_re = (double *)(base + L.eta_re);
    d.eta_im = (double *)(base + L.eta_im);
    d.epair = (double2 *)(base + L.epair);
    d.chains = (uint64_t *)(base + L.chains);
    d.samples = (uint64_t *)(base + L.samples);
    d.sbits = (uint32_t *)(base + L.sbits);
    d.R = (double2 *)(base + L.R);
    d.eloc = (double2 *)(base + L.eloc);
    d.acc = (uint32_t *)(base + L.acc);
    d.dw = (double *)(base + L.dw);
    d.bmean = (double2 *)(base + L.bmean);
    d.G = (double2 *)(base + L.G);
    d.gbar = (double2 *)(base + L.gbar);
    d.obar = (double *)(base + L.obar);
    d.obarc = (double2 *)(base + L.obarc);
    d.w_re = (double *)(base + L.w_re);
    d.w_im = (double *)(base + L.w_im);
    d.cT = (double2 *)(base + L.cT);
    d.sT = (double2 *)(base + L.sT);
    d.cW = (double2 *)(base + L.cW);
    d.sW = (double2 *)(base + L.sW);
    d.tt = (double2 *)(base + L.tt);
    d.mp = (m + RQ_T - 1) / RQ_T * RQ_T;
    d.rbmP = (uint16_t *)(base + L.rbmP);
    d.ss = use_sample_space(c, a, m);
    d.ssrow = (double2 *)(base + L.ssrow);
    d.ssrhs = (double2 *)(base + L.ssrhs);
    d.ssu = (double2 *)(base + L.ssu);
    d.ssbar = (double *)(base + L.ssbar);
    d.D = (double2 *)(base + L.D);
    d.S = (double *)(base + L.S);
    d.linv = (double *)(base + L.linv);
    d.mom_part = (double *)(base + L.mom_part);
    d.momtab = (double2 *)(base + L.momtab);
    d.mom = (double *)(base + L.mom);
    d.hist = (double *)(base + L.hist);
    d.ens = (double *)(base + L.ens);
    d.flags = (int *)(base + L.flags);
    d.dstep = (int *)(base + L.dstep);
    d.linear = c->unravelling == TVMC_SSE_LINEAR;
    d.lognorm = (double *)(base + L.lognorm);
    d.dq0 = d.lognorm + T;
    d.momlq = d.lognorm + 2 * (size_t)T;
    d.qhist = (double *)(base + L.qhist);
    d.reg = c->regulariser;
    d.snr_tau = c->snr_tau;
    d.snr_nxb = (c->n_samples + 63) / 64;
    d.snrV = (double *)(base + L.snrV);
    d.snrRho = (double2 *)(base + L.snrRho);
    d.snrW = (double2 *)(base + L.snrW);
    d.snrEig = (double *)(base + L.snrEig);
    d.snrPart = (double *)(base + L.snrPart);
    d.snrRot = (double2 *)(base + L.snrRot);
    d.snrSweeps = (int *)(base + L.snrSweeps);
    d.ar = c->proposal;
    d.ah = c->proposal ? c->ar_hidden : 0;
    d.arnp = c->proposal ? ar_params(n, c->ar_hidden) : 0;
    d.arP = (float *)(base + L.arP);
    d.arG = (float *)(base + L.arG);
    d.arM = (float *)(base + L.arM);
    d.arV = (float *)(base + L.arV);
    d.arW1Tb = (uint16_t *)(base + L.arW1Tb);
    d.arW2Tb = (uint16_t *)(base + L.arW2Tb);
    d.arh = (float *)(base + L.arh);
    d.arda = (float *)(base + L.arda);
    d.arg = (float *)(base + L.arg);
    d.arlogq = (float *)(base + L.arlogq);
    d.arlogqb = (float *)(base + L.arlogqb);
    d.arloss = (double *)(base + L.arloss);
    d.aracc = (uint32_t *)(base + L.aracc);

    // what each O_k is: pb = -1: s_pa; pb >= 0: s_pa s_pb; pb = -2: the sum of s_j s_{j+pa}
    // over the chain (a shared LJPHd distance).  pidx: theta index of the eta of each pair.
    std::vector<int> pa(m, 0), pb(m, -1), pidx((size_t)n * n, 0);
    for (int i = 0; i < n; ++i) pa[i] = i;
    if (a->kind != TVMC_ANSATZ_RBM)
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) {
                const int q = eta_param(a, n, j, k);
                pidx[(size_t)j * n + k] = pidx[(size_t)k * n + j] = q;
                if (a->kind == TVMC_ANSATZ_LJPH && k - j > a->range) {
                    pa[q] = k - j;
                    pb[q] = -2;
                } else {
                    pa[q] = j;
                    pb[q] = k;
                }
            }
    std::vector<double2> th((size_t)T * m);
    for (int t = 0; t < T; ++t)
        for (int k = 0; k < m; ++k)
            th[(size_t)t * m + k] = theta0 ? make_double2(theta0[2 * k], theta0[2 * k + 1]) : make_double2(0.0, 0.0);
    auto fail = [&](tvmc_status s) {
        snprintf(g_err, sizeof(g_err), "%s", ctx->err);
        for (int g = 0; g < NSIDE; ++g) {
            if (ctx->side[g]) (void)hipStreamDestroy(ctx->side[g]);
            if (ctx->join[g]) (void)hipEventDestroy(ctx->join[g]);
        }
        if (ctx->fork) (void)hipEventDestroy(ctx->fork);
        delete ctx;
        return s;
    };
#define INITCHECK(call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            set_err(ctx, "%s failed: %s", #call, hipGetErrorString(e_));                   \
            return fail(TVMC_E_DEVICE);                                                    \
        }                                                                                  \
    } while (0)
    for (int q = 0; q < np; ++q) {
        INITCHECK(hipMemcpyAsync((void *)(d.J + (size_t)q * n * n), pbs[q].J, sizeof(double) * n * n,
                                 hipMemcpyHostToDevice, ctx->stream));
        if (nch > 0)
            INITCHECK(hipMemcpyAsync((void *)(d.jrate + (size_t)q * nch), pbs[q].jump_rate, sizeof(double) * nch,
                                     hipMemcpyHostToDevice, ctx->stream));
    }
    if (nch > 0) {
        INITCHECK(hipMemcpyAsync((void *)d.jkind, p->jump_kind, sizeof(int) * nch, hipMemcpyHostToDevice, ctx->stream));
        INITCHECK(hipMemcpyAsync((void *)d.jsite, p->jump_site, sizeof(int) * nch, hipMemcpyHostToDevice, ctx->stream));
    }
    INITCHECK(hipMemcpyAsync((void *)d.pa, pa.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
    INITCHECK(hipMemcpyAsync((void *)d.pb, pb.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
    INITCHECK(hipMemcpyAsync((void *)d.pidx, pidx.data(), sizeof(int) * pidx.size(), hipMemcpyHostToDevice,
                             ctx->stream));
    INITCHECK(hipMemcpyAsync(d.theta, th.data(), sizeof(double2) * th.size(), hipMemcpyHostToDevice, ctx->stream));
    INITCHECK(hipMemsetAsync(d.flags, 0, sizeof(int) * T, ctx->stream));
    INITCHECK(hipMemsetAsync(d.lognorm, 0, sizeof(double) * 3 * (size_t)T, ctx->stream));
    INITCHECK(hipMemsetAsync(d.qhist, 0, sizeof(double) * (size_t)(d.nobs > 0 ? d.nobs : 1) * T, ctx->stream));
    INITCHECK(hipMemsetAsync(d.hist, 0, sizeof(double) * 9 * (size_t)(d.nobs > 0 ? d.nobs : 1) * T, ctx->stream));
    INITCHECK(hipMemsetAsync(d.mom, 0, sizeof(double) * 9 * (size_t)T, ctx->stream));
    INITCHECK(hipMemsetAsync(d.d0, 0, sizeof(double2) * (size_t)T * m, ctx->stream));
    INITCHECK(hipMemsetAsync(d.d1, 0, sizeof(double2) * (size_t)T * m, ctx->stream));
    hipLaunchKernelGGL(k_init_chains, dim3((c->n_chains + 63) / 64, T), dim3(64), 0, ctx->stream, d);
    INITCHECK(hipGetLastError());
    if (d.ar) {
        hipLaunchKernelGGL(k_ar_init, dim3((unsigned)((d.arnp + 255) / 256), T), dim3(256), 0, ctx->stream, d);
        INITCHECK(hipGetLastError());
        hipLaunchKernelGGL(k_ar_copy, dim3((d.ah * n + 255) / 256, T), dim3(256), 0, ctx->stream, d);
        INITCHECK(hipGetLastError());
    }
    if (side_streams) {
        for (int g = 0; g < NSIDE; ++g) {
            INITCHECK(hipStreamCreateWithFlags(&ctx->side[g], hipStreamNonBlocking));
            INITCHECK(hipEventCreateWithFlags(&ctx->join[g], hipEventDisableTiming));
        }
        INITCHECK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    }
    INITCHECK(hipStreamSynchronize(ctx->stream));
#undef INITCHECK
    *out = ctx;
    return TVMC_OK;
}

// The static workspace of tvmc_init_static: one array per device (each device that loads the
// library holds its own copy until the process ends).  Host code never uses the array's name as
// an address: the device address comes from hipGetSymbolAddress, once per device, with that
// device current.  At most one live context per device uses it.
constexpr size_t STATIC_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[STATIC_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[MAX_DEVICES] = {};
bool g_static_busy[MAX_DEVICES] = {};

}  // namespace

extern "C" {

tvmc_status tvmc_init_batch(const tvmc_problem *pbs, int32_t np, const tvmc_ansatz *a, const tvmc_config *c,
                            const double *theta0, void *ws, size_t ws_bytes, void *stream, tvmc_ctx **out) {
    return init_impl(pbs, np, a, c, theta0, ws, ws_bytes, stream, true, out);
}

tvmc_status tvmc_static_workspace_bytes(size_t *bytes) {
    if (!bytes) return TVMC_E_INVAL;
    *bytes = STATIC_BYTES;
    return TVMC_OK;
}

tvmc_status tvmc_init_static(const tvmc_problem *p, const tvmc_ansatz *a, const tvmc_config *c, const double *theta0,
                             void *stream, tvmc_ctx **out) {
    if (!out) return TVMC_E_INVAL;
    *out = nullptr;
    size_t need = 0;
    tvmc_status st = tvmc_workspace_size(p, a, c, &need);
    if (st != TVMC_OK) return st;
    if (need > STATIC_BYTES)
        return snprintf(g_err, sizeof(g_err), "tvmc_init_static: the problem needs %zu bytes of workspace, more than the "
                        "static %zu", need, STATIC_BYTES), TVMC_E_NOMEM;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return snprintf(g_err, sizeof(g_err), "tvmc_init_static: no usable current device"), TVMC_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev])
        return snprintf(g_err, sizeof(g_err), "tvmc_init_static: device %d's static workspace is held by a live "
                        "context (destroy it first)", dev), TVMC_E_STATE;
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return snprintf(g_err, sizeof(g_err), "tvmc_init_static: hipGetSymbolAddress failed: %s",
                            hipGetErrorString(e)), TVMC_E_DEVICE;
        g_static_ptr[dev] = ptr;
    }
    st = init_impl(p, 1, a, c, theta0, g_static_ptr[dev], STATIC_BYTES, stream, false, out);
    if (st != TVMC_OK) return st;
    (*out)->static_dev = dev;
    g_static_busy[dev] = true;
    return TVMC_OK;
}

tvmc_status tvmc_init(const tvmc_problem *p, const tvmc_ansatz *a, const tvmc_config *c, const double *theta0,
                      void *ws, size_t ws_bytes, void *stream, tvmc_ctx **out) {
    return tvmc_init_batch(p, 1, a, c, theta0, ws, ws_bytes, stream, out);
}

tvmc_status tvmc_sample(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    if (c->phase != 0) return set_err(c, "tvmc_sample: the previous evaluation was not completed"), TVMC_E_STATE;
    return run_sample(c);
}

tvmc_status tvmc_estimate(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    if (c->phase != 1) return set_err(c, "tvmc_estimate: call tvmc_sample first"), TVMC_E_STATE;
    return run_estimate(c);
}

tvmc_status tvmc_sr_solve(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    if (c->phase != 2) return set_err(c, "tvmc_sr_solve: call tvmc_estimate first"), TVMC_E_STATE;
    return run_solve(c);
}

tvmc_status tvmc_update(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    if (c->phase != 3) return set_err(c, "tvmc_update: call tvmc_sr_solve first"), TVMC_E_STATE;
    return run_update(c);
}

// One step through the captured graph: capture it on first use (the captured calls advance the
// host-side position as an eager step does), then replay with the step index set beforehand.
static tvmc_status graph_step(tvmc_ctx *c) {
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, c->stream, c->d, c->step);
    LAUNCHCHECK(c, "k_set_step");
    if (!c->gexec) {
        const int step0 = c->step, stage0 = c->stage, phase0 = c->phase;
        HIPCHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        tvmc_status st = TVMC_OK;
        for (int stage = 0; stage < 2 && st == TVMC_OK; ++stage) {
            if ((st = run_sample(c)) != TVMC_OK) break;
            if ((st = run_estimate(c)) != TVMC_OK) break;
            if ((st = run_solve(c)) != TVMC_OK) break;
            st = run_update(c);
        }
        c->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (st != TVMC_OK || e != hipSuccess) {   // nothing ran: back to the step boundary
            if (g) (void)hipGraphDestroy(g);
            c->step = step0;
            c->stage = stage0;
            c->phase = phase0;
            if (st == TVMC_OK) set_err(c, "step capture failed: %s", hipGetErrorString(e));
            return st != TVMC_OK ? st : TVMC_E_DEVICE;
        }
        c->graph = g;
        hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (ie == hipSuccess) ie = hipGraphLaunch(c->gexec, c->stream);
        if (ie != hipSuccess) {
            if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
            (void)hipGraphDestroy(g);
            c->gexec = nullptr;
            c->graph = nullptr;
            c->step = step0;
            c->stage = stage0;
            c->phase = phase0;
            set_err(c, "step graph instantiate / launch failed: %s", hipGetErrorString(ie));
            return TVMC_E_DEVICE;
        }
        return TVMC_OK;
    }
    HIPCHECK(c, hipGraphLaunch(c->gexec, c->stream));
    ++c->step;
    return TVMC_OK;
}

tvmc_status tvmc_sde_step(tvmc_ctx *c, int32_t n_steps) {
    if (!c || n_steps < 0) return TVMC_E_INVAL;
    if (c->phase != 0 || c->stage != 0) return set_err(c, "tvmc_sde_step: a step is half done"), TVMC_E_STATE;
    for (int s = 0; s < n_steps; ++s) {
        const bool obs = c->cfg.obs_every > 0 && c->step % c->cfg.obs_every == 0 && c->nobs < c->d.nobs;
        const bool train = c->d.ar && c->cfg.ar_train_every > 0 && c->step % c->cfg.ar_train_every == 0;
        if (c->cfg.use_graph && c->step >= 1 && !obs && !train && !c->timing) {
            tvmc_status st = graph_step(c);
            if (st != TVMC_OK) return st;
            continue;
        }
        for (int stage = 0; stage < 2; ++stage) {
            tvmc_status st = run_sample(c);
            if (st != TVMC_OK) return st;
            if (stage == 0 && c->cfg.obs_every > 0 && c->step % c->cfg.obs_every == 0 && c->nobs < c->d.nobs) {
                st = run_moments(c, c->nobs++);
                if (st != TVMC_OK) return st;
            }
            if (stage == 0 && c->d.ar && c->cfg.ar_train_every > 0 && c->step % c->cfg.ar_train_every == 0) {
                st = run_train(c, c->cfg.ar_train_iters);
                if (st != TVMC_OK) return st;
            }
            if ((st = run_estimate(c)) != TVMC_OK) return st;
            if ((st = run_solve(c)) != TVMC_OK) return st;
            if ((st = run_update(c)) != TVMC_OK) return st;
        }
    }
    return TVMC_OK;
}

tvmc_status tvmc_train_proposal(tvmc_ctx *c, int32_t n_iters) {
    if (!c || n_iters < 0) return TVMC_E_INVAL;
    if (!c->d.ar) return set_err(c, "tvmc_train_proposal: the learned proposal is not enabled"), TVMC_E_STATE;
    if (c->phase < 1) return set_err(c, "tvmc_train_proposal: no samples at the current evaluation point"), TVMC_E_STATE;
    return run_train(c, n_iters);
}

tvmc_status tvmc_observables(tvmc_ctx *c, double *out) {
    if (!c) return TVMC_E_INVAL;
    if (c->phase < 1) return set_err(c, "tvmc_observables: no samples at the current evaluation point"), TVMC_E_STATE;
    tvmc_status st = run_moments(c, -1);
    if (st != TVMC_OK) return st;
    if (out) {
        HIPCHECK(c, hipMemcpyAsync(out, c->d.mom, sizeof(double) * 9 * c->d.nt, hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    return TVMC_OK;
}

tvmc_status tvmc_ensemble(tvmc_ctx *c, double *out) { return tvmc_ensemble_at(c, -1, out, nullptr); }

tvmc_status tvmc_ensemble_at(tvmc_ctx *c, int32_t slot, double *out, double *loo_xi2) {
    if (!c || !out) return TVMC_E_INVAL;
    const Dev &d = c->d;
    if (slot >= c->nobs) return set_err(c, "tvmc_ensemble_at: history record %d not taken yet", slot), TVMC_E_INVAL;
    if (loo_xi2 && d.nt < 2) return set_err(c, "tvmc_ensemble_at: the jackknife needs two trajectories"), TVMC_E_INVAL;
    const int blocks = loo_xi2 ? d.nt + 1 : 1;
    hipLaunchKernelGGL(k_ensemble, dim3(blocks), dim3(64), 0, c->stream, d, slot < 0 ? -1 : slot, d.ens);
    LAUNCHCHECK(c, "k_ensemble");
    std::vector<double> buf((size_t)16 * blocks);
    HIPCHECK(c, hipMemcpyAsync(buf.data(), d.ens, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    memcpy(out, buf.data(), sizeof(double) * 13);
    if (loo_xi2)
        for (int t = 0; t < d.nt; ++t) loo_xi2[t] = buf[(size_t)16 * (t + 1) + 12];
    return TVMC_OK;
}

tvmc_status tvmc_get(tvmc_ctx *c, int32_t what, int32_t traj, void *host, size_t bytes) {
    if (!c || !host) return TVMC_E_INVAL;
    const Dev &d = c->d;
    if (traj < 0 || traj >= d.nt) return set_err(c, "tvmc_get: trajectory out of range"), TVMC_E_INVAL;
    const size_t nb = q_bytes(c, what);
    if (nb == 0) return set_err(c, "tvmc_get: unknown quantity %d", what), TVMC_E_INVAL;
    if (bytes < nb) return set_err(c, "tvmc_get: buffer too small (%zu < %zu)", bytes, nb), TVMC_E_INVAL;
    const size_t t = (size_t)traj;
    const void *src = nullptr;
    switch (what) {
    case TVMC_Q_THETA: src = d.theta + t * d.m; break;
    case TVMC_Q_THETA_EVAL: src = d.theta_eval + t * d.m; break;
    case TVMC_Q_DELTA0: src = d.d0 + t * d.m; break;
    case TVMC_Q_DELTA1: src = d.d1 + t * d.m; break;
    case TVMC_Q_SAMPLES: src = d.samples + t * d.ns * d.nw; break;
    case TVMC_Q_ELOC: src = d.eloc + t * d.ns; break;
    case TVMC_Q_S: src = d.S + t * s_doubles(d.kind, d.ss ? d.ns : d.m); break;
    case TVMC_Q_D: src = d.D + t * d.m; break;
    case TVMC_Q_OBAR: src = d.kind == TVMC_ANSATZ_RBM ? (const void *)(d.obarc + t * d.m) : (const void *)(d.obar + t * d.m); break;
    case TVMC_Q_BMEAN: src = d.bmean + t * d.nch; break;
    case TVMC_Q_DW: src = d.dw + t * d.nch; break;
    case TVMC_Q_ACCEPTS: src = d.acc + t * d.nc; break;
    case TVMC_Q_CHAINS: src = d.chains + t * d.nc * d.nw; break;
    case TVMC_Q_MOMENTS: src = d.mom + t * 9; break;
    case TVMC_Q_AR_PARAMS: src = d.arP + t * d.arnp; break;
    case TVMC_Q_AR_GRAD: src = d.arG + t * d.arnp; break;
    case TVMC_Q_AR_LOGQ: src = d.arlogq + t * d.ns; break;
    case TVMC_Q_AR_LOGQ_BF16:
        hipLaunchKernelGGL(k_ar_logq_bf16, dim3((d.ns + 3) / 4 < 1024 ? (d.ns + 3) / 4 : 1024), dim3(256), 0, c->stream,
                           d, traj);
        LAUNCHCHECK(c, "k_ar_logq_bf16");
        src = d.arlogqb + t * d.ns;
        break;
    case TVMC_Q_AR_LOSS: src = d.arloss + t; break;
    case TVMC_Q_AR_ACCEPTS: src = d.aracc + t * d.nc; break;
    case TVMC_Q_LOGNORM: src = d.lognorm + t; break;
    case TVMC_Q_EIG: src = d.snrEig + t * 2 * d.m; break;
    default: break;
    }
    if (what == TVMC_Q_OBS_HIST) {
        for (int s = 0; s < d.nobs; ++s)
            HIPCHECK(c, hipMemcpyAsync((double *)host + 9 * s, d.hist + ((size_t)s * d.nt + t) * 9, sizeof(double) * 9,
                                       hipMemcpyDeviceToHost, c->stream));
    } else if (what == TVMC_Q_LOGNORM_HIST) {
        if (d.nobs > 0)
            HIPCHECK(c, hipMemcpy2DAsync(host, sizeof(double), d.qhist + t, sizeof(double) * d.nt, sizeof(double),
                                         d.nobs, hipMemcpyDeviceToHost, c->stream));
    } else if (nb > 0) {
        HIPCHECK(c, hipMemcpyAsync(host, src, nb, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TVMC_OK;
}

tvmc_status tvmc_set(tvmc_ctx *c, int32_t what, int32_t traj, const void *host, size_t bytes) {
    if (!c || !host) return TVMC_E_INVAL;
    const Dev &d = c->d;
    if (traj < 0 || traj >= d.nt) return set_err(c, "tvmc_set: trajectory out of range"), TVMC_E_INVAL;
    if (what != TVMC_Q_THETA && what != TVMC_Q_CHAINS && what != TVMC_Q_AR_PARAMS)
        return set_err(c, "tvmc_set: only theta, chains and the proposal parameters"), TVMC_E_INVAL;
    const size_t nb = q_bytes(c, what);
    if (nb == 0) return set_err(c, "tvmc_set: quantity not present"), TVMC_E_INVAL;
    if (bytes < nb) return set_err(c, "tvmc_set: buffer too small"), TVMC_E_INVAL;
    if (what == TVMC_Q_AR_PARAMS) {
        for (size_t i = 0; i < d.arnp; ++i)
            if (!std::isfinite(((const float *)host)[i])) return set_err(c, "tvmc_set: parameters not finite"), TVMC_E_INVAL;
        HIPCHECK(c, hipMemcpyAsync(d.arP + (size_t)traj * d.arnp, host, nb, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_ar_copy, dim3((d.ah * d.n + 255) / 256, d.nt), dim3(256), 0, c->stream, d);
        LAUNCHCHECK(c, "k_ar_copy");
        HIPCHECK(c, hipStreamSynchronize(c->stream));
        return TVMC_OK;
    }
    void *dst = what == TVMC_Q_THETA ? (void *)(d.theta + (size_t)traj * d.m) : (void *)(d.chains + (size_t)traj * d.nc * d.nw);
    if (what == TVMC_Q_CHAINS)
        for (int i = 0; i < d.nc; ++i)
            for (int q = 0; q < d.nw; ++q) {
                const int bits = d.n - 64 * q;
                const uint64_t v = ((const uint64_t *)host)[(size_t)i * d.nw + q];
                if (bits < 64 && (v >> bits)) return set_err(c, "tvmc_set: chain word has bits above N"), TVMC_E_INVAL;
            }
    if (what == TVMC_Q_THETA)
        for (size_t i = 0; i < 2 * (size_t)d.m; ++i)
            if (!std::isfinite(((const double *)host)[i])) return set_err(c, "tvmc_set: theta not finite"), TVMC_E_INVAL;
    HIPCHECK(c, hipMemcpyAsync(dst, host, nb, hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TVMC_OK;
}

}  // extern "C"

namespace {

// Checkpoint blob: a header of 16 int64 (magic, version, N, M, T, chains, proposal parameters,
// history slots, kind, step, slots used, Adam step, reserved...), then theta [T][M] double2,
// chains [T][C] u64, log Q / predictor increment / log Q of the last moments [3][T] double,
// last moments [T][9], moment history [nobs][T][9], log Q history [nobs][T], and with the
// learned proposal its parameters and Adam moments [3][T][P] float.
constexpr int64_t STATE_MAGIC = 0x31455441534d5654ll;   // "TVMSATE1"
struct StatePart {
    void *dev;
    size_t bytes;
};
std::vector<StatePart> state_parts(const tvmc_ctx *c) {
    const Dev &d = c->d;
    const size_t T = (size_t)d.nt, nobs = (size_t)(d.nobs > 0 ? d.nobs : 0);
    std::vector<StatePart> p = {{d.theta, sizeof(double2) * T * d.m}, {d.chains, sizeof(uint64_t) * T * d.nc * d.nw},
                                {d.lognorm, sizeof(double) * 3 * T}, {d.mom, sizeof(double) * T * 9}};
    if (nobs) {
        p.push_back({d.hist, sizeof(double) * nobs * T * 9});
        p.push_back({d.qhist, sizeof(double) * nobs * T});
    }
    if (d.ar) {
        p.push_back({d.arP, sizeof(float) * T * d.arnp});
        p.push_back({d.arM, sizeof(float) * T * d.arnp});
        p.push_back({d.arV, sizeof(float) * T * d.arnp});
    }
    return p;
}
void state_header(const tvmc_ctx *c, int64_t h[16]) {
    const Dev &d = c->d;
    for (int i = 0; i < 16; ++i) h[i] = 0;
    h[0] = STATE_MAGIC;
    h[1] = 1;
    h[2] = d.n;
    h[3] = d.m;
    h[4] = d.nt;
    h[5] = d.nc;
    h[6] = (int64_t)d.arnp;
    h[7] = d.nobs;
    h[8] = d.kind;
    h[9] = c->step;
    h[10] = c->nobs;
    h[11] = c->adam_t;
}
size_t state_bytes(const tvmc_ctx *c) {
    size_t b = sizeof(int64_t) * 16;
    for (const auto &p : state_parts(c)) b += p.bytes;
    return b;
}

}  // namespace

extern "C" {

tvmc_status tvmc_state_size(const tvmc_ctx *c, size_t *bytes) {
    if (!c || !bytes) return TVMC_E_INVAL;
    *bytes = state_bytes(c);
    return TVMC_OK;
}

tvmc_status tvmc_save_state(tvmc_ctx *c, void *host, size_t bytes) {
    if (!c || !host) return TVMC_E_INVAL;
    if (c->stage != 0 || c->phase != 0) return set_err(c, "tvmc_save_state: not at a step boundary"), TVMC_E_STATE;
    if (bytes < state_bytes(c)) return set_err(c, "tvmc_save_state: buffer too small"), TVMC_E_INVAL;
    int64_t h[16];
    state_header(c, h);
    memcpy(host, h, sizeof(h));
    char *o = (char *)host + sizeof(h);
    for (const auto &p : state_parts(c)) {
        HIPCHECK(c, hipMemcpyAsync(o, p.dev, p.bytes, hipMemcpyDeviceToHost, c->stream));
        o += p.bytes;
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return TVMC_OK;
}

tvmc_status tvmc_load_state(tvmc_ctx *c, const void *host, size_t bytes) {
    if (!c || !host) return TVMC_E_INVAL;
    if (c->stage != 0 || c->phase != 0) return set_err(c, "tvmc_load_state: not at a step boundary"), TVMC_E_STATE;
    if (bytes != state_bytes(c)) return set_err(c, "tvmc_load_state: blob of another size"), TVMC_E_INVAL;
    int64_t h[16], mine[16];
    memcpy(h, host, sizeof(h));
    state_header(c, mine);
    for (int i = 0; i < 9; ++i)
        if (h[i] != mine[i]) return set_err(c, "tvmc_load_state: blob of another shape (header word %d)", i), TVMC_E_INVAL;
    if (h[9] < 0 || h[10] < 0 || h[10] > c->d.nobs || h[11] < 0)
        return set_err(c, "tvmc_load_state: bad counters"), TVMC_E_INVAL;
    const char *in = (const char *)host + sizeof(h);
    for (const auto &p : state_parts(c)) {
        HIPCHECK(c, hipMemcpyAsync(p.dev, in, p.bytes, hipMemcpyHostToDevice, c->stream));
        in += p.bytes;
    }
    if (c->d.ar) {
        hipLaunchKernelGGL(k_ar_copy, dim3((c->d.ah * c->d.n + 255) / 256, c->d.nt), dim3(256), 0, c->stream, c->d);
        LAUNCHCHECK(c, "k_ar_copy");
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->step = (int)h[9];
    c->nobs = (int)h[10];
    c->adam_t = (int)h[11];
    return TVMC_OK;
}

tvmc_status tvmc_position(const tvmc_ctx *c, int32_t *step, int32_t *stage) {
    if (!c || !step || !stage) return TVMC_E_INVAL;
    *step = c->step;
    *stage = c->stage;
    return TVMC_OK;
}

tvmc_status tvmc_synchronize(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    std::vector<int> f(c->d.nt);
    HIPCHECK(c, hipMemcpy(f.data(), c->d.flags, sizeof(int) * f.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < c->d.nt; ++t)
        if (f[t]) {
            set_err(c, "trajectory %d: non-positive pivot or non-finite increment", c->d.traj0 + t);
            return TVMC_E_NUMERIC;
        }
    return TVMC_OK;
}

tvmc_status tvmc_set_timing(tvmc_ctx *c, int32_t enable) {
    if (!c) return TVMC_E_INVAL;
    c->timing = enable != 0;
    for (auto &t : c->timers) t.used = 0;
    return TVMC_OK;
}

tvmc_status tvmc_timing(tvmc_ctx *c, const char *group, double *avg_ms, int32_t *count) {
    if (!c || !group || !avg_ms || !count) return TVMC_E_INVAL;
    *avg_ms = 0.0;
    *count = 0;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (size_t g = 0; g < c->groups.size(); ++g) {
        if (c->groups[g] != group) continue;
        Timer &tm = c->timers[g];
        double tot = 0.0;
        for (size_t i = 0; i < tm.used; ++i) {
            float ms = 0.f;
            HIPCHECK(c, hipEventElapsedTime(&ms, tm.start[i], tm.stop[i]));
            tot += ms;
        }
        *count = (int32_t)tm.used;
        *avg_ms = tm.used ? tot / tm.used : 0.0;
    }
    return TVMC_OK;
}

const char *tvmc_last_error(const tvmc_ctx *c) { return c ? c->err : g_err; }

tvmc_status tvmc_destroy(tvmc_ctx *c) {
    if (!c) return TVMC_E_INVAL;
    (void)hipStreamSynchronize(c->stream);
    for (int g = 0; g < NSIDE; ++g) {
        if (c->side[g]) {
            (void)hipStreamSynchronize(c->side[g]);
            (void)hipStreamDestroy(c->side[g]);
        }
        if (c->join[g]) (void)hipEventDestroy(c->join[g]);
    }
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[c->static_dev] = false;
    }
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto &t : c->timers) {
        for (auto e : t.start) (void)hipEventDestroy(e);
        for (auto e : t.stop) (void)hipEventDestroy(e);
    }
    delete c;
    return TVMC_OK;
}

}  // extern "C"
