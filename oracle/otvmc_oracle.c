/*
 * ORACLE -- test infrastructure, not product code.
 *
 * A plain, slow, double-precision CPU implementation of trajectory-unravelled
 * time-dependent variational Monte Carlo (otVMC) as defined in "Unraveling Open Quantum
 * Dynamics with Time-Dependent Variational Monte Carlo" (Apostoli, D'Alberto, Genoni,
 * Bertaina, Galli).  Equation numbers below are those of the paper:
 *   (1) Lindblad equation, (2) nonlinear Ito SSE, (4)-(5) Stratonovich SSE and H_eff^Strat,
 *   (8) the otVMC equations with the definitions of O_k, E_eff, B^n, S, F, N^n that follow
 *   it, (10) LITF Hamiltonian, (11) RBM, (12) Jastrow, the LJPHd ansatz of the LITF section,
 *   App. B (linear SSE), App. C (SDE solvers).
 *
 * Parity unpinned against the paper: the functional form of the SNR regulariser (snr_solve,
 * snr_solve_herm).  The paper names the scheme and its threshold but takes the form from a
 * reference it does not reproduce; the form used here is stated where it is defined.  The tests
 * pin its arithmetic against an independent vectorised statement of the same form (oracle/exact.py),
 * its limits (tau = 0, tau -> infinity), a one-spin case and its scale invariance, not the form.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no source with the GPU library; the two only meet in the seeded
 * inputs handed to both.  Every loop below is the plain definition in the paper's order:
 * no blocking, no fusion, sums run over samples in sample order.
 *
 * Sampling uses one counter-based generator, Philox4x32-10, written here from its
 * published definition (Salmon, Moraes, Dror, Shaw, SC'11).  Counter layout:
 *   key = (seed_lo32, seed_hi32)
 *   Metropolis proposal p of chain c: ctr = (p, stage<<31 | c, step, 1<<24 | traj)
 *   Wiener increments, channel pair q:  ctr = (q, 0, step, 2<<24 | traj)
 *   initial chain configuration block b: ctr = (b, c, 0, 3<<24 | traj)
 * Uniforms carry 53 bits: u = ((a>>5)*2^26 + (b>>6)) * 2^-53.
 */
#define _POSIX_C_SOURCE 199309L
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <time.h>
#include <string.h>

typedef double complex cplx;

enum { ORC_OK = 0, ORC_E_INVAL = 1, ORC_E_NOMEM = 2, ORC_E_NUMERIC = 4 };
enum { ORC_JASTROW = 0, ORC_RBM = 1, ORC_LJPH = 2 };
enum { ORC_SIGMA_MINUS = 0, ORC_SIGMA_PLUS = 1, ORC_SIGMA_Z = 2 };
enum { ORC_HEUN = 0, ORC_MIDPOINT = 1, ORC_EULER = 2 };

typedef struct {
    int32_t n;             /* number of spins N */
    const double *J;       /* N*N, symmetric, zero diagonal: H_diag = sum_{i<j} J_ij s_i s_j */
    double hx;             /* H_offdiag = hx * sum_i sigma^x_i */
    int32_t n_ch;          /* number of jump operators L_c = sqrt(rate_c) op_c(site_c) */
    const int32_t *kind;   /* ORC_SIGMA_MINUS / PLUS / Z */
    const int32_t *site;
    const double *rate;
} orc_problem;

typedef struct {
    int32_t kind;          /* ORC_JASTROW (all-pair two-body Jastrow), ORC_RBM or ORC_LJPH */
    int32_t n_hidden;      /* RBM hidden units N' */
    int32_t range;         /* LJPHd: d, pairs with |j-k| <= d keep their own eta */
} orc_ansatz;

typedef struct {
    int32_t n_samples, n_chains, burn_sweeps, thin_sweeps, init_sweeps;
    int32_t enumerate;     /* 1: exact |psi|^2-weighted sums over all 2^N configurations */
    double dt, diag_shift;
    int32_t scheme;        /* ORC_HEUN, ORC_MIDPOINT, ORC_EULER (negative control) */
    int32_t n_steps, obs_every;
    uint64_t seed;
    int32_t linear;        /* 1: the linear SSE of App. B (E_eff^lin, norm SDE, weighted averages) */
    int32_t regulariser;   /* ORC_REG_SHIFT: (S + eps I) delta = D by Cholesky; ORC_REG_SNR: the
                              signal-to-noise filter in the eigenbasis of S + eps I */
    double snr_tau;        /* SNR threshold of the filter */
} orc_config;

enum { ORC_REG_SHIFT = 0, ORC_REG_SNR = 1 };

typedef struct {           /* optional outputs of one evaluation (any pointer may be NULL) */
    int8_t *samples;       /* [n_samples][N], +-1 */
    double *eloc;          /* [n_samples][2]  local energy of H (not H_eff) */
    double *S;             /* [M][M][2] */
    double *F;             /* [M][2] */
    double *Nn;            /* [n_ch][M][2] */
    double *D;             /* [M][2] */
    double *bmean;         /* [n_ch][2] Monte Carlo mean of B^n */
    double *obar;          /* [M][2] */
    double *delta;         /* [M][2] */
    int64_t *accepts;      /* [n_chains] */
    double *obs;           /* [9] per-trajectory moments (see orc_moments) */
    double *seconds;       /* [3] wall time of: sampling and local quantities; means, S, F, N^n, D; solve */
    double *dlognorm;      /* [1] linear SSE: increment of log Q over the step (App. B, norm SDE) */
    double *eig;           /* [M][2] SNR solve: eigenvalue of S + eps I and the SNR of D's component */
    double *G;             /* [n_samples][2] G(x) = -i dt E_eff(x) + sum_n B^n(x) dW_n per sample */
} orc_eval_out;

/* ------------------------------------------------------------------ Philox4x32-10 */

void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double orc_u53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

static void key_of(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
}

/* Real Gaussian Wiener increments dW_c ~ N(0, dt), one per channel per step, shared by
 * predictor and corrector (Eq. 2: real increments of variance dt; App. C).
 * Box-Muller on two 53-bit uniforms, with 1-u1 in (0,1]. */
void orc_draw_dw(uint64_t seed, int32_t traj, int32_t step, int32_t n_ch, double dt, double *dw)
{
    uint32_t key[2];
    key_of(seed, key);
    const double two_pi = 6.283185307179586476925286766559;
    for (int q = 0; 2 * q < n_ch; ++q) {
        uint32_t ctr[4] = {(uint32_t)q, 0u, (uint32_t)step, (2u << 24) | (uint32_t)traj}, r[4];
        orc_philox(ctr, key, r);
        double u1 = orc_u53(r[0], r[1]), u2 = orc_u53(r[2], r[3]);
        double rad = sqrt(-2.0 * log(1.0 - u1));
        double z0 = rad * cos(two_pi * u2), z1 = rad * sin(two_pi * u2);
        dw[2 * q] = sqrt(dt) * z0;
        if (2 * q + 1 < n_ch) dw[2 * q + 1] = sqrt(dt) * z1;
    }
}

/* Initial chain configurations: uniform random spins (exact samples of |psi|^2 when all
 * Jastrow parameters vanish, which is the +x coherent state, Eq. 12 and the text after it). */
void orc_init_chains(uint64_t seed, int32_t traj, int32_t n, int32_t n_chains, int8_t *chains)
{
    uint32_t key[2];
    key_of(seed, key);
    for (int c = 0; c < n_chains; ++c) {
        for (int b = 0; 128 * b < n; ++b) {
            uint32_t ctr[4] = {(uint32_t)b, (uint32_t)c, 0u, (3u << 24) | (uint32_t)traj}, r[4];
            orc_philox(ctr, key, r);
            for (int i = 128 * b; i < n && i < 128 * (b + 1); ++i) {
                int j = i - 128 * b;
                int bit = (r[j / 32] >> (j % 32)) & 1u;
                chains[(size_t)c * n + i] = bit ? 1 : -1;
            }
        }
    }
}

/* ------------------------------------------------------------------ problem */

/* Kac-normalised power-law couplings of the LITF Hamiltonian (Eq. 10):
 *   J_ij = Jscale * r_ij^-alpha / K(alpha),  K(alpha) = sum_{i<j} r_ij^-alpha / (N-1).
 * geom 0: open chain, r = |i-j|;  geom 1: periodic chain with the nearest replica only,
 * r = min(|i-j|, N-|i-j|);  geom 2: open Lx x Ly lattice, Euclidean r. */
int orc_couplings(int32_t geom, int32_t lx, int32_t ly, double alpha, double jscale, double *J)
{
    int n = (geom == 2) ? lx * ly : lx;
    if (n < 2) return ORC_E_INVAL;
    double kac = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double r;
            if (geom == 2) {
                double dx = (double)(i % lx - j % lx), dy = (double)(i / lx - j / lx);
                r = sqrt(dx * dx + dy * dy);
            } else {
                int d = abs(i - j);
                if (geom == 1 && n - d < d) d = n - d;
                r = (double)d;
            }
            J[(size_t)i * n + j] = (i == j) ? 0.0 : pow(r, -alpha);
            if (i < j) kac += pow(r, -alpha);
        }
    kac /= (double)(n - 1);
    for (int i = 0; i < n * n; ++i) J[i] = jscale * J[i] / kac;
    return ORC_OK;
}

/* ------------------------------------------------------------------ ansatz */

/* LJPHd (the partially inhomogeneous Jastrow of the LITF section): the biases a_i and the
 * pairs at distance |j-k| <= d keep their own parameters, every farther pair shares one eta per
 * distance D = d+1 .. N-1 (open chain).  Pairs with their own eta: d(2N-d-1)/2. */
static int ljph_own_pairs(int n, int d) { return d * (2 * n - d - 1) / 2; }

int32_t orc_n_params(const orc_ansatz *a, int32_t n)
{
    if (a->kind == ORC_JASTROW) return n + n * (n - 1) / 2;
    if (a->kind == ORC_LJPH) return n + ljph_own_pairs(n, a->range) + (n - 1 - a->range);
    return n + a->n_hidden + n * a->n_hidden;
}

/* Jastrow pair index of eta_{jk}, j<k, row-major upper triangle after the N one-body terms */
static int pair_index(int n, int j, int k)
{
    if (j > k) { int t = j; j = k; k = t; }
    return n + j * n - j * (j + 1) / 2 + (k - j - 1);
}

/* index of the parameter that plays eta_{jk} (j != k): the Jastrow pair itself, or for LJPHd
 * the pair's own parameter (same row-major order, rows cut at distance d) when |j-k| <= d and
 * the shared parameter of its distance otherwise */
static int eta_index(const orc_ansatz *an, int n, int j, int k)
{
    if (an->kind != ORC_LJPH) return pair_index(n, j, k);
    if (j > k) { int t = j; j = k; k = t; }
    int d = an->range, dist = k - j;
    if (dist > d) return n + ljph_own_pairs(n, d) + (dist - d - 1);
    int at = n;
    for (int r = 0; r < j; ++r) at += (n - 1 - r < d) ? n - 1 - r : d;
    return at + dist - 1;
}

/* log cosh(z) without overflow: cosh is even, and for Re z >= 0
 * log cosh z = z + log(1 + e^{-2z}) - log 2. */
static cplx lncosh(cplx z)
{
    if (creal(z) < 0.0) z = -z;
    return z + clog(1.0 + cexp(-2.0 * z)) - log(2.0);
}

static void rbm_angles(int n, int nh, const cplx *th, const int8_t *s, cplx *gam)
{
    const cplx *b = th + n, *w = th + n + nh;
    for (int j = 0; j < nh; ++j) {
        cplx g = b[j];
        for (int i = 0; i < n; ++i) g += w[(size_t)i * nh + j] * (double)s[i];
        gam[j] = g;
    }
}

/* log psi(sigma): Eq. 12 (Jastrow) and Eq. 11 (RBM) */
static cplx logpsi(const orc_ansatz *an, int n, const cplx *th, const int8_t *s)
{
    cplx lp = 0.0;
    for (int i = 0; i < n; ++i) lp += th[i] * (double)s[i];
    if (an->kind != ORC_RBM) {
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) lp += th[eta_index(an, n, j, k)] * (double)(s[j] * s[k]);
    } else {
        int nh = an->n_hidden;
        cplx *g = malloc(sizeof(cplx) * nh);
        rbm_angles(n, nh, th, s, g);
        for (int j = 0; j < nh; ++j) lp += log(2.0) + lncosh(g[j]);
        free(g);
    }
    return lp;
}

/* log psi(sigma with spin i flipped) - log psi(sigma).  gam: RBM angles of sigma. */
static cplx flip1(const orc_ansatz *an, int n, const cplx *th, const int8_t *s, const cplx *gam, int i)
{
    double si = (double)s[i];
    if (an->kind != ORC_RBM) {
        cplx f = th[i];
        for (int k = 0; k < n; ++k)
            if (k != i) f += th[eta_index(an, n, i, k)] * (double)s[k];
        return -2.0 * si * f;
    }
    int nh = an->n_hidden;
    const cplx *w = th + n + nh;
    cplx d = -2.0 * th[i] * si;
    for (int j = 0; j < nh; ++j) d += lncosh(gam[j] - 2.0 * w[(size_t)i * nh + j] * si) - lncosh(gam[j]);
    return d;
}

/* log psi(sigma with spins i and k flipped) - log psi(sigma), i != k */
static cplx flip2(const orc_ansatz *an, int n, const cplx *th, const int8_t *s, const cplx *gam, int i, int k)
{
    double si = (double)s[i], sk = (double)s[k];
    if (an->kind != ORC_RBM)
        return flip1(an, n, th, s, gam, i) + flip1(an, n, th, s, gam, k) + 4.0 * si * sk * th[eta_index(an, n, i, k)];
    int nh = an->n_hidden;
    const cplx *w = th + n + nh;
    cplx d = -2.0 * th[i] * si - 2.0 * th[k] * sk;
    for (int j = 0; j < nh; ++j)
        d += lncosh(gam[j] - 2.0 * w[(size_t)i * nh + j] * si - 2.0 * w[(size_t)k * nh + j] * sk) - lncosh(gam[j]);
    return d;
}

/* O_k(sigma) = d log psi / d theta_k (definition after Eq. 8) */
static void log_derivs(const orc_ansatz *an, int n, const cplx *th, const int8_t *s, const cplx *gam, cplx *O,
                       size_t stride)
{
    for (int i = 0; i < n; ++i) O[i * stride] = (double)s[i];
    if (an->kind == ORC_JASTROW) {
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) O[pair_index(n, j, k) * stride] = (double)(s[j] * s[k]);
    } else if (an->kind == ORC_LJPH) {
        /* a shared eta multiplies every pair of its distance: O is the sum of their s_j s_k */
        int m = orc_n_params(an, n);
        for (int k = n; k < m; ++k) O[k * stride] = 0.0;
        for (int j = 0; j < n; ++j)
            for (int k = j + 1; k < n; ++k) O[eta_index(an, n, j, k) * stride] += (double)(s[j] * s[k]);
    } else {
        int nh = an->n_hidden;
        for (int j = 0; j < nh; ++j) O[(n + j) * stride] = ctanh(gam[j]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < nh; ++j) O[(n + nh + (size_t)i * nh + j) * stride] = (double)s[i] * ctanh(gam[j]);
    }
    (void)th;
}

/* exported single-configuration helpers (tests check them against brute force) */
static void unpack_theta(int m, const double *t2, cplx *th)
{
    for (int k = 0; k < m; ++k) th[k] = t2[2 * k] + I * t2[2 * k + 1];
}

void orc_logpsi(const orc_ansatz *an, int32_t n, const double *theta, const int8_t *s, double *out)
{
    int m = orc_n_params(an, n);
    cplx *th = malloc(sizeof(cplx) * m);
    unpack_theta(m, theta, th);
    cplx v = logpsi(an, n, th, s);
    out[0] = creal(v); out[1] = cimag(v);
    free(th);
}

void orc_local_quantities(const orc_ansatz *an, int32_t n, const double *theta, const int8_t *s,
                          double *flip1_out /*[n][2]*/, double *flip2_out /*[n][n][2] or NULL*/,
                          double *O_out /*[M][2]*/)
{
    int m = orc_n_params(an, n), nh = an->kind == ORC_RBM ? an->n_hidden : 0;
    cplx *th = malloc(sizeof(cplx) * m), *gam = malloc(sizeof(cplx) * (nh + 1)), *O = malloc(sizeof(cplx) * m);
    unpack_theta(m, theta, th);
    if (nh) rbm_angles(n, nh, th, s, gam);
    for (int i = 0; i < n; ++i) {
        cplx d = flip1(an, n, th, s, gam, i);
        flip1_out[2 * i] = creal(d); flip1_out[2 * i + 1] = cimag(d);
        if (flip2_out)
            for (int k = 0; k < n; ++k) {
                cplx e = (k == i) ? 0.0 : flip2(an, n, th, s, gam, i, k);
                flip2_out[2 * ((size_t)i * n + k)] = creal(e);
                flip2_out[2 * ((size_t)i * n + k) + 1] = cimag(e);
            }
    }
    log_derivs(an, n, th, s, gam, O, 1);
    for (int k = 0; k < m; ++k) { O_out[2 * k] = creal(O[k]); O_out[2 * k + 1] = cimag(O[k]); }
    free(th); free(gam); free(O);
}

/* ------------------------------------------------------------------ sampling */

/* Metropolis sampling of |psi_theta|^2 (text after Eq. 9): single-spin-flip chains, random
 * site per proposal, accept iff log u < 2 Re[log psi(s') - log psi(s)].  One evaluation runs
 * `burn` sweeps and then records n_samples/n_chains samples per chain, one every `thin` sweeps
 * (a sweep is N proposals).  Chains continue from where the previous evaluation left them. */
static void metropolis(const orc_ansatz *an, int n, const cplx *th, const orc_config *cf, int traj, int step,
                       int stage, int burn, int8_t *chains, int8_t *samples, int64_t *accepts)
{
    uint32_t key[2];
    key_of(cf->seed, key);
    int per = cf->n_samples / cf->n_chains, nh = an->kind == ORC_RBM ? an->n_hidden : 0;
    cplx *gam = malloc(sizeof(cplx) * (nh + 1));
    for (int c = 0; c < cf->n_chains; ++c) {
        int8_t *s = chains + (size_t)c * n;
        uint32_t p = 0;
        int64_t acc = 0;
        int64_t total = (int64_t)burn * n + (int64_t)per * cf->thin_sweeps * n;
        int rec = 0;
        for (int64_t q = 0; q < total; ++q) {
            uint32_t ctr[4] = {p++, ((uint32_t)stage << 31) | (uint32_t)c, (uint32_t)step, (1u << 24) | (uint32_t)traj};
            uint32_t r[4];
            orc_philox(ctr, key, r);
            int i = (int)(((uint64_t)r[0] * (uint64_t)n) >> 32);
            double u = orc_u53(r[1], r[2]);
            if (nh) rbm_angles(n, nh, th, s, gam);
            double re = creal(flip1(an, n, th, s, gam, i));
            if (log(u) < 2.0 * re) { s[i] = (int8_t)-s[i]; ++acc; }
            if (q >= (int64_t)burn * n && (q - (int64_t)burn * n + 1) % ((int64_t)cf->thin_sweeps * n) == 0) {
                memcpy(samples + ((size_t)c * per + rec) * n, s, n);
                ++rec;
            }
        }
        if (accepts) accepts[c] = acc;
    }
    free(gam);
}

/* ------------------------------------------------------------------ estimators */

/* Per-configuration moments of the collective spin used by the magnetisation and the
 * covariance C_ab = (1/2)<{M_a, M_b}> - M_a M_b (LITF section, observables paragraph).
 * out = (mx, my, mz, sxx, syy, szz, sxy, sxz, syz) with s_ab = (1/2)<{M_a,M_b}>. */
static void config_moments(const orc_ansatz *an, int n, const cplx *th, const int8_t *s, const cplx *gam,
                           const cplx *R, double *out)
{
    cplx mx = 0, my = 0, mz = 0, xx = 0, yy = 0, zz = 0, xy = 0, xz = 0, yz = 0;
    for (int a = 0; a < n; ++a) {
        double sa = (double)s[a];
        mx += R[a];
        my += -I * sa * R[a];
        mz += sa;
        for (int b = 0; b < n; ++b) {
            if (b == a) continue;
            double sb = (double)s[b];
            cplx Rab = cexp(flip2(an, n, th, s, gam, a, b));
            zz += sa * sb;
            xx += Rab;
            yy += -sa * sb * Rab;
            xy += -I * sb * Rab;
            xz += sb * R[a];
            yz += -I * sa * sb * R[a];
        }
    }
    double N = (double)n;
    out[0] = creal(mx) / N; out[1] = creal(my) / N; out[2] = creal(mz) / N;
    out[3] = (N + creal(xx)) / (N * N);
    out[4] = (N + creal(yy)) / (N * N);
    out[5] = (N + creal(zz)) / (N * N);
    out[6] = creal(xy) / (N * N);
    out[7] = creal(xz) / (N * N);
    out[8] = creal(yz) / (N * N);
}

/* Complex Hermitian Cholesky A = L L^H (lower, in place) and solve A x = b. */
static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------ SNR-regularised solve */

/* Eigen-decomposition A = V diag(lam) V^T of a real symmetric m x m matrix (row-major, destroyed)
 * by cyclic Jacobi rotations: every off-diagonal pair (p, q) in turn is zeroed by the plane
 * rotation with t = tan(phi) the smaller root of t^2 + 2 t theta - 1 = 0,
 * theta = (A_qq - A_pp) / (2 A_pq), until the off-diagonal mass is below 1e-30 of the total. */
int orc_eigh_sym(int32_t m, double *A, double *V, double *lam)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V[(size_t)i * m + j] = (i == j) ? 1.0 : 0.0;
    int sweep = 0;
    for (; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                double a = A[(size_t)i * m + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = A[(size_t)p * m + q];
                if (apq == 0.0) continue;
                double theta = (A[(size_t)q * m + q] - A[(size_t)p * m + p]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < m; ++k) {   /* columns p, q: A J */
                    double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - sn * akq;
                    A[(size_t)k * m + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {   /* rows p, q: J^T (A J) */
                    double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - sn * aqk;
                    A[(size_t)q * m + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {   /* V J */
                    double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - sn * vkq;
                    V[(size_t)k * m + q] = sn * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) lam[i] = A[(size_t)i * m + i];
    return sweep < 100 ? ORC_OK : ORC_E_NUMERIC;
}

/* The regulariser named in the text after Eq. 9: D is written in the eigenbasis of S, and each
 * component rho_k = (V^T D)_k is kept in proportion to its signal-to-noise ratio.  With the
 * per-sample contributions q_k(x) = u_k(x) (G(x) - <G>), u_k(x) = sum_l V_lk (O_l(x) - <O_l>),
 * whose mean is rho_k: SNR_k = |rho_k| sqrt(N_s) / sqrt(<|q_k|^2> - |rho_k|^2), and
 *   delta = sum_k V_k rho_k / lam_k * 1 / (1 + (tau / SNR_k)^6),
 * the smooth cutoff of Schmitt and Heyl's scheme; eigenvalues below 1e-14 of the largest are
 * dropped.  Real S (O_k real): the Jastrow ansaetze; the RBM's Hermitian S below. */
static int snr_solve(int m, int ns, const double *wgt, double norm, const cplx *O, const cplx *ob, const cplx *S,
                     double eps, const cplx *dG, double tau, cplx *D, double *eig_out)
{
    double *A = malloc(sizeof(double) * (size_t)m * m), *V = malloc(sizeof(double) * (size_t)m * m);
    double *lam = malloc(sizeof(double) * m), *u = malloc(sizeof(double) * ns);
    cplx *rho = malloc(sizeof(cplx) * m), *dl = calloc(m, sizeof(cplx));
    if (!A || !V || !lam || !u || !rho || !dl) return ORC_E_NOMEM;
    for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) A[(size_t)k * m + l] = creal(S[(size_t)k * m + l]) + (k == l ? eps : 0.0);
    int st = orc_eigh_sym(m, A, V, lam);
    double lmax = 0.0;
    for (int k = 0; k < m; ++k) lmax = fmax(lmax, lam[k]);
    for (int k = 0; k < m && st == ORC_OK; ++k) {
        cplx r = 0.0;
        for (int l = 0; l < m; ++l) r += V[(size_t)l * m + k] * D[l];
        rho[k] = r;
        double q2 = 0.0;
        for (int x = 0; x < ns; ++x) {
            double v = 0.0;
            for (int l = 0; l < m; ++l) v += V[(size_t)l * m + k] * creal(O[(size_t)l * ns + x] - ob[l]);
            u[x] = v;
            q2 += wgt[x] * v * v * (creal(dG[x]) * creal(dG[x]) + cimag(dG[x]) * cimag(dG[x]));
        }
        double var = q2 * norm - (creal(r) * creal(r) + cimag(r) * cimag(r));
        double snr = var > 0.0 ? cabs(r) * sqrt((double)ns) / sqrt(var) : INFINITY;
        double keep = (lam[k] > 1e-14 * lmax && cabs(r) > 0.0) ? 1.0 / (1.0 + pow(tau / snr, 6.0)) : 0.0;
        if (eig_out) { eig_out[2 * k] = lam[k]; eig_out[2 * k + 1] = snr; }
        if (keep > 0.0)
            for (int l = 0; l < m; ++l) dl[l] += V[(size_t)l * m + k] * (keep * rho[k] / lam[k]);
    }
    for (int l = 0; l < m; ++l) D[l] = dl[l];
    free(A); free(V); free(lam); free(u); free(rho); free(dl);
    return st;
}

/* The same for a complex Hermitian matrix: the rotation of (p, q) first turns A_pq real by the
 * phase e^{-i phi} on q (phi = arg A_pq), then applies the real rotation of |A_pq|; with
 * U_pp = c, U_pq = s, U_qp = -s e^{-i phi}, U_qq = c e^{-i phi}: A <- U^H A U, V <- V U. */
int orc_eigh_herm(int32_t m, cplx *A, cplx *V, double *lam)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V[(size_t)i * m + j] = (i == j) ? 1.0 : 0.0;
    int sweep = 0;
    for (; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                cplx a = A[(size_t)i * m + j];
                double a2 = creal(a) * creal(a) + cimag(a) * cimag(a);
                tot += a2;
                if (i != j) off += a2;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                cplx apq = A[(size_t)p * m + q];
                double aa = cabs(apq);
                if (aa == 0.0) continue;
                cplx ph = apq / aa;
                double theta = (creal(A[(size_t)q * m + q]) - creal(A[(size_t)p * m + p])) / (2.0 * aa);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < m; ++k) {   /* A U */
                    cplx akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
                    A[(size_t)k * m + p] = c * akp - sn * conj(ph) * akq;
                    A[(size_t)k * m + q] = sn * akp + c * conj(ph) * akq;
                }
                for (int k = 0; k < m; ++k) {   /* U^H (A U) */
                    cplx apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
                    A[(size_t)p * m + k] = c * apk - sn * ph * aqk;
                    A[(size_t)q * m + k] = sn * apk + c * ph * aqk;
                }
                for (int k = 0; k < m; ++k) {   /* V U */
                    cplx vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
                    V[(size_t)k * m + p] = c * vkp - sn * conj(ph) * vkq;
                    V[(size_t)k * m + q] = sn * vkp + c * conj(ph) * vkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) lam[i] = creal(A[(size_t)i * m + i]);
    return sweep < 100 ? ORC_OK : ORC_E_NUMERIC;
}

/* The SNR solve for a complex Hermitian S (the RBM): rho = V^H D, u_k(x) = sum_l V_lk
 * (O_l(x) - <O_l>), q_k(x) = conj(u_k(x)) (G(x) - <G>), otherwise as for the real S. */
static int snr_solve_herm(int m, int ns, const double *wgt, double norm, const cplx *O, const cplx *ob,
                          const cplx *S, double eps, const cplx *dG, double tau, cplx *D, double *eig_out)
{
    cplx *A = malloc(sizeof(cplx) * (size_t)m * m), *V = malloc(sizeof(cplx) * (size_t)m * m);
    double *lam = malloc(sizeof(double) * m);
    cplx *rho = malloc(sizeof(cplx) * m), *dl = calloc(m, sizeof(cplx));
    if (!A || !V || !lam || !rho || !dl) return ORC_E_NOMEM;
    for (int k = 0; k < m; ++k)
        for (int l = 0; l < m; ++l) A[(size_t)k * m + l] = S[(size_t)k * m + l] + (k == l ? eps : 0.0);
    int st = orc_eigh_herm(m, A, V, lam);
    double lmax = 0.0;
    for (int k = 0; k < m; ++k) lmax = fmax(lmax, lam[k]);
    for (int k = 0; k < m && st == ORC_OK; ++k) {
        cplx r = 0.0;
        for (int l = 0; l < m; ++l) r += conj(V[(size_t)l * m + k]) * D[l];
        rho[k] = r;
        double q2 = 0.0;
        for (int x = 0; x < ns; ++x) {
            cplx v = 0.0;
            for (int l = 0; l < m; ++l) v += V[(size_t)l * m + k] * (O[(size_t)l * ns + x] - ob[l]);
            double u2 = creal(v) * creal(v) + cimag(v) * cimag(v);
            q2 += wgt[x] * u2 * (creal(dG[x]) * creal(dG[x]) + cimag(dG[x]) * cimag(dG[x]));
        }
        double var = q2 * norm - (creal(r) * creal(r) + cimag(r) * cimag(r));
        double snr = var > 0.0 ? cabs(r) * sqrt((double)ns) / sqrt(var) : INFINITY;
        double keep = (lam[k] > 1e-14 * lmax && cabs(r) > 0.0) ? 1.0 / (1.0 + pow(tau / snr, 6.0)) : 0.0;
        if (eig_out) { eig_out[2 * k] = lam[k]; eig_out[2 * k + 1] = snr; }
        if (keep > 0.0)
            for (int l = 0; l < m; ++l) dl[l] += V[(size_t)l * m + k] * (keep * rho[k] / lam[k]);
    }
    for (int l = 0; l < m; ++l) D[l] = dl[l];
    free(A); free(V); free(lam); free(rho); free(dl);
    return st;
}

static int chol_solve(int m, cplx *A, cplx *b)
{
    for (int j = 0; j < m; ++j) {
        double d = creal(A[(size_t)j * m + j]);
        for (int k = 0; k < j; ++k) {
            cplx l = A[(size_t)j * m + k];
            d -= creal(l * conj(l));
        }
        if (!(d > 0.0) || !isfinite(d)) return ORC_E_NUMERIC;
        d = sqrt(d);
        A[(size_t)j * m + j] = d;
        for (int i = j + 1; i < m; ++i) {
            cplx v = A[(size_t)i * m + j];
            for (int k = 0; k < j; ++k) v -= A[(size_t)i * m + k] * conj(A[(size_t)j * m + k]);
            A[(size_t)i * m + j] = v / d;
        }
    }
    for (int i = 0; i < m; ++i) {
        cplx v = b[i];
        for (int k = 0; k < i; ++k) v -= A[(size_t)i * m + k] * b[k];
        b[i] = v / creal(A[(size_t)i * m + i]);
    }
    for (int i = m - 1; i >= 0; --i) {
        cplx v = b[i];
        for (int k = i + 1; k < m; ++k) v -= conj(A[(size_t)k * m + i]) * b[k];
        b[i] = v / creal(A[(size_t)i * m + i]);
    }
    for (int i = 0; i < m; ++i)
        if (!isfinite(creal(b[i])) || !isfinite(cimag(b[i]))) return ORC_E_NUMERIC;
    return ORC_OK;
}

/*
 * One evaluation of the right-hand side of the otVMC equations (Eq. 8) at theta:
 *   sample |psi|^2 -> local O_k, E_eff, B^n -> S, F, N^n -> D = -i F dt + sum_n N^n dW_n
 *   -> delta = (S + eps I)^{-1} D.
 * E_eff uses H_eff^Strat of Eq. 5 without its c-number terms (they cancel in F, which is a
 * covariance); <L_n + L_n^dag> is the Monte Carlo estimate 2 Re<B^n> from the same samples.
 * want_solve = 0 samples and evaluates observables only; 2 also computes the means, F, N^n
 * and D but neither S nor the solve (for large-N checks where S is checked separately);
 * 3 solves in sample space (Monte Carlo mode only) and returns T = O_c O_c^H / ns in S.
 */
int orc_eval(const orc_problem *pb, const orc_ansatz *an, const orc_config *cf, const double *theta,
             int8_t *chains, int32_t traj, int32_t step, int32_t stage, int32_t first, const double *dw,
             int32_t want_solve, orc_eval_out *out)
{
    int n = pb->n, m = orc_n_params(an, n), nch = pb->n_ch;
    int nh = an->kind == ORC_RBM ? an->n_hidden : 0;
    int ns;
    double t0 = wall_seconds();
    int8_t *conf;
    double *wgt;
    if (cf->enumerate) {
        if (n > 20 || want_solve == 3) return ORC_E_INVAL;
        ns = 1 << n;
    } else {
        if (cf->n_chains <= 0 || cf->n_samples % cf->n_chains) return ORC_E_INVAL;
        ns = cf->n_samples;
    }
    cplx *th = malloc(sizeof(cplx) * m);
    conf = malloc((size_t)ns * n);
    wgt = malloc(sizeof(double) * ns);
    cplx *O = malloc(sizeof(cplx) * (size_t)ns * m);
    cplx *eh = malloc(sizeof(cplx) * ns), *B = malloc(sizeof(cplx) * (size_t)ns * (nch + 1));
    double *ll = malloc(sizeof(double) * ns);
    cplx *gam = malloc(sizeof(cplx) * (nh + 1)), *R = malloc(sizeof(cplx) * n);
    if (!th || !conf || !wgt || !O || !eh || !B || !ll || !gam || !R) return ORC_E_NOMEM;
    unpack_theta(m, theta, th);

    if (cf->enumerate) {
        double *lre = malloc(sizeof(double) * ns), mx = -INFINITY, z = 0.0;
        for (int x = 0; x < ns; ++x) {
            for (int i = 0; i < n; ++i) conf[(size_t)x * n + i] = ((x >> i) & 1) ? 1 : -1;
            lre[x] = creal(logpsi(an, n, th, conf + (size_t)x * n));
            if (lre[x] > mx) mx = lre[x];
        }
        for (int x = 0; x < ns; ++x) { wgt[x] = exp(2.0 * (lre[x] - mx)); z += wgt[x]; }
        for (int x = 0; x < ns; ++x) wgt[x] /= z;
        free(lre);
    } else {
        int burn = cf->burn_sweeps + (first ? cf->init_sweeps : 0);
        metropolis(an, n, th, cf, traj, step, stage, burn, chains, conf, out ? out->accepts : NULL);
        for (int x = 0; x < ns; ++x) wgt[x] = 1.0;  /* divided by ns after summing */
        if (out && out->samples) memcpy(out->samples, conf, (size_t)ns * n);
    }
    double norm = cf->enumerate ? 1.0 : 1.0 / (double)ns;

    /* local quantities: O_k, E_H, B^n, sum_n [(L^dag L)_loc + (L^2)_loc] */
    double mom_acc[9] = {0};
    for (int x = 0; x < ns; ++x) {
        const int8_t *s = conf + (size_t)x * n;
        if (nh) rbm_angles(n, nh, th, s, gam);
        for (int i = 0; i < n; ++i) R[i] = cexp(flip1(an, n, th, s, gam, i));
        cplx e = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) e += pb->J[(size_t)i * n + j] * (double)(s[i] * s[j]);
        for (int i = 0; i < n; ++i) e += pb->hx * R[i];
        eh[x] = e;
        double l2 = 0.0;
        for (int c = 0; c < nch; ++c) {
            int st = pb->site[c];
            double g = pb->rate[c], sq = sqrt(g);
            cplx b;
            if (pb->kind[c] == ORC_SIGMA_MINUS) {
                b = (s[st] == -1) ? sq * R[st] : 0.0;
                l2 += (s[st] == 1) ? g : 0.0;
            } else if (pb->kind[c] == ORC_SIGMA_PLUS) {
                b = (s[st] == 1) ? sq * R[st] : 0.0;
                l2 += (s[st] == -1) ? g : 0.0;
            } else {
                b = sq * (double)s[st];
                l2 += g + g;
            }
            B[(size_t)c * ns + x] = b;
        }
        ll[x] = l2;
        log_derivs(an, n, th, s, gam, O + x, (size_t)ns);
        if (out && out->obs) {
            double mo[9];
            config_moments(an, n, th, s, gam, R, mo);
            for (int q = 0; q < 9; ++q) mom_acc[q] += wgt[x] * mo[q];
        }
        if (out && out->eloc && !cf->enumerate) { out->eloc[2 * x] = creal(e); out->eloc[2 * x + 1] = cimag(e); }
    }
    if (out && out->obs)
        for (int q = 0; q < 9; ++q) out->obs[q] = mom_acc[q] * norm;

    int status = ORC_OK;
    double t1 = wall_seconds(), t2 = t1;
    if (want_solve) {
        cplx *ob = calloc(m, sizeof(cplx)), *bm = calloc(nch + 1, sizeof(cplx));
        cplx *S = malloc(sizeof(cplx) * (want_solve == 1 ? (size_t)m * m : 1)), *F = malloc(sizeof(cplx) * m);
        cplx *Nn = malloc(sizeof(cplx) * (size_t)(nch + 1) * m), *D = malloc(sizeof(cplx) * m);
        cplx *eeff = malloc(sizeof(cplx) * ns);
        if (!ob || !bm || !S || !F || !Nn || !D || !eeff) return ORC_E_NOMEM;
        /* means */
        for (int k = 0; k < m; ++k) {
            cplx v = 0.0;
            for (int x = 0; x < ns; ++x) v += wgt[x] * O[(size_t)k * ns + x];
            ob[k] = v * norm;
        }
        for (int c = 0; c < nch; ++c) {
            cplx v = 0.0;
            for (int x = 0; x < ns; ++x) v += wgt[x] * B[(size_t)c * ns + x];
            bm[c] = v * norm;
        }
        /* E_eff(x) = E_H(x) - (i/2) sum_n [ (L^dag L)_loc - 2 <L+L^dag> B^n + (L^2)_loc ];
         * for the linear SSE (App. B) E_eff^lin(x) = E_H(x) - (i/2) sum_n [ (L^dag L)_loc + (L^2)_loc ],
         * the Stratonovich H_eff of the linear equation, which has no <L+L^dag> term */
        cplx eb = 0.0;
        for (int x = 0; x < ns; ++x) {
            cplx drive = 0.0;
            if (!cf->linear)
                for (int c = 0; c < nch; ++c) drive += 2.0 * (2.0 * creal(bm[c])) * B[(size_t)c * ns + x];
            eeff[x] = eh[x] - 0.5 * I * (ll[x] - drive);
            eb += wgt[x] * eeff[x];
        }
        eb *= norm;
        /* norm SDE of App. B: dQ = Q (2 Im<E_eff^lin> dt + 2 sum_n Re<B^n> o dW_n), i.e. in
         * log Q the increment 2 Im<E_eff^lin> dt + 2 sum_n Re<B^n> dW_n at this evaluation point;
         * the nonlinear SSE keeps the norm, Q = 1 */
        if (out && out->dlognorm) {
            double dq = 2.0 * cimag(eb) * cf->dt;
            for (int c = 0; c < nch; ++c) dq += 2.0 * creal(bm[c]) * dw[c];
            out->dlognorm[0] = cf->linear ? dq : 0.0;
        }
        /* S_kl = <O_k^* O_l> - <O_k^*><O_l>;  F_k = <O_k^* E_eff> - <O_k^*><E_eff>;
         * N^n_k = <O_k^* B^n> - <O_k^*><B^n>  (definitions after Eq. 8) */
        for (int k = 0; k < m; ++k) {
            const cplx *ok = O + (size_t)k * ns;
            for (int l = k; l < m && want_solve == 1; ++l) {   /* S is Hermitian by definition: fill l >= k, mirror */
                const cplx *ol = O + (size_t)l * ns;
                cplx v = 0.0;
                for (int x = 0; x < ns; ++x) v += wgt[x] * conj(ok[x]) * ol[x];
                S[(size_t)k * m + l] = v * norm - conj(ob[k]) * ob[l];
                S[(size_t)l * m + k] = conj(S[(size_t)k * m + l]);
            }
            cplx f = 0.0;
            for (int x = 0; x < ns; ++x) f += wgt[x] * conj(ok[x]) * eeff[x];
            F[k] = f * norm - conj(ob[k]) * eb;
            for (int c = 0; c < nch; ++c) {
                cplx v = 0.0;
                for (int x = 0; x < ns; ++x) v += wgt[x] * conj(ok[x]) * B[(size_t)c * ns + x];
                Nn[(size_t)c * m + k] = v * norm - conj(ob[k]) * bm[c];
            }
        }
        /* D = -i F dt + sum_n N^n dW_n  (the regularised-solve paragraph after Eq. 9) */
        for (int k = 0; k < m; ++k) {
            cplx d = -I * F[k] * cf->dt;
            for (int c = 0; c < nch; ++c) d += Nn[(size_t)c * m + k] * dw[c];
            D[k] = d;
        }
        if (out && out->G && !cf->enumerate)
            for (int x = 0; x < ns; ++x) {   /* G(x), whose covariance with O^* is D */
                cplx g = -I * cf->dt * eeff[x];
                for (int c = 0; c < nch; ++c) g += dw[c] * B[(size_t)c * ns + x];
                out->G[2 * x] = creal(g);
                out->G[2 * x + 1] = cimag(g);
            }
        if (out) {
            for (int k = 0; k < m; ++k) {
                if (out->F) { out->F[2 * k] = creal(F[k]); out->F[2 * k + 1] = cimag(F[k]); }
                if (out->D) { out->D[2 * k] = creal(D[k]); out->D[2 * k + 1] = cimag(D[k]); }
                if (out->obar) { out->obar[2 * k] = creal(ob[k]); out->obar[2 * k + 1] = cimag(ob[k]); }
                if (out->Nn)
                    for (int c = 0; c < nch; ++c) {
                        out->Nn[2 * ((size_t)c * m + k)] = creal(Nn[(size_t)c * m + k]);
                        out->Nn[2 * ((size_t)c * m + k) + 1] = cimag(Nn[(size_t)c * m + k]);
                    }
                if (out->S && want_solve == 1)
                    for (int l = 0; l < m; ++l) {
                        out->S[2 * ((size_t)k * m + l)] = creal(S[(size_t)k * m + l]);
                        out->S[2 * ((size_t)k * m + l) + 1] = cimag(S[(size_t)k * m + l]);
                    }
            }
            if (out->bmean)
                for (int c = 0; c < nch; ++c) { out->bmean[2 * c] = creal(bm[c]); out->bmean[2 * c + 1] = cimag(bm[c]); }
        }
        /* regularised solve (S + eps I) delta = D */
        t2 = wall_seconds();
        if (want_solve == 1 && cf->regulariser == ORC_REG_SNR) {
            cplx *dG = malloc(sizeof(cplx) * ns), gm = 0.0;
            if (!dG) return ORC_E_NOMEM;
            for (int x = 0; x < ns; ++x) {   /* G(x) = -i dt E_eff(x) + sum_n dW_n B^n(x) */
                cplx g = -I * cf->dt * eeff[x];
                for (int c = 0; c < nch; ++c) g += dw[c] * B[(size_t)c * ns + x];
                dG[x] = g;
                gm += wgt[x] * g;
            }
            gm *= norm;
            for (int x = 0; x < ns; ++x) dG[x] -= gm;
            if (an->kind == ORC_RBM)
                status = snr_solve_herm(m, ns, wgt, norm, O, ob, S, cf->diag_shift, dG, cf->snr_tau, D,
                                        out ? out->eig : NULL);
            else
                status = snr_solve(m, ns, wgt, norm, O, ob, S, cf->diag_shift, dG, cf->snr_tau, D,
                                   out ? out->eig : NULL);
            free(dG);
        } else if (want_solve == 1) {
            for (int k = 0; k < m; ++k) S[(size_t)k * m + k] += cf->diag_shift;
            status = chol_solve(m, S, D);
        } else if (want_solve == 3) {
            /* The same solve in sample space.  With A[x][k] = (O_k(x) - <O_k>) / sqrt(ns) and
             * g[x] = (G(x) - <G>) / sqrt(ns), G(x) = -i dt E_eff(x) + sum_n dW_n B^n(x), one has
             * S = A^H A and D = A^H g, and (A^H A + eps I)^-1 A^H = A^H (A A^H + eps I)^-1, so
             *   delta = A^H u / sqrt(ns),  (T + eps I) u = G - <G>,  T = A A^H (ns x ns). */
            cplx *T = malloc(sizeof(cplx) * (size_t)ns * ns), *u = malloc(sizeof(cplx) * ns);
            if (!T || !u) return ORC_E_NOMEM;
            cplx gm = 0.0;
            for (int x = 0; x < ns; ++x) {
                cplx g = -I * cf->dt * eeff[x];
                for (int c = 0; c < nch; ++c) g += dw[c] * B[(size_t)c * ns + x];
                u[x] = g;
                gm += g;
            }
            gm *= norm;
            for (int x = 0; x < ns; ++x) u[x] -= gm;
            for (int x = 0; x < ns; ++x)
                for (int y = 0; y <= x; ++y) {
                    cplx v = 0.0;
                    for (int k = 0; k < m; ++k)
                        v += (O[(size_t)k * ns + x] - ob[k]) * conj(O[(size_t)k * ns + y] - ob[k]);
                    T[(size_t)x * ns + y] = v * norm;
                    T[(size_t)y * ns + x] = conj(v) * norm;
                }
            if (out && out->S)
                for (size_t e = 0; e < (size_t)ns * ns; ++e) { out->S[2 * e] = creal(T[e]); out->S[2 * e + 1] = cimag(T[e]); }
            for (int x = 0; x < ns; ++x) T[(size_t)x * ns + x] += cf->diag_shift;
            status = chol_solve(ns, T, u);
            for (int k = 0; k < m; ++k) {
                cplx v = 0.0;
                for (int x = 0; x < ns; ++x) v += conj(O[(size_t)k * ns + x] - ob[k]) * u[x];
                D[k] = v * norm;
            }
            free(T); free(u);
        }
        if (out && out->delta && (want_solve == 1 || want_solve == 3))
            for (int k = 0; k < m; ++k) { out->delta[2 * k] = creal(D[k]); out->delta[2 * k + 1] = cimag(D[k]); }
        free(ob); free(bm); free(S); free(F); free(Nn); free(D); free(eeff);
    }
    if (out && out->seconds) {
        double t3 = wall_seconds();
        out->seconds[0] = t1 - t0;
        out->seconds[1] = t2 - t1;
        out->seconds[2] = t3 - t2;
    }
    free(th); free(conf); free(wgt); free(O); free(eh); free(B); free(ll); free(gam); free(R);
    return status;
}

/* ------------------------------------------------------------------ trajectories */

typedef struct {
    const orc_problem *pb;
    const orc_ansatz *an;
    const orc_config *cf;
    const double *theta0;
    int32_t n_traj, traj0;
    double *theta_out;     /* [n_traj][M][2] */
    double *obs_out;       /* [n_traj][n_out][9] */
    int32_t *status_out;   /* [n_traj] */
    double *lognorm_out;   /* [n_traj][n_out] log Q at the output times (may be NULL) */
    int next;
    pthread_mutex_t lock;
} run_job;

/* One trajectory: N_T independent trajectories start from theta0 (text after Eq. 9); each
 * step draws dW once and applies the predictor-corrector of App. C:
 *   Heun (trapezoid): thb = th + d(th);  th' = th + (d(th) + d(thb))/2
 *   midpoint:         thb = th + d(th);  th' = th + d((th + thb)/2)
 *   Euler:            th' = th + d(th)   (not Stratonovich-consistent; a negative control)
 * Observables come from the predictor samples at steps that are multiples of obs_every,
 * and from one extra sampling pass after the last step. */
static int run_one(const orc_problem *pb, const orc_ansatz *an, const orc_config *cf, const double *theta0,
                   int traj, double *th_out, double *obs_out, double *lq_out)
{
    int n = pb->n, m = orc_n_params(an, n), nch = pb->n_ch;
    double *th = malloc(sizeof(double) * 2 * m), *te = malloc(sizeof(double) * 2 * m);
    double *d0 = malloc(sizeof(double) * 2 * m), *d1 = malloc(sizeof(double) * 2 * m);
    double *dw = malloc(sizeof(double) * (nch + 1));
    int8_t *chains = malloc((size_t)(cf->n_chains > 0 ? cf->n_chains : 1) * n);
    memcpy(th, theta0, sizeof(double) * 2 * m);
    if (!cf->enumerate) orc_init_chains(cf->seed, traj, n, cf->n_chains, chains);
    int st = ORC_OK, iout = 0;
    /* log Q of the linear SSE, integrated by the same scheme as theta (the norm SDE is in
     * Stratonovich form); Q = 1 at t = 0 */
    double lq = 0.0, q0 = 0.0, q1 = 0.0;
    for (int step = 0; step < cf->n_steps && st == ORC_OK; ++step) {
        orc_draw_dw(cf->seed, traj, step, nch, cf->dt, dw);
        orc_eval_out o0 = {0};
        o0.delta = d0;
        o0.dlognorm = &q0;
        if (cf->obs_every > 0 && step % cf->obs_every == 0) {
            if (lq_out) lq_out[iout] = lq;
            o0.obs = obs_out + 9 * (size_t)iout++;
        }
        st = orc_eval(pb, an, cf, th, chains, traj, step, 0, step == 0, dw, 1, &o0);
        if (st) break;
        if (cf->scheme == ORC_EULER) {
            for (int k = 0; k < 2 * m; ++k) th[k] = th[k] + d0[k];
            lq += q0;
            continue;
        }
        for (int k = 0; k < 2 * m; ++k) te[k] = (cf->scheme == ORC_HEUN) ? th[k] + d0[k] : th[k] + 0.5 * d0[k];
        orc_eval_out o1 = {0};
        o1.delta = d1;
        o1.dlognorm = &q1;
        st = orc_eval(pb, an, cf, te, chains, traj, step, 1, 0, dw, 1, &o1);
        if (st) break;
        for (int k = 0; k < 2 * m; ++k)
            th[k] = (cf->scheme == ORC_HEUN) ? th[k] + 0.5 * (d0[k] + d1[k]) : th[k] + d1[k];
        lq += (cf->scheme == ORC_HEUN) ? 0.5 * (q0 + q1) : q1;
    }
    if (st == ORC_OK && cf->obs_every > 0) {
        orc_eval_out o = {0};
        if (lq_out) lq_out[iout] = lq;
        o.obs = obs_out + 9 * (size_t)iout;
        st = orc_eval(pb, an, cf, th, chains, traj, cf->n_steps, 0, cf->n_steps == 0, dw, 0, &o);
    }
    memcpy(th_out, th, sizeof(double) * 2 * m);
    free(th); free(te); free(d0); free(d1); free(dw); free(chains);
    return st;
}

static void *run_worker(void *arg)
{
    run_job *jb = (run_job *)arg;
    int m = orc_n_params(jb->an, jb->pb->n);
    int n_out = jb->cf->obs_every > 0 ? jb->cf->n_steps / jb->cf->obs_every + 1 : 0;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int t = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (t >= jb->n_traj) break;
        jb->status_out[t] = run_one(jb->pb, jb->an, jb->cf, jb->theta0, jb->traj0 + t,
                                    jb->theta_out + (size_t)t * 2 * m, jb->obs_out + (size_t)t * n_out * 9,
                                    jb->lognorm_out ? jb->lognorm_out + (size_t)t * n_out : NULL);
    }
    return NULL;
}

/* Run n_traj independent trajectories (ids traj0 .. traj0+n_traj-1) on n_threads threads;
 * lognorm_out (may be NULL) receives log Q at the output times (zero unless cf->linear). */
int orc_run(const orc_problem *pb, const orc_ansatz *an, const orc_config *cf, const double *theta0,
            int32_t n_traj, int32_t traj0, int32_t n_threads, double *theta_out, double *obs_out, int32_t *status_out,
            double *lognorm_out)
{
    if (cf->obs_every > 0 && cf->n_steps % cf->obs_every) return ORC_E_INVAL;
    run_job jb = {pb, an, cf, theta0, n_traj, traj0, theta_out, obs_out, status_out, lognorm_out, 0,
                  PTHREAD_MUTEX_INITIALIZER};
    if (n_threads < 1) n_threads = 1;
    pthread_t *tid = malloc(sizeof(pthread_t) * n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&tid[i], NULL, run_worker, &jb);
    for (int i = 0; i < n_threads; ++i) pthread_join(tid[i], NULL);
    free(tid);
    for (int t = 0; t < n_traj; ++t)
        if (status_out[t]) return status_out[t];
    return ORC_OK;
}
