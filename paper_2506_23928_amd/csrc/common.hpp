// Device-side building blocks shared by the otVMC kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvmc {

// ---------------------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// two 32x32->64 multiplications with multipliers 0xD2511F53 / 0xCD9E8D57, key schedule
// bumped by the Weyl constants 0x9E3779B9 / 0xBB67AE85.
// Counter layout used by this library:
//   Metropolis proposal p of chain c : (p, stage<<31 | c, step, 1<<24 | traj)
//   Wiener increments, channel pair q: (q, 0, step, 2<<24 | traj)
//   initial configuration of chain c : (0, c, 0, 3<<24 | traj)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// 53-bit uniform in [0, 1) from the top 27 bits of a and the top 26 bits of b.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reductions over the 64 lanes through DPP lane moves (no LDS round trips): within each row
// of 16 lanes by quad permutations and mirrors, then across rows by the row broadcasts of
// lanes 15 and 31, which leave the total in lane 63; it is returned to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double old, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_1032 = 0xB1, DPP_QUAD_2301 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140,
              DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

__device__ __forceinline__ double wave_prod(double v) {
    v *= dpp_d<DPP_QUAD_1032, 0xF>(v, v);
    v *= dpp_d<DPP_QUAD_2301, 0xF>(v, v);
    v *= dpp_d<DPP_HALF_MIRROR, 0xF>(v, v);
    v *= dpp_d<DPP_MIRROR, 0xF>(v, v);
    v *= dpp_d<DPP_BCAST15, 0xA>(1.0, v);
    v *= dpp_d<DPP_BCAST31, 0xC>(1.0, v);
    return readlane_d(v, 63);
}

__device__ __forceinline__ int wave_sum_i(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, DPP_QUAD_1032, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_QUAD_2301, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_HALF_MIRROR, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_MIRROR, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_BCAST15, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, DPP_BCAST31, 0xC, 0xF, false);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ double spin(uint64_t mask, int i) { return ((mask >> i) & 1ull) ? 1.0 : -1.0; }

// A configuration of up to 64 W spins as W words: bit i % 64 of word i / 64 set <=> s_i = +1;
// bits at and above N are zero.  Stored as W consecutive words per configuration.
constexpr int MAX_WORDS = 3;   // N <= 192
template <int W>
struct Cfg {
    uint64_t w[W];
};
template <int W>
__device__ __forceinline__ Cfg<W> cfg_load(const uint64_t *p) {
    Cfg<W> c;
#pragma unroll
    for (int q = 0; q < W; ++q) c.w[q] = p[q];
    return c;
}
template <int W>
__device__ __forceinline__ void cfg_store(uint64_t *p, const Cfg<W> &c) {
#pragma unroll
    for (int q = 0; q < W; ++q) p[q] = c.w[q];
}
template <int W>
__device__ __forceinline__ bool cfg_up(const Cfg<W> &c, int i) {
    if constexpr (W == 1) return (c.w[0] >> i) & 1ull;
    else return (c.w[i >> 6] >> (i & 63)) & 1ull;
}
template <int W>
__device__ __forceinline__ double spin(const Cfg<W> &c, int i) { return cfg_up(c, i) ? 1.0 : -1.0; }
template <int W>
__device__ __forceinline__ void cfg_flip(Cfg<W> &c, int i) {
    if constexpr (W == 1) c.w[0] ^= 1ull << i;
    else c.w[i >> 6] ^= 1ull << (i & 63);
}
// number of sites where two configurations differ
template <int W>
__device__ __forceinline__ int cfg_diff(const Cfg<W> &x, const Cfg<W> &y) {
    int d = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) d += __popcll(x.w[q] ^ y.w[q]);
    return d;
}
// word q of the configuration shifted down by p sites (site j + p moves to site j), 0 < p < 64 W
template <int W>
__device__ __forceinline__ uint64_t cfg_shr_word(const Cfg<W> &c, int p, int q) {
    const int ws = p >> 6, bs = p & 63;
    const uint64_t lo = q + ws < W ? c.w[q + ws] : 0ull;
    const uint64_t hi = q + ws + 1 < W ? c.w[q + ws + 1] : 0ull;
    return bs ? ((lo >> bs) | (hi << (64 - bs))) : lo;
}
// sum over j of s_j s_{j+p}, j = 0 .. n-p-1: pairs that agree minus pairs that differ
template <int W>
__device__ __forceinline__ int cfg_dist_sum(const Cfg<W> &c, int p, int n) {
    const int len = n - p;
    int diff = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int bits = len - 64 * q;
        if (bits <= 0) break;
        const uint64_t low = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
        diff += __popcll((c.w[q] ^ cfg_shr_word(c, p, q)) & low);
    }
    return len - 2 * diff;
}

// Jastrow pair index of eta_{jk} (j < k) after the N one-body parameters.
__host__ __device__ __forceinline__ int pair_index(int n, int j, int k) {
    return n + j * n - j * (j + 1) / 2 + (k - j - 1);
}

// O_k of a packed configuration (bit i set <=> s_i = +1), as an integer.  DIST = false: the
// +-1 log-derivatives of the all-pair Jastrow only (no shared distances to test for).
template <bool DIST = true>
__device__ __forceinline__ int o_int(uint64_t mk, int p, int q, int n) {
    if (DIST && q == -2) {   // sum over j of s_j s_{j+p}: pairs that agree minus pairs that differ
        const int len = n - p;
        const uint64_t low = len >= 64 ? ~0ull : ((1ull << len) - 1ull);
        return len - 2 * __popcll((mk ^ (mk >> p)) & low);
    }
    const uint64_t par = (q < 0) ? (((mk >> p) & 1ull) ^ 1ull) : (((mk >> p) ^ (mk >> q)) & 1ull);
    return par ? -1 : 1;   // par = 1 <=> O = -1
}
template <bool DIST = true, int W>
__device__ __forceinline__ int o_int(const Cfg<W> &c, int p, int q, int n) {
    if constexpr (W == 1) {
        return o_int<DIST>(c.w[0], p, q, n);
    } else {
        if (DIST && q == -2) return cfg_dist_sum(c, p, n);
        const bool par = (q < 0) ? !cfg_up(c, p) : (cfg_up(c, p) != cfg_up(c, q));
        return par ? -1 : 1;
    }
}

// Everything a kernel may touch, as raw device pointers into the caller's workspace.
struct Dev {
    int n, m, nch, ns, nc, per, nt, nobs;
    int nw;                   // 64-bit words per configuration (1 for N <= 64, 2 for N <= 128, 3 for N <= 192)
    int kind, nh;             // ansatz (0 Jastrow, 1 RBM), hidden units
    int mp;                   // M rounded up to 128 (rows of the RBM's BF16 operand planes)
    int ss;                   // 1: the solve runs in sample space (S holds T = O_c O_c^H / N_s)
    double2 *ssrow, *ssrhs, *ssu;  // sample space: row means of K, G - <G>, solution u   [T][N_s]
    double *ssbar;            // mean of the row means [T]
    uint16_t *rbmP;           // RBM precision form: [T][4][mp][ns] BF16 split of the centred O
    int burn, thin, init_sweeps, scheme, traj0;
    uint32_t key0, key1;
    double hx, dt, eps;
    const double *J;          // [N*N] or [T][N*N] (j_stride = N*N when each trajectory has its own)
    size_t j_stride, r_stride;  // per-trajectory strides of J and of the jump rates (0: shared)
    const int *jkind;         // [nch]
    const int *jsite;         // [nch]
    const double *jrate;      // [nch] or [T][nch]
    const int *pa;            // [M] first site of O_k (k < N: the site itself)
    const int *pb;            // [M] second site of O_k (-1 for one-body terms, -2 for a shared
                              //     LJPHd distance pa: O_k = sum_j s_j s_{j+pa})
    const int *pidx;          // [N*N] theta index of the eta multiplying s_j s_k (j != k)
    double2 *theta, *theta_eval, *d0, *d1;   // [T][M]
    double *eta_re, *eta_im;  // [T][N*N] dense symmetric pair parameters of the evaluation point
    double2 *epair;           // [T][2][N*N] exp(+-4 eta_jk) for two-flip ratios
    uint64_t *chains;         // [T][C][nw]
    uint64_t *samples;        // [T][Ns][nw]
    uint32_t *sbits;          // [T][N][Ns/32] site-major bit planes of the samples
    double2 *R;               // [T][Ns][N] single-flip ratios psi(s^(i))/psi(s)
    double2 *eloc;            // [T][Ns] local energy of H
    uint32_t *acc;            // [T][C]
    double *dw;               // [T][nch]
    double2 *bmean;           // [T][nch]
    double2 *G;               // [T][Ns]
    double2 *gbar;            // [T]
    double *obar;             // [T][M] (Jastrow, real)
    double2 *obarc;           // [T][M] (RBM, complex)
    double *w_re, *w_im;      // [T][N][N'] RBM weights, split planes
    double2 *cT, *sT;         // [T][N'][N] cosh 2w, sinh 2w (transposed)
    double2 *cW, *sW;         // [T][N][N'] cosh 2w, sinh 2w (the sampler's single-flip ratios)
    double2 *tt;              // [T][Ns][N'] tanh g_j per sample
    double2 *D;               // [T][M]
    double *S;                // [T][M][M]
    double *linv;             // [T][panels][64*64] inverses of the Cholesky diagonal blocks
    double *mom_part;         // [T][mom_blocks][9]
    double2 *momtab;          // RBM moments with N > 64 or N N' > 4096: [T][mom_blocks][2][N'][N] tables
    double *mom;              // [T][9]
    double *hist;             // [nobs][T][9]
    double *ens;              // [16]
    int *flags;               // [T]
    int mom_blocks;
    // linear SSE (App. B): no <L+L^dag> drive in E_eff; log Q per trajectory
    int linear;
    double *lognorm;          // [T] log Q at the current step
    double *dq0;              // [T] predictor-stage increment of log Q
    double *momlq;            // [T] log Q when the moments in mom were taken
    double *qhist;            // [nobs][T] log Q at the history records
    // SNR-regularised solve (real S)
    int reg, snr_nxb;         // regulariser (1: SNR), 64-sample blocks of the variance sums
    double snr_tau;
    double *snrV;             // [T][M][M] eigenvectors as rows (V^T)
    double2 *snrRho, *snrW;   // [T][M] V^T D and the kept, scaled components
    double *snrEig;           // [T][M][2] eigenvalue, SNR
    double *snrPart;          // [T][snr_nxb][M] partial sums of u_k^2 |G - <G>|^2
    double2 *snrRot;          // [T][sweeps][rounds][pairs] recorded rotations (c, s) of the LDS Jacobi
    int *snrSweeps;           // [T] sweeps the LDS Jacobi ran
    int *dstep;               // [1] the step index that keys this step's Philox streams (device
                              //     resident, so a captured step graph replays for any step)
    // learned proposal (MADE): hidden width, parameter count per trajectory, buffers
    int ar, ah;
    size_t arnp;
    float *arP, *arG, *arM, *arV;     // [T][arnp] master parameters, gradient, Adam moments
    uint16_t *arW1Tb, *arW2Tb;       // [T][N][H], [T][H][N] BF16 inference copies (transposed)
    float *arh, *arda;                // [T][Ns][H] training activations
    float *arg;                       // [T][Ns][N]
    float *arlogq;                    // [T][Ns]
    float *arlogqb;                   // [T][Ns] log q under the sampler's BF16 network (on request)
    double *arloss;                   // [T]
    uint32_t *aracc;                  // [T][C] accepted learned proposals
};

}  // namespace tvmc
