// Assembly of S + eps I for the Jastrow ansatz (definition after Eq. 8, diagonal shift of the
// regularised solve).  Every O_k is +-1 (s_i, or s_j s_k), or for a shared LJPHd distance D
// the integer sum of s_j s_{j+D}, so sum_s O_sk O_sl is an exact integer in either variant
// below (the int8 one takes +-1 only), and the centring S_kl = sum/N_s - <O_k><O_l> uses the same
// separately rounded operations in both: they produce the same bits for any N_s (and S is
// exact outright when N_s is a power of two).  Only the lower triangle (k >= l) is written;
// the Cholesky factorisation reads nothing else.
#pragma once
#include "common.hpp"

namespace tvmc {

// sum/N_s - <O_k><O_l>, each product and the difference rounded separately (no fused
// multiply-add), so the result does not depend on how the compiler contracts it.
__device__ __forceinline__ double centre(double sum, double inv, double ok, double ol) {
#pragma clang fp contract(off)
    const double a = sum * inv;
    const double b = ok * ol;
    return a - b;
}

__device__ __forceinline__ double add_shift(double v, double eps) {
#pragma clang fp contract(off)
    return v + eps;
}

template <int W>
__device__ __forceinline__ double o_value(const Cfg<W> &mk, int p, int q, int n) { return (double)o_int<true>(mk, p, q, n); }

// Plain form: 64x64 tile per workgroup, 4x4 register tile per thread, FP64 FMAs.
template <int W>
__global__ __launch_bounds__(256) void k_sbuild_f64(Dev a) {
    __shared__ Cfg<W> smask[256];
    const int t = blockIdx.y;
    // lower-triangular tile index -> (bi, bj), bi >= bj
    const int tile = blockIdx.x;
    int bi = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    while (bi * (bi + 1) / 2 > tile) --bi;
    const int bj = tile - bi * (bi + 1) / 2;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    int rp[4], rq[4], cp[4], cq[4];
    for (int u = 0; u < 4; ++u) {
        const int k = bi * 64 + ty * 4 + u, l = bj * 64 + tx * 4 + u;
        rp[u] = k < a.m ? a.pa[k] : 0;
        rq[u] = k < a.m ? a.pb[k] : -1;
        cp[u] = l < a.m ? a.pa[l] : 0;
        cq[u] = l < a.m ? a.pb[l] : -1;
    }
    double acc[4][4] = {};
    const uint64_t *smp = a.samples + (size_t)t * a.ns * W;
    for (int s0 = 0; s0 < a.ns; s0 += 256) {
        __syncthreads();
        if (s0 + threadIdx.x < a.ns) smask[threadIdx.x] = cfg_load<W>(smp + (size_t)(s0 + threadIdx.x) * W);
        __syncthreads();
        const int cnt = (a.ns - s0) < 256 ? (a.ns - s0) : 256;
        for (int s = 0; s < cnt; ++s) {
            const Cfg<W> mk = smask[s];
            double ov[4], cv[4];
            for (int u = 0; u < 4; ++u) {
                ov[u] = o_value(mk, rp[u], rq[u], a.n);
                cv[u] = o_value(mk, cp[u], cq[u], a.n);
            }
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[u][v] += ov[u] * cv[v];
        }
    }
    const double inv = 1.0 / (double)a.ns;
    const double *ob = a.obar + (size_t)t * a.m;
    double *S = a.S + (size_t)t * a.m * a.m;
    for (int u = 0; u < 4; ++u) {
        const int k = bi * 64 + ty * 4 + u;
        if (k >= a.m) continue;
        for (int v = 0; v < 4; ++v) {
            const int l = bj * 64 + tx * 4 + v;
            if (l >= a.m || l > k) continue;
            double sv = centre(acc[u][v], inv, ob[k], ob[l]);
            if (k == l) sv = add_shift(sv, a.eps);
            S[(size_t)k * a.m + l] = sv;
        }
    }
}

}  // namespace tvmc
