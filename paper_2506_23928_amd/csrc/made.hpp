// Learned proposal: a two-layer masked autoregressive network (MADE) per trajectory, trained on
// the trajectory's own samples and used for independent Metropolis-Hastings moves.  The paper
// has no learned proposal; its definition (degrees, masks, loss) is this library's:
//   hidden unit k has degree d(k) = 1 + k mod (N-1) and sees spins j < d(k);
//   output i sees hidden units with d(k) <= i;  q(s_i = +1 | s_<i) = sigmoid(l_i);
//   a_k = b1_k + sum_{j<d(k)} W1[k][j] s_j,  h = relu(a),  l_i = b2_i + sum_{d(k)<=i} W2[i][k] h_k.
// Training: full-batch Adam on the mean negative log-likelihood, FP32 master weights; the
// sampler reads BF16 copies and accumulates in FP32.  Every
// independent proposal uses the same BF16 network for q(s') and q(s), so the chain stays exact.
#pragma once
#include "common.hpp"

namespace tvmc {

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                      // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ int ar_degree(int k, int n) { return 1 + (n > 1 ? k % (n - 1) : 0); }

__device__ __forceinline__ float log_sigmoid_f(float x) { return x >= 0.f ? -log1pf(expf(-x)) : x - log1pf(expf(x)); }

// parameter block of one trajectory: W1 [H][N] | b1 [H] | W2 [N][H] | b2 [N]
struct ArView {
    float *W1, *b1, *W2, *b2;
};
__device__ __forceinline__ ArView ar_view(float *base, int n, int h) {
    return ArView{base, base + (size_t)h * n, base + (size_t)h * n + h, base + (size_t)h * n + h + (size_t)n * h};
}
__host__ __device__ inline size_t ar_params(int n, int h) { return (size_t)2 * n * h + n + h; }

// refresh the BF16 inference copies of trajectory t: W1T [N][H] (W1 transposed), W2 [N][H]
// (row i = the weights of output i) and W2T [H][N]; element (k, j) of W1 is W1T[j H + k]
__device__ __forceinline__ void ar_copy_one(const Dev &a, int t, size_t e) {
    const int n = a.n, h = a.ah;
    ArView p = ar_view(a.arP + (size_t)t * a.arnp, n, h);
    if (e < (size_t)h * n) {
        const int k = (int)(e / n), j = (int)(e % n);
        const size_t base = (size_t)t * h * n;
        a.arW1Tb[base + (size_t)j * h + k] = f2bf(p.W1[e]);
        a.arW2b[base + (size_t)j * h + k] = f2bf(p.W2[(size_t)j * h + k]);
        a.arW2Tb[base + (size_t)k * n + j] = f2bf(p.W2[(size_t)j * h + k]);
    }
}

// Weights an independent proposal reads, in the [site][hidden unit] layout (consecutive lanes
// read consecutive hidden units): from LDS when they fit there, else from global memory.
constexpr int AR_LDS_W = 8192;    // H N entries per matrix staged in LDS (H <= 128 at N = 64)
struct ArNet {
    const uint16_t *W1T, *W2;      // element (k, i) at [i H + k]
    const float *b1, *b2;
};
// Stage trajectory t's draw weights into LDS (whole workgroup; a barrier must follow).
__device__ __forceinline__ ArNet ar_net(const Dev &a, int t, uint16_t *sW1T, uint16_t *sW2, float *sb1, float *sb2) {
    const int n = a.n, h = a.ah;
    const size_t base = (size_t)t * h * n;
    const float *b1 = a.arP + (size_t)t * a.arnp + (size_t)h * n;
    const float *b2 = b1 + h + (size_t)n * h;
    for (int i = threadIdx.x; i < h; i += blockDim.x) sb1[i] = b1[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sb2[i] = b2[i];
    if (h * n <= AR_LDS_W) {
        for (int e = threadIdx.x; e < h * n; e += blockDim.x) {
            sW1T[e] = a.arW1Tb[base + e];
            sW2[e] = a.arW2b[base + e];
        }
        return ArNet{sW1T, sW2, sb1, sb2};
    }
    return ArNet{a.arW1Tb + base, a.arW2b + base, sb1, sb2};
}

// deterministic initialisation: W ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) on unmasked entries,
// biases zero, Adam moments zero (Philox stream 7: (index, 0, 0, 7<<24 | traj)).
__global__ void k_ar_init(Dev a) {
    const int t = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.n, h = a.ah;
    if (e >= a.arnp) return;
    float v = 0.f;
    if (e < (size_t)h * n) {
        const int k = (int)(e / n), j = (int)(e % n);
        uint32_t r[4];
        philox4x32_10((uint32_t)e, 0u, 0u, (7u << 24) | (uint32_t)(a.traj0 + t), a.key0, a.key1, r);
        const float u = (float)((r[0] >> 8) * (1.0 / 16777216.0)) * 2.f - 1.f;
        v = j < ar_degree(k, n) ? u / sqrtf((float)n) : 0.f;
    } else if (e >= (size_t)h * n + h && e < (size_t)2 * h * n + h) {
        const size_t o = e - (size_t)h * n - h;
        const int i = (int)(o / h), k = (int)(o % h);
        uint32_t r[4];
        philox4x32_10((uint32_t)e, 0u, 0u, (7u << 24) | (uint32_t)(a.traj0 + t), a.key0, a.key1, r);
        const float u = (float)((r[0] >> 8) * (1.0 / 16777216.0)) * 2.f - 1.f;
        v = ar_degree(k, n) <= i ? u / sqrtf((float)h) : 0.f;
    }
    a.arP[(size_t)t * a.arnp + e] = v;
    a.arM[(size_t)t * a.arnp + e] = 0.f;
    a.arV[(size_t)t * a.arnp + e] = 0.f;
}

__global__ void k_ar_copy(Dev a) {
    const int t = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (size_t)a.ah * a.n) ar_copy_one(a, t, e);
}

// Training forward/backward per sample (one wavefront per sample, lanes over hidden units and
// sites).  Writes log q, the hidden activations h, g = d(loss)/d(logits) and da = d(loss)/da.
constexpr int AR_WAVES = 4;
__global__ __launch_bounds__(64 * AR_WAVES) void k_ar_forward(Dev a, int want_grad) {
    __shared__ float hs[AR_WAVES][256];
    __shared__ float gs[AR_WAVES][64];
    const int t = blockIdx.y, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int s = blockIdx.x * AR_WAVES + w;
    const int n = a.n, h = a.ah;
    if (s >= a.ns) return;
    const ArView p = ar_view(a.arP + (size_t)t * a.arnp, n, h);
    const uint64_t mk = a.samples[(size_t)t * a.ns + s];
    float av[4];
    for (int q = 0; q < 4; ++q) {
        const int k = lane + 64 * q;
        av[q] = 0.f;
        if (k < h) {
            float x = p.b1[k];
            const int dk = ar_degree(k, n);
            for (int j = 0; j < dk; ++j) x += p.W1[(size_t)k * n + j] * (float)spin(mk, j);
            av[q] = x;
            hs[w][k] = fmaxf(x, 0.f);
        }
    }
    float lq = 0.f, gi = 0.f;
    if (lane < n) {
        float l = p.b2[lane];
        for (int k = 0; k < h; ++k)
            if (ar_degree(k, n) <= lane) l += p.W2[(size_t)lane * h + k] * hs[w][k];
        const float si = (float)spin(mk, lane);
        lq = log_sigmoid_f(si * l);
        // d(-log sigmoid(s l))/dl / B
        gi = -si * expf(log_sigmoid_f(-si * l)) / (float)a.ns;
        gs[w][lane] = gi;
    }
    lq = (float)wave_sum((double)lq);
    if (lane == 0) a.arlogq[(size_t)t * a.ns + s] = lq;
    if (!want_grad) return;
    const size_t sb = (size_t)t * a.ns + s;
    if (lane < n) a.arg[sb * n + lane] = gi;
    for (int q = 0; q < 4; ++q) {
        const int k = lane + 64 * q;
        if (k >= h) continue;
        float dh = 0.f;
        const int dk = ar_degree(k, n);
        for (int i = dk; i < n; ++i) dh += gs[w][i] * p.W2[(size_t)i * h + k];
        a.arh[sb * h + k] = hs[w][k];
        a.arda[sb * h + k] = av[q] > 0.f ? dh : 0.f;
    }
}

// Gradient reductions over the batch, as two small GEMMs per trajectory:
//   gW2[i][k] = sum_s g[s][i] h[s][k] (masked), gb2[i] = sum_s g[s][i]
//   gW1[k][j] = sum_s da[s][k] s_j     (masked), gb1[k] = sum_s da[s][k]
// Workgroup = 32 x 32 output tile, samples staged 64 at a time through LDS; a fixed order.
__global__ __launch_bounds__(256) void k_ar_grad(Dev a) {
    __shared__ float X[64][33];
    __shared__ float Y[64][33];
    const int t = blockIdx.z, which = blockIdx.y;     // 0: W2 tile (rows i, cols k); 1: W1 tile (rows k, cols j)
    const int n = a.n, h = a.ah;
    const int rows = which == 0 ? n : h, cols = which == 0 ? h : n;
    const int tiles_c = (cols + 31) / 32;
    const int r0 = (blockIdx.x / tiles_c) * 32, c0 = (blockIdx.x % tiles_c) * 32;
    if (r0 >= rows) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows of 32 columns per pass, 4 rows each
    float acc[4] = {0.f, 0.f, 0.f, 0.f}, bacc[4] = {0.f, 0.f, 0.f, 0.f};
    const size_t tb = (size_t)t * a.ns;
    for (int s0 = 0; s0 < a.ns; s0 += 64) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            const int ss = e >> 5, cc = e & 31, s = s0 + ss;
            float xv = 0.f, yv = 0.f;
            if (s < a.ns) {
                const int r = r0 + cc, c = c0 + cc;
                if (which == 0) {
                    xv = r < n ? a.arg[(tb + s) * n + r] : 0.f;
                    yv = c < h ? a.arh[(tb + s) * h + c] : 0.f;
                } else {
                    xv = r < h ? a.arda[(tb + s) * h + r] : 0.f;
                    yv = c < n ? (float)spin(a.samples[tb + s], c) : 0.f;
                }
            }
            X[ss][cc] = xv;
            Y[ss][cc] = yv;
        }
        __syncthreads();
        for (int ss = 0; ss < 64; ++ss) {
            const float y = Y[ss][tx];
            for (int u = 0; u < 4; ++u) {
                const float x = X[ss][ty * 4 + u];
                acc[u] += x * y;
                bacc[u] += x;
            }
        }
    }
    ArView gv = ar_view(a.arG + (size_t)t * a.arnp, n, h);
    for (int u = 0; u < 4; ++u) {
        const int r = r0 + ty * 4 + u, c = c0 + tx;
        if (r >= rows || c >= cols) continue;
        if (which == 0) {
            gv.W2[(size_t)r * h + c] = ar_degree(c, n) <= r ? acc[u] : 0.f;
            if (c == 0) gv.b2[r] = bacc[u];
        } else {
            gv.W1[(size_t)r * n + c] = c < ar_degree(r, n) ? acc[u] : 0.f;
            if (c == 0) gv.b1[r] = bacc[u];
        }
    }
}

// mean loss per trajectory (for monitoring) and one Adam step over every parameter
__global__ void k_ar_loss(Dev a) {
    const int t = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < a.ns; i += blockDim.x) s += a.arlogq[(size_t)t * a.ns + i];
    s = wave_sum(s);
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) a.arloss[t] = -(part[0] + part[1] + part[2] + part[3]) / (double)a.ns;
}

__global__ void k_ar_adam(Dev a, float lr, int step) {
    const int t = blockIdx.y;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.arnp) return;
    const size_t i = (size_t)t * a.arnp + e;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float g = a.arG[i];
    const float m = b1 * a.arM[i] + (1.f - b1) * g;
    const float v = b2 * a.arV[i] + (1.f - b2) * g * g;
    a.arM[i] = m;
    a.arV[i] = v;
    const float mh = m / (1.f - powf(b1, (float)step)), vh = v / (1.f - powf(b2, (float)step));
    a.arP[i] -= lr * mh / (sqrtf(vh) + eps);
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// log q(s) of the BF16 network for configuration mk (every lane returns the same value).
// hs: this wave's LDS scratch of H floats.
__device__ float ar_logq(const Dev &a, int t, uint64_t mk, int lane, float *hs) {
    const int n = a.n, h = a.ah;
    const float *b1 = a.arP + (size_t)t * a.arnp + (size_t)h * n;
    const float *b2 = b1 + h + (size_t)n * h;
    const uint16_t *W1T = a.arW1Tb + (size_t)t * h * n, *W2T = a.arW2Tb + (size_t)t * h * n;
    for (int k = lane; k < h; k += 64) {
        float x = b1[k];
        const int dk = ar_degree(k, n);
        for (int j = 0; j < dk; ++j) x += bf2f(W1T[(size_t)j * h + k]) * (float)spin(mk, j);
        hs[k] = fmaxf(x, 0.f);
    }
    float lq = 0.f;
    if (lane < n) {
        float l = b2[lane];
        for (int k = 0; k < h; ++k)
            if (ar_degree(k, n) <= lane) l += bf2f(W2T[(size_t)k * n + lane]) * hs[k];
        lq = log_sigmoid_f((float)spin(mk, lane) * l);
    }
    return wave_sum_f(lq);
}

// One independent proposal s' ~ q drawn autoregressively with the BF16 network (every lane
// returns the same s', log q(s') and accept uniform).  Philox stream 6, counter
// (17 idx + block, ctr1, step, 6 << 24 | traj): blocks 0..15 give one 24-bit site uniform per
// site (word lane & 3 of block lane >> 2), block 16 gives the 53-bit accept uniform.
__device__ uint64_t ar_draw(const Dev &a, const ArNet &net, int t, uint32_t ctr1, int step, uint32_t idx, int lane,
                            float &lqn, double &uacc) {
    const int n = a.n, h = a.ah;
    uint32_t rr[4] = {0u, 0u, 0u, 0u};
    if (lane < 17)
        philox4x32_10(idx * 17u + (uint32_t)lane, ctr1, (uint32_t)step, (6u << 24) | (uint32_t)(a.traj0 + t), a.key0,
                      a.key1, rr);
    uint32_t word = 0u;
    for (int q4 = 0; q4 < 4; ++q4) {
        const uint32_t v = (uint32_t)__shfl((int)rr[q4], lane >> 2, 64);
        if ((lane & 3) == q4) word = v;
    }
    const float usite = ((float)(word >> 8) + 0.5f) * (1.0f / 16777216.0f);
    uacc = u53((uint32_t)__builtin_amdgcn_readlane((int)rr[0], 16), (uint32_t)__builtin_amdgcn_readlane((int)rr[1], 16));
    const float *b2 = net.b2;
    const uint16_t *W1T = net.W1T, *W2 = net.W2;
    float ak[4];
    for (int q = 0; q < 4; ++q) ak[q] = (lane + 64 * q < h) ? net.b1[lane + 64 * q] : 0.f;
    uint64_t mnew = 0ull;
    float lq = 0.f;
    for (int ii = 0; ii < n; ++ii) {
        float part = 0.f;
        for (int q = 0; q < 4; ++q) {
            const int k = lane + 64 * q;
            if (k < h && ar_degree(k, n) <= ii) part += bf2f(W2[(size_t)ii * h + k]) * fmaxf(ak[q], 0.f);
        }
        const float l = b2[ii] + wave_sum_f(part);
        const float pu = 1.f / (1.f + expf(-l));
        const float ui = __shfl(usite, ii, 64);
        const bool up = ui < pu;
        const float sv = up ? 1.f : -1.f;
        lq += log_sigmoid_f(sv * l);
        if (up) mnew |= (1ull << ii);
        for (int q = 0; q < 4; ++q) {
            const int k = lane + 64 * q;
            if (k < h && ar_degree(k, n) > ii) ak[q] += bf2f(W1T[(size_t)ii * h + k]) * sv;
        }
    }
    lqn = lq;
    return mnew;
}

}  // namespace tvmc
