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

// float -> bfloat16, round to nearest even (the hardware conversion, v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
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

// refresh the BF16 inference copies of trajectory t: W1T [N][H] (W1 transposed) and W2T [H][N]
// (W2 transposed); element (k, j) of W1 is W1T[j H + k], element (i, k) of W2 is W2T[k N + i]
__device__ __forceinline__ void ar_copy_one(const Dev &a, int t, size_t e) {
    const int n = a.n, h = a.ah;
    ArView p = ar_view(a.arP + (size_t)t * a.arnp, n, h);
    if (e < (size_t)h * n) {
        const int k = (int)(e / n), j = (int)(e % n);
        const size_t base = (size_t)t * h * n;
        // masked entries are written as exact zeros: the sampler's walk relies on them
        const int dk = ar_degree(k, n);
        a.arW1Tb[base + (size_t)j * h + k] = j < dk ? f2bf(p.W1[e]) : (uint16_t)0;
        a.arW2Tb[base + (size_t)k * n + j] = dk <= j ? f2bf(p.W2[(size_t)j * h + k]) : (uint16_t)0;
    }
}

// BF16 weights the sampler reads, staged in LDS per workgroup (all its chains belong to one
// trajectory): W1T (element (k, j) of W1 at [j H + k]: consecutive lanes read consecutive
// hidden units) and W2T (element (i, k) of W2 at [k N + i]: consecutive lanes read
// consecutive outputs).  H N <= AR_LDS_W is checked at initialisation.
constexpr int AR_LDS_W = 8192;    // H N entries per matrix (H <= 128 at N = 64)
struct ArNet {
    const uint16_t *W1T, *W2T;
    const float *b1, *b2;
};
// Stage trajectory t's weights into LDS (whole workgroup; a barrier must follow).
__device__ __forceinline__ ArNet ar_net(const Dev &a, int t, uint16_t *sW1T, uint16_t *sW2T, float *sb1, float *sb2) {
    const int n = a.n, h = a.ah;
    const size_t base = (size_t)t * h * n;
    const float *b1 = a.arP + (size_t)t * a.arnp + (size_t)h * n;
    const float *b2 = b1 + h + (size_t)n * h;
    for (int i = threadIdx.x; i < h; i += blockDim.x) sb1[i] = b1[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sb2[i] = b2[i];
    for (int e = threadIdx.x; e < h * n; e += blockDim.x) {
        sW1T[e] = a.arW1Tb[base + e];
        sW2T[e] = a.arW2Tb[base + e];
    }
    return ArNet{sW1T, sW2T, sb1, sb2};
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

// Training forward/backward per sample (a wavefront takes AR_SB samples at a time, lanes over
// hidden units and sites).  Writes log q, the hidden activations h, g = d(loss)/d(logits) and da = d(loss)/da.
// A workgroup takes AR_SAMPLES samples of one trajectory and first stages that trajectory's
// FP32 weights in LDS with the masks applied (masked entries exactly zero, so the loops run
// over all inputs without degree tests): W1 as [k][j] with rows padded to N + 1 and W2 as
// [i][k] with rows padded to H + 1, which keeps every loop below on distinct banks.
constexpr int AR_WAVES = 8;
constexpr int AR_SAMPLES = 128;
constexpr int AR_SB = 4;          // samples per wavefront pass: each weight read serves four
__global__ __launch_bounds__(64 * AR_WAVES) void k_ar_forward(Dev a, int want_grad) {
    __shared__ float sW1[AR_LDS_W + 256];     // [k][j], row stride N + 1
    __shared__ float sW2[AR_LDS_W + 64];      // [i][k], row stride H + 1
    __shared__ float sb1[256], sb2[64];
    __shared__ float hs[AR_WAVES][AR_SB][256];
    __shared__ float gs[AR_WAVES][AR_SB][64];
    const int t = blockIdx.y, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, h = a.ah, s1 = n + 1, s2 = h + 1;
    const ArView p = ar_view(a.arP + (size_t)t * a.arnp, n, h);
    for (int e = threadIdx.x; e < h * n; e += blockDim.x) {
        const int k = e / n, j = e % n;
        sW1[k * s1 + j] = j < ar_degree(k, n) ? p.W1[e] : 0.f;
    }
    for (int e = threadIdx.x; e < n * h; e += blockDim.x) {
        const int i = e / h, k = e % h;
        sW2[i * s2 + k] = ar_degree(k, n) <= i ? p.W2[e] : 0.f;
    }
    for (int k = threadIdx.x; k < h; k += blockDim.x) sb1[k] = p.b1[k];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sb2[i] = p.b2[i];
    __syncthreads();
    const int s_end = min(a.ns, (int)(blockIdx.x + 1) * AR_SAMPLES);
    for (int s0 = blockIdx.x * AR_SAMPLES + w * AR_SB; s0 < s_end; s0 += AR_WAVES * AR_SB) {
        uint64_t mk[AR_SB];
        for (int b = 0; b < AR_SB; ++b) mk[b] = s0 + b < s_end ? a.samples[(size_t)t * a.ns + s0 + b] : 0ull;
        // per sample, the same multiply-adds in the same order as one sample at a time
        float av[4][AR_SB];
        for (int q = 0; q < 4; ++q) {
            const int k = lane + 64 * q;
            for (int b = 0; b < AR_SB; ++b) av[q][b] = 0.f;
            if (k < h) {
                float x[AR_SB];
                for (int b = 0; b < AR_SB; ++b) x[b] = sb1[k];
                for (int j = 0; j < n; ++j) {
                    const float wv = sW1[k * s1 + j];
                    for (int b = 0; b < AR_SB; ++b) x[b] += wv * (float)spin(mk[b], j);
                }
                for (int b = 0; b < AR_SB; ++b) {
                    av[q][b] = x[b];
                    hs[w][b][k] = fmaxf(x[b], 0.f);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        float lq[AR_SB], gi[AR_SB];
        for (int b = 0; b < AR_SB; ++b) lq[b] = gi[b] = 0.f;
        if (lane < n) {
            float l[AR_SB];
            for (int b = 0; b < AR_SB; ++b) l[b] = sb2[lane];
            for (int k = 0; k < h; ++k) {
                const float wv = sW2[lane * s2 + k];
                for (int b = 0; b < AR_SB; ++b) l[b] += wv * hs[w][b][k];
            }
            for (int b = 0; b < AR_SB; ++b) {
                const float si = (float)spin(mk[b], lane);
                lq[b] = log_sigmoid_f(si * l[b]);
                // d(-log sigmoid(s l))/dl / B
                gi[b] = -si * expf(log_sigmoid_f(-si * l[b])) / (float)a.ns;
                gs[w][b][lane] = gi[b];
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int b = 0; b < AR_SB; ++b) {
            const float lqs = (float)wave_sum((double)lq[b]);
            if (lane == 0 && s0 + b < s_end) a.arlogq[(size_t)t * a.ns + s0 + b] = lqs;
        }
        if (want_grad) {
            for (int b = 0; b < AR_SB; ++b)
                if (lane < n && s0 + b < s_end) a.arg[((size_t)t * a.ns + s0 + b) * n + lane] = gi[b];
            for (int q = 0; q < 4; ++q) {
                const int k = lane + 64 * q;
                if (k >= h) continue;
                float dh[AR_SB];
                for (int b = 0; b < AR_SB; ++b) dh[b] = 0.f;
                for (int i = 0; i < n; ++i) {
                    const float wv = sW2[i * s2 + k];
                    for (int b = 0; b < AR_SB; ++b) dh[b] += gs[w][b][i] * wv;
                }
                for (int b = 0; b < AR_SB; ++b) {
                    if (s0 + b >= s_end) continue;
                    const size_t sb = (size_t)t * a.ns + s0 + b;
                    a.arh[sb * h + k] = hs[w][b][k];
                    a.arda[sb * h + k] = av[q][b] > 0.f ? dh[b] : 0.f;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
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

// The autoregressive walk over sites 0..N-1 that draws s' ~ q together with log q(s')
// (ar_logq evaluates log q of a given configuration with the same operations in the same
// order).  Lane k (and k + 64, ...) holds the pre-activation a_k of hidden unit k; lane i holds the logit l_i of site i.  Hidden unit k has inputs j <
// d(k) and outputs i >= d(k), so it is complete once site d(k) - 1 is known: at site ii the
// units of degree ii (k = ii - 1 + c (N - 1)) add W2[i][k] relu(a_k) to the logits (the
// masked weights W2[i][k], i < d(k), are exactly zero), site ii is decided from l_ii, and
// every unit adds W1[k][ii] s_ii (zero for the units with d(k) <= ii).  No cross-lane
// reductions: only scalar reads of one lane.  draw: s_ii = +1 iff logit(u_ii) < l_ii, i.e.
// u_ii < sigmoid(l_ii), with u_ii the site uniform of lane ii; otherwise s_ii is read from mk.
// Inlined into the samplers, so the weight reads compile to LDS instructions.  Returns the
// configuration and log q of it (all lanes).
// value of lane l (uniform l): a scalar read instead of a cross-lane permute
__device__ __forceinline__ float readlane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

struct ArWalk {
    uint64_t cfg;
    float lq;
};
__device__ __forceinline__ ArWalk ar_walk(int n, int h, const uint16_t *W1T, const uint16_t *W2T, const float *b1,
                                          const float *b2, uint64_t mk, float usite, int lane, int draw) {
    const int nm1 = n > 1 ? n - 1 : 1, nq = (h + 63) >> 6;
    float ak[4];
    for (int q = 0; q < 4; ++q) ak[q] = (lane + 64 * q < h) ? b1[lane + 64 * q] : 0.f;
    const int li = lane < n ? lane : n - 1;          // W2T column this lane reads
    float logit = lane < n ? b2[lane] : 0.f;
    // logit of the site uniform, so that a site is decided without a transcendental
    const float ulog = draw ? logf(usite) - log1pf(-usite) : 0.f;
    float arg = 0.f;                                 // lane i: s_i l_i
    uint64_t out = 0ull;
    for (int ii = 0; ii < n; ++ii) {
        if (ii >= 1)
            for (int k = ii - 1; k < h; k += nm1) {
                const int q = k >> 6;
                const float av = q == 0 ? ak[0] : q == 1 ? ak[1] : q == 2 ? ak[2] : ak[3];
                const float hk = fmaxf(readlane_f(av, k & 63), 0.f);
                logit += bf2f(W2T[(size_t)k * n + li]) * hk;
            }
        const float l = readlane_f(logit, ii);
        const bool up = draw ? (readlane_f(ulog, ii) < l) : (bool)((mk >> ii) & 1ull);
        const float sv = up ? 1.f : -1.f;
        arg = lane == ii ? sv * l : arg;
        if (up) out |= (1ull << ii);
        for (int q = 0; q < nq; ++q) {
            const int k = lane + 64 * q;
            ak[q] += (k < h ? bf2f(W1T[(size_t)ii * h + k]) : 0.f) * sv;
        }
    }
    const float mylq = lane < n ? log_sigmoid_f(arg) : 0.f;
    return ArWalk{out, wave_sum_f(mylq)};
}

// log q(s) of the BF16 network for a given configuration mk (every lane returns the same
// value).  Nothing is decided on the way, so the pre-activations are formed first and the
// logits afterwards, but with the walk's operations in the walk's order: each a_k adds the
// input rows site by site, and each logit adds the hidden units in the order the walk
// completes them (site ii = 1 .. N-1, units ii - 1 + c (N - 1)).  Units the walk adds after it
// has read a logit, and rows it adds after a unit's last input, carry masked weights that are
// exactly zero, so the result is the walk's log q bit for bit.
__device__ __forceinline__ float ar_logq(const Dev &a, const ArNet &net, uint64_t mk, int lane) {
    const int n = a.n, h = a.ah, nm1 = n > 1 ? n - 1 : 1, nq = (h + 63) >> 6;
    float ak[4];
    for (int q = 0; q < 4; ++q) ak[q] = (lane + 64 * q < h) ? net.b1[lane + 64 * q] : 0.f;
    for (int ii = 0; ii < n; ++ii) {
        const float sv = ((mk >> ii) & 1ull) ? 1.f : -1.f;
        for (int q = 0; q < nq; ++q) {
            const int k = lane + 64 * q;
            ak[q] += (k < h ? bf2f(net.W1T[(size_t)ii * h + k]) : 0.f) * sv;
        }
    }
    const int li = lane < n ? lane : n - 1;
    float logit = lane < n ? net.b2[lane] : 0.f;
    for (int ii = 1; ii < n; ++ii)
        for (int k = ii - 1; k < h; k += nm1) {
            const int q = k >> 6;
            const float av = q == 0 ? ak[0] : q == 1 ? ak[1] : q == 2 ? ak[2] : ak[3];
            const float hk = fmaxf(readlane_f(av, k & 63), 0.f);
            logit += bf2f(net.W2T[(size_t)k * n + li]) * hk;
        }
    const float sv = ((mk >> li) & 1ull) ? 1.f : -1.f;
    const float mylq = lane < n ? log_sigmoid_f(sv * logit) : 0.f;
    return wave_sum_f(mylq);
}

// log q of trajectory t's last samples under the sampler's BF16 network (ar_logq, one
// wavefront per sample), the value the sampler's acceptance test uses, for checking it
// against a float64 evaluation of the same rounded weights.
__global__ __launch_bounds__(256) void k_ar_logq_bf16(Dev a, int t) {
    __shared__ uint16_t sW1T[AR_LDS_W], sW2T[AR_LDS_W];
    __shared__ float sb1[256], sb2[64];
    const ArNet net = ar_net(a, t, sW1T, sW2T, sb1, sb2);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s = blockIdx.x * 4 + w; s < a.ns; s += gridDim.x * 4) {
        const float lq = ar_logq(a, net, a.samples[(size_t)t * a.ns + s], lane);
        if (lane == 0) a.arlogqb[(size_t)t * a.ns + s] = lq;
    }
}

// One independent proposal s' ~ q drawn autoregressively with the BF16 network (every lane
// returns the same s', log q(s') and accept uniform).  Philox stream 6, counter
// (17 idx + block, ctr1, step, 6 << 24 | traj): blocks 0..15 give one 24-bit site uniform per
// site (word lane & 3 of block lane >> 2), block 16 gives the 53-bit accept uniform.
__device__ uint64_t ar_draw(const Dev &a, const ArNet &net, int t, uint32_t ctr1, int step, uint32_t idx, int lane,
                            float &lqn, double &uacc) {
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
    const ArWalk r = ar_walk(a.n, a.ah, net.W1T, net.W2T, net.b1, net.b2, 0ull, usite, lane, 1);
    lqn = r.lq;
    return r.cfg;
}

}  // namespace tvmc
