// mlp.hip -- learned |a| seed for the relative opening criterion.
//
// The paper seeds the relative criterion (eq. eqnrelcriterion) for the very
// first force with a geometric walk (footnote to that equation).  This module
// replaces that pre-walk by a small network that predicts log10 |a| of each
// particle from cheap tree features: an 8 -> 64 -> 64 -> 1 perceptron with
// SiLU activations, BF16 weights and FP32 arithmetic.  Parameter layout (4801
// values): W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3.
//
// Kernels: per-particle features from the particle's leaf, forward pass,
// loss gradient (per-particle backpropagation, block-level reduction of the
// weight gradients through LDS, one atomic per weight per block) and an Adam
// step that keeps FP32 master weights and writes the BF16 copy.
#include "g4_device.h"
#include "g4_internal.h"

#define MLP_NP 4801
#define OFF_B1 512
#define OFF_W2 576
#define OFF_B2 4672
#define OFF_W3 4736
#define OFF_B3 4800

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// ------------------------------------------------------------------ features
// Cheap per-particle features from the particle's leaf L, its parent P and
// grandparent (no tree walk):
//   f0 log10 M_L, f1 log10 l_L, f2 level of L,
//   f3 log10(|x - s_L| / l_L + 1e-3), f4 log10(|x - s_P| / l_P + 1e-3),
//   f5 log10 M_P, f6 log10 M_grandparent,
//   f7 log10 |a_near|: the pair force of the other particles of L plus the
//      monopole forces of the siblings of L and of P (same softened kernel as
//      the walk), about 20 interactions per particle.
// A missing ancestor is replaced by the node itself.  Optionally
// standardised: (f - norm[k]) * norm[8 + k].
// One wavefront per leaf.  Lane = (particle a of the leaf, slot k): the
// near-field sum of particle a is split over S = 64 / (particles in the chunk)
// slots, each taking every S-th source, and the partial sums are added in LDS;
// lanes with k = 0 then form and write the particle's eight features.
template <int KER>
__global__ __launch_bounds__(256) void k_mlp_features(const DevCounters *__restrict__ C, const WNode *__restrict__ wn,
                                                      const double *__restrict__ mom,
                                                      const uint32_t *__restrict__ parent,
                                                      const uint4 *__restrict__ parts, const uint32_t *__restrict__ perm,
                                                      double boxd, double unit_d, float asplit, float h2,
                                                      float hinv, const float *__restrict__ norm,
                                                      float *__restrict__ feat)
{
    __shared__ float part[4][64][3];
    const uint32_t nn = C->node_count;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const float unit = (float)unit_d;
    for (uint32_t q = blockIdx.x * 4 + wv; q < nn; q += gridDim.x * 4) {
        const WNode w = wn[q];
        if (!(w.meta & WN_LEAF)) continue;
        const uint32_t p = parent[q];
        const uint32_t gp = p != 0xffffffffu ? parent[p] : 0xffffffffu;
        // monopoles of the siblings of the leaf (slots 0-7) and of its parent (slots 8-15), one per lane
        uint32_t sx = 0, sy = 0, sz = 0;
        float sm = 0.f;
        if (lane < 16) {
            const uint32_t self = lane < 8 ? q : p, up = lane < 8 ? p : gp;
            if (self != 0xffffffffu && up != 0xffffffffu) {
                const uint32_t nc = wn[up].num, c = wn[up].next + (lane & 7);
                if ((uint32_t)(lane & 7) < nc && c != self) {
                    const WNode wc = wn[c];
                    sx = wc.cx;
                    sy = wc.cy;
                    sz = wc.cz;
                    sm = wc.mass;
                }
            }
        }
        for (uint32_t c0 = 0; c0 < w.num; c0 += 64) {
            const uint32_t nc = min(w.num - c0, 64u);
            const uint32_t S = 64u / nc;
            const uint32_t a = (uint32_t)lane % nc, k = (uint32_t)lane / nc;
            const bool act = k < S;
            const uint32_t j = w.next + c0 + a;
            const uint4 pj = parts[j];
            float ax = 0.f, ay = 0.f, az = 0.f, K, W;
            for (uint32_t s = (act ? k : w.num); s < w.num; s += S) {
                const uint4 pk = parts[w.next + s];
                const float dx = (float)(int32_t)(pk.x - pj.x) * unit, dy = (float)(int32_t)(pk.y - pj.y) * unit,
                            dz = (float)(int32_t)(pk.z - pj.z) * unit;
                pair_kernel<KER, false>(dx * dx + dy * dy + dz * dz, asplit, h2, hinv, K, W);
                const float mk = w.next + s != j ? __uint_as_float(pk.w) * K : 0.f;
                ax += mk * dx;
                ay += mk * dy;
                az += mk * dz;
            }
            for (uint32_t e = 0; e < 16; e += S) {
                // sibling slot e + k, fetched from its lane
                const int from = (int)min(e + k, 15u);
                const uint32_t kx = (uint32_t)__shfl((int)sx, from), ky = (uint32_t)__shfl((int)sy, from),
                               kz = (uint32_t)__shfl((int)sz, from);
                const float km = __uint_as_float((uint32_t)__shfl((int)__float_as_uint(sm), from));
                if (act && e + k < 16 && km != 0.f) {
                    const float dx = (float)(int32_t)(kx - pj.x) * unit, dy = (float)(int32_t)(ky - pj.y) * unit,
                                dz = (float)(int32_t)(kz - pj.z) * unit;
                    pair_kernel<KER, false>(dx * dx + dy * dy + dz * dz, asplit, h2, hinv, K, W);
                    const float mk = km * K;
                    ax += mk * dx;
                    ay += mk * dy;
                    az += mk * dz;
                }
            }
            part[wv][lane][0] = ax;
            part[wv][lane][1] = ay;
            part[wv][lane][2] = az;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if ((uint32_t)lane < nc) {
                // slot sums in slot order: leaf particles first, then siblings, as one sequence per slot
                float tx = 0.f, ty = 0.f, tz = 0.f;
                for (uint32_t kk = 0; kk < S; kk++) {
                    tx += part[wv][kk * nc + a][0];
                    ty += part[wv][kk * nc + a][1];
                    tz += part[wv][kk * nc + a][2];
                }
                const int level = (int)(w.meta & 0xffu);
                const uint32_t pp = p != 0xffffffffu ? p : q;
                const WNode wp = wn[pp];
                const double *dl = mom + (size_t)q * MOM_STRIDE + 1, *dp = mom + (size_t)pp * MOM_STRIDE + 1;
                const double il = 1.0 / ldexp(boxd, -level), ilp = 1.0 / ldexp(boxd, -(int)(wp.meta & 0xffu));
                float f[8];
                f[0] = log10f((float)mom[(size_t)q * MOM_STRIDE]);
                f[1] = log10f((float)ldexp(boxd, -level));
                f[2] = (float)level;
                // offsets from the centres of mass in FP64 (they may nearly cancel), logarithms in FP32
                double a0 = (double)(int32_t)(pj.x - w.gx) * unit_d - dl[0],
                       a1 = (double)(int32_t)(pj.y - w.gy) * unit_d - dl[1],
                       a2 = (double)(int32_t)(pj.z - w.gz) * unit_d - dl[2];
                f[3] = log10f((float)(sqrt(a0 * a0 + a1 * a1 + a2 * a2) * il + 1e-3));
                a0 = (double)(int32_t)(pj.x - wp.gx) * unit_d - dp[0];
                a1 = (double)(int32_t)(pj.y - wp.gy) * unit_d - dp[1];
                a2 = (double)(int32_t)(pj.z - wp.gz) * unit_d - dp[2];
                f[4] = log10f((float)(sqrt(a0 * a0 + a1 * a1 + a2 * a2) * ilp + 1e-3));
                const float Mp = (float)mom[(size_t)pp * MOM_STRIDE];
                f[5] = log10f(Mp);
                f[6] = gp != 0xffffffffu ? log10f((float)mom[(size_t)gp * MOM_STRIDE]) : log10f(Mp);
                f[7] = log10f(fmaxf(sqrtf(tx * tx + ty * ty + tz * tz), 1e-30f));
                float *o = feat + (size_t)perm[j] * 8;
                for (int kk = 0; kk < 8; kk++) o[kk] = norm ? (f[kk] - norm[kk]) * norm[8 + kk] : f[kk];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

int g4_launch_mlp_features(g4_ctx *ctx, const g4_tree *t, const g4_walk_params *wp, const float *norm, float *feat)
{
    int blocks = (int)((t->cap + 3) / 4);
    if (blocks > 4096) blocks = 4096;
    const double h = 2.8 * wp->eps0;
    const float asplit = wp->kernel == 1 ? (float)(0.5 / wp->r_s) : 0.f;
    const float h2 = (float)(h * h), hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    if (wp->kernel == 1)
        k_mlp_features<1><<<blocks, 256, 0, ctx->stream>>>(t->ctr, t->wn, t->mom, t->parent, t->parts, t->perm1,
                                                           t->tp.box, t->unit, asplit, h2, hinv, norm, feat);
    else
        k_mlp_features<0><<<blocks, 256, 0, ctx->stream>>>(t->ctr, t->wn, t->mom, t->parent, t->parts, t->perm1,
                                                           t->tp.box, t->unit, asplit, h2, hinv, norm, feat);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ forward
// One thread per particle; weights converted to FP32 once per block into LDS
// and read at wave-uniform addresses (broadcast).  mode 0 writes y = log10|a|,
// mode 1 writes 10^(y + shift).
__global__ __launch_bounds__(256, 2) void k_mlp_forward(const uint16_t *__restrict__ w, const float *__restrict__ feat,
                                                     int64_t n, float *__restrict__ out, float shift, int mode)
{
    __shared__ float W[MLP_NP + 3];
    for (int k = threadIdx.x; k < MLP_NP; k += blockDim.x) W[k] = bf16_to_f32(w[k]);
    __syncthreads();
    // one particle per thread: no particle loop, so the weight reads from LDS
    // are not hoisted into registers across particles
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) {
        const float4 xa = reinterpret_cast<const float4 *>(feat)[2 * p];
        const float4 xb = reinterpret_cast<const float4 *>(feat)[2 * p + 1];
        const float x[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        float h1[64];
#pragma unroll
        for (int o = 0; o < 64; o++) {
            float z = W[OFF_B1 + o];
#pragma unroll
            for (int i = 0; i < 8; i++) z = fmaf(W[o * 8 + i], x[i], z);
            h1[o] = z * sigm(z);
        }
        float y = W[OFF_B3];
#pragma unroll 1
        for (int o = 0; o < 64; o += 4) {
            // four independent dot products per pass for instruction-level parallelism
            float z0 = W[OFF_B2 + o], z1 = W[OFF_B2 + o + 1], z2 = W[OFF_B2 + o + 2], z3 = W[OFF_B2 + o + 3];
            const float *r = W + OFF_W2 + o * 64;
#pragma unroll
            for (int i = 0; i < 64; i++) {
                z0 = fmaf(r[i], h1[i], z0);
                z1 = fmaf(r[64 + i], h1[i], z1);
                z2 = fmaf(r[128 + i], h1[i], z2);
                z3 = fmaf(r[192 + i], h1[i], z3);
            }
            y = fmaf(W[OFF_W3 + o], z0 * sigm(z0), y);
            y = fmaf(W[OFF_W3 + o + 1], z1 * sigm(z1), y);
            y = fmaf(W[OFF_W3 + o + 2], z2 * sigm(z2), y);
            y = fmaf(W[OFF_W3 + o + 3], z3 * sigm(z3), y);
        }
        out[p] = mode ? exp10f(y + shift) : y;
    }
}

int g4_launch_mlp_forward(g4_ctx *ctx, const uint16_t *w, const float *feat, int64_t n, float *out, float shift,
                          int mode)
{
    const int64_t blocks = (n + 255) / 256;
    if (n > 0) k_mlp_forward<<<(unsigned)blocks, 256, 0, ctx->stream>>>(w, feat, n, out, shift, mode);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ gradient
// Loss L = (1/n) sum (y - t)^2 (or the pinball loss for a quantile target).
// Each block takes TB particles,
// backpropagates each in its own thread, stores the per-particle layer
// inputs and output gradients in LDS, then forms the weight-gradient sums
// over its particles (outer products) and adds them to grad with atomics.
#define TB 128

__global__ __launch_bounds__(TB) void k_mlp_grad(const uint16_t *__restrict__ w, const float *__restrict__ feat,
                                                 const float *__restrict__ target, int64_t n, float inv_n, float tau,
                                                 float *__restrict__ grad, float *__restrict__ loss)
{
    __shared__ float W[MLP_NP + 3];
    __shared__ float sH1[TB][65];   // h1 per particle
    __shared__ float sD2[TB][65];   // dL/dz2
    __shared__ float sD1[TB][65];   // first dy*h2, then dL/dz1
    __shared__ float sX[TB][9];
    __shared__ float sDy[TB];
    const int t = threadIdx.x;
    for (int k = t; k < MLP_NP; k += TB) W[k] = bf16_to_f32(w[k]);
    __syncthreads();
    const int64_t p = blockIdx.x * (int64_t)TB + t;
    const bool valid = p < n;
    float x[8];
    for (int i = 0; i < 8; i++) x[i] = valid ? feat[p * 8 + i] : 0.f;
    // forward; h1 stays in registers for layer 2, z2 is parked in sD2
    float h1[64];
#pragma unroll
    for (int o = 0; o < 64; o++) {
        float z = W[OFF_B1 + o];
#pragma unroll
        for (int i = 0; i < 8; i++) z = fmaf(W[o * 8 + i], x[i], z);
        h1[o] = z * sigm(z);
        sH1[t][o] = h1[o];
    }
    float y = W[OFF_B3];
#pragma unroll 1
    for (int o = 0; o < 64; o++) {
        float z = W[OFF_B2 + o];
#pragma unroll
        for (int i = 0; i < 64; i++) z = fmaf(W[OFF_W2 + o * 64 + i], h1[i], z);
        sD2[t][o] = z;
        y = fmaf(W[OFF_W3 + o], z * sigm(z), y);
    }
    // tau <= 0: mean squared error; 0 < tau < 1: pinball (quantile) loss
    // rho(u) = u (tau - [u < 0]) of u = target - y, whose minimiser is the
    // tau-quantile of the target given the features
    const float e = valid ? y - target[p] : 0.f;
    const float dy = tau > 0.f ? (e > 0.f ? (1.f - tau) : -tau) * inv_n * (valid ? 1.f : 0.f) : 2.f * e * inv_n;
    const float lterm = tau > 0.f ? (e > 0.f ? (1.f - tau) * e : -tau * e) : e * e;
    sDy[t] = dy;
    for (int i = 0; i < 8; i++) sX[t][i] = x[i];
    // backward through layer 2: dL/dz2 and dL/dh1
    float dh1[64];
#pragma unroll
    for (int i = 0; i < 64; i++) dh1[i] = 0.f;
#pragma unroll 1
    for (int o = 0; o < 64; o++) {
        const float z2 = sD2[t][o];
        const float s = sigm(z2);
        sD1[t][o] = dy * z2 * s;                                   // dy * h2 (for dL/dw3)
        const float d2 = dy * W[OFF_W3 + o] * s * (1.f + z2 * (1.f - s));  // SiLU' = s (1 + z (1 - s))
        sD2[t][o] = d2;
#pragma unroll
        for (int i = 0; i < 64; i++) dh1[i] = fmaf(W[OFF_W2 + o * 64 + i], d2, dh1[i]);
    }
    // loss: block sum of e^2 / n
    float e2 = lterm * inv_n;
    for (int off = 32; off > 0; off >>= 1) e2 += __shfl_xor(e2, off);
    if ((t & 63) == 0) atomicAdd(loss, e2);
    __syncthreads();
    // dL/dw3 and dL/db3 from the dy*h2 table
    if (t < 64) {
        float s = 0.f;
        for (int q = 0; q < TB; q++) s += sD1[q][t];
        atomicAdd(&grad[OFF_W3 + t], s);
    }
    if (t == 64) {
        float s = 0.f;
        for (int q = 0; q < TB; q++) s += sDy[q];
        atomicAdd(&grad[OFF_B3], s);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 64; i++) {
        float z1 = W[OFF_B1 + i];  // recompute the layer-1 pre-activation
#pragma unroll
        for (int k = 0; k < 8; k++) z1 = fmaf(W[i * 8 + k], x[k], z1);
        const float s = sigm(z1);
        sD1[t][i] = dh1[i] * s * (1.f + z1 * (1.f - s));
    }
    __syncthreads();
    // dL/dW2[o][i] = sum_q dz2[q][o] h1[q][i]; 4096 entries, 32 per thread
    for (int k = 0; k < 4096 / TB; k++) {
        const int e_ = t + TB * k, o = e_ >> 6, i = e_ & 63;
        float s = 0.f;
        for (int q = 0; q < TB; q++) s = fmaf(sD2[q][o], sH1[q][i], s);
        atomicAdd(&grad[OFF_W2 + e_], s);
    }
    // dL/dW1[o][i] = sum_q dz1[q][o] x[q][i]; 512 entries, 4 per thread
    for (int k = 0; k < 512 / TB; k++) {
        const int e_ = t + TB * k, o = e_ >> 3, i = e_ & 7;
        float s = 0.f;
        for (int q = 0; q < TB; q++) s = fmaf(sD1[q][o], sX[q][i], s);
        atomicAdd(&grad[e_], s);
    }
    if (t < 64) {
        float s1 = 0.f, s2 = 0.f;
        for (int q = 0; q < TB; q++) {
            s1 += sD1[q][t];
            s2 += sD2[q][t];
        }
        atomicAdd(&grad[OFF_B1 + t], s1);
        atomicAdd(&grad[OFF_B2 + t], s2);
    }
}

int g4_launch_mlp_grad(g4_ctx *ctx, const uint16_t *w, const float *feat, const float *target, int64_t n, float tau,
                       float *grad, float *loss)
{
    G4_HIP(ctx, hipMemsetAsync(grad, 0, MLP_NP * sizeof(float), ctx->stream));
    G4_HIP(ctx, hipMemsetAsync(loss, 0, sizeof(float), ctx->stream));
    if (n > 0)
        k_mlp_grad<<<(unsigned)((n + TB - 1) / TB), TB, 0, ctx->stream>>>(w, feat, target, n, 1.0f / (float)n, tau,
                                                                        grad, loss);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ Adam
// Kingma & Ba (2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps); the BF16 copy is the
// round-to-nearest-even of the FP32 master weight.
__global__ void k_mlp_adam(uint16_t *__restrict__ w, float *__restrict__ master, float *__restrict__ m,
                           float *__restrict__ v, const float *__restrict__ grad, float lr, float b1, float b2,
                           float eps, float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_NP) return;
    const float g = grad[k];
    const float mk = b1 * m[k] + (1.f - b1) * g;
    const float vk = b2 * v[k] + (1.f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    const float wk = master[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    master[k] = wk;
    w[k] = f32_to_bf16(wk);
}

int g4_launch_mlp_adam(g4_ctx *ctx, uint16_t *w, float *master, float *m, float *v, const float *grad, float lr,
                       float b1, float b2, float eps, int64_t step)
{
    const float c1 = (float)(1.0 - pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - pow((double)b2, (double)step));
    k_mlp_adam<<<(MLP_NP + 255) / 256, 256, 0, ctx->stream>>>(w, master, m, v, grad, lr, b1, b2, eps, c1, c2);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
