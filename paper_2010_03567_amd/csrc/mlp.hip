// mlp.hip -- learned |a| seed for the relative opening criterion.
//
// The paper seeds the relative criterion (eq. eqnrelcriterion) for the very
// first force with a geometric walk (footnote to that equation).  This module
// replaces that pre-walk by a small network that predicts log10 |a| of each
// particle from cheap tree features: an 8 -> 64 -> 64 -> 1 perceptron with
// SiLU activations, BF16 weights and FP32 arithmetic (the forward pass puts
// the hidden 64 x 64 layer on the matrix cores).  Parameter layout (4801
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
// One lane per particle j (sorted order). Its leaf comes from the moments
// pass (leafof), and the lanes of one leaf read the same records, so a
// wavefront's loads touch few distinct lines. The near-field sum runs over
// the leaf's particles in order, then over the sibling monopoles (children
// of the parent other than the leaf, then children of the grandparent other
// than the parent); the source loads go out four at a time (clamped
// indices), so the loop is not a chain of single trips to memory.
template <int KER>
__global__ __launch_bounds__(256) void k_mlp_features(const WNode *__restrict__ wn, const double *__restrict__ mom,
                                                      const uint32_t *__restrict__ parent,
                                                      const uint32_t *__restrict__ leafof,
                                                      const uint4 *__restrict__ parts, const uint32_t *__restrict__ perm,
                                                      int64_t n, double boxd, double unit_d, float asplit, float h2,
                                                      float hinv, const float *__restrict__ norm,
                                                      float *__restrict__ feat)
{
    const float unit = (float)unit_d;
    const uint32_t NONE = 0xffffffffu;
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < n; jj += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t j = (uint32_t)jj;
        const uint32_t q = leafof[j];
        const uint4 pj = parts[j];
        const uint32_t row = perm[j];
        const WNode w = wn[q];
        const uint32_t p = parent[q];
        const uint32_t gp = p != NONE ? parent[p] : NONE;
        const uint32_t pp = p != NONE ? p : q;
        const WNode wp = wn[pp];
        const double *ml = mom + (size_t)q * MOM_STRIDE, *mpp = mom + (size_t)pp * MOM_STRIDE;
        const double mq = ml[0], mp = mpp[0];
        const double mg = gp != NONE ? mom[(size_t)gp * MOM_STRIDE] : mp;
        float ax = 0.f, ay = 0.f, az = 0.f, K, W;
        const uint32_t stop = w.next + w.num;
        for (uint32_t s0 = w.next; s0 < stop; s0 += 4) {
            uint4 pk[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) pk[u] = parts[s0 + u < stop ? s0 + u : stop - 1];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const float dx = (float)(int32_t)(pk[u].x - pj.x) * unit, dy = (float)(int32_t)(pk[u].y - pj.y) * unit,
                            dz = (float)(int32_t)(pk[u].z - pj.z) * unit;
                pair_kernel<KER, false>(dx * dx + dy * dy + dz * dz, asplit, h2, hinv, K, W);
                const float mk = s0 + u < stop && s0 + u != j ? __uint_as_float(pk[u].w) * K : 0.f;
                ax += mk * dx;
                ay += mk * dy;
                az += mk * dz;
            }
        }
        for (int side = 0; side < 2; side++) {
            const uint32_t self = side ? p : q, up = side ? gp : p;
            if (self == NONE || up == NONE) continue;
            const WNode wu = side ? wn[up] : wp;
            // centre of mass and mass of each child (the first 16 bytes of its record)
            uint4 ch[8];
#pragma unroll
            for (uint32_t c = 0; c < 8; c++)
                ch[c] = reinterpret_cast<const uint4 *>(wn + wu.next + (c < wu.num ? c : 0))[0];
#pragma unroll
            for (uint32_t c = 0; c < 8; c++) {
                if (c >= wu.num || wu.next + c == self) continue;
                const float km = __uint_as_float(ch[c].w);
                if (km == 0.f) continue;
                const float dx = (float)(int32_t)(ch[c].x - pj.x) * unit, dy = (float)(int32_t)(ch[c].y - pj.y) * unit,
                            dz = (float)(int32_t)(ch[c].z - pj.z) * unit;
                pair_kernel<KER, false>(dx * dx + dy * dy + dz * dz, asplit, h2, hinv, K, W);
                const float mk = km * K;
                ax += mk * dx;
                ay += mk * dy;
                az += mk * dz;
            }
        }
        const int level = (int)(w.meta & 0xffu);
        const double il = 1.0 / ldexp(boxd, -level), ilp = 1.0 / ldexp(boxd, -(int)(wp.meta & 0xffu));
        float f[8];
        f[0] = log10f((float)mq);
        f[1] = log10f((float)ldexp(boxd, -level));
        f[2] = (float)level;
        // offsets from the centres of mass in FP64 (they may nearly cancel), logarithms in FP32
        double a0 = (double)(int32_t)(pj.x - w.gx) * unit_d - ml[1], a1 = (double)(int32_t)(pj.y - w.gy) * unit_d - ml[2],
               a2 = (double)(int32_t)(pj.z - w.gz) * unit_d - ml[3];
        f[3] = log10f((float)(sqrt(a0 * a0 + a1 * a1 + a2 * a2) * il + 1e-3));
        a0 = (double)(int32_t)(pj.x - wp.gx) * unit_d - mpp[1];
        a1 = (double)(int32_t)(pj.y - wp.gy) * unit_d - mpp[2];
        a2 = (double)(int32_t)(pj.z - wp.gz) * unit_d - mpp[3];
        f[4] = log10f((float)(sqrt(a0 * a0 + a1 * a1 + a2 * a2) * ilp + 1e-3));
        f[5] = log10f((float)mp);
        f[6] = log10f((float)mg);
        f[7] = log10f(fmaxf(sqrtf(ax * ax + ay * ay + az * az), 1e-30f));
        float *o = feat + (size_t)row * 8;
        for (int kk = 0; kk < 8; kk++) o[kk] = norm ? (f[kk] - norm[kk]) * norm[8 + kk] : f[kk];
    }
}

int g4_launch_mlp_features(g4_ctx *ctx, const g4_tree *t, const g4_walk_params *wp, const float *norm, float *feat)
{
    int64_t blocks = (t->n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    const double h = 2.8 * wp->eps0;
    const float asplit = wp->kernel == 1 ? (float)(0.5 / wp->r_s) : 0.f;
    const float h2 = (float)(h * h), hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    if (wp->kernel == 1)
        k_mlp_features<1><<<(unsigned)blocks, 256, 0, ctx->stream>>>(t->wn, t->mom, t->parent, t->leafof, t->parts,
                                                                     t->perm1, t->n, t->tp.box, t->unit, asplit, h2,
                                                                     hinv, norm, feat);
    else
        k_mlp_features<0><<<(unsigned)blocks, 256, 0, ctx->stream>>>(t->wn, t->mom, t->parent, t->leafof, t->parts,
                                                                     t->perm1, t->n, t->tp.box, t->unit, asplit, h2,
                                                                     hinv, norm, feat);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ forward
// One wavefront per tile of 32 particles. Lane (c, h), c = lane % 32, takes
// particle c of the tile and hidden units 8h + 16s + j (s < 4, j < 8) of the
// first layer in FP32. The 64 x 64 second layer runs on the matrix cores
// (32x32x16 BF16 products, FP32 accumulation): W2 is exact in BF16, and each
// first-layer output is split as hi + lo with hi = bf16(h), lo = bf16(h - hi),
// so the two products per step carry h to about 2^-17 relative, close to
// FP32. A lane's 16 + 16 accumulator values are rows 8 (r / 4) + 4 h + r % 4
// of the two 32-row output tiles for its particle; the last layer sums them
// and the two halves of the wave are added. mode 0 writes y = log10|a|,
// mode 1 writes 10^(y + shift).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define FWD_TILE 32

__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *__restrict__ w, const float *__restrict__ feat,
                                                     int64_t n, float *__restrict__ out, float shift, int mode)
{
    // W1 rows (8 weights + bias, padded to 12 for 16-byte reads), then b2 and w3
    __shared__ __attribute__((aligned(16))) float L1[64][12];
    __shared__ float E[2][64];
    for (int k = threadIdx.x; k < 64 * 9; k += blockDim.x) {
        const int u = k / 9, i = k % 9;
        L1[u][i] = bf16_to_f32(w[i < 8 ? u * 8 + i : OFF_B1 + u]);
    }
    for (int k = threadIdx.x; k < 64; k += blockDim.x) {
        E[0][k] = bf16_to_f32(w[OFF_B2 + k]);
        E[1][k] = bf16_to_f32(w[OFF_W3 + k]);
    }
    const float b3 = bf16_to_f32(w[OFF_B3]);
    __syncthreads();
    const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
    // second-layer weights as matrix-core A operands: row 32 t + c, columns 16 s + 8 h + j
    bf16x8 A[2][4];
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
        for (int s = 0; s < 4; s++) {
            u16x8 v;
            const uint16_t *r = w + OFF_W2 + (32 * t + c) * 64 + 16 * s + 8 * h;
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] = r[j];
            A[t][s] = __builtin_bit_cast(bf16x8, v);
        }
    const int64_t tiles = (n + FWD_TILE - 1) / FWD_TILE;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t tile = wave; tile < tiles; tile += nwave) {
        const int64_t p = tile * FWD_TILE + c;
        const bool valid = p < n;
        float x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (valid) {
            const float4 xa = reinterpret_cast<const float4 *>(feat)[2 * p];
            const float4 xb = reinterpret_cast<const float4 *>(feat)[2 * p + 1];
            x[0] = xa.x; x[1] = xa.y; x[2] = xa.z; x[3] = xa.w;
            x[4] = xb.x; x[5] = xb.y; x[6] = xb.z; x[7] = xb.w;
        }
        // an offset the compiler cannot see through, so the first-layer
        // weights are read from LDS per tile instead of held in registers
        int row0 = 8 * h;
        asm volatile("" : "+v"(row0));
        bf16x8 Bh[4], Bl[4];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const float *r = L1[row0 + 16 * s + j];
                const float4 ra = *reinterpret_cast<const float4 *>(r);
                const float4 rb = *reinterpret_cast<const float4 *>(r + 4);
                float z = r[8];
                z = fmaf(ra.x, x[0], z); z = fmaf(ra.y, x[1], z); z = fmaf(ra.z, x[2], z); z = fmaf(ra.w, x[3], z);
                z = fmaf(rb.x, x[4], z); z = fmaf(rb.y, x[5], z); z = fmaf(rb.z, x[6], z); z = fmaf(rb.w, x[7], z);
                const float a = z * sigm(z);
                const __bf16 hi = (__bf16)a;
                Bh[s][j] = hi;
                Bl[s][j] = (__bf16)(a - (float)hi);
            }
        f32x16 acc0 = {}, acc1 = {};
#pragma unroll
        for (int s = 0; s < 4; s++) {
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][s], Bh[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][s], Bh[s], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][s], Bl[s], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][s], Bl[s], acc1, 0, 0, 0);
        }
        float y = 0.f;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int o = 8 * (r >> 2) + 4 * h + (r & 3);
            const float z0 = acc0[r] + E[0][o], z1 = acc1[r] + E[0][32 + o];
            y = fmaf(E[1][o], z0 * sigm(z0), y);
            y = fmaf(E[1][32 + o], z1 * sigm(z1), y);
        }
        y += __shfl_xor(y, 32);
        if (h == 0 && valid) {
            y += b3;
            out[p] = mode ? exp10f(y + shift) : y;
        }
    }
}

int g4_launch_mlp_forward(g4_ctx *ctx, const uint16_t *w, const float *feat, int64_t n, float *out, float shift,
                          int mode)
{
    // about eight tiles per wavefront, so the A operands load once per eight tiles
    const int64_t tiles = (n + FWD_TILE - 1) / FWD_TILE;
    int64_t blocks = (tiles + 31) / 32;
    if (blocks > 4096) blocks = 4096;
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
    if (int st = g4_launch_zero(ctx, grad, MLP_NP * sizeof(float))) return st;
    if (int st = g4_launch_zero(ctx, loss, sizeof(float))) return st;
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
