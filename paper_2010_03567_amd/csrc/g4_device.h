// g4_device.h -- device functions shared by the HIP kernels: fast hardware
// reciprocals, an erfc approximation, the spline-softening factors and the
// softened (short-range) pair kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define INV_SQRTPI 0.564189583547756287f

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ uint32_t uabs(int32_t d) { return d < 0 ? 0u - (uint32_t)d : (uint32_t)d; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float expneg(float x2) { return __builtin_amdgcn_exp2f(-1.44269504088896341f * x2); }

// erfc(x) for x >= 0 by Abramowitz & Stegun 7.1.26 (Hastings' rational
// approximation, |error| <= 1.5e-7): erfc(x) = t P(t) exp(-x^2), t = 1/(1+px).
// ex = exp(-x^2) is passed in because the kernel needs it anyway.
__device__ __forceinline__ float erfc_hastings(float x, float ex)
{
    float t = rcp(1.0f + 0.3275911f * x);
    float p = fmaf(t, 1.061405429f, -1.453152027f);
    p = fmaf(t, p, 1.421413741f);
    p = fmaf(t, p, -0.284496736f);
    p = fmaf(t, p, 0.254829592f);
    return t * p * ex;
}

// Spline-softened force factor K(u)/h^3 and potential W(u)/h, u = r/h < 1.
__device__ __forceinline__ float soft_force(float u, float hinv)
{
    float h3 = hinv * hinv * hinv, u2 = u * u;
    if (u < 0.5f) return h3 * (10.666666666666667f + u2 * (-38.4f + 32.0f * u));
    return h3 * (21.333333333333333f - 48.0f * u + 38.4f * u2 - 10.666666666666667f * u2 * u -
                 0.066666666666666667f * rcp(u2 * u));
}
__device__ __forceinline__ float soft_pot(float u, float hinv)
{
    float u2 = u * u;
    if (u < 0.5f) return hinv * (2.8f + u2 * (-5.333333333333333f + u2 * (9.6f - 6.4f * u)));
    return hinv * (3.2f - 0.066666666666666667f * rcp(u) +
                   u2 * (-10.666666666666667f + u * (16.0f + u * (-9.6f + 2.1333333333333333f * u))));
}

// Long-range pair factors for x = alpha r, needed only inside the softening edge:
//   lrf(x) = (erf x - 2x e^{-x^2}/sqrt(pi)) / x^3,   erfx(x) = erf(x)/x,
// by their Taylor series below x = 0.5 and in closed form above.  Inside the softening
// length x is usually far below 0.5 (h alpha << 1), so the closed form sits behind a branch
// on the wavefront's vote and is skipped when no active lane needs it.
__device__ __forceinline__ float lr_force_x3(float x)
{
    const float x2 = x * x;
    float v = 4.0f * INV_SQRTPI *
              (1.0f / 3 + x2 * (-1.0f / 5 + x2 * (1.0f / 14 + x2 * (-1.0f / 54 + x2 * (1.0f / 264 - x2 * (1.0f / 1560))))));
    if (__builtin_amdgcn_ballot_w64(x >= 0.5f)) {
        // an empty statement that the compiler must assume changes y: it keeps the closed form
        // inside the branch instead of evaluating it for every lane beside the series
        float y = x;
        asm volatile("" : "+v"(y));
        if (y >= 0.5f) {
            const float ex = expneg(y * y);
            const float erfv = 1.0f - erfc_hastings(y, ex);
            v = (erfv - 2.0f * INV_SQRTPI * y * ex) * rcp(y * y * y);
        }
    }
    return v;
}
__device__ __forceinline__ float erf_over_x(float x)
{
    const float x2 = x * x;
    float v = 2.0f * INV_SQRTPI *
              (1.0f + x2 * (-1.0f / 3 + x2 * (1.0f / 10 + x2 * (-1.0f / 42 + x2 * (1.0f / 216 - x2 * (1.0f / 1320))))));
    if (__builtin_amdgcn_ballot_w64(x >= 0.5f)) {
        float y = x;
        asm volatile("" : "+v"(y));  // as in lr_force_x3
        if (y >= 0.5f) v = (1.0f - erfc_hastings(y, expneg(y * y))) * rcp(y);
    }
    return v;
}

// Pair interaction (softened, optionally short-range): returns the force
// factor K (a += m K d) and the potential factor W (phi -= m W).
template <int KER, bool POT>
__device__ __forceinline__ void pair_kernel(float r2, float asplit, float h2, float hinv, float &K, float &W)
{
    float rinv = r2 > 0.f ? rsq(r2) : 0.f;
    float rinv2 = rinv * rinv;
    if (KER == 0) {
        K = rinv * rinv2;
        if (POT) W = rinv;
    } else {
        float r = r2 * rinv;
        float x = asplit * r;
        float ex = expneg(x * x);
        float ec = erfc_hastings(x, ex);
        K = (ec + 2.0f * INV_SQRTPI * x * ex) * rinv * rinv2;
        if (POT) W = ec * rinv;
    }
    // the softened branch for r < h; a pair at zero separation (a particle with itself) adds no
    // force whatever K is, so without the potential it takes the plain branch (rinv = 0, K = 0)
    // and does not pull the whole wavefront into the softened one
    if (r2 < h2 && (POT || r2 > 0.f)) {
        float r = r2 * rinv;
        float u = r * hinv;
        K = soft_force(u, hinv);
        if (POT) W = soft_pot(u, hinv);
        if (KER == 1) {
            float x = asplit * r;
            float a3 = asplit * asplit * asplit;
            K -= a3 * lr_force_x3(x);
            if (POT) W -= asplit * erf_over_x(x);
        }
    }
}

// Short-range factors by table (Sec. "TreePM approach": one-dimensional
// look-up table instead of erfc per interaction).  With x = alpha_split r,
//   S_0 = erfc x,  S_n = erfc x + (2x/sqrt(pi)) e^{-x^2} P_n(x^2),
//   P_1 = 1, P_2 = 1 + 2x^2/3, P_3 = 1 + 2x^2/3 + 4x^4/15,
// so that the short-range g_0..g_3 are the Newtonian ones (1/r, -1/r^3,
// 3/r^5, -15/r^7) times S_0..S_3.  tab[f * n + k] holds the cubic Hermite
// piece of S_f on interval k, in u in [0, 1]; t = r * tscale = x n / x_max.
__device__ __forceinline__ void sr_locate(float r, float tscale, uint32_t n, uint32_t &k, float &u)
{
    const float t = fminf(r * tscale, (float)n);
    k = min((uint32_t)t, n - 1u);
    u = t - (float)k;
}
__device__ __forceinline__ float sr_eval(const float4 &c, float u)
{
    return fmaf(u, fmaf(u, fmaf(u, c.w, c.z), c.y), c.x);
}

// pair_kernel<1, POT> with the short-range factors from the table
template <bool POT>
__device__ __forceinline__ void pair_kernel_tab(float r2, const float4 *__restrict__ tab, uint32_t n, float tscale,
                                                float asplit, float h2, float hinv, float &K, float &W)
{
    float rinv = r2 > 0.f ? rsq(r2) : 0.f;
    float rinv2 = rinv * rinv;
    float r = r2 * rinv;
    uint32_t k;
    float u;
    sr_locate(r, tscale, n, k, u);
    K = sr_eval(tab[n + k], u) * rinv * rinv2;
    if (POT) W = sr_eval(tab[k], u) * rinv;
    if (r2 < h2 && (POT || r2 > 0.f)) {  // as in pair_kernel
        float uh = r * hinv;
        K = soft_force(uh, hinv);
        if (POT) W = soft_pot(uh, hinv);
        float x = asplit * r;
        float a3 = asplit * asplit * asplit;
        K -= a3 * lr_force_x3(x);
        if (POT) W -= asplit * erf_over_x(x);
    }
}
