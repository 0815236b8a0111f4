// ewald.h -- periodic correction potential psi on the device: table layout
// and the third-order Taylor evaluation used by the walk.
//
// Paper: Sec. "Periodic boundary conditions" (eqs. eqnpo1, eqnpo2, eqnewal;
// the derivative tensors of psi tabulated on a grid and evaluated at a point
// by a Taylor expansion around the nearest grid point, third order).
//
// psi is even in every coordinate and symmetric under axis permutations, so
// one octant [0, L/2]^3 is tabulated: (ne + 1)^3 points x = (i, j, k) h,
// h = L / (2 ne), with the 84 derivatives D^(a,b,c) psi of orders 0..6 per
// point (FP32, 336 bytes).  Within a point the components run order by order,
// and within an order with a descending, then b descending:
//   index(a, b, c) = o (o + 1)(o + 2)/6 + (b + c)(b + c + 1)/2 + c,  o = a + b + c.
// An offset d = (s_x u_x, s_y u_y, s_z u_z) with signs s and u >= 0 maps to
// the octant point u, and D^(a,b,c) psi(d) = s_x^a s_y^b s_z^c D^(a,b,c) psi(u).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define G4_EWALD_NCOMP 84
#define G4_EWALD_NE_MIN 4
#define G4_EWALD_NE_MAX 128

__host__ __device__ constexpr int ew_idx(int a, int b, int c)
{
    return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

// Located point: the table row of the nearest grid point x0, the monomials
// (u - x0)^b / b! for |b| <= 3 (indexed like the components), and the signs
// of the offset.
struct EwPoint {
    const float *row;
    float m[20];
    float sx, sy, sz;
};

__device__ __forceinline__ EwPoint ew_locate(const float *__restrict__ tab, int ne, float h, float hinv, float dx,
                                             float dy, float dz)
{
    EwPoint p;
    p.sx = dx < 0.f ? -1.f : 1.f;
    p.sy = dy < 0.f ? -1.f : 1.f;
    p.sz = dz < 0.f ? -1.f : 1.f;
    const float ux = fabsf(dx), uy = fabsf(dy), uz = fabsf(dz);
    const int i = min((int)fmaf(ux, hinv, 0.5f), ne);
    const int j = min((int)fmaf(uy, hinv, 0.5f), ne);
    const int k = min((int)fmaf(uz, hinv, 0.5f), ne);
    const float ex = fmaf(-(float)i, h, ux), ey = fmaf(-(float)j, h, uy), ez = fmaf(-(float)k, h, uz);
    p.row = tab + ((size_t)(i * (ne + 1) + j) * (ne + 1) + k) * G4_EWALD_NCOMP;
    const float xx = ex * ex, yy = ey * ey, zz = ez * ez;
    float *m = p.m;
    m[ew_idx(0, 0, 0)] = 1.f;
    m[ew_idx(1, 0, 0)] = ex;
    m[ew_idx(0, 1, 0)] = ey;
    m[ew_idx(0, 0, 1)] = ez;
    m[ew_idx(2, 0, 0)] = 0.5f * xx;
    m[ew_idx(1, 1, 0)] = ex * ey;
    m[ew_idx(1, 0, 1)] = ex * ez;
    m[ew_idx(0, 2, 0)] = 0.5f * yy;
    m[ew_idx(0, 1, 1)] = ey * ez;
    m[ew_idx(0, 0, 2)] = 0.5f * zz;
    m[ew_idx(3, 0, 0)] = (1.f / 6.f) * xx * ex;
    m[ew_idx(2, 1, 0)] = 0.5f * xx * ey;
    m[ew_idx(2, 0, 1)] = 0.5f * xx * ez;
    m[ew_idx(1, 2, 0)] = 0.5f * ex * yy;
    m[ew_idx(1, 1, 1)] = ex * ey * ez;
    m[ew_idx(1, 0, 2)] = 0.5f * ex * zz;
    m[ew_idx(0, 3, 0)] = (1.f / 6.f) * yy * ey;
    m[ew_idx(0, 2, 1)] = 0.5f * yy * ez;
    m[ew_idx(0, 1, 2)] = 0.5f * ey * zz;
    m[ew_idx(0, 0, 3)] = (1.f / 6.f) * zz * ez;
    return p;
}

// D^(A,B,C) psi at the located point (octant frame): sum_{|b| <= 3} D^(A,B,C)+b (x0) m_b
template <int A, int B, int C>
__device__ __forceinline__ float ew_taylor(const EwPoint &p)
{
    float s = 0.f;
#pragma unroll
    for (int o = 3; o >= 0; o--)
#pragma unroll
        for (int b1 = o; b1 >= 0; b1--)
#pragma unroll
            for (int b2 = o - b1; b2 >= 0; b2--) {
                const int b3 = o - b1 - b2;
                s = fmaf(p.row[ew_idx(A + b1, B + b2, C + b3)], p.m[ew_idx(b1, b2, b3)], s);
            }
    return s;
}

// grad psi(d) (and psi(d) with POT) for a single source at offset d
template <bool POT>
__device__ __forceinline__ void ew_grad(const float *__restrict__ tab, int ne, float h, float hinv, float dx, float dy,
                                        float dz, float &gx, float &gy, float &gz, float &ps)
{
    const EwPoint p = ew_locate(tab, ne, h, hinv, dx, dy, dz);
    gx = p.sx * ew_taylor<1, 0, 0>(p);
    gy = p.sy * ew_taylor<0, 1, 0>(p);
    gz = p.sz * ew_taylor<0, 0, 1>(p);
    if (POT) ps = ew_taylor<0, 0, 0>(p);
}

// Correction of a node with mass M, second moments q (xx xy xz yy yz zz) and,
// for the potential, third moments o (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz)
// about its centre of mass at offset d from the target:
//   force  f = M grad psi + (1/2) Q2 : grad^3 psi       (ORD3; M grad psi otherwise)
//   potential  M psi + (1/2) Q2 : grad^2 psi (+ (1/6) Q3 . grad^3 psi with ORD3)
// (the node terms of eq. eqnpo1 with the multipole expansion of psi).
template <bool POT, bool ORD3>
__device__ __forceinline__ void ew_node(const float *__restrict__ tab, int ne, float h, float hinv, float dx, float dy,
                                        float dz, float M, float4 qa, float2 qb, const float *__restrict__ o,
                                        float &fx, float &fy, float &fz, float &fp)
{
    const EwPoint p = ew_locate(tab, ne, h, hinv, dx, dy, dz);
    const float sx = p.sx, sy = p.sy, sz = p.sz;
    // moments reflected into the octant frame
    const float qxx = qa.x, qxy = sx * sy * qa.y, qxz = sx * sz * qa.z, qyy = qa.w, qyz = sy * sz * qb.x, qzz = qb.y;
    float gx = M * ew_taylor<1, 0, 0>(p), gy = M * ew_taylor<0, 1, 0>(p), gz = M * ew_taylor<0, 0, 1>(p);
    float t300 = 0.f, t210 = 0.f, t201 = 0.f, t120 = 0.f, t111 = 0.f, t102 = 0.f, t030 = 0.f, t021 = 0.f, t012 = 0.f,
          t003 = 0.f;
    if (ORD3 || POT) {
        t300 = ew_taylor<3, 0, 0>(p);
        t210 = ew_taylor<2, 1, 0>(p);
        t201 = ew_taylor<2, 0, 1>(p);
        t120 = ew_taylor<1, 2, 0>(p);
        t111 = ew_taylor<1, 1, 1>(p);
        t102 = ew_taylor<1, 0, 2>(p);
        t030 = ew_taylor<0, 3, 0>(p);
        t021 = ew_taylor<0, 2, 1>(p);
        t012 = ew_taylor<0, 1, 2>(p);
        t003 = ew_taylor<0, 0, 3>(p);
    }
    if (ORD3) {
        gx += 0.5f * (qxx * t300 + qyy * t120 + qzz * t102) + qxy * t210 + qxz * t201 + qyz * t111;
        gy += 0.5f * (qxx * t210 + qyy * t030 + qzz * t012) + qxy * t120 + qxz * t111 + qyz * t021;
        gz += 0.5f * (qxx * t201 + qyy * t021 + qzz * t003) + qxy * t111 + qxz * t102 + qyz * t012;
    }
    fx = sx * gx;
    fy = sy * gy;
    fz = sz * gz;
    if (POT) {
        const float d2 = 0.5f * (qxx * ew_taylor<2, 0, 0>(p) + qyy * ew_taylor<0, 2, 0>(p) + qzz * ew_taylor<0, 0, 2>(p)) +
                         qxy * ew_taylor<1, 1, 0>(p) + qxz * ew_taylor<1, 0, 1>(p) + qyz * ew_taylor<0, 1, 1>(p);
        const float sxyz = sx * sy * sz;
        const float d3 = sx * o[0] * t300 + sy * o[6] * t030 + sz * o[9] * t003 +
                         3.f * (sy * o[1] * t210 + sz * o[2] * t201 + sx * o[3] * t120 + sx * o[5] * t102 +
                                sz * o[7] * t021 + sy * o[8] * t012) +
                         6.f * sxyz * o[4] * t111;
        fp = M * ew_taylor<0, 0, 0>(p) + d2 + (ORD3 ? d3 * (1.f / 6.f) : 0.f);
    }
}

// D0..D3 of psi at offset d, packed as 1 + 3 + 6 + 10 values in the order of
// the components above (D2: xx xy xz yy yz zz; D3: xxx xxy xxz xyy xyz xzz
// yyy yyz yzz zzz), for the field expansions of the periodic FMM.
__device__ __forceinline__ void ew_d20(const float *__restrict__ tab, int ne, float h, float hinv, float dx, float dy,
                                       float dz, float D[20])
{
    const EwPoint p = ew_locate(tab, ne, h, hinv, dx, dy, dz);
    const float sx = p.sx, sy = p.sy, sz = p.sz;
    D[0] = ew_taylor<0, 0, 0>(p);
    D[1] = sx * ew_taylor<1, 0, 0>(p);
    D[2] = sy * ew_taylor<0, 1, 0>(p);
    D[3] = sz * ew_taylor<0, 0, 1>(p);
    D[4] = ew_taylor<2, 0, 0>(p);
    D[5] = sx * sy * ew_taylor<1, 1, 0>(p);
    D[6] = sx * sz * ew_taylor<1, 0, 1>(p);
    D[7] = ew_taylor<0, 2, 0>(p);
    D[8] = sy * sz * ew_taylor<0, 1, 1>(p);
    D[9] = ew_taylor<0, 0, 2>(p);
    D[10] = sx * ew_taylor<3, 0, 0>(p);
    D[11] = sy * ew_taylor<2, 1, 0>(p);
    D[12] = sz * ew_taylor<2, 0, 1>(p);
    D[13] = sx * ew_taylor<1, 2, 0>(p);
    D[14] = sx * sy * sz * ew_taylor<1, 1, 1>(p);
    D[15] = sx * ew_taylor<1, 0, 2>(p);
    D[16] = sy * ew_taylor<0, 3, 0>(p);
    D[17] = sz * ew_taylor<0, 2, 1>(p);
    D[18] = sy * ew_taylor<0, 1, 2>(p);
    D[19] = sz * ew_taylor<0, 0, 3>(p);
}
