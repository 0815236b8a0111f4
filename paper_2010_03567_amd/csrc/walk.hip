// walk.hip -- one-sided tree walk (Newtonian and TreePM short-range) on gfx950.
//
// Paper: Sec. "One-sided multipole expansion" (eqs. eqonesidetreeacc /
// eqonesidetreepotential at p = 3: a = -G[M D1 + Q2:D3/2]), Sec. "Tree walk
// and opening criterion" (geometric l/r < theta, relative eq. eqnrelcriterion,
// exclusion zone), Sec. "TreePM approach" (eq. eqnpo4 kernel, node dropped when
// its nearest edge lies beyond r_cut), Sec. "Softened potential in periodic
// systems" (spline softening of edge h = 2.8 eps0).
//
// Mapping to CDNA4: one 64-lane wavefront walks the tree for a group of up to
// 64 consecutive Morton-sorted particles.  Every target takes its own opening
// decisions, exactly as in the per-particle walk of the paper, but the work is
// packed so that lanes stay busy: (node, target) visits, particle-node and
// particle-particle interactions are each issued 64 at a time from LDS (see
// the kernel below).  Interactions are FP32 arithmetic on int32 nearest-image
// differences, summed per target in FP64.
#include <algorithm>
#include <cstdlib>
#include <new>
#include <vector>

#include "ewald.h"
#include "g4_device.h"
#include "g4_internal.h"

struct WalkArgs {
    const uint4 *parts;
    const WNode *wn;
    const float *q3;
    const float *aseed;
    const uint32_t *perm;
    int64_t n;
    int group;
    int S;
    int exclusion;    // bit 0: exclusion zone around each node; bit 1: per-target decisions only (diagnostic)
    int order;
    float unit;       // physical length per integer step
    float box;        // physical root side
    float h, h2, hinv;
    float asplit;     // 1/(2 r_s)
    const float4 *tab;  // short-range factor table (kernel 2), tn intervals, t = r * tscale
    uint32_t tn;
    float tscale;
    const double *q4;   // fourth moments (15 per node, packed), orders p = 4, 5
    const float *ew;    // periodic correction table (kernel 3): ew_n intervals of ew_h over [0, L/2]
    int ew_n;
    float ew_h, ew_hinv;
    float rcut2;
    float theta2;
    float alpha;      // relative-criterion accuracy parameter
    double G;
    double *ax, *ay, *az, *pot;
    uint32_t *counts;
    float *aout_caller, *aout_sorted;
    unsigned long long *stat;   // 3 counters: p2p, p2m, visits
    unsigned long long *wstat;  // passes, deepest stack, entries, leaves, chunks, group decisions (slots 9..17)
    const uint4 *items;         // work items (first particle, count, root node), or null: groups of `group`
    uint32_t nitems;
    uint32_t *item_ctr;         // zeroed before the launch
    uint4 *spill;               // per-wavefront spill area of the traversal stack
    int64_t spill_waves;        // wavefronts the spill area has room for (a multiple of 4)
    int lds_stk;                // stack entries kept in LDS (<= WK_LDS_STK)
    uint32_t *flags;            // tree flags: G4_FLAG_WALK_STACK if the stack bound is ever broken
};

// Kernels: 0 Newtonian (isolated), 1 TreePM short range, 2 the same with the
// short-range factors from a table, 3 periodic Newtonian: the nearest image
// with the Newtonian kernel plus the correction potential psi of every node
// and particle (eq. eqnpo1), its derivatives from the Taylor table.
// g1, g2, g3 (and g0) of the interaction kernel at r (r2, rinv given), r >= h.
template <int KER>
__device__ __forceinline__ void gfun(float r2, float rinv, const WalkArgs &A, float &g0, float &g1, float &g2,
                                     float &g3)
{
    float ri2 = rinv * rinv;
    if (KER == 0 || KER == 3) {
        g0 = rinv;
        g1 = -rinv * ri2;
        g2 = -3.0f * g1 * ri2;
        g3 = -5.0f * g2 * ri2;
    } else if (KER == 2) {
        // the short-range factors from the table: g_n = (Newtonian g_n) S_n
        uint32_t k;
        float u;
        sr_locate(r2 * rinv, A.tscale, A.tn, k, u);
        const float s1 = sr_eval(A.tab[A.tn + k], u), s2 = sr_eval(A.tab[2 * A.tn + k], u),
                    s3 = sr_eval(A.tab[3 * A.tn + k], u);
        const float ri3 = rinv * ri2;
        g0 = sr_eval(A.tab[k], u) * rinv;
        g1 = -s1 * ri3;
        g2 = 3.0f * s2 * ri3 * ri2;
        g3 = -15.0f * s3 * ri3 * ri2 * ri2;
    } else {
        float r = r2 * rinv;
        float x = A.asplit * r;
        float ex = expneg(x * x);
        float ec = erfc_hastings(x, ex);
        float E = 2.0f * INV_SQRTPI * A.asplit * ex;
        float a2 = A.asplit * A.asplit;
        float t1 = ec * rinv * ri2;
        float e2 = E * ri2;
        g0 = ec * rinv;
        g1 = -(t1 + e2);
        g2 = 3.0f * t1 * ri2 + e2 * (3.0f * ri2 + 2.0f * a2);
        g3 = -(15.0f * t1 * ri2 * ri2 + e2 * (ri2 * (15.0f * ri2 + 10.0f * a2) + 4.0f * a2 * a2));
    }
}

// Dimensionless s_n = g_n r^(2n+1), n = 2..5, of the Newtonian kernel
// ((-1)^n (2n-1)!!) or of erfc(alpha r)/r, from the recursion
// g_{n+1} = r^-1 d g_n/dr; with x = alpha r and e = (2/sqrt(pi)) exp(-x^2):
//   s2 = 3 erfc(x) + e (3x + 2x^3),  s3 = -15 erfc(x) - e (15x + 10x^3 + 4x^5),
//   s4 = 105 erfc(x) + e (105x + 70x^3 + 28x^5 + 8x^7),
//   s5 = -945 erfc(x) - e (945x + 630x^3 + 252x^5 + 72x^7 + 16x^9).
// The orders above p = 3 are written with them and the unit vector of r, the
// power of 1/r applied last: g5 itself (~ 1/r^11) leaves the FP32 range at the
// node distances of a 128^3 box.
template <int KER>
__device__ __forceinline__ void sfun_hi(float r, const WalkArgs &A, float &s2, float &s3, float &s4, float &s5)
{
    if (KER == 0) {
        s2 = 3.f;
        s3 = -15.f;
        s4 = 105.f;
        s5 = -945.f;
    } else {
        const float x = A.asplit * r, x2 = x * x;
        const float ex = expneg(x2), ec = erfc_hastings(x, ex);
        const float e = 2.0f * INV_SQRTPI * ex * x;
        s2 = 3.f * ec + e * (3.f + 2.f * x2);
        s3 = -15.f * ec - e * (15.f + x2 * (10.f + 4.f * x2));
        s4 = 105.f * ec + e * (105.f + x2 * (70.f + x2 * (28.f + 8.f * x2)));
        s5 = -945.f * ec - e * (945.f + x2 * (630.f + x2 * (252.f + x2 * (72.f + 16.f * x2))));
    }
}

// Terms of the orders above p = 3 for a node at r = |r| n from the target
// (Appendix A): the force adds Q3:D4/6 (p >= 4) and Q4:D5/24 (p = 5), the
// potential Q4:D4/24 (p >= 4), with the radial D_n written through s_n:
//   Q3:D4 = r^-5 [3 s2 t + 3 s3 (T:nn + (t.n) n) + s4 (T.nnn) n],  t_i = T_ikk,
//   Q4:D5 = r^-6 [12 s3 W n + 3 s3 w n + 4 s4 U.nnn + 6 s4 (n.W.n) n + s5 (U.nnnn) n],
//   Q4:D4 = r^-5 [3 s2 w + 6 s3 (n.W.n) + s4 (U.nnnn)],  W_ij = U_ijkk, w = W_ii,
// with T, U the packed third and fourth moments about the node's centre of mass.
template <int HI, bool POT>
__device__ __forceinline__ void eval_high(const float *o, const double *u4, float nx, float ny, float nz, float rinv,
                                          float s2, float s3, float s4, float s5, float &fx, float &fy, float &fz,
                                          float &fp)
{
    const float n[3] = {nx, ny, nz};
    const float ri2 = rinv * rinv, r5 = ri2 * ri2 * rinv, r6 = ri2 * ri2 * ri2;
    float T[10];
#pragma unroll
    for (int a = 0; a < 10; a++) T[a] = o[a];
    auto t3 = [&](int i, int j, int k) {
        const int c[3] = {(i == 0) + (j == 0) + (k == 0), (i == 1) + (j == 1) + (k == 1), (i == 2) + (j == 2) + (k == 2)};
        return T[ew_idx(c[0], c[1], c[2]) - 10];
    };
    float tnn[3], tv[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        float sacc = 0.f;
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int k = 0; k < 3; k++) sacc = fmaf(t3(i, j, k), n[j] * n[k], sacc);
        tnn[i] = sacc;
        tv[i] = t3(i, 0, 0) + t3(i, 1, 1) + t3(i, 2, 2);
    }
    const float tnnn = nx * tnn[0] + ny * tnn[1] + nz * tnn[2], tn = nx * tv[0] + ny * tv[1] + nz * tv[2];
    const float c4 = (3.f * s3 * tn + s4 * tnnn) * (1.f / 6.f);
    const float h5 = r5;
    fx += h5 * (0.5f * (s2 * tv[0] + s3 * tnn[0]) + c4 * nx);
    fy += h5 * (0.5f * (s2 * tv[1] + s3 * tnn[1]) + c4 * ny);
    fz += h5 * (0.5f * (s2 * tv[2] + s3 * tnn[2]) + c4 * nz);
    float U[15];
#pragma unroll
    for (int a = 0; a < 15; a++) U[a] = (float)u4[a];
    auto u = [&](int i, int j, int k, int l) {
        const int c[3] = {(i == 0) + (j == 0) + (k == 0) + (l == 0), (i == 1) + (j == 1) + (k == 1) + (l == 1),
                          (i == 2) + (j == 2) + (k == 2) + (l == 2)};
        return U[ew_idx(c[0], c[1], c[2]) - 20];
    };
    float Wm[3][3], V[3][3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            Wm[i][j] = u(i, j, 0, 0) + u(i, j, 1, 1) + u(i, j, 2, 2);
            float sacc = 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++)
#pragma unroll
                for (int l = 0; l < 3; l++) sacc = fmaf(u(i, j, k, l), n[k] * n[l], sacc);
            V[i][j] = sacc;
        }
    float wn[3], vn[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        wn[i] = Wm[i][0] * nx + Wm[i][1] * ny + Wm[i][2] * nz;
        vn[i] = V[i][0] * nx + V[i][1] * ny + V[i][2] * nz;
    }
    const float w = Wm[0][0] + Wm[1][1] + Wm[2][2];
    const float nwn = nx * wn[0] + ny * wn[1] + nz * wn[2], unnnn = nx * vn[0] + ny * vn[1] + nz * vn[2];
    if (HI >= 5) {
        const float c5 = (3.f * s3 * w + 6.f * s4 * nwn + s5 * unnnn) * (1.f / 24.f);
        fx += r6 * ((12.f * s3 * wn[0] + 4.f * s4 * vn[0]) * (1.f / 24.f) + c5 * nx);
        fy += r6 * ((12.f * s3 * wn[1] + 4.f * s4 * vn[1]) * (1.f / 24.f) + c5 * ny);
        fz += r6 * ((12.f * s3 * wn[2] + 4.f * s4 * vn[2]) * (1.f / 24.f) + c5 * nz);
    }
    if (POT) fp += r5 * (3.f * s2 * w + 6.f * s3 * nwn + s4 * unnnn) * (1.f / 24.f);
}

// ---------------------------------------------------------------------------
// Decide-then-evaluate wavefront walk.
//
// A wavefront owns one group of up to 64 targets (one per lane) and keeps, in
// its own slice of LDS, the targets, their FP64 accumulators, the top of a
// traversal stack and rings of pending work.  A stack entry is a set of
// sibling nodes [first, first + c) together with the mask of target lanes that
// must look at them.  Every (node, target) pair of an entry gets one lane of a
// visit pass, so a pass is full however sparse the mask; each lane takes the
// per-target decision of the paper (drop beyond r_cut, open, or use the
// multipoles).  Accepted pairs go to the node ring, evaluated 64 at a time and
// added to the target's accumulator with an LDS atomic.  An opened leaf gives
// a (leaf, target) item in the leaf ring; a lane-level queue then walks each
// item's particles for its target, one pair per lane per step, refilling
// lanes as their items run out, and adds the item's sum once.  Opened internal
// nodes are collected per child into the masks of new stack entries.
// Before the visit passes of a large entry, each sibling is tested once
// against the bounding box of the group's targets: a sibling that every
// target would use goes straight into the node ring for all targets of the
// mask, one that every target would drop (beyond r_cut) is skipped, and only
// the rest get per-target slots.  The bounds reproduce the per-target tests
// (see group_decision), so every target's decisions are unchanged.
// ---------------------------------------------------------------------------

// Stack depth bound (entries of 16 bytes; the constants are in g4_internal.h):
// entries hold sibling nodes of one level, 0..G4_MAXLEV; processing an entry
// pushes at most 8, and at most 7 of them wait per level below the current
// path, so at most 7 (G4_MAXLEV - 1) + 8 entries are live after the root's.
// The top entries (WK_LDS_STK, or fewer if asked for) live in LDS, deeper ones
// in a per-wavefront spill area of the tree workspace.
#define WK_STK G4_WALK_STACK
#define WK_LDS_STK G4_WALK_LDS_STACK
#define WK_SPILL G4_WALK_SPILL
#define WK_RING 128  // ring capacity: < 64 pending before an append of <= 64

#define NUM_LEAF (1u << 31)  // leaf bit of VisitRec::numleaf
// Entries with fewer (child, target) slots than this skip the decisions for the
// whole group (their cost per entry outweighs the visit passes they save).
#define WK_GROUP_MIN_SLOTS 128

// Per-child visit record, staged in LDS for the passes over one entry.
struct __attribute__((aligned(16))) VisitRec {
    uint32_t cx, cy, cz;
    float crit;         // relative: M l^p; geometric: l^2; +inf at level 0 (the root is never used)
    uint32_t gx, gy, gz;
    int32_t lm1;        // exclusion: cube half-size on the grid minus 1 (-1: no exclusion zone)
    float hl;           // half side (physical); negative: every target is within r_cut of the cube (no test)
    uint32_t node;      // node index
    uint32_t next;      // first child, or first particle of a leaf
    uint32_t numleaf;   // number of children or particles, NUM_LEAF for a leaf
};
static_assert(sizeof(VisitRec) == 48, "VisitRec is 48 bytes");

// One wavefront's LDS: 5848 bytes without the potential (7 wavefronts per
// SIMD fit in the 160 KiB of a CU), 6360 with it.
#define FLAG_OPEN 1
#define FLAG_USE 2
template <bool POT>
struct __attribute__((aligned(16))) WaveLds {
    uint4 tgt[64];                 // target x, y, z (grid) and alpha |a_old| (bits)
    double acc[POT ? 4 : 3][64];   // a_x, a_y, a_z (, potential), before the factor G, component-major
    uint32_t pm_idx[WK_RING];      // node of each pending particle-node pair
    uint32_t lt_first[WK_RING];    // first particle of each pending opened leaf
    uint32_t lt_num[WK_RING];      // its particle count
    uint8_t pm_tgt[WK_RING];       // target lane of each pending particle-node pair
    uint8_t lt_tgt[WK_RING];       // target lane of each pending opened leaf
    VisitRec rec[8];               // children of the current entry
    uint8_t flag[8][64];           // flag[j][t]: FLAG_OPEN / FLAG_USE of child j for target t (t in the mask)
    uint8_t rmap[64];              // rank within the entry mask -> lane
    uint8_t anyopen[8];            // anyopen[j]: some target opened child j, an internal node
    int32_t gbox[6];               // the group's bounding box: lower x y z, upper x y z (offsets from target 0)
    float gamin;                   // its smallest alpha |a| (relative criterion); negative: no group decisions
    uint4 stk[WK_LDS_STK];         // (first node, count, mask lo, mask hi), top of the stack
};

// mask of the active lanes for which c holds
__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// readfirstlane/readlane return int: go through uint32_t so no half of a mask sign-extends
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint32_t lane_val(uint32_t x, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}
__device__ __forceinline__ void wave_sync_lds()
{
    // LDS operations of one wavefront execute in order; this only keeps the
    // compiler from moving LDS accesses across the point.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// M (l/r)^p / r^2 < alpha |a|  <=>  M l^p < alpha |a| r^(p+2): r^(p+2) from r^2 and 1/r
template <bool ORD3, int HI>
__device__ __forceinline__ float crit_rpow(float r2, float rinv)
{
    return HI == 5 ? r2 * r2 * r2 * r2 * rinv : (HI == 4 ? r2 * r2 * r2 : (ORD3 ? r2 * r2 * r2 * rinv : r2 * r2));
}

// The decisions of a visit taken once for every target of the group: 1 if
// every target uses the node, 2 if every target drops it (beyond r_cut), 0 if
// the targets must decide one by one, 4 if they must but none of them can find
// the node's cube beyond r_cut (the kernels with a cut-off).  box: the group's
// bounding box on the grid as offsets from target 0 (t0), lower corner in
// box[0..2], upper in box[3..5]; amin: the group's smallest alpha |a|.
// Each bound evaluates the per-target expression of the visit pass with the
// box's least (or most) favourable offsets in place of the target's; rounding
// is monotonic in every operation there, so a bound that passes implies the
// same outcome for every target.  The one exception, the hardware reciprocal
// square root of the relative criterion, is covered by a margin of 1e-5.  The
// offsets of a target are int32 differences modulo 2^32; the bounds apply only
// where none of them can wrap (node and centre of mass within 2^30 grid steps
// of target 0, box within 2^29).
template <int KER, int CRIT, bool ORD3, int HI>
__device__ __forceinline__ uint32_t group_decision(const WalkArgs &A, const WNode &nd, float crit, float hl,
                                                   int32_t lm1, uint4 t0, const int32_t *box, float amin)
{
    const int32_t lim = 1 << 30;
    bool safe = true, outside = false;
    float sn = 0.f, sf = 0.f, r2 = 0.f;  // sums over the axes z, y, x (the visit's order of operations)
#pragma unroll
    for (int a = 2; a >= 0; a--) {
        const int32_t gq = (int32_t)((a == 0 ? nd.gx : a == 1 ? nd.gy : nd.gz) - (a == 0 ? t0.x : a == 1 ? t0.y : t0.z));
        const int32_t cq = (int32_t)((a == 0 ? nd.cx : a == 1 ? nd.cy : nd.cz) - (a == 0 ? t0.x : a == 1 ? t0.y : t0.z));
        const int32_t b0 = box[a], b1 = box[3 + a];
        safe = safe && gq > -lim && gq < lim && cq > -lim && cq < lim;
        // nearest and farthest offsets of the box from the node's centre, nearest from its centre of mass
        const int32_t dmin = max(max(b0 - gq, gq - b1), 0);
        const int32_t dmax = max(gq - b0, b1 - gq);
        const int32_t cmin = max(max(b0 - cq, cq - b1), 0);
        outside = outside || dmin > lm1;  // no target inside the exclusion cube
        const float qn = fmaxf(fmaf((float)dmin, A.unit, -hl), 0.f);
        const float qf = fmaxf(fmaf((float)dmax, A.unit, -hl), 0.f);
        const float cm = (float)cmin * A.unit;
        sn = a == 2 ? qn * qn : fmaf(qn, qn, sn);
        sf = a == 2 ? qf * qf : fmaf(qf, qf, sf);
        r2 = a == 2 ? cm * cm : fmaf(cm, cm, r2);
    }
    if (!safe) return 0u;
    if (KER == 1 || KER == 2) {
        if (sn > A.rcut2) return 2u;
        if (!(sf <= A.rcut2)) return 0u;
    }
    const uint32_t within = (KER == 1 || KER == 2) ? 4u : 0u;  // no target can drop the node
    if (!outside || !(r2 >= A.h2)) return within;
    if (CRIT == 0) return crit < A.theta2 * r2 ? 1u : within;
    return crit < (amin * crit_rpow<ORD3, HI>(r2, rsq(r2))) * 0.99999f ? 1u : within;
}

// 64 particle-node interactions from the node ring, one per lane (lanes >= n idle).
template <int KER, bool POT, bool ORD3, int HI = 0>
__device__ __forceinline__ void eval_p2m(const WalkArgs &A, WaveLds<POT> &W, uint32_t head, uint32_t n, int lane)
{
    if ((uint32_t)lane >= n) return;
    const uint32_t q = (head + lane) & (WK_RING - 1);
    const uint32_t node = W.pm_idx[q], t = W.pm_tgt[q];
    const uint4 T = W.tgt[t];
    const WNode *nd = A.wn + node;
    const uint4 c4 = *reinterpret_cast<const uint4 *>(nd);
    const float4 qa = *reinterpret_cast<const float4 *>(&nd->q[0]);
    const float2 qb = *reinterpret_cast<const float2 *>(&nd->q[4]);
    const float mass = __uint_as_float(c4.w);
    const float dx = (float)(int32_t)(c4.x - T.x) * A.unit;
    const float dy = (float)(int32_t)(c4.y - T.y) * A.unit;
    const float dz = (float)(int32_t)(c4.z - T.z) * A.unit;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float rinv = rsq(r2);
    float g0, g1, g2, g3;
    gfun<KER>(r2, rinv, A, g0, g1, g2, g3);
    float fx, fy, fz, fp = 0.f;
    // Q2 packed xx xy xz yy yz zz
    const float qx = fmaf(qa.x, dx, fmaf(qa.y, dy, qa.z * dz));
    const float qy = fmaf(qa.y, dx, fmaf(qa.w, dy, qb.x * dz));
    const float qz = fmaf(qa.z, dx, fmaf(qb.x, dy, qb.y * dz));
    const float rqr = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    const float tr = qa.x + qa.w + qb.y;
    // the node's contribution is -(fx, fy, fz): the sign goes into the FP64 conversion below
    if (ORD3) {
        const float fac = fmaf(mass, g1, 0.5f * fmaf(g2, tr, g3 * rqr));
        fx = fmaf(fac, dx, g2 * qx);
        fy = fmaf(fac, dy, g2 * qy);
        fz = fmaf(fac, dz, g2 * qz);
        if (POT) {
            const float *o = A.q3 + (size_t)node * 10;
            // Q3 . D3 = 3 g2 (t . r) + g3 Q3(r, r, r), t_k = sum_i Q3_iik
            const float tx = o[0] + o[3] + o[5], ty = o[1] + o[6] + o[8], tz = o[2] + o[7] + o[9];
            const float c3 = o[0] * dx * dx * dx + o[6] * dy * dy * dy + o[9] * dz * dz * dz +
                             3.f * (o[1] * dx * dx * dy + o[2] * dx * dx * dz + o[3] * dx * dy * dy +
                                    o[5] * dx * dz * dz + o[7] * dy * dy * dz + o[8] * dy * dz * dz) +
                             6.f * o[4] * dx * dy * dz;
            const float q3d3 = 3.f * g2 * (tx * dx + ty * dy + tz * dz) + g3 * c3;
            fp = mass * g0 + 0.5f * (g1 * tr + g2 * rqr) + q3d3 * (1.0f / 6.0f);
        }
    } else {
        const float fac = mass * g1;
        fx = fac * dx;
        fy = fac * dy;
        fz = fac * dz;
        if (POT) fp = mass * g0 + 0.5f * (g1 * tr + g2 * rqr);
    }
    if constexpr (HI >= 4) {
        float s2, s3, s4, s5;
        sfun_hi<KER>(r2 * rinv, A, s2, s3, s4, s5);
        eval_high<HI, POT>(A.q3 + (size_t)node * 10, A.q4 + (size_t)node * 15, dx * rinv, dy * rinv, dz * rinv, rinv,
                           s2, s3, s4, s5, fx, fy, fz, fp);
    }
    if constexpr (KER == 3) {
        // the other images: g = 1/r - psi, so the node adds +f (force) and +phi_psi (potential)
        float cx, cy, cz, cp = 0.f;
        ew_node<POT, ORD3>(A.ew, A.ew_n, A.ew_h, A.ew_hinv, dx, dy, dz, mass, qa, qb, A.q3 + (size_t)node * 10, cx, cy,
                           cz, cp);
        fx -= cx;
        fy -= cy;
        fz -= cz;
        if (POT) fp -= cp;
    }
    lds_add(&W.acc[0][t], -(double)fx);
    lds_add(&W.acc[1][t], -(double)fy);
    lds_add(&W.acc[2][t], -(double)fz);
    if constexpr (POT) lds_add(&W.acc[3][t], -(double)fp);
}

// Wavefronts per SIMD the register budget must allow: the LDS of the walks
// without the potential leaves room for 7, which the Newtonian and TreePM
// kernels at p <= 3 reach within 72 VGPRs without spilling; the others keep
// the compiler's own choice.
#define WALK_MIN_WAVES(KER, POT, HI) ((!(POT) && (KER) <= 1 && (HI) == 0) ? 7 : 1)

// ORD3: p = 3, the force includes the quadrupole term (p = 2: monopole force);
// HI = 4 or 5: the orders above (ORD3 set as well)
template <int KER, int CRIT, bool POT, bool ORD3, int HI = 0>
__global__ __launch_bounds__(256, WALK_MIN_WAVES(KER, POT, HI)) void k_walk(const WalkArgs A)
{
    __shared__ WaveLds<POT> lds[4];
    const int lane = threadIdx.x & 63;
    WaveLds<POT> &W = lds[threadIdx.x >> 6];
    uint4 *const spill = A.spill + (size_t)(blockIdx.x * 4 + (threadIdx.x >> 6)) * WK_SPILL;
    uint32_t t_pp = 0;                                 // per-lane total of particle-particle pairs
    uint32_t u_pm = 0, u_visit = 0;                    // wavefront totals (per launch < 2^32 per wave)
    uint32_t w_pass = 0, w_pm = 0, w_pp = 0;           // 64-lane steps: visits, node pairs, particle pairs
    int max_sp = 0;                                    // deepest stack seen
    uint32_t w_entry = 0, w_leaf = 0, w_phase = 0;     // sibling sets, (leaf, target) items, pair phases
    uint32_t g_use = 0, g_drop = 0;                    // (node, target) pairs decided for the whole group

    for (;;) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(A.item_ctr, 1u);
    it = uni(it);  // all lanes are active here, so the first lane is lane 0
    if (it >= A.nitems) break;
    int64_t i0;
    uint32_t gcount, root;
    if (A.items) {
        const uint4 w = A.items[it];
        i0 = uni(w.x);
        gcount = uni(w.y);
        root = uni(w.z);
    } else {
        i0 = (int64_t)it * A.group;
        gcount = (uint32_t)min((int64_t)A.group, A.n - i0);
        root = 0;
    }
    const int64_t i = i0 + lane;
    const bool act = (uint32_t)lane < gcount;
    uint4 me = make_uint4(0u, 0u, 0u, 0u);
    float arel = __builtin_huge_valf();
    if (act) {
        me = A.parts[i];
        arel = CRIT == 1 ? A.alpha * A.aseed[i] : 0.f;
        W.tgt[lane] = make_uint4(me.x, me.y, me.z, __float_as_uint(arel));
    }
    {
        // the group's bounding box as offsets from target 0 (every group has it) and its
        // smallest alpha |a|, for the decisions taken once for the whole group
        const uint32_t t0x = uni(me.x), t0y = uni(me.y), t0z = uni(me.z);
        int32_t lo[3] = {act ? (int32_t)(me.x - t0x) : 0, act ? (int32_t)(me.y - t0y) : 0,
                         act ? (int32_t)(me.z - t0z) : 0};
        int32_t hi[3] = {lo[0], lo[1], lo[2]};
        // a seed that is not a non-negative number (NaN) would make the bound unsafe: no group decisions
        float am = arel >= 0.f ? arel : -1.f;
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int a = 0; a < 3; a++) {
                lo[a] = min(lo[a], __shfl_xor(lo[a], off));
                hi[a] = max(hi[a], __shfl_xor(hi[a], off));
            }
            am = fminf(am, __shfl_xor(am, off));
        }
        const int32_t ext = max(max(max(-lo[0], hi[0]), max(-lo[1], hi[1])), max(-lo[2], hi[2]));
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < 3; a++) {
                W.gbox[a] = lo[a];
                W.gbox[3 + a] = hi[a];
            }
            W.gamin = ext < (1 << 29) && am >= 0.f ? (CRIT == 1 ? am : 0.f) : -1.f;
        }
    }
    W.acc[0][lane] = 0.0;
    W.acc[1][lane] = 0.0;
    W.acc[2][lane] = 0.0;
    if constexpr (POT) W.acc[3][lane] = 0.0;
    const uint64_t amask = ballot(act);
    if (lane == 0) W.stk[0] = make_uint4(root, 1u, (uint32_t)amask, (uint32_t)(amask >> 32));
    uint32_t n_pp = 0, n_pm = 0;                      // counts of target `lane` (only with A.counts)
    int sp = 1;
    uint32_t pm_h = 0, pm_t = 0, lt_h = 0, lt_t = 0;  // ring heads and tails (uniform)
    // this lane's (leaf, target) item: next source, sources left, target lane and position, partial sums
    uint32_t q_src = 0, q_rem = 0, q_t = 0, q_self = 0;
    uint32_t q_x = 0, q_y = 0, q_z = 0;
    float q_fx = 0.f, q_fy = 0.f, q_fz = 0.f, q_fp = 0.f;
    wave_sync_lds();

    // Particle pairs from the leaf ring: idle lanes take the next items in ring
    // order; every step evaluates one pair per busy lane.  Without `drain` the
    // phase ends as soon as a lane cannot be refilled, so every step is full;
    // lanes keep their unfinished items for the next phase.
    // One pair for every lane that holds an item.  The target itself is among
    // the sources of its own leaf: its separation is zero, where the kernel
    // is finite, so its force term is exactly zero and only the potential
    // needs the mass masked.
    auto pair_step = [&]() {
        const uint4 src = A.parts[q_src];
        const float mj = (POT && q_src == q_self) ? 0.f : __uint_as_float(src.w);
        const float sx = (float)(int32_t)(src.x - q_x) * A.unit;
        const float sy = (float)(int32_t)(src.y - q_y) * A.unit;
        const float sz = (float)(int32_t)(src.z - q_z) * A.unit;
        const float s2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
        float K, Wp;
        if constexpr (KER == 2) pair_kernel_tab<POT>(s2, A.tab, A.tn, A.tscale, A.asplit, A.h2, A.hinv, K, Wp);
        else pair_kernel<KER == 3 ? 0 : KER, POT>(s2, A.asplit, A.h2, A.hinv, K, Wp);
        const float mk = mj * K;
        q_fx = fmaf(mk, sx, q_fx);
        q_fy = fmaf(mk, sy, q_fy);
        q_fz = fmaf(mk, sz, q_fz);
        if (POT) q_fp = fmaf(-mj, Wp, q_fp);
        if constexpr (KER == 3) {
            // + m grad psi(d), + m psi(d) (grad psi(0) = 0, so the target's own slot adds nothing)
            float ex, ey, ez, ep = 0.f;
            ew_grad<POT>(A.ew, A.ew_n, A.ew_h, A.ew_hinv, sx, sy, sz, ex, ey, ez, ep);
            q_fx = fmaf(mj, ex, q_fx);
            q_fy = fmaf(mj, ey, q_fy);
            q_fz = fmaf(mj, ez, q_fz);
            if (POT) q_fp = fmaf(mj, ep, q_fp);
        }
        q_src++;
        q_rem--;
        if (q_rem == 0) {
            lds_add(&W.acc[0][q_t], (double)q_fx);
            lds_add(&W.acc[1][q_t], (double)q_fy);
            lds_add(&W.acc[2][q_t], (double)q_fz);
            if constexpr (POT) lds_add(&W.acc[3][q_t], (double)q_fp);
            q_fx = q_fy = q_fz = q_fp = 0.f;
        }
    };
    auto run_pairs = [&](bool drain) {
        w_phase++;
        for (;;) {
            const uint64_t idle = ballot(q_rem == 0);
            const uint32_t avail = lt_t - lt_h;
            if (idle && avail) {
                const uint32_t r = lanes_below(idle);
                if (q_rem == 0 && r < avail) {
                    const uint32_t q = (lt_h + r) & (WK_RING - 1);
                    q_src = W.lt_first[q];
                    q_rem = W.lt_num[q];
                    q_t = W.lt_tgt[q];
                    const uint4 T = W.tgt[q_t];
                    q_x = T.x;
                    q_y = T.y;
                    q_z = T.z;
                    q_self = (uint32_t)i0 + q_t;  // sorted index of the target itself
                    if (A.stat) {
                        // the pair count only when it is read; the empty statement keeps the
                        // count behind the branch instead of a select after it
                        uint32_t nq = q_rem;
                        asm volatile("" : "+v"(nq));
                        t_pp += nq - ((q_self - q_src) < nq ? 1u : 0u);
                    }
                }
                lt_h += min((uint32_t)__builtin_popcountll(idle), avail);
            }
            const uint64_t busy = ballot(q_rem != 0);
            if (drain) {
                if (!busy) break;
                w_pp++;
                if (q_rem != 0) pair_step();
            } else {
                // every lane holds an item (busy is all ones)
                if (busy != ~0ull) break;
                w_pp++;
                pair_step();
            }
        }
    };

    while (sp > 0) {
        // ---- pop an entry: nodes [first, first + c) for the lanes in mask m; stage the nodes ----
        sp--;
        w_entry++;
        uint4 e;
        if (sp < A.lds_stk) {
            e = W.stk[sp];
        } else {
            // deeper entries were written by lane 0; lane 0 reads them back
            e = make_uint4(0u, 0u, 0u, 0u);
            if (lane == 0) e = spill[sp - A.lds_stk];
        }
        const uint32_t first = uni(e.x), c = uni(e.y);
        const uint64_t m = ((uint64_t)uni(e.w) << 32) | (uint64_t)uni(e.z);
        const uint32_t k = (uint32_t)__builtin_popcountll(m);
        // p / k for p < 576 as the float fma(p, 1/k, 1/2k), exact with the hardware reciprocal
        const float invk = rcp((float)k), hinvk = 0.5f * invk;
        if ((m >> lane) & 1ull) W.rmap[lanes_below(m)] = (uint8_t)lane;
        uint32_t v_next = 0, v_numleaf = 0;  // lane j < c: child j (after the decisions below: the
                                             // j-th of the children the targets decide one by one)
        uint32_t v_dec = 0;                  // lane j < c: 1 every target uses child j, 2 every target drops it
        if ((uint32_t)lane < c) {
            VisitRec r;
            const WNode nd = A.wn[first + lane];
            const int level = (int)(nd.meta & 0xffu);
            const float l = ldexpf(A.box, -level);
            r.cx = nd.cx;
            r.cy = nd.cy;
            r.cz = nd.cz;
            if (level == 0) r.crit = __builtin_huge_valf();
            else if (CRIT == 0) r.crit = l * l;
            else r.crit = nd.mass * (HI == 5 ? l * l * l * l * l : (HI == 4 ? l * l * l * l : (ORD3 ? l * l * l : l * l)));
            r.gx = nd.gx;
            r.gy = nd.gy;
            r.gz = nd.gz;
            r.lm1 = ((A.exclusion & 1) && level > 0) ? (int32_t)((1u << (A.S - level)) - 1u) : -1;
            r.hl = 0.5f * l;
            r.node = first + lane;
            r.next = nd.next;
            r.numleaf = nd.num | ((nd.meta & WN_LEAF) ? NUM_LEAF : 0u);
            v_next = r.next;
            v_numleaf = r.numleaf;
            W.rec[lane] = r;
            const float gamin = W.gamin;
            if (c * k >= WK_GROUP_MIN_SLOTS && !(A.exclusion & 2) && level > 0 && gamin >= 0.f) {
                v_dec = group_decision<KER, CRIT, ORD3, HI>(A, nd, r.crit, r.hl, r.lm1, W.tgt[0], W.gbox, gamin);
                if (v_dec == 4u) {
                    // left to the targets, none of which can see the cube beyond r_cut
                    W.rec[lane].hl = -r.hl;
                    v_dec = 0;
                }
            }
        }
        // the children left to the targets get consecutive records, slots and child registers;
        // the node indices of the children every target uses follow them (in the records' node field)
        uint32_t cmix = c, uslots = 0;
        const uint64_t decm = ballot(v_dec != 0);
        if (decm) {
            const bool pert = (uint32_t)lane < c && v_dec == 0, guse = v_dec == 1u;
            const uint64_t mixm = ballot(pert), usem = ballot(guse);
            cmix = (uint32_t)__builtin_popcountll(mixm);
            uslots = (uint32_t)__builtin_popcountll(usem) * k;
            g_drop += k * (uint32_t)__builtin_popcountll(ballot(v_dec == 2u));
            if (A.counts && ((m >> lane) & 1ull)) n_pm += (uint32_t)__builtin_popcountll(usem);
            wave_sync_lds();
            const uint4 *src = reinterpret_cast<const uint4 *>(&W.rec[lane & 7]);
            const uint4 r0 = src[0], r1 = src[1], r2 = src[2];
            wave_sync_lds();
            if (pert) {
                uint4 *dst = reinterpret_cast<uint4 *>(&W.rec[lanes_below(mixm)]);
                dst[0] = r0;
                dst[1] = r1;
                dst[2] = r2;
            }
            if (guse) W.rec[cmix + lanes_below(usem)].node = first + lane;
            wave_sync_lds();
            v_next = (uint32_t)lane < cmix ? W.rec[lane].next : 0u;
            v_numleaf = (uint32_t)lane < cmix ? W.rec[lane].numleaf : 0u;
        }
        const uint32_t slots = cmix * k, ubase = (uslots + 63u) & ~63u;
        if (lane == 0) *reinterpret_cast<uint2 *>(W.anyopen) = make_uint2(0u, 0u);
        wave_sync_lds();

        // ---- children every target uses: their (node, target) pairs go straight into the node
        // ring, 64 at a time; then visit passes, 64 (child, target) slots at a time ----
        for (uint32_t base = 0; base < ubase + slots; base += 64) {
          if (base < ubase) {
            const uint32_t p = base + lane;
            if (p < uslots) {
                const uint32_t u = (uint32_t)fmaf((float)p, invk, hinvk);
                const uint32_t q = (pm_t + lane) & (WK_RING - 1);
                W.pm_idx[q] = W.rec[cmix + u].node;
                W.pm_tgt[q] = W.rmap[p - u * k];
            }
            const uint32_t nu = min(64u, uslots - base);
            pm_t += nu;
            u_pm += nu;
            u_visit += nu;
            g_use += nu;
          } else {
            const uint32_t p = base - ubase + lane;
            const bool valid = p < slots;
            uint32_t j = (uint32_t)fmaf((float)p, invk, hinvk);
            uint32_t rank = p - j * k;
            if (!valid) j = rank = 0;
            const uint32_t t = W.rmap[rank];
            const uint4 T = W.tgt[t];
            const VisitRec R = W.rec[j];
            const float dx = (float)(int32_t)(R.cx - T.x) * A.unit;
            const float dy = (float)(int32_t)(R.cy - T.y) * A.unit;
            const float dz = (float)(int32_t)(R.cz - T.z) * A.unit;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            // offsets from the cube centre (grid units): |d| < half-size on all axes is the
            // exclusion zone; the nearest-edge distance is max(|d| unit - l/2, 0) per axis
            const int32_t gx = (int32_t)(R.gx - T.x), gy = (int32_t)(R.gy - T.y), gz = (int32_t)(R.gz - T.z);
            bool ok = valid;
            if ((KER == 1 || KER == 2) && R.hl >= 0.f) {
                // nearest edge of the node's cube farther than r_cut: drop it
                const float qx = fmaxf(fmaf(fabsf((float)gx), A.unit, -R.hl), 0.f);
                const float qy = fmaxf(fmaf(fabsf((float)gy), A.unit, -R.hl), 0.f);
                const float qz = fmaxf(fmaf(fabsf((float)gz), A.unit, -R.hl), 0.f);
                ok = ok && (fmaf(qx, qx, fmaf(qy, qy, qz * qz)) <= A.rcut2);
            }
            const bool inside = max(gx, max(gy, gz)) <= R.lm1 && min(gx, min(gy, gz)) >= -R.lm1;
            const float rinv = rsq(r2);
            bool accept = !inside && r2 >= A.h2;
            if (CRIT == 0) {
                accept = accept && (R.crit < A.theta2 * r2);
            } else {
                accept = accept && (R.crit < __uint_as_float(T.w) * crit_rpow<ORD3, HI>(r2, rinv));
            }
            const bool use = ok && accept;
            const bool open = ok && !accept;
            const uint64_t um = ballot(use);
            if (use) {
                const uint32_t q = (pm_t + lanes_below(um)) & (WK_RING - 1);
                W.pm_idx[q] = R.node;
                W.pm_tgt[q] = (uint8_t)t;
            }
            // opened leaves become (leaf, target) items
            const bool oleaf = open && (R.numleaf & NUM_LEAF);
            const uint64_t lm = ballot(oleaf);
            if (lm) {
                if (oleaf) {
                    const uint32_t q = (lt_t + lanes_below(lm)) & (WK_RING - 1);
                    W.lt_first[q] = R.next;
                    W.lt_num[q] = R.numleaf & ~NUM_LEAF;
                    W.lt_tgt[q] = (uint8_t)t;
                }
                const uint32_t nl = (uint32_t)__builtin_popcountll(lm);
                lt_t += nl;
                w_leaf += nl;
            }
            // every (child, target) pair of the entry has exactly one slot: no clearing needed
            if (valid) W.flag[j][t] = (uint8_t)(use ? FLAG_USE : (open ? FLAG_OPEN : 0));
            if (open && !(R.numleaf & NUM_LEAF)) W.anyopen[j] = 1;
            const uint32_t nu = (uint32_t)__builtin_popcountll(um);
            pm_t += nu;
            u_pm += nu;
            u_visit += (uint32_t)__builtin_popcountll(ballot(ok));
            w_pass++;
          }
            if (pm_t - pm_h >= 64) {
                wave_sync_lds();
                eval_p2m<KER, POT, ORD3, HI>(A, W, pm_h, 64u, lane);
                pm_h += 64;
                w_pm++;
            }
            if (lt_t - lt_h >= 64) {
                wave_sync_lds();
                run_pairs(false);
            }
        }
        wave_sync_lds();

        // ---- interaction counts per target (only if asked for) ----
        const bool inm = (m >> lane) & 1ull;
        if (A.counts) {
            for (uint32_t jj = 0; jj < cmix; jj++) {
                const uint32_t next = lane_val(v_next, jj), nl = lane_val(v_numleaf, jj);
                const uint32_t num = nl & ~NUM_LEAF;
                const uint32_t f = W.flag[jj][lane];
                n_pm += (inm && f == FLAG_USE) ? 1u : 0u;
                if ((nl & NUM_LEAF) && inm && f == FLAG_OPEN) n_pp += num - ((uint32_t)(i - next) < num ? 1u : 0u);
            }
        }
        // ---- opened internal children become entries ----
        const uint2 ao = *reinterpret_cast<const uint2 *>(W.anyopen);
        uint64_t anyb = ((uint64_t)uni(ao.y) << 32) | (uint64_t)uni(ao.x);
        while (anyb) {
            const uint32_t jj = (uint32_t)__builtin_ctzll(anyb) >> 3;
            anyb &= ~(0xffull << (8 * jj));
            const uint32_t next = lane_val(v_next, jj), num = lane_val(v_numleaf, jj) & ~NUM_LEAF;
            const uint64_t om = ballot(W.flag[jj][lane] == FLAG_OPEN) & m;
            if (sp < WK_STK) {
                const uint4 ne = make_uint4(next, num, (uint32_t)om, (uint32_t)(om >> 32));
                if (lane == 0) {
                    if (sp < A.lds_stk) W.stk[sp] = ne;
                    else spill[sp - A.lds_stk] = ne;
                }
                sp++;
                max_sp = max(max_sp, sp);
            } else if (lane == 0) {
                // beyond the depth bound above: never expected, but never silent
                atomicOr(A.flags, G4_FLAG_WALK_STACK);
            }
        }
    }
    // ---- drain the rings ----
    wave_sync_lds();
    while (pm_t != pm_h) {
        const uint32_t n = min(pm_t - pm_h, 64u);
        eval_p2m<KER, POT, ORD3, HI>(A, W, pm_h, n, lane);
        pm_h += n;
        w_pm++;
    }
    run_pairs(true);
    wave_sync_lds();

    if (act) {
        const uint32_t o = A.perm[i];
        const double gx = A.G * W.acc[0][lane], gy = A.G * W.acc[1][lane], gz = A.G * W.acc[2][lane];
        A.ax[o] = gx;
        A.ay[o] = gy;
        A.az[o] = gz;
        if constexpr (POT) {
            if (A.pot) A.pot[o] = A.G * W.acc[3][lane];
        }
        const float amag = (float)sqrt(gx * gx + gy * gy + gz * gz);
        if (A.aout_sorted) A.aout_sorted[i] = amag;
        if (A.aout_caller) A.aout_caller[o] = amag;
        if (A.counts) {
            A.counts[2 * (size_t)o] = n_pp;
            A.counts[2 * (size_t)o + 1] = n_pm;
        }
    }
    wave_sync_lds();
    }  // work items
    if (A.stat) {
        // wavefront sums of the interaction counters, one atomic per wavefront
        unsigned long long s0 = t_pp;
        for (int off = 32; off > 0; off >>= 1) s0 += __shfl_xor(s0, off);
        if (lane == 0) {
            atomicAdd(&A.stat[0], s0);
            atomicAdd(&A.stat[1], (unsigned long long)u_pm);
            atomicAdd(&A.stat[2], (unsigned long long)u_visit);
            // 64-lane steps of each kind, the deepest stack and the bookkeeping counts (slots 9..15
            // of the counter block, walk call only)
            if (A.wstat) {
                atomicAdd(&A.wstat[0], (unsigned long long)w_pass);
                atomicAdd(&A.wstat[1], (unsigned long long)w_pm);
                atomicAdd(&A.wstat[2], (unsigned long long)w_pp);
                atomicMax(&A.wstat[3], (unsigned long long)max_sp);  // slot 12
                atomicAdd(&A.wstat[4], (unsigned long long)w_entry);
                atomicAdd(&A.wstat[5], (unsigned long long)w_leaf);
                atomicAdd(&A.wstat[6], (unsigned long long)w_phase);
                atomicAdd(&A.wstat[7], (unsigned long long)g_use);  // slots 16, 17
                atomicAdd(&A.wstat[8], (unsigned long long)g_drop);
            }
        }
    }
}

template <int KER, int CRIT, bool POT>
static void launch_walk(const WalkArgs &A, hipStream_t s)
{
    // persistent grid: 4 wavefronts per block, each with its own spill area
    int64_t blocks = ((int64_t)A.nitems + 3) / 4;
    if (blocks > A.spill_waves / 4) blocks = A.spill_waves / 4;
    if (blocks < 1) blocks = 1;
    if constexpr (KER <= 1) {
        if (A.order == 5) {
            k_walk<KER, CRIT, POT, true, 5><<<(unsigned)blocks, 256, 0, s>>>(A);
            return;
        }
        if (A.order == 4) {
            k_walk<KER, CRIT, POT, true, 4><<<(unsigned)blocks, 256, 0, s>>>(A);
            return;
        }
    }
    if (A.order >= 3) k_walk<KER, CRIT, POT, true><<<(unsigned)blocks, 256, 0, s>>>(A);
    else k_walk<KER, CRIT, POT, false><<<(unsigned)blocks, 256, 0, s>>>(A);
}

// Cubic Hermite pieces of S_0..S_3 (see pair_kernel_tab) on n intervals of
// x in [0, G4_SRTAB_XMAX], from FP64 values and derivatives at the interval
// ends; dS_f/dx = -2^(f+1) x^(2f) e^{-x^2} / ((2f-1)!! sqrt(pi)).
__device__ inline void sr_value(int f, double x, double &v, double &d)
{
    const double e = exp(-x * x), c = 1.1283791670955126;  // 2/sqrt(pi)
    const double x2 = x * x;
    const double P = f == 0 ? 0.0 : (f == 1 ? 1.0 : (f == 2 ? 1.0 + x2 * (2.0 / 3) : 1.0 + x2 * (2.0 / 3 + x2 * (4.0 / 15))));
    v = erfc(x) + c * x * e * P;
    const double dfac = f == 0 ? 1.0 : (f == 1 ? 2.0 * x2 : (f == 2 ? 4.0 / 3 * x2 * x2 : 8.0 / 15 * x2 * x2 * x2));
    d = -c * e * dfac;
}

__global__ void k_srtab(float4 *__restrict__ tab, int n)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= G4_SRTAB_FUNCS * n) return;
    const int f = idx / n, k = idx % n;
    const double dx = G4_SRTAB_XMAX / n;
    double f0, d0, f1, d1;
    sr_value(f, k * dx, f0, d0);
    sr_value(f, (k + 1) * dx, f1, d1);
    d0 *= dx;
    d1 *= dx;
    tab[idx] = make_float4((float)f0, (float)d0, (float)(3.0 * (f1 - f0) - 2.0 * d0 - d1),
                           (float)(2.0 * (f0 - f1) + d0 + d1));
}

int g4_launch_walk(g4_ctx *ctx, g4_tree *t, const g4_walk_params *wp, int kernel, int criterion, double *ax,
                   double *ay, double *az, double *pot, uint32_t *counts, float *aout_caller, float *aout_sorted,
                   int stat_slot, bool count)
{
    WalkArgs A;
    A.parts = t->parts;
    A.wn = t->wn;
    A.q3 = t->q3;
    A.aseed = t->aseed;
    A.perm = t->perm1;
    A.n = t->n;
    A.group = wp->group_size > 0 && wp->group_size <= 64 ? wp->group_size : 64;
    A.S = t->S;
    A.exclusion = wp->exclusion ? 1 : 0;
    A.order = wp->order;
    A.unit = (float)t->unit;
    A.box = (float)t->tp.box;
    const double h = 2.8 * wp->eps0;
    A.h = (float)h;
    A.h2 = (float)(h * h);
    A.hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    A.asplit = kernel == 1 ? (float)(0.5 / wp->r_s) : 0.f;
    const bool tabulated = kernel == 1 && wp->sr_table > 0;
    A.tab = t->srtab;
    A.tn = tabulated ? (uint32_t)wp->sr_table : 0u;
    A.tscale = tabulated ? (float)(0.5 / wp->r_s * wp->sr_table / G4_SRTAB_XMAX) : 0.f;
    if (tabulated && t->tab_n != wp->sr_table) {
        // the table is in units of x = alpha_split r, so it depends on its length only
        k_srtab<<<(G4_SRTAB_FUNCS * wp->sr_table + 63) / 64, 64, 0, ctx->stream>>>(t->srtab, wp->sr_table);
        G4_HIP(ctx, hipGetLastError());
        t->tab_n = wp->sr_table;
    }
    A.q4 = t->q4d;
    A.ew = static_cast<const float *>(wp->ewald_table);
    A.ew_n = wp->ewald_n;
    A.ew_h = kernel == 2 ? (float)(0.5 * t->tp.box / wp->ewald_n) : 0.f;
    A.ew_hinv = kernel == 2 ? (float)(2.0 * wp->ewald_n / t->tp.box) : 0.f;
    A.rcut2 = (float)(wp->r_cut * wp->r_cut);
    A.theta2 = (float)(criterion == 0 ? (wp->criterion == 0 ? wp->theta * wp->theta : wp->theta_seed * wp->theta_seed)
                                      : 0.0);
    A.alpha = (float)wp->alpha;
    A.G = wp->G;
    A.ax = ax;
    A.ay = ay;
    A.az = az;
    A.pot = pot;
    A.counts = counts;
    A.aout_caller = aout_caller;
    A.aout_sorted = aout_sorted;
    // interaction and pass counters only when the caller reads them: the kernel then skips
    // the per-lane counting as well
    A.stat = count ? t->ctr->stat + stat_slot : nullptr;
    if (t->nbox > 1 && t->items_group != A.group) {
        // work items of a forest: every box cut into groups; largest boxes first so the
        // persistent wavefronts finish together (longest-processing-time order)
        if (!t->items_host) {
            t->items_host = new (std::nothrow) uint4[t->items_cap];
            if (!t->items_host) return g4_set_err(ctx, G4_ENOMEM, "host allocation failed");
        }
        std::vector<int> order(t->nbox);
        for (int b = 0; b < t->nbox; b++) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return t->box_off[a + 1] - t->box_off[a] > t->box_off[b + 1] - t->box_off[b];
        });
        // wait for earlier work that may still read the previous items
        G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
        int64_t k = 0;
        for (int b : order)
            for (int64_t f = t->box_off[b]; f < t->box_off[b + 1]; f += A.group) {
                const int64_t c = std::min<int64_t>(A.group, t->box_off[b + 1] - f);
                t->items_host[k++] = make_uint4((uint32_t)f, (uint32_t)c, (uint32_t)b, 0u);
            }
        t->nitems = (uint32_t)k;
        t->items_group = A.group;
        G4_HIP(ctx, hipMemcpyAsync(t->items, t->items_host, (size_t)k * sizeof(uint4), hipMemcpyHostToDevice,
                                   ctx->stream));
    }
    if (t->nitems) {
        A.items = t->items;
        A.nitems = t->nitems;
    } else {
        A.items = nullptr;
        A.nitems = (uint32_t)((A.n + A.group - 1) / A.group);
    }
    A.item_ctr = &t->ctr->item_ctr;
    A.spill = t->walk_spill;
    A.spill_waves = t->walk_spill_waves;
    A.lds_stk = WK_LDS_STK;
    A.flags = &t->ctr->flags;
    if (const char *env = getenv("G4_WALK_PER_TARGET")) {
        // diagnostic: every (node, target) pair decided in the visit passes, none for the whole group
        if (atoi(env) != 0) A.exclusion |= 2;
    }
    if (const char *env = getenv("G4_WALK_LDS_STACK")) {
        // diagnostic: keep fewer entries in LDS so that the spill path runs
        const int v = atoi(env);
        if (v >= 1 && v <= WK_LDS_STK) A.lds_stk = v;
    }
    if (int st = g4_launch_zero(ctx, A.item_ctr, sizeof(uint32_t))) return st;
    A.wstat = count && stat_slot == 0 ? t->ctr->stat + 9 : nullptr;
    hipStream_t s = ctx->stream;
    const bool P = pot != nullptr;
    if (kernel == 0) {
        if (criterion == 0) { if (P) launch_walk<0, 0, true>(A, s); else launch_walk<0, 0, false>(A, s); }
        else { if (P) launch_walk<0, 1, true>(A, s); else launch_walk<0, 1, false>(A, s); }
    } else if (kernel == 2) {
        if (criterion == 0) { if (P) launch_walk<3, 0, true>(A, s); else launch_walk<3, 0, false>(A, s); }
        else { if (P) launch_walk<3, 1, true>(A, s); else launch_walk<3, 1, false>(A, s); }
    } else if (tabulated) {
        if (criterion == 0) { if (P) launch_walk<2, 0, true>(A, s); else launch_walk<2, 0, false>(A, s); }
        else { if (P) launch_walk<2, 1, true>(A, s); else launch_walk<2, 1, false>(A, s); }
    } else {
        if (criterion == 0) { if (P) launch_walk<1, 0, true>(A, s); else launch_walk<1, 0, false>(A, s); }
        else { if (P) launch_walk<1, 1, true>(A, s); else launch_walk<1, 1, false>(A, s); }
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
