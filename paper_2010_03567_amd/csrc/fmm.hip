// fmm.hip -- symmetric Cartesian fast multipole method at p = 3 on gfx950.
//
// Paper: Sec. "Fast multipole method": the interaction of two cells is
// expanded about both centres of mass, giving field expansions
// F_k = sum_n D_{n+k} . Q_n / n! at each side (the other side's expansion is
// the same formula with r -> -r), which conserves momentum; the node-node
// criterion (l_A + l_B)/r < theta (eq. eqnNodeDec); nodes that touch never
// interact; a cell's self-interaction is the interaction of all pairs of its
// daughters; the three phases (upward moments, dual walk storing field
// expansions, downward shift and evaluation at the particles).  Sec. "The
// FMM-PM approach": the short-range kernel with pairs dropped when their
// nearest sides are farther apart than r_cut.
//
// Mapping to the GPU.  The dual walk is a breadth-first frontier of entity
// pairs (nodes, or single particles once a leaf is opened).  Each pass
// classifies every pair and appends, with one atomic per wavefront per list,
// (a) new pairs to the next frontier or (b) per-target entries
// (target, source) entries: a node target collects the field of a node (M2L) or a
// particle (P2L); a particle target collects the force of a node (M2P), of a
// single particle, or of all particles of a leaf (P2P).  Both sides of every
// symmetric interaction become an entry; entries are sorted by target and,
// within a target, by the source's first particle and level, so each target
// sums its own list in an order that depends neither on the order of
// appends nor on node numbering: no floating-point atomics, bitwise
// reproducible.  Then L2L runs level by level and one pass per particle does
// M2P + P2P + L2P with FP64 accumulation.
#include <cstring>


#include "ewald.h"
#include "g4_device.h"
#include "g4_internal.h"

#define PF 0x80000000u           // frontier entity: particle (sorted index) when set
#define ENT_NODE 0x00000000u     // entry source types (top two bits)
#define ENT_PART 0x40000000u
#define ENT_LEAF 0x80000000u
#define ENT_IDX(e) ((e) & 0x3fffffffu)
#define ENT_TYPE(e) ((e) & 0xc0000000u)

struct FmmArgs {
    const WNode *wn;
    const uint32_t *bfirst;  // first particle of each node
    const uint4 *parts;
    const float *q3;
    const DevCounters *ctr;
    const uint32_t *parent;
    int S;
    float unit, box;
    float theta, h2, asplit, hinv, rcut2;
    int kernel;
    int crit;            // 0 geometric, 1 relative node-node criterion
    float alpha;
    const float *pseed;  // |a| per particle (sorted order), criterion 1
    const float *amin;   // smallest |a| of each node's particles, criterion 1
    const float *ew;     // periodic correction table (kernel 2)
    int ew_n;
    float ew_h, ew_hinv;
    // frontier and entry lists
    const uint2 *fin;
    uint2 *fout;
    uint32_t *cnt;   // [0] in-count (read), [1] out-count, [2] node entries, [3] particle entries, [4] overflow
    uint32_t cap_pairs;
    // entries: key = target << 32 | order key of the source, value = source (type bits | index)
    uint64_t *nkey;
    uint32_t *nval;
    uint32_t cap_node;
    uint64_t *pkey;
    uint32_t *pval;
    uint32_t cap_part;
    unsigned long long *stat;  // pp, pn, nn
};

// ---------------------------------------------------------------- geometry
// |d| of an int32 nearest-image offset given as u32 (2^31 for the most negative one)
__device__ __forceinline__ uint32_t fm_uabs(uint32_t u) { return (int32_t)u < 0 ? 0u - u : u; }

// Separation of two cubes (or of a point and a cube) on the integer grid: centre offsets
// (b - a, nearest image) against hs, the sum of the half sides.  g2: the squared distance
// between the nearest faces (physical, only axes with a gap count); returns whether the
// cubes touch or overlap (|d| <= hs on every axis).  Offsets are at most 2^31 and hs fits
// 32 bits below the root level, so the test runs in 32-bit integers (a larger hs only
// arises for two root cubes, which always touch).
__device__ __forceinline__ bool fm_cube_gap(uint32_t ax, uint32_t ay, uint32_t az, uint32_t bx, uint32_t by,
                                            uint32_t bz, uint64_t hs64, float unit, float &g2)
{
    const uint32_t hs = hs64 > 0xffffffffull ? 0xffffffffu : (uint32_t)hs64;
    const uint32_t d[3] = {fm_uabs(bx - ax), fm_uabs(by - ay), fm_uabs(bz - az)};
    bool touching = true;
    g2 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (d[k] > hs) {
            const float gf = (float)(d[k] - hs) * unit;
            g2 += gf * gf;
            touching = false;
        }
    }
    return touching;
}

struct Ent {
    uint32_t gx, gy, gz;     // integer centre (position for a particle)
    uint32_t cx, cy, cz;     // integer centre of mass
    uint64_t half;           // integer half side (0 for a particle)
    float l;                 // side length (0 for a particle)
    float mass;
    bool part, leaf;
    uint32_t next, num;      // node: children or particle range
    float amin;              // smallest |a| of its particles (relative criterion)
};

// The node-node opening criterion (p = 3): geometric (l_a + l_b)/r < theta
// (eq. eqnNodeDec), or relative (M_max / r^2)(l_max / r)^(p-1) < alpha |a|_min.
__device__ __forceinline__ bool fmm_accept(int crit, float theta2, float alpha, float la, float lb, float ma,
                                           float mb, float aa, float ab, float r2)
{
    if (crit == 0) {
        const float ls = la + lb;
        return ls * ls < theta2 * r2;
    }
    const float lm = fmaxf(la, lb);
    return fmaxf(ma, mb) * lm * lm < alpha * fminf(aa, ab) * (r2 * r2);
}

// |a|_min of every node of one level: the smallest seed of a leaf's particles,
// or of the children's minima (levels are processed from the deepest up)
__global__ void k_fmm_amin(const DevCounters *__restrict__ C, const WNode *__restrict__ wn,
                           const float *__restrict__ pseed, float *__restrict__ amin, int level)
{
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    for (uint32_t q = beg + blockIdx.x * blockDim.x + threadIdx.x; q < end; q += gridDim.x * blockDim.x) {
        const WNode w = wn[q];
        const float *src = (w.meta & WN_LEAF) ? pseed : amin;
        float m = __builtin_huge_valf();
        for (uint32_t k = 0; k < w.num; k++) m = fminf(m, src[w.next + k]);
        amin[q] = m;
    }
}

__device__ __forceinline__ Ent load_ent(const FmmArgs &A, uint32_t e)
{
    Ent E;
    if (e & PF) {
        const uint4 p = A.parts[e & ~PF];
        E.gx = E.cx = p.x;
        E.gy = E.cy = p.y;
        E.gz = E.cz = p.z;
        E.half = 0;
        E.l = 0.f;
        E.mass = __uint_as_float(p.w);
        E.part = true;
        E.leaf = false;
        E.next = E.num = 0;
        E.amin = A.crit ? A.pseed[e & ~PF] : 0.f;
    } else {
        const WNode w = A.wn[e];
        const int lev = (int)(w.meta & 0xffu);
        E.gx = w.gx; E.gy = w.gy; E.gz = w.gz;
        E.cx = w.cx; E.cy = w.cy; E.cz = w.cz;
        E.half = 1ull << (A.S - lev - 1);
        E.l = ldexpf(A.box, -lev);
        E.mass = w.mass;
        E.part = false;
        E.leaf = (w.meta & WN_LEAF) != 0;
        E.next = w.next;
        E.num = w.num;
        E.amin = A.crit ? A.amin[e] : 0.f;
    }
    return E;
}

// what happens to one frontier pair
enum { ACT_NONE = 0, ACT_SELF_LEAF, ACT_SELF_SPLIT, ACT_PP, ACT_NN, ACT_PN, ACT_OPEN_PP, ACT_OPEN };

struct Act {
    int kind;
    Ent a, b;
    uint32_t ea, eb;
    uint32_t na, nb;  // opened counts per side (ACT_OPEN*, ACT_SELF_*)
    uint32_t n_pairs, n_node, n_part;
};

__device__ __forceinline__ uint32_t open_count(const Ent &E) { return E.part ? 1u : E.num; }

__device__ __forceinline__ uint32_t open_item(const Ent &E, uint32_t e, uint32_t k)
{
    if (E.part) return e;
    return E.leaf ? (PF | (E.next + k)) : (E.next + k);
}

__device__ Act classify(const FmmArgs &A, uint32_t ea, uint32_t eb)
{
    Act X;
    X.ea = ea;
    X.eb = eb;
    X.n_pairs = X.n_node = X.n_part = 0;
    X.a = load_ent(A, ea);
    X.kind = ACT_NONE;
    if (ea == eb) {
        if (X.a.part) return X;
        if (X.a.leaf) {
            X.kind = ACT_SELF_LEAF;
            X.n_part = X.a.num;
        } else {
            X.kind = ACT_SELF_SPLIT;
            X.n_pairs = X.a.num * (X.a.num + 1) / 2;
        }
        return X;
    }
    X.b = load_ent(A, eb);
    const Ent &a = X.a, &b = X.b;
    if (a.part && b.part) {
        X.kind = ACT_PP;
        X.n_part = 2;
        return X;
    }
    float g2;
    const bool touching = fm_cube_gap(a.gx, a.gy, a.gz, b.gx, b.gy, b.gz, a.half + b.half, A.unit, g2);
    if (A.kernel == 1 && g2 > A.rcut2) return X;  // nearest sides beyond r_cut: dropped
    const float rx = (float)(int32_t)(b.cx - a.cx) * A.unit, ry = (float)(int32_t)(b.cy - a.cy) * A.unit,
                rz = (float)(int32_t)(b.cz - a.cz) * A.unit;
    const float r2 = rx * rx + ry * ry + rz * rz;
    if (!touching && fmm_accept(A.crit, A.theta * A.theta, A.alpha, a.l, b.l, a.mass, b.mass, a.amin, b.amin, r2) &&
        r2 >= A.h2) {
        if (!a.part && !b.part) {
            X.kind = ACT_NN;
            X.n_node = 2;
        } else {
            X.kind = ACT_PN;
            X.n_node = 1;
            X.n_part = 1;
        }
        return X;
    }
    X.na = open_count(a);
    X.nb = open_count(b);
    const bool fa = a.part || a.leaf, fb = b.part || b.leaf;
    if (fa && fb) {
        X.kind = ACT_OPEN_PP;  // every resulting pair is particle-particle
        X.n_part = X.na + X.nb;
    } else {
        X.kind = ACT_OPEN;
        X.n_pairs = X.na * X.nb;
    }
    return X;
}

// Order key of a source that does not depend on how nodes were numbered:
// its first particle (sorted order) and its level (31 for a single particle).
__device__ __forceinline__ uint32_t src_order(const FmmArgs &A, uint32_t src)
{
    const uint32_t id = ENT_IDX(src);
    if (ENT_TYPE(src) == ENT_PART) return (id << 5) | 31u;
    return (A.bfirst[id] << 5) | (A.wn[id].meta & 0x1fu);
}

__device__ __forceinline__ void put(uint64_t *key, uint32_t *val, uint32_t at, const FmmArgs &A, uint32_t target,
                                    uint32_t src)
{
    key[at] = ((uint64_t)target << 32) | src_order(A, src);
    val[at] = src;
}


// Block-aggregated append to three counters at once (all 256 threads call it):
// one atomic per counter and block instead of per wavefront, since every
// block appends to the same three counters and same-address atomics are
// serialised across the chip.  Returns this thread's base index in each list.
__device__ __forceinline__ uint3 block_append3(uint32_t *c0, uint32_t *c1, uint32_t *c2, uint32_t n0, uint32_t n1,
                                               uint32_t n2)
{
    __shared__ uint32_t wsum[4][3], base[3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t i0 = n0, i1 = n1, i2 = n2;  // inclusive scans within the wavefront
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v0 = __shfl_up(i0, off), v1 = __shfl_up(i1, off), v2 = __shfl_up(i2, off);
        if (lane >= off) {
            i0 += v0;
            i1 += v1;
            i2 += v2;
        }
    }
    if (lane == 63) {
        wsum[wv][0] = i0;
        wsum[wv][1] = i1;
        wsum[wv][2] = i2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t0 = wsum[0][0] + wsum[1][0] + wsum[2][0] + wsum[3][0];
        const uint32_t t1 = wsum[0][1] + wsum[1][1] + wsum[2][1] + wsum[3][1];
        const uint32_t t2 = wsum[0][2] + wsum[1][2] + wsum[2][2] + wsum[3][2];
        base[0] = t0 ? atomicAdd(c0, t0) : 0u;
        base[1] = t1 ? atomicAdd(c1, t1) : 0u;
        base[2] = t2 ? atomicAdd(c2, t2) : 0u;
    }
    __syncthreads();
    uint32_t b0 = base[0], b1 = base[1], b2 = base[2];
    for (int w = 0; w < wv; w++) {
        b0 += wsum[w][0];
        b1 += wsum[w][1];
        b2 += wsum[w][2];
    }
    __syncthreads();  // wsum and base are reused by the next call
    return make_uint3(b0 + i0 - n0, b1 + i1 - n1, b2 + i2 - n2);
}

__global__ __launch_bounds__(256) void k_fmm_traverse(FmmArgs A)
{
    // after an overflow the lists are incomplete: stop touching them (decided once per
    // block, since every thread of the block must reach the barriers of the appends)
    __shared__ uint32_t s_over;
    if (threadIdx.x == 0) s_over = A.cnt[4];
    __syncthreads();
    if (s_over) return;
    const uint32_t nin = min(A.cnt[0], A.cap_pairs);
    // interaction counters: particle pairs, particle-node, node-node (summed over the loop,
    // one atomic per wavefront at the end)
    unsigned long long c_pp = 0, c_pn = 0, c_nn = 0;
    for (uint32_t base = blockIdx.x * blockDim.x; base < nin; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        Act X;
        X.kind = ACT_NONE;
        X.n_pairs = X.n_node = X.n_part = 0;
        if (t < nin) {
            const uint2 pr = A.fin[t];
            X = classify(A, pr.x, pr.y);
        }
        const uint3 off3 = block_append3(&A.cnt[1], &A.cnt[2], &A.cnt[3], X.n_pairs, X.n_node, X.n_part);
        const uint32_t op = off3.x, on = off3.y, ok = off3.z;
        if (X.kind == ACT_PP) c_pp += 1;
        if (X.kind == ACT_OPEN_PP) c_pp += (unsigned long long)X.na * X.nb;
        if (X.kind == ACT_SELF_LEAF) c_pp += (unsigned long long)X.a.num * (X.a.num - 1) / 2;
        if (X.kind == ACT_PN) c_pn += 1;
        if (X.kind == ACT_NN) c_nn += 1;
        if (t >= nin) continue;
        if ((uint64_t)op + X.n_pairs > A.cap_pairs || (uint64_t)on + X.n_node > A.cap_node ||
            (uint64_t)ok + X.n_part > A.cap_part) {
            atomicOr(&A.cnt[4], 1u);
            continue;
        }
        switch (X.kind) {
        case ACT_SELF_LEAF:
            for (uint32_t k = 0; k < X.a.num; k++) put(A.pkey, A.pval, ok + k, A, X.a.next + k, ENT_LEAF | X.ea);
            break;
        case ACT_SELF_SPLIT: {
            uint32_t o = op;
            for (uint32_t c1 = 0; c1 < X.a.num; c1++)
                for (uint32_t c2 = c1; c2 < X.a.num; c2++) A.fout[o++] = make_uint2(X.a.next + c1, X.a.next + c2);
            break;
        }
        case ACT_PP:
            put(A.pkey, A.pval, ok, A, X.ea & ~PF, ENT_PART | (X.eb & ~PF));
            put(A.pkey, A.pval, ok + 1, A, X.eb & ~PF, ENT_PART | (X.ea & ~PF));
            break;
        case ACT_NN:
            put(A.nkey, A.nval, on, A, X.ea, ENT_NODE | X.eb);
            put(A.nkey, A.nval, on + 1, A, X.eb, ENT_NODE | X.ea);
            break;
        case ACT_PN: {
            const uint32_t node = X.a.part ? X.eb : X.ea, part = (X.a.part ? X.ea : X.eb) & ~PF;
            put(A.nkey, A.nval, on, A, node, ENT_PART | part);
            put(A.pkey, A.pval, ok, A, part, ENT_NODE | node);
            break;
        }
        case ACT_OPEN_PP: {
            // side a's particles see all of side b, and vice versa
            const uint32_t srcb = X.b.part ? (ENT_PART | (X.eb & ~PF)) : (ENT_LEAF | X.eb);
            const uint32_t srca = X.a.part ? (ENT_PART | (X.ea & ~PF)) : (ENT_LEAF | X.ea);
            uint32_t o = ok;
            for (uint32_t k = 0; k < X.na; k++) put(A.pkey, A.pval, o++, A, open_item(X.a, X.ea, k) & ~PF, srcb);
            for (uint32_t k = 0; k < X.nb; k++) put(A.pkey, A.pval, o++, A, open_item(X.b, X.eb, k) & ~PF, srca);
            break;
        }
        case ACT_OPEN: {
            uint32_t o = op;
            for (uint32_t i = 0; i < X.na; i++)
                for (uint32_t j = 0; j < X.nb; j++)
                    A.fout[o++] = make_uint2(open_item(X.a, X.ea, i), open_item(X.b, X.eb, j));
            break;
        }
        default:
            break;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        c_pp += __shfl_xor(c_pp, off);
        c_pn += __shfl_xor(c_pn, off);
        c_nn += __shfl_xor(c_nn, off);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c_pp) atomicAdd(&A.stat[0], c_pp);
        if (c_pn) atomicAdd(&A.stat[1], c_pn);
        if (c_nn) atomicAdd(&A.stat[2], c_nn);
    }
}

// counts: in <- out, clear out (a single thread between passes)
__global__ void k_fmm_rotate(uint32_t *cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        cnt[0] = cnt[1];
        cnt[1] = 0;
    }
}

// the walk starts from the self-pair of every root (one root per box of a forest)
__global__ void k_fmm_init(uint32_t *cnt, uint2 *f0, unsigned long long *stat, int nroot)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nroot) f0[b] = make_uint2((uint32_t)b, (uint32_t)b);
    if (b == 0) {
        cnt[0] = (uint32_t)nroot;
        for (int k = 1; k < 8; k++) cnt[k] = 0;
        stat[0] = stat[1] = stat[2] = 0;
    }
}

// ------------------------------------------------------------ CSR of entries
__global__ void k_fmm_csr(const uint64_t *__restrict__ key, uint32_t n, uint32_t *__restrict__ start,
                          uint32_t *__restrict__ end)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t k = (uint32_t)(key[i] >> 32);
        if (i == 0 || (uint32_t)(key[i - 1] >> 32) != k) start[k] = i;
        if (i == n - 1 || (uint32_t)(key[i + 1] >> 32) != k) end[k] = i + 1;
    }
}

// ------------------------------------------------------------ field algebra
// packed symmetric storage: F2 xx xy xz yy yz zz, F3 xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
__device__ __forceinline__ int i2(int i, int j)
{
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
__device__ __forceinline__ int i3(int i, int j, int k)
{
    // sort the triple
    int a = i, b = j, c = k, t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    if (a == 0) return b == 0 ? c : (b == 1 ? 2 + c : 5);
    if (a == 1) return b == 1 ? 5 + c : 8;
    return 9;
}

// g0..g3 of the interaction kernel at r: short-range for kernel 1, Newtonian
// otherwise (kernel 2 adds the periodic correction psi separately)
__device__ __forceinline__ void gfun_f(int kernel, float r2, float asplit, float &g0, float &g1, float &g2, float &g3)
{
    const float rinv = rsq(r2), ri2 = rinv * rinv;
    if (kernel != 1) {
        g0 = rinv;
        g1 = -rinv * ri2;
        g2 = -3.0f * g1 * ri2;
        g3 = -5.0f * g2 * ri2;
    } else {
        const float r = r2 * rinv, x = asplit * r;
        const float ex = expneg(x * x), ec = erfc_hastings(x, ex);
        const float E = 2.0f * INV_SQRTPI * asplit * ex, a2 = asplit * asplit;
        const float t1 = ec * rinv * ri2, e2 = E * ri2;
        g0 = ec * rinv;
        g1 = -(t1 + e2);
        g2 = 3.0f * t1 * ri2 + e2 * (3.0f * ri2 + 2.0f * a2);
        g3 = -(15.0f * t1 * ri2 * ri2 + e2 * (ri2 * (15.0f * ri2 + 10.0f * a2) + 4.0f * a2 * a2));
    }
}

// add the field of a source (mass M, Q2, Q3; Q2 = Q3 = null for a particle)
// seen at r = s_source - s_sink: F0 += M D0 + Q2:D2/2 + Q3.D3/6,
// F1 += M D1 + Q2:D3/2, F2 += M D2, F3 += M D3.
__device__ __forceinline__ void add_field_f(float F[20], const float r[3], float g0, float g1, float g2, float g3,
                                            float M, const float *Q2, const float *Q3)
{
    float D2[6], D3[10];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) D2[i2(i, j)] = (i == j ? g1 : 0.f) + g2 * r[i] * r[j];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++)
#pragma unroll
            for (int k = j; k < 3; k++) {
                float t = 0.f;
                if (i == j) t += r[k];
                if (j == k) t += r[i];
                if (i == k) t += r[j];
                D3[i3(i, j, k)] = g2 * t + g3 * r[i] * r[j] * r[k];
            }
    float f0 = M * g0;
    float f1[3] = {M * g1 * r[0], M * g1 * r[1], M * g1 * r[2]};
    if (Q2) {
        const float tr = Q2[0] + Q2[3] + Q2[5];
        const float qr[3] = {Q2[0] * r[0] + Q2[1] * r[1] + Q2[2] * r[2], Q2[1] * r[0] + Q2[3] * r[1] + Q2[4] * r[2],
                             Q2[2] * r[0] + Q2[4] * r[1] + Q2[5] * r[2]};
        const float rqr = r[0] * qr[0] + r[1] * qr[1] + r[2] * qr[2];
        f0 += 0.5f * (g1 * tr + g2 * rqr);
        const float c = 0.5f * (g2 * tr + g3 * rqr);
#pragma unroll
        for (int i = 0; i < 3; i++) f1[i] += g2 * qr[i] + c * r[i];
        if (Q3) {
            const float tv[3] = {Q3[0] + Q3[3] + Q3[5], Q3[1] + Q3[6] + Q3[8], Q3[2] + Q3[7] + Q3[9]};
            float c3 = 0.f;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
#pragma unroll
                    for (int k = 0; k < 3; k++) c3 += Q3[i3(i, j, k)] * r[i] * r[j] * r[k];
            f0 += (3.f * g2 * (tv[0] * r[0] + tv[1] * r[1] + tv[2] * r[2]) + g3 * c3) * (1.0f / 6.0f);
        }
    }
    F[0] += f0;
    F[1] += f1[0];
    F[2] += f1[1];
    F[3] += f1[2];
#pragma unroll
    for (int a = 0; a < 6; a++) F[4 + a] += M * D2[a];
#pragma unroll
    for (int a = 0; a < 10; a++) F[10 + a] += M * D3[a];
}

// Periodic FMM (kernel 2): the Green's function is 1/r - psi, so the field of
// a source gets the same expansion with psi's derivatives D (packed D0..D3 at
// r = s_source - s_sink) subtracted: F0 -= M D0 + Q2:D2/2 + Q3.D3/6,
// F1 -= M D1 + Q2:D3/2, F2 -= M D2, F3 -= M D3.
__device__ __forceinline__ void sub_field_psi(float F[20], const float D[20], float M, const float *Q2,
                                              const float *Q3)
{
    const float *D1 = D + 1, *D2 = D + 4, *D3 = D + 10;
    float f0 = M * D[0];
    float f1[3] = {M * D1[0], M * D1[1], M * D1[2]};
    if (Q2) {
        // symmetric contractions in packed storage (off-diagonal terms twice)
        f0 += 0.5f * (Q2[0] * D2[0] + Q2[3] * D2[3] + Q2[5] * D2[5]) + Q2[1] * D2[1] + Q2[2] * D2[2] +
              Q2[4] * D2[4];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            float c = 0.f;
#pragma unroll
            for (int j = 0; j < 3; j++)
#pragma unroll
                for (int k = 0; k < 3; k++) c += Q2[i2(j, k)] * D3[i3(i, j, k)];
            f1[i] += 0.5f * c;
        }
        if (Q3) {
            float c3 = 0.f;
#pragma unroll
            for (int i = 0; i < 3; i++)
#pragma unroll
                for (int j = 0; j < 3; j++)
#pragma unroll
                    for (int k = 0; k < 3; k++) c3 += Q3[i3(i, j, k)] * D3[i3(i, j, k)];
            f0 += c3 * (1.0f / 6.0f);
        }
    }
    F[0] -= f0;
    F[1] -= f1[0];
    F[2] -= f1[1];
    F[3] -= f1[2];
#pragma unroll
    for (int a = 0; a < 6; a++) F[4 + a] -= M * D2[a];
#pragma unroll
    for (int a = 0; a < 10; a++) F[10 + a] -= M * D3[a];
}

// psi's packed D0..D3 at -r from those at r (psi is even: odd orders change sign)
__device__ __forceinline__ void psi_mirror(float D[20])
{
#pragma unroll
    for (int a = 1; a < 4; a++) D[a] = -D[a];
#pragma unroll
    for (int a = 10; a < 20; a++) D[a] = -D[a];
}

// M2L / P2L: each node sums the fields of its sources
template <bool EW>
__global__ __launch_bounds__(256) void k_fmm_m2l(FmmArgs A, const uint32_t *__restrict__ start,
                                                 const uint32_t *__restrict__ end, float *__restrict__ F)
{
    const uint32_t nn = A.ctr->node_count;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += gridDim.x * blockDim.x) {
        float f[20];
#pragma unroll
        for (int a = 0; a < 20; a++) f[a] = 0.f;
        const WNode w = A.wn[q];
        for (uint32_t e = start[q]; e < end[q]; e++) {
            const uint32_t src = A.nval[e];
            const uint32_t id = ENT_IDX(src);
            float r[3], M;
            const float *Q2 = nullptr, *Q3 = nullptr;
            float q2[6], q3[10];
            if (ENT_TYPE(src) == ENT_PART) {
                const uint4 p = A.parts[id];
                r[0] = (float)(int32_t)(p.x - w.cx) * A.unit;
                r[1] = (float)(int32_t)(p.y - w.cy) * A.unit;
                r[2] = (float)(int32_t)(p.z - w.cz) * A.unit;
                M = __uint_as_float(p.w);
            } else {
                const WNode s = A.wn[id];
                r[0] = (float)(int32_t)(s.cx - w.cx) * A.unit;
                r[1] = (float)(int32_t)(s.cy - w.cy) * A.unit;
                r[2] = (float)(int32_t)(s.cz - w.cz) * A.unit;
                M = s.mass;
#pragma unroll
                for (int a = 0; a < 6; a++) q2[a] = s.q[a];
#pragma unroll
                for (int a = 0; a < 10; a++) q3[a] = A.q3[(size_t)id * 10 + a];
                Q2 = q2;
                Q3 = q3;
            }
            float g0, g1, g2, g3;
            gfun_f(A.kernel, r[0] * r[0] + r[1] * r[1] + r[2] * r[2], A.asplit, g0, g1, g2, g3);
            add_field_f(f, r, g0, g1, g2, g3, M, Q2, Q3);
            if constexpr (EW) {
                float D[20];
                ew_d20(A.ew, A.ew_n, A.ew_h, A.ew_hinv, r[0], r[1], r[2], D);
                sub_field_psi(f, D, M, Q2, Q3);
            }
        }
#pragma unroll
        for (int a = 0; a < 20; a++) F[(size_t)q * 20 + a] = f[a];
    }
}

// L2L for one level: F_child += shift of F_parent by d = s_child - s_parent:
// F'0 = F0 - F1.d + F2:dd/2 - F3:ddd/6, F'1 = F1 - F2.d + F3:dd/2,
// F'2 = F2 - F3.d, F'3 = F3 (exact re-centring of the cubic expansion).
__global__ void k_fmm_l2l(FmmArgs A, int level, float *__restrict__ F)
{
    const uint32_t beg = A.ctr->lvl_start[level], end = beg + A.ctr->lvl_count[level];
    for (uint32_t q = beg + blockIdx.x * blockDim.x + threadIdx.x; q < end; q += gridDim.x * blockDim.x) {
        const uint32_t p = A.parent[q];
        const WNode wc = A.wn[q], wp = A.wn[p];
        const float d[3] = {(float)(int32_t)(wc.cx - wp.cx) * A.unit, (float)(int32_t)(wc.cy - wp.cy) * A.unit,
                            (float)(int32_t)(wc.cz - wp.cz) * A.unit};
        float P[20];
#pragma unroll
        for (int a = 0; a < 20; a++) P[a] = F[(size_t)p * 20 + a];
        const float *F1 = P + 1, *F2 = P + 4, *F3 = P + 10;
        float o[20];
        float s0 = P[0];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            s0 -= F1[i] * d[i];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                s0 += 0.5f * F2[i2(i, j)] * d[i] * d[j];
#pragma unroll
                for (int k = 0; k < 3; k++) s0 -= F3[i3(i, j, k)] * d[i] * d[j] * d[k] * (1.0f / 6.0f);
            }
        }
        o[0] = s0;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            float s = F1[i];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                s -= F2[i2(i, j)] * d[j];
#pragma unroll
                for (int k = 0; k < 3; k++) s += 0.5f * F3[i3(i, j, k)] * d[j] * d[k];
            }
            o[1 + i] = s;
        }
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = i; j < 3; j++) {
                float s = F2[i2(i, j)];
#pragma unroll
                for (int k = 0; k < 3; k++) s -= F3[i3(i, j, k)] * d[k];
                o[4 + i2(i, j)] = s;
            }
#pragma unroll
        for (int a = 0; a < 10; a++) o[10 + a] = F3[a];
#pragma unroll
        for (int a = 0; a < 20; a++) F[(size_t)q * 20 + a] += o[a];
    }
}

__global__ void k_fmm_leafmap(const DevCounters *__restrict__ C, const WNode *__restrict__ wn,
                              uint32_t *__restrict__ leafid)
{
    const uint32_t nn = C->node_count;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += gridDim.x * blockDim.x) {
        const WNode w = wn[q];
        if (w.meta & WN_LEAF)
            for (uint32_t j = w.next; j < w.next + w.num; j++) leafid[j] = q;
    }
}

// Per particle: M2P from node sources, P2P from particle or leaf sources,
// then L2P of the leaf's field expansion: a = G[-F1 + F2.a - F3:aa/2],
// phi = -G[F0 - F1.a + F2:aa/2 - F3:aaa/6], a = x - s_leaf.
template <int KER, bool POT>
__global__ __launch_bounds__(256) void k_fmm_particles(FmmArgs A, const uint32_t *__restrict__ start,
                                                       const uint32_t *__restrict__ end,
                                                       const float *__restrict__ F,
                                                       const uint32_t *__restrict__ leafid, const uint32_t *perm,
                                                       int64_t n, double G, double *ax, double *ay, double *az,
                                                       double *pot)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 me = A.parts[i];
    double dx_ = 0, dy_ = 0, dz_ = 0, dp_ = 0;
    for (uint32_t e = start[i]; e < end[i]; e++) {
        const uint32_t src = A.pval[e];
        const uint32_t id = ENT_IDX(src);
        float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
        if (ENT_TYPE(src) == ENT_NODE) {
            const WNode s = A.wn[id];
            const float r[3] = {(float)(int32_t)(s.cx - me.x) * A.unit, (float)(int32_t)(s.cy - me.y) * A.unit,
                                (float)(int32_t)(s.cz - me.z) * A.unit};
            float g0, g1, g2, g3;
            gfun_f(KER, r[0] * r[0] + r[1] * r[1] + r[2] * r[2], A.asplit, g0, g1, g2, g3);
            float f[20];
#pragma unroll
            for (int a = 0; a < 20; a++) f[a] = 0.f;
            float q2[6], q3[10];
#pragma unroll
            for (int a = 0; a < 6; a++) q2[a] = s.q[a];
            if (POT) {
#pragma unroll
                for (int a = 0; a < 10; a++) q3[a] = A.q3[(size_t)id * 10 + a];
            }
            add_field_f(f, r, g0, g1, g2, g3, s.mass, q2, POT ? q3 : nullptr);
            if constexpr (KER == 2) {
                float D[20];
                ew_d20(A.ew, A.ew_n, A.ew_h, A.ew_hinv, r[0], r[1], r[2], D);
                sub_field_psi(f, D, s.mass, q2, POT ? q3 : nullptr);
            }
            fx = -f[1];
            fy = -f[2];
            fz = -f[3];
            fp = -f[0];
        } else {
            const uint32_t j0 = ENT_TYPE(src) == ENT_LEAF ? A.wn[id].next : id;
            const uint32_t j1 = ENT_TYPE(src) == ENT_LEAF ? j0 + A.wn[id].num : id + 1;
            for (uint32_t j = j0; j < j1; j++) {
                if ((int64_t)j == i) continue;
                const uint4 p = A.parts[j];
                const float sx = (float)(int32_t)(p.x - me.x) * A.unit, sy = (float)(int32_t)(p.y - me.y) * A.unit,
                            sz = (float)(int32_t)(p.z - me.z) * A.unit;
                float K, W;
                pair_kernel<KER == 2 ? 0 : KER, POT>(sx * sx + sy * sy + sz * sz, A.asplit, A.h2, A.hinv, K, W);
                const float mj = __uint_as_float(p.w), mk = mj * K;
                fx += mk * sx;
                fy += mk * sy;
                fz += mk * sz;
                if (POT) fp -= mj * W;
                if constexpr (KER == 2) {
                    float ex, ey, ez, ep = 0.f;
                    ew_grad<POT>(A.ew, A.ew_n, A.ew_h, A.ew_hinv, sx, sy, sz, ex, ey, ez, ep);
                    fx += mj * ex;
                    fy += mj * ey;
                    fz += mj * ez;
                    if (POT) fp += mj * ep;
                }
            }
        }
        dx_ += fx;
        dy_ += fy;
        dz_ += fz;
        if (POT) dp_ += fp;
    }
    // L2P
    const uint32_t L = leafid[i];
    const WNode wl = A.wn[L];
    const float a[3] = {(float)(int32_t)(me.x - wl.cx) * A.unit, (float)(int32_t)(me.y - wl.cy) * A.unit,
                        (float)(int32_t)(me.z - wl.cz) * A.unit};
    float P[20];
#pragma unroll
    for (int k = 0; k < 20; k++) P[k] = F[(size_t)L * 20 + k];
    const float *F1 = P + 1, *F2 = P + 4, *F3 = P + 10;
    float g[3], ph = P[0];
#pragma unroll
    for (int ii = 0; ii < 3; ii++) {
        float s = -F1[ii];
        ph -= F1[ii] * a[ii];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            s += F2[i2(ii, k)] * a[k];
            ph += 0.5f * F2[i2(ii, k)] * a[ii] * a[k];
#pragma unroll
            for (int m = 0; m < 3; m++) {
                s -= 0.5f * F3[i3(ii, k, m)] * a[k] * a[m];
                ph -= F3[i3(ii, k, m)] * a[ii] * a[k] * a[m] * (1.0f / 6.0f);
            }
        }
        g[ii] = s;
    }
    dx_ += g[0];
    dy_ += g[1];
    dz_ += g[2];
    dp_ -= ph;
    const uint32_t o = perm[i];
    ax[o] = G * dx_;
    ay[o] = G * dy_;
    az[o] = G * dz_;
    if (POT && pot) pot[o] = G * dp_;
}


// ==================================================================== fast path
// The same interactions as the list-based walk above, organised for the GPU
// without per-interaction lists (Sec. "Fast multipole method" fixes which pairs
// interact and how; the order of the floating-point sums is free):
//  1. node-level dual walk, breadth first: a frontier item is a pair of
//     internal nodes to be opened (or an internal node's self pair); one
//     wavefront takes an item and gives one lane to every pair of daughters.
//     Accepted pairs add both field expansions, summed per daughter in LDS and
//     then added to the node fields with one contiguous atomic per coefficient.
//     Opened pairs of internal nodes form the next frontier; an opened pair of
//     two leaves goes to the leaf-pair list, a leaf against an internal node
//     to the leaf-node list.
//  2. particle pairs, one wavefront per leaf: the pairs inside the leaf and
//     with every partner leaf of the leaf-pair list (grouped per leaf by a
//     counting sort), each pair evaluated from both of its leaves; sums go
//     straight to the leaf's particles, no atomics.
//  3. leaf-node pairs, one wavefront each: every particle of the leaf walks
//     the internal node's subtree with the particle-node rules; particle-node
//     interactions also put the particle's field on the node, opened leaves
//     give particle pairs (both sides); sums go out with atomics.
//  4. downward shift (the kernel above) and evaluation at the particles.
// Summation order follows the scheduling of the atomics, so results agree
// with the list-based path to round-off but are not bitwise reproducible.
#define FT_STK 32  // traversal stack of a leaf-node pair: one sibling entry per level
#define FT_SB 16   // source block of the particle pairs with an opened leaf
#define FP_SRC 512 // partner particles listed in LDS at a time by the leaf-pair kernel
#define FT_NC 2     // copies of the daughters' field sums in the node-pair passes

__constant__ uint8_t c_tri[36][2] = {{0, 0}, {0, 1}, {1, 1}, {0, 2}, {1, 2}, {2, 2}, {0, 3}, {1, 3}, {2, 3}, {3, 3}, {0, 4}, {1, 4}, {2, 4}, {3, 4}, {4, 4}, {0, 5}, {1, 5}, {2, 5}, {3, 5}, {4, 5}, {5, 5}, {0, 6}, {1, 6}, {2, 6}, {3, 6}, {4, 6}, {5, 6}, {6, 6}, {0, 7}, {1, 7}, {2, 7}, {3, 7}, {4, 7}, {5, 7}, {6, 7}, {7, 7}};  // daughter pairs (i <= j) of a self pair, j-major

struct FastArgs {
    const WNode *wn;
    const uint4 *parts;
    const float *q3;
    int S;
    float unit, box, theta2, h2, asplit, hinv, rcut2;
    int kernel;
    int crit;            // 0 geometric, 1 relative node-node criterion
    float alpha;
    const float *pseed;  // |a| per particle (sorted order), criterion 1
    const float *amin;   // smallest |a| of each node's particles, criterion 1
    const float *ew;     // periodic correction table (kernel 2)
    int ew_n;
    float ew_h, ew_hinv;
    const uint2 *fin;
    uint2 *fout;
    uint32_t *cnt;  // [0] frontier in, [1] frontier out, [2] leaf pairs, [3] leaf-node pairs, [4] overflow
    uint32_t cap_pairs;
    uint2 *ll;      // opened (leaf, leaf) pairs
    uint2 *ln;      // opened (leaf, internal node) pairs
    uint32_t cap_ll, cap_ln;
    uint32_t *pstart;  // CSR of partner leaves per node (node_count + 1)
    uint32_t *plist;   // partner leaf of each entry (2 per leaf pair)
    float *F;       // 20 field coefficients per node
    double *acc;    // 4 per particle (sorted order): a_x, a_y, a_z, potential, before the factor G
    unsigned long long *stat;  // pp, pn, nn
    uint32_t *flags;           // tree flags: G4_FLAG_FMM_STACK if a leaf-node stack overflows
};

__device__ __forceinline__ uint32_t fm_uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t fm_ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ uint32_t fm_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ void fm_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Two nodes: 0 dropped (beyond r_cut), 1 interact, 2 open.  Same arithmetic
// as classify() above; r = s_b - s_a.
__device__ __forceinline__ int fm_classify(const FastArgs &A, const WNode &a, const WNode &b, uint32_t ia,
                                           uint32_t ib, float r[3], float &r2)
{
    const int la = (int)(a.meta & 0xffu), lb = (int)(b.meta & 0xffu);
    float g2;
    const bool touching = fm_cube_gap(a.gx, a.gy, a.gz, b.gx, b.gy, b.gz,
                                      (1ull << (A.S - la - 1)) + (1ull << (A.S - lb - 1)), A.unit, g2);
    if (A.kernel == 1 && g2 > A.rcut2) return 0;
    r[0] = (float)(int32_t)(b.cx - a.cx) * A.unit;
    r[1] = (float)(int32_t)(b.cy - a.cy) * A.unit;
    r[2] = (float)(int32_t)(b.cz - a.cz) * A.unit;
    r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const float aa = A.crit ? A.amin[ia] : 0.f, ab = A.crit ? A.amin[ib] : 0.f;
    const bool acc = fmm_accept(A.crit, A.theta2, A.alpha, ldexpf(A.box, -la), ldexpf(A.box, -lb), a.mass, b.mass,
                                aa, ab, r2);
    return (!touching && acc && r2 >= A.h2) ? 1 : 2;
}

// the walk starts from the self pair of every internal root (a root leaf only
// has its own particle pairs, which phase 2 does for every leaf)
__global__ void k_fast_init(FastArgs A, int nroot)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nroot || (A.wn[b].meta & WN_LEAF)) return;
    const uint32_t o = atomicAdd(&A.cnt[0], 1u);
    if (o < A.cap_pairs) A.fout[o] = make_uint2((uint32_t)b, (uint32_t)b);
    else atomicOr(&A.cnt[4], 1u);
}

// Wavefront-local staging of appended pairs: up to 127 pending entries in LDS,
// written out 64 at a time with one atomic on the global counter.
template <uint32_t CAP>
struct Stage {
    uint2 *buf;        // LDS, CAP entries; a push adds at most 64, writes go out CAP - 64 at a time
    uint32_t n;        // pending (wavefront-uniform)
};

// append one pair per lane that wants it (all lanes active)
template <uint32_t CAP>
__device__ __forceinline__ void st_push(Stage<CAP> &S, bool want, uint2 v)
{
    const uint64_t m = fm_ballot(want);
    if (want) S.buf[S.n + fm_below(m)] = v;
    S.n += (uint32_t)__builtin_popcountll(m);
}

// write out cap - 64 pending pairs (or all, if final) to out[] behind counter.
// Every wavefront appends to the same counter, and same-address atomics are
// serialised across the chip, so larger batches mean fewer of them.
template <uint32_t CAP>
__device__ __forceinline__ void st_flush(Stage<CAP> &S, bool final, uint2 *out, uint32_t *counter, uint32_t cap,
                                         uint32_t *overflow)
{
    const int lane = threadIdx.x & 63;
    constexpr uint32_t chunk = CAP - 64u;
    while (S.n >= chunk || (final && S.n > 0)) {
        const uint32_t k = min(S.n, chunk);
        fm_sync();
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(counter, k);
        base = fm_uni(base);
#pragma unroll
        for (uint32_t l0 = 0; l0 < chunk; l0 += 64u) {
            const uint32_t l = l0 + (uint32_t)lane;
            if (l < k) {
                if (base + l < cap) out[base + l] = S.buf[l];
                else atomicOr(overflow, 1u);
            }
        }
        // move the rest (< 64) to the front
        const uint2 rest = (uint32_t)lane + k < S.n ? S.buf[lane + k] : make_uint2(0u, 0u);
        fm_sync();
        if ((uint32_t)lane + k < S.n) S.buf[lane] = rest;
        S.n -= k;
        fm_sync();
    }
}

// value of lane + S within this lane's row of 16 (0 past the row's end): DPP row_shl
template <int S>
__device__ __forceinline__ uint32_t fm_from_next(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 + S, 0xf, 0xf, false);
}
// adds the expansions of lane + S to this lane's where it takes them (bit B of take)
template <int S, int B>
__device__ __forceinline__ void fm_combine(float f[20], uint32_t take)
{
#pragma unroll
    for (int k = 0; k < 20; k++) {
        const float o = __uint_as_float(fm_from_next<S>(__float_as_uint(f[k])));
        if ((take >> B) & 1u) f[k] += o;
    }
}

template <bool POT, bool EW>
__global__ __launch_bounds__(256) void k_fast_open(FastArgs A)
{
    // field sums of the daughters, FT_NC copies: the lanes of one daughter spread over the
    // copies, since float atomics to one LDS address serialise
    __shared__ float Floc[4][FT_NC][16][20];
    __shared__ uint2 sbf[4][128], sbl[4][256], sbn[4][128];  // staging: frontier, leaf pairs, leaf-node pairs
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float(*FL)[16][20] = Floc[wv];
    for (int v = lane; v < FT_NC * 320; v += 64) (&FL[0][0][0])[v] = 0.f;
    if (A.cnt[4]) return;  // a list overflowed: the host retries with more room
    const uint32_t nin = min(A.cnt[0], A.cap_pairs);
    uint32_t c_nn = 0;
    Stage<128> sf{sbf[wv], 0u}, sn{sbn[wv], 0u};
    Stage<256> sl{sbl[wv], 0u};
    const uint32_t stride = gridDim.x * 4;
    uint32_t it = blockIdx.x * 4 + wv;
    uint2 pr = it < nin ? A.fin[it] : make_uint2(0u, 0u);
    fm_sync();
    for (; it < nin; it += stride) {
        const uint32_t pa = fm_uni(pr.x), pb = fm_uni(pr.y);
        // the next item's pair, loaded while this one is worked on
        if (it + stride < nin) pr = A.fin[it + stride];
        const bool self = pa == pb;
        const uint32_t ca = fm_uni(A.wn[pa].next), na = fm_uni(A.wn[pa].num);
        const uint32_t cb = fm_uni(A.wn[pb].next), nb = fm_uni(A.wn[pb].num);
        uint32_t i = 0, j = 0;
        bool valid;
        if (self) {
            valid = (uint32_t)lane < na * (na + 1) / 2;
            if (valid) {
                i = c_tri[lane][0];
                j = c_tri[lane][1];
            }
        } else {
            valid = (uint32_t)lane < na * nb;
            if (valid) {
                i = (uint32_t)lane / nb;
                j = (uint32_t)lane - i * nb;
            }
        }
        int act = 0;  // 1 interact, 2 open, 3 self pair of a daughter
        WNode w1, w2;
        float r[3] = {0.f, 0.f, 0.f}, r2 = 0.f;
        if (valid) {
            w1 = A.wn[ca + i];
            w2 = A.wn[cb + j];
            act = (self && i == j) ? 3 : fm_classify(A, w1, w2, ca + i, cb + j, r, r2);
        }
        const bool inter = act == 1;
        const uint64_t im = fm_ballot(inter);
        if (im) {
            // The two expansions of each interacting pair are summed per daughter with LDS float
            // atomics, which serialise on one address.  Lanes that add to the same daughter and
            // sit next to each other first combine their expansions by a tree of cross-lane
            // moves within rows of 16 lanes: the pairs (i, j), (i, j + 1), ... for side i of a
            // pair of distinct nodes, (i, j), (i + 1, j), ... for side j of a node with itself.
            // m is the pair's position in that run, n the run's length.
            const uint32_t cm = self ? i : j, cn = self ? j + 1 : nb;
            const bool comb = valid;
            uint32_t lvl_take = 0, anyi = inter ? 1u : 0u;  // bit s: took at distance 2^s
            bool given = false;
            auto level = [&](uint32_t st, uint32_t b, uint32_t nbr) {
                const bool take = comb && !given && (cm % (2 * st)) == 0 && cm + st < cn && (lane & 15) + st <= 15;
                if (comb && !given && (cm % (2 * st)) == st && (uint32_t)(lane & 15) >= st) given = true;
                if (take) {
                    lvl_take |= 1u << b;
                    anyi |= nbr;
                }
            };
            level(1, 0, fm_from_next<1>(anyi));
            level(2, 1, fm_from_next<2>(anyi));
            level(4, 2, fm_from_next<4>(anyi));
            // the other side's pairs of one daughter are not adjacent: two steps of a tree of
            // lane-indexed moves, the pair at position m taking position m + 1 (m even), then
            // m + 2 (m a multiple of 4)
            const uint32_t sm = self ? j - i : i, sn = self ? na - i : na;
            const uint32_t s_src1 = self ? (uint32_t)lane + j + 1 : (uint32_t)lane + nb;
            const uint32_t s_src2 = self ? (uint32_t)lane + 2 * j + 3 : (uint32_t)lane + 2 * nb;
            const bool s_take1 = valid && (sm & 1u) == 0 && sm + 1 < sn;
            const bool s_take2 = valid && (sm & 3u) == 0 && sm + 2 < sn;
            const bool s_give = valid && (sm & 3u) != 0;
            const int s_lane1 = (int)(s_take1 ? s_src1 : (uint32_t)lane);
            const int s_lane2 = (int)(s_take2 ? s_src2 : (uint32_t)lane);
            int s_any = inter ? 1 : 0;
            const int s_any1 = __shfl(s_any, s_lane1);  // every lane takes part in the moves
            if (s_take1) s_any |= s_any1;
            const int s_any2 = __shfl(s_any, s_lane2);
            if (s_take2) s_any |= s_any2;
            float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
            if (inter) gfun_f(A.kernel, r2, A.asplit, g0, g1, g2, g3);
            float f[20], q2[6], q3[10];
            const float mr[3] = {-r[0], -r[1], -r[2]};
            float Dp[20];  // psi's D0..D3 at +r (kernel 2)
            if constexpr (EW) {
                if (inter) ew_d20(A.ew, A.ew_n, A.ew_h, A.ew_hinv, r[0], r[1], r[2], Dp);
            }
            // daughter i sees daughter j at +r ...
#pragma unroll
            for (int k = 0; k < 20; k++) f[k] = 0.f;
            if (inter) {
#pragma unroll
                for (int k = 0; k < 6; k++) q2[k] = w2.q[k];
                if (POT) {
#pragma unroll
                    for (int k = 0; k < 10; k++) q3[k] = A.q3[(size_t)(cb + j) * 10 + k];
                }
                add_field_f(f, r, g0, g1, g2, g3, w2.mass, q2, POT ? q3 : nullptr);
                if constexpr (EW) sub_field_psi(f, Dp, w2.mass, q2, POT ? q3 : nullptr);
            }
            if (!self) {
                fm_combine<1, 0>(f, lvl_take);
                fm_combine<2, 1>(f, lvl_take);
                fm_combine<4, 2>(f, lvl_take);
            } else {
#pragma unroll
                for (int k = 0; k < 20; k++) {
                    const float o = __shfl(f[k], s_lane1);
                    if (s_take1) f[k] += o;
                }
#pragma unroll
                for (int k = 0; k < 20; k++) {
                    const float o = __shfl(f[k], s_lane2);
                    if (s_take2) f[k] += o;
                }
            }
            if (self ? (s_any && !s_give) : (anyi && !given)) {
                const uint32_t cA = (self ? sm >> 2 : j >> 1) % FT_NC;
#pragma unroll
                for (int k = 0; k < 20; k++) atomicAdd(&FL[cA][i][k], f[k]);
            }
            // ... and j sees i at -r (the mirrored expansion)
#pragma unroll
            for (int k = 0; k < 20; k++) f[k] = 0.f;
            if (inter) {
#pragma unroll
                for (int k = 0; k < 6; k++) q2[k] = w1.q[k];
                if (POT) {
#pragma unroll
                    for (int k = 0; k < 10; k++) q3[k] = A.q3[(size_t)(ca + i) * 10 + k];
                }
                add_field_f(f, mr, g0, g1, g2, g3, w1.mass, q2, POT ? q3 : nullptr);
                if constexpr (EW) {
                    psi_mirror(Dp);
                    sub_field_psi(f, Dp, w1.mass, q2, POT ? q3 : nullptr);
                }
            }
            if (self) {
                fm_combine<1, 0>(f, lvl_take);
                fm_combine<2, 1>(f, lvl_take);
                fm_combine<4, 2>(f, lvl_take);
            } else {
#pragma unroll
                for (int k = 0; k < 20; k++) {
                    const float o = __shfl(f[k], s_lane1);
                    if (s_take1) f[k] += o;
                }
#pragma unroll
                for (int k = 0; k < 20; k++) {
                    const float o = __shfl(f[k], s_lane2);
                    if (s_take2) f[k] += o;
                }
            }
            if (self ? (anyi && !given) : (s_any && !s_give)) {
                const uint32_t sj = self ? j : 8 + j;
                const uint32_t cB = (self ? i >> 1 : i >> 2) % FT_NC;
#pragma unroll
                for (int k = 0; k < 20; k++) atomicAdd(&FL[cB][sj][k], f[k]);
            }
            c_nn += (uint32_t)__builtin_popcountll(im);
            fm_sync();
            for (int v = lane; v < 320; v += 64) {
                const uint32_t s = (uint32_t)v / 20, k = (uint32_t)v - s * 20;
                const bool have = s < 8 ? s < na : (!self && s - 8 < nb);
                float val = 0.f;
#pragma unroll
                for (int c = 0; c < FT_NC; c++) {
                    val += FL[c][s][k];
                    FL[c][s][k] = 0.f;
                }
                if (have && val != 0.f) atomicAdd(&A.F[(size_t)(s < 8 ? ca + s : cb + (s - 8)) * 20 + k], val);
            }
            fm_sync();
        }
        const bool l1 = valid && (w1.meta & WN_LEAF), l2 = valid && (w2.meta & WN_LEAF);
        const uint2 pij = make_uint2(ca + i, cb + j);
        st_push(sf, (act == 3 && !l1) || (act == 2 && !l1 && !l2), pij);
        st_push(sl, act == 2 && l1 && l2, pij);
        st_push(sn, act == 2 && (l1 != l2), l1 ? pij : make_uint2(cb + j, ca + i));
        st_flush(sf, false, A.fout, &A.cnt[1], A.cap_pairs, &A.cnt[4]);
        st_flush(sl, false, A.ll, &A.cnt[2], A.cap_ll, &A.cnt[4]);
        st_flush(sn, false, A.ln, &A.cnt[3], A.cap_ln, &A.cnt[4]);
    }
    st_flush(sf, true, A.fout, &A.cnt[1], A.cap_pairs, &A.cnt[4]);
    st_flush(sl, true, A.ll, &A.cnt[2], A.cap_ll, &A.cnt[4]);
    st_flush(sn, true, A.ln, &A.cnt[3], A.cap_ln, &A.cnt[4]);
    if (lane == 0 && c_nn) atomicAdd(&A.stat[2], (unsigned long long)c_nn);
}

// ---- partner lists of the leaf pairs: count, exclusive scan, scatter
// The dual walk emits the pairs of one leaf close together, so neighbouring lanes often
// name the same leaf: each run of equal values in consecutive lanes makes one atomic.
// ll_run gives the first and last lane of this lane's run; all 64 lanes must be active.
__device__ __forceinline__ void ll_run(uint32_t v, int lane, int &first, int &last)
{
    const uint32_t up = (uint32_t)__shfl_up((int)v, 1), dn = (uint32_t)__shfl_down((int)v, 1);
    const uint64_t heads = __builtin_amdgcn_ballot_w64(lane == 0 || up != v);
    const uint64_t tails = __builtin_amdgcn_ballot_w64(lane == 63 || dn != v);
    first = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));  // lane 0 is always a head
    last = __builtin_ctzll(tails & ~((1ull << lane) - 1ull));       // lane 63 is always a tail
}

// loops run over whole blocks (uniform), so every lane takes part in the run detection;
// lanes past the end hold ~0, which no leaf index equals
__global__ __launch_bounds__(256) void k_ll_count(const uint2 *__restrict__ ll, uint32_t n, uint32_t *__restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    for (uint32_t b = blockIdx.x * blockDim.x; b < n; b += gridDim.x * blockDim.x) {
        const uint32_t k = b + threadIdx.x;
        const uint2 p = k < n ? ll[k] : make_uint2(~0u, ~0u);
        int f, l;
        ll_run(p.x, lane, f, l);
        if (k < n && lane == l) atomicAdd(&cnt[p.x], (uint32_t)(l - f + 1));
        ll_run(p.y, lane, f, l);
        if (k < n && lane == l) atomicAdd(&cnt[p.y], (uint32_t)(l - f + 1));
    }
}

// exclusive scan of v[0..m) in place, 1024 values per block; block totals to bsum
__global__ __launch_bounds__(256) void k_scan_blocks(uint32_t *__restrict__ v, uint32_t m, uint32_t *__restrict__ bsum)
{
    __shared__ uint32_t s[256];
    const uint32_t base = blockIdx.x * 1024 + threadIdx.x * 4;
    uint32_t x[4], t = 0;
    for (int k = 0; k < 4; k++) {
        x[k] = base + k < m ? v[base + k] : 0u;
        t += x[k];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - t;  // exclusive prefix of this thread's four values
    for (int k = 0; k < 4; k++) {
        if (base + k < m) v[base + k] = run;
        run += x[k];
    }
    if (threadIdx.x == 255) bsum[blockIdx.x] = s[255];
}

// exclusive scan of the block totals (one block), then the total at v[m]
__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *__restrict__ bsum, uint32_t nb, uint32_t *__restrict__ total)
{
    __shared__ uint32_t s[1024];
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += 1024) {
        const uint32_t k = c0 + threadIdx.x;
        const uint32_t x = k < nb ? bsum[k] : 0u;
        s[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t add = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < nb) bsum[k] = carry + s[threadIdx.x] - x;
        const uint32_t sum = s[1023];
        __syncthreads();
        carry += sum;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(uint32_t *__restrict__ v, uint32_t m, const uint32_t *__restrict__ bsum,
                           uint32_t *__restrict__ cursor)
{
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        const uint32_t o = v[k] + bsum[k / 1024];
        v[k] = o;
        cursor[k] = o;
    }
}

// the last lane of a run reserves the run's slots; the run's lanes fill them in lane order
__global__ __launch_bounds__(256) void k_ll_scatter(const uint2 *__restrict__ ll, uint32_t n,
                                                    uint32_t *__restrict__ cursor, uint32_t *__restrict__ plist)
{
    const int lane = threadIdx.x & 63;
    for (uint32_t b = blockIdx.x * blockDim.x; b < n; b += gridDim.x * blockDim.x) {
        const uint32_t k = b + threadIdx.x;
        const uint2 p = k < n ? ll[k] : make_uint2(~0u, ~0u);
        int f, l;
        uint32_t o = 0;
        ll_run(p.x, lane, f, l);
        if (k < n && lane == l) o = atomicAdd(&cursor[p.x], (uint32_t)(l - f + 1));
        o = (uint32_t)__shfl((int)o, l);
        if (k < n) plist[o + (uint32_t)(lane - f)] = p.y;
        o = 0;
        ll_run(p.y, lane, f, l);
        if (k < n && lane == l) o = atomicAdd(&cursor[p.y], (uint32_t)(l - f + 1));
        o = (uint32_t)__shfl((int)o, l);
        if (k < n) plist[o + (uint32_t)(lane - f)] = p.x;
    }
}

// force (and potential factor) on a target from one source particle of mass m
template <int KER, bool POT>
__device__ __forceinline__ void fm_pair(const FastArgs &A, const uint4 &t, const uint4 &s, float m, float &fx,
                                        float &fy, float &fz, float &fp)
{
    const float sx = (float)(int32_t)(s.x - t.x) * A.unit;
    const float sy = (float)(int32_t)(s.y - t.y) * A.unit;
    const float sz = (float)(int32_t)(s.z - t.z) * A.unit;
    float K, W;
    pair_kernel<KER == 2 ? 0 : KER, POT>(sx * sx + sy * sy + sz * sz, A.asplit, A.h2, A.hinv, K, W);
    const float mk = m * K;
    fx += mk * sx;
    fy += mk * sy;
    fz += mk * sz;
    if (POT) fp -= m * W;
    if constexpr (KER == 2) {
        float ex, ey, ez, ep = 0.f;
        ew_grad<POT>(A.ew, A.ew_n, A.ew_h, A.ew_hinv, sx, sy, sz, ex, ey, ez, ep);
        fx += m * ex;
        fy += m * ey;
        fz += m * ez;
        if (POT) fp += m * ep;
    }
}

// Phase 2: all particle pairs of one leaf per wavefront.  Lane = (particle a,
// stride slot k): slot k takes every S-th particle of each source leaf; the S
// partial sums of a particle are added in LDS.  Writes acc (the first sum a
// particle receives; phase 3 adds to it).
template <int KER, bool POT>
__global__ __launch_bounds__(256) void k_fast_pp(FastArgs A, uint32_t nnodes)
{
    __shared__ float part[4][64][4];
    __shared__ uint32_t srcs[4][FP_SRC];  // partner particles of the current window
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long n_pairs = 0;  // this lane's share of the pair count
    for (uint32_t q = blockIdx.x * 4 + wv; q < nnodes; q += gridDim.x * 4) {
        const uint32_t meta = fm_uni(A.wn[q].meta);
        if (!(meta & WN_LEAF)) continue;
        const uint32_t ja = fm_uni(A.wn[q].next), na = fm_uni(A.wn[q].num);
        const uint32_t p0 = fm_uni(A.pstart[q]), p1 = fm_uni(A.pstart[q + 1]);
        if (lane == 0) n_pairs += (unsigned long long)na * (na - 1) / 2;  // pairs inside the leaf
        for (uint32_t c0 = 0; c0 < na; c0 += 64) {
            const uint32_t nc = min(na - c0, 64u);               // targets in this chunk
            const uint32_t S = 64u / nc;                          // stride slots per target
            const uint32_t a = (uint32_t)lane % nc, k = (uint32_t)lane / nc;
            const bool act = k < S;
            const uint32_t t = ja + c0 + a;
            const uint4 me = A.parts[t];
            float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
            // the leaf's own particles
            for (uint32_t s = (act ? k : na); s < na; s += S) {
                const uint4 src = A.parts[ja + s];
                fm_pair<KER, POT>(A, me, src, (ja + s != t) ? __uint_as_float(src.w) : 0.f, fx, fy, fz, fp);
            }
            // partner leaves, their records fetched 64 at a time; their particles are listed
            // one after another in LDS, so that the S slots of a target stride over all of
            // them at once (small leaves would otherwise leave most slots idle)
            for (uint32_t e0 = p0; e0 < p1; e0 += 64) {
                const uint32_t ne = min(64u, p1 - e0);
                uint32_t pj = 0, pn = 0;
                if ((uint32_t)lane < ne) {
                    const uint32_t b = A.plist[e0 + lane];
                    pj = A.wn[b].next;
                    pn = A.wn[b].num;
                    // each leaf pair is listed at both leaves: count it at the lower node index
                    if (c0 == 0 && b > q) n_pairs += (unsigned long long)na * pn;
                }
                // exclusive prefix of the partners' particle counts
                uint32_t incl = pn;
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t v = (uint32_t)__shfl_up((int)incl, d);
                    if (lane >= d) incl += v;
                }
                const uint32_t excl = incl - pn;
                const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                for (uint32_t w0 = 0; w0 < total; w0 += FP_SRC) {
                    const uint32_t wn = min((uint32_t)FP_SRC, total - w0);
                    const uint32_t lo = max(excl, w0), hi = min(excl + pn, w0 + wn);
                    for (uint32_t x = lo; x < hi; x++) srcs[wv][x - w0] = pj + (x - excl);
                    fm_sync();
                    for (uint32_t s = (act ? k : wn); s < wn; s += S) {
                        const uint4 src = A.parts[srcs[wv][s]];
                        fm_pair<KER, POT>(A, me, src, __uint_as_float(src.w), fx, fy, fz, fp);
                    }
                    fm_sync();
                }
            }
            part[wv][lane][0] = fx;
            part[wv][lane][1] = fy;
            part[wv][lane][2] = fz;
            part[wv][lane][3] = fp;
            fm_sync();
            if ((uint32_t)lane < nc) {
                double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
                for (uint32_t kk = 0; kk < S; kk++) {
                    const uint32_t l = kk * nc + a;
                    sx += part[wv][l][0];
                    sy += part[wv][l][1];
                    sz += part[wv][l][2];
                    sp += part[wv][l][3];
                }
                double *o = A.acc + (size_t)t * 4;
                o[0] = sx;
                o[1] = sy;
                o[2] = sz;
                o[3] = POT ? sp : 0.0;
            }
            fm_sync();
        }
    }
    for (int off = 32; off > 0; off >>= 1) n_pairs += __shfl_xor(n_pairs, off);
    if (lane == 0 && n_pairs) atomicAdd(&A.stat[0], n_pairs);
}

template <bool POT>
__device__ __forceinline__ void fm_deposit(const FastArgs &A, uint32_t j, float fx, float fy, float fz, float fp)
{
    double *a = A.acc + (size_t)j * 4;
    atomicAdd(a + 0, (double)fx);
    atomicAdd(a + 1, (double)fy);
    atomicAdd(a + 2, (double)fz);
    if (POT) atomicAdd(a + 3, (double)fp);
}

// sums of the 20 values over each aligned 16-lane group (a DPP row), in the group's first
// lane; the other lanes end with partial sums.  Row shifts with the adds, no LDS traffic;
// every lane of the wavefront must be active.  `span` (wavefront-uniform: 4, 8 or 16) bounds
// the lanes of every group that may hold nonzero values: the shifts that would only add
// zeros are skipped, which leaves every sum bitwise unchanged.
__device__ __forceinline__ void fm_gsum20(float v[20], uint32_t span)
{
#pragma unroll
    for (int q = 0; q < 20; q++) {
        v[q] += __uint_as_float(fm_from_next<1>(__float_as_uint(v[q])));
        v[q] += __uint_as_float(fm_from_next<2>(__float_as_uint(v[q])));
    }
    if (span > 4) {
#pragma unroll
        for (int q = 0; q < 20; q++) v[q] += __uint_as_float(fm_from_next<4>(__float_as_uint(v[q])));
    }
    if (span > 8) {
#pragma unroll
        for (int q = 0; q < 20; q++) v[q] += __uint_as_float(fm_from_next<8>(__float_as_uint(v[q])));
    }
}
// this lane's group's 16 bits of a wavefront mask
__device__ __forceinline__ uint32_t fm_gbits(uint64_t m, uint32_t g) { return (uint32_t)(m >> (16 * g)) & 0xffffu; }

// Phase 3: leaf-node pairs, four per wavefront.  Each 16-lane group takes one
// pair at a time (16 of the leaf's particles per chunk) and walks the
// daughters of the internal node with the particle-node rules, with its own
// stack of (first sibling, count, group lane mask) entries; a group whose walk
// ends deposits its particles' sums and takes the wavefront's next pair.
// Leaves opened in a step give particle pairs for the targets that opened
// them only; these are spread one pair per lane over the whole wavefront.
template <int KER, bool POT>
__global__ __launch_bounds__(256) void k_fast_ln(FastArgs A, uint32_t npairs)
{
    __shared__ uint2 stk[4][4][FT_STK];     // (first sibling, count | group lane mask << 16)
    __shared__ float red[4][4][20];
    __shared__ uint4 tpos[4][64];           // targets (grid position, mass bits) for the leaf pairs
    __shared__ float tacc[4][64][4];        // their pair sums
    __shared__ float sacc[4][4][FT_SB][4];  // pair sums of the current source block of each group
    __shared__ uint2 gblk[4][4];            // each group's source block: first particle, count
    __shared__ uint8_t trank[4][4][16];     // each group's open targets: rank -> lane in the group
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t g = (uint32_t)lane >> 4, gl = (uint32_t)lane & 15u;
    tacc[wv][lane][0] = tacc[wv][lane][1] = tacc[wv][lane][2] = tacc[wv][lane][3] = 0.f;
    for (uint32_t v = (uint32_t)lane; v < 4u * FT_SB * 4u; v += 64u) (&sacc[wv][0][0][0])[v] = 0.f;
    // this wavefront's contiguous share of the pairs
    const uint32_t nw = gridDim.x * 4, wid = blockIdx.x * 4 + wv;
    const uint32_t per = (npairs + nw - 1) / nw;
    uint32_t next = min(npairs, wid * per);  // wavefront-uniform
    const uint32_t end = min(npairs, next + per);
    // group state (uniform within a group)
    int sp = 0;
    uint32_t ja = 0, na = 0, c0 = 0, tb = 0;
    // lane state: one target particle
    uint32_t t = 0;
    bool act = false;
    uint4 me = make_uint4(0u, 0u, 0u, 0u);
    float mt = 0.f, fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
    uint32_t n_pp = 0, n_pn = 0;
    for (;;) {
        // ---- groups whose walk ended: deposit, then the next chunk of the pair or the next pair
        const bool done = sp == 0;
        if (done && act) fm_deposit<POT>(A, t, fx, fy, fz, fp);
        if (done) fx = fy = fz = fp = 0.f;
        const bool more = done && c0 + 16 < na;
        if (more) c0 += 16;
        const bool want = done && !more;
        const uint64_t wm = fm_ballot(want && gl == 0);  // one bit per group that needs a pair
        const uint32_t k = next + (uint32_t)__builtin_popcountll(wm & ((1ull << (16 * g)) - 1ull));
        next = min(end, next + (uint32_t)__builtin_popcountll(wm));
        bool start = more;
        if (want) {
            if (k < end) {
                const uint2 pr = A.ln[k];
                ja = A.wn[pr.x].next;
                na = A.wn[pr.x].num;
                tb = pr.y;
                c0 = 0;
                start = true;
            } else {
                na = 0;
                c0 = 0;
            }
        }
        if (start) {
            t = ja + c0 + gl;
            act = c0 + gl < na;
            me = A.parts[act ? t : ja];
            mt = act ? __uint_as_float(me.w) : 0.f;
        } else if (done) {
            act = false;
        }
        const uint32_t am = fm_gbits(fm_ballot(act), g);
        if (start) {
            if (gl == 0) stk[wv][g][0] = make_uint2(A.wn[tb].next, A.wn[tb].num | (am << 16));
            sp = 1;
        }
        if (!fm_ballot(sp > 0)) break;
        fm_sync();
        // ---- one step of every live group's walk
        const bool live = sp > 0;
        uint2 e = make_uint2(0u, 0u);
        if (live) e = stk[wv][g][sp - 1];
        const uint32_t node = e.x, cnt = e.y & 0xffffu, gm = e.y >> 16;
        if (live) {
            if (cnt > 1) {
                if (gl == 0) stk[wv][g][sp - 1] = make_uint2(node + 1, (cnt - 1) | (gm << 16));
            } else {
                sp--;
            }
        }
        const WNode w = A.wn[live ? node : 0u];
        const bool mine = live && ((gm >> gl) & 1u);
        const int lev = (int)(w.meta & 0xffu);
        // particle (l = 0) against the node: the rules of fm_classify
        float g2;
        const bool touching = fm_cube_gap(me.x, me.y, me.z, w.gx, w.gy, w.gz, 1ull << (A.S - lev - 1), A.unit, g2);
        const bool drop = A.kernel == 1 && g2 > A.rcut2;
        const float r[3] = {(float)(int32_t)(w.cx - me.x) * A.unit, (float)(int32_t)(w.cy - me.y) * A.unit,
                            (float)(int32_t)(w.cz - me.z) * A.unit};
        const float r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const float l = ldexpf(A.box, -lev);
        const float a_t = A.crit ? A.pseed[act ? t : ja] : 0.f, a_n = A.crit ? A.amin[live ? node : 0u] : 0.f;
        const bool inter = mine && !drop && !touching &&
                           fmm_accept(A.crit, A.theta2, A.alpha, 0.f, l, mt, w.mass, a_t, a_n, r2) && r2 >= A.h2;
        const bool open = mine && !drop && !inter;
        const uint64_t im = fm_ballot(inter);
        if (im) {
            float pf[20];
#pragma unroll
            for (int q = 0; q < 20; q++) pf[q] = 0.f;
            if (inter) {
                float g0, g1, g2, g3;
                gfun_f(KER, r2, A.asplit, g0, g1, g2, g3);
                // the node's field at the particle: a = -F1, phi = -F0
                float f[20], q2[6], q3[10];
#pragma unroll
                for (int q = 0; q < 20; q++) f[q] = 0.f;
#pragma unroll
                for (int q = 0; q < 6; q++) q2[q] = w.q[q];
                if (POT) {
#pragma unroll
                    for (int q = 0; q < 10; q++) q3[q] = A.q3[(size_t)node * 10 + q];
                }
                add_field_f(f, r, g0, g1, g2, g3, w.mass, q2, POT ? q3 : nullptr);
                float Dp[20];
                if constexpr (KER == 2) {
                    ew_d20(A.ew, A.ew_n, A.ew_h, A.ew_hinv, r[0], r[1], r[2], Dp);
                    sub_field_psi(f, Dp, w.mass, q2, POT ? q3 : nullptr);
                }
                fx -= f[1];
                fy -= f[2];
                fz -= f[3];
                if (POT) fp -= f[0];
                // the particle's field at the node (source at -r)
                const float mr[3] = {-r[0], -r[1], -r[2]};
                add_field_f(pf, mr, g0, g1, g2, g3, mt, nullptr, nullptr);
                if constexpr (KER == 2) {
                    psi_mirror(Dp);
                    sub_field_psi(pf, Dp, mt, nullptr, nullptr);
                }
                n_pn++;
            }
            // only the lanes in im hold nonzero values: within each group, lanes 0-3, 0-7 or all 16
            const uint32_t span = (im & 0xff00ff00ff00ff00ull) ? 16u : (im & 0xfff0fff0fff0fff0ull) ? 8u : 4u;
            fm_gsum20(pf, span);  // read by lane 0 of the group
            const bool gi = fm_gbits(im, g) != 0;
            if (gi && gl == 0) {
#pragma unroll
                for (int q = 0; q < 20; q++) red[wv][g][q] = pf[q];
            }
            fm_sync();
            if (gi) {
                atomicAdd(&A.F[(size_t)node * 20 + gl], red[wv][g][gl]);
                if (gl < 4) atomicAdd(&A.F[(size_t)node * 20 + 16 + gl], red[wv][g][16 + gl]);
            }
            fm_sync();
        }
        const uint64_t om = fm_ballot(open);
        if (om) {
            const uint32_t go = fm_gbits(om, g);
            const bool gleaf = go && (w.meta & WN_LEAF);
            const uint64_t lm = fm_ballot(gleaf);
            if (lm) {
                // particle pairs with the opened leaves of the wavefront's groups, one pair per
                // lane: group g pairs its open targets with the leaf's sources in blocks of
                // FT_SB; both sides are summed in LDS and the sources' sums deposited per block
                const uint32_t om16 = fm_gbits(om, g);
                if (open && gleaf) {
                    trank[wv][g][__builtin_popcount(om16 & ((1u << gl) - 1u))] = (uint8_t)gl;
                    tpos[wv][lane] = make_uint4(me.x, me.y, me.z, __float_as_uint(mt));
                }
                // the longest opened leaf of the wavefront
                // (the node and gleaf are uniform within a group: one lane of each group suffices)
                const uint32_t nl = gleaf ? w.num : 0u;
                const uint32_t nmax = max(max((uint32_t)__builtin_amdgcn_readlane((int)nl, 0),
                                              (uint32_t)__builtin_amdgcn_readlane((int)nl, 16)),
                                          max((uint32_t)__builtin_amdgcn_readlane((int)nl, 32),
                                              (uint32_t)__builtin_amdgcn_readlane((int)nl, 48)));
                const uint32_t gk = gleaf ? (uint32_t)__builtin_popcount(om16) : 0u;
                for (uint32_t b0 = 0; b0 < nmax; b0 += FT_SB) {
                    const uint32_t nb = gleaf && b0 < w.num ? min(w.num - b0, (uint32_t)FT_SB) : 0u;
                    // pair ranges of the four groups (uniform)
                    const uint32_t P0 = __builtin_amdgcn_readlane((int)(gk * nb), 0),
                                   P1 = __builtin_amdgcn_readlane((int)(gk * nb), 16),
                                   P2 = __builtin_amdgcn_readlane((int)(gk * nb), 32),
                                   P3 = __builtin_amdgcn_readlane((int)(gk * nb), 48);
                    if (gl == 0) gblk[wv][g] = make_uint2(w.next + b0, nb);
                    fm_sync();
                    const uint32_t e1 = P0, e2 = e1 + P1, e3 = e2 + P2, ptot = e3 + P3;
                    for (uint32_t base = 0; base < ptot; base += 64) {
                        const uint32_t p = base + (uint32_t)lane;
                        if (p < ptot) {
                            const uint32_t gg = (p >= e1 ? 1u : 0u) + (p >= e2 ? 1u : 0u) + (p >= e3 ? 1u : 0u);
                            const uint32_t pl = p - (gg == 0 ? 0u : gg == 1 ? e1 : gg == 2 ? e2 : e3);
                            const uint2 gb = gblk[wv][gg];
                            // pl = rank nb + k, k < nb <= FT_SB
                            uint32_t rk = (uint32_t)((float)pl * __builtin_amdgcn_rcpf((float)gb.y));
                            if (rk * gb.y > pl) rk--;
                            else if ((rk + 1u) * gb.y <= pl) rk++;
                            const uint32_t ks = pl - rk * gb.y;
                            const uint32_t tl = 16u * gg + trank[wv][gg][rk];
                            const uint4 T = tpos[wv][tl];
                            const uint4 src = A.parts[gb.x + ks];
                            const float sx = (float)(int32_t)(src.x - T.x) * A.unit;
                            const float sy = (float)(int32_t)(src.y - T.y) * A.unit;
                            const float sz = (float)(int32_t)(src.z - T.z) * A.unit;
                            float K, W;
                            pair_kernel<KER == 2 ? 0 : KER, POT>(sx * sx + sy * sy + sz * sz, A.asplit, A.h2,
                                                                 A.hinv, K, W);
                            // force per unit source mass on the target (the source gets minus it)
                            float vx = K * sx, vy = K * sy, vz = K * sz;
                            if constexpr (KER == 2) {
                                float ex, ey, ez, ep = 0.f;
                                ew_grad<POT>(A.ew, A.ew_n, A.ew_h, A.ew_hinv, sx, sy, sz, ex, ey, ez, ep);
                                vx += ex;
                                vy += ey;
                                vz += ez;
                                if (POT) W -= ep;
                            }
                            const float ms = __uint_as_float(src.w), mo = __uint_as_float(T.w);
                            atomicAdd(&tacc[wv][tl][0], ms * vx);
                            atomicAdd(&tacc[wv][tl][1], ms * vy);
                            atomicAdd(&tacc[wv][tl][2], ms * vz);
                            if (POT) atomicAdd(&tacc[wv][tl][3], -ms * W);
                            atomicAdd(&sacc[wv][gg][ks][0], -mo * vx);
                            atomicAdd(&sacc[wv][gg][ks][1], -mo * vy);
                            atomicAdd(&sacc[wv][gg][ks][2], -mo * vz);
                            if (POT) atomicAdd(&sacc[wv][gg][ks][3], -mo * W);
                        }
                    }
                    fm_sync();
                    // the sources' sums of this block, cleared for the next
                    if (gk) {
                        for (uint32_t kk = gl; kk < nb; kk += 16) {
                            float *sa = sacc[wv][g][kk];
                            fm_deposit<POT>(A, w.next + b0 + kk, sa[0], sa[1], sa[2], sa[3]);
                            sa[0] = sa[1] = sa[2] = sa[3] = 0.f;
                        }
                    }
                    fm_sync();
                }
                // the targets' sums into their registers
                fx += tacc[wv][lane][0];
                fy += tacc[wv][lane][1];
                fz += tacc[wv][lane][2];
                if (POT) fp += tacc[wv][lane][3];
                tacc[wv][lane][0] = tacc[wv][lane][1] = tacc[wv][lane][2] = tacc[wv][lane][3] = 0.f;
                if (open && gleaf) n_pp += w.num;
            }
            if (go && !gleaf && sp < FT_STK) {
                if (gl == 0) stk[wv][g][sp] = make_uint2(w.next, w.num | (go << 16));
                sp++;
            } else if (go && !gleaf && gl == 0) {
                atomicOr(A.flags, G4_FLAG_FMM_STACK);  // one entry per level: never expected
            }
        }
        fm_sync();
    }
    // counters: one atomic per wavefront
    unsigned long long c_pp = n_pp, c_pn = n_pn;
    for (int off = 32; off > 0; off >>= 1) {
        c_pp += __shfl_xor(c_pp, off);
        c_pn += __shfl_xor(c_pn, off);
    }
    if (lane == 0) {
        if (c_pp) atomicAdd(&A.stat[0], c_pp);
        if (c_pn) atomicAdd(&A.stat[1], c_pn);
    }
}

// L2P at each particle plus its accumulated particle sums, written in caller order
template <bool POT>
__global__ void k_fast_finish(const FastArgs A, const uint32_t *__restrict__ leafid, const uint32_t *__restrict__ perm,
                              int64_t n, double G, double *ax, double *ay, double *az, double *pot)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 me = A.parts[i];
    const uint32_t L = leafid[i];
    const WNode wl = A.wn[L];
    const float a[3] = {(float)(int32_t)(me.x - wl.cx) * A.unit, (float)(int32_t)(me.y - wl.cy) * A.unit,
                        (float)(int32_t)(me.z - wl.cz) * A.unit};
    float P[20];
#pragma unroll
    for (int k = 0; k < 20; k++) P[k] = A.F[(size_t)L * 20 + k];
    const float *F1 = P + 1, *F2 = P + 4, *F3 = P + 10;
    float g[3], ph = P[0];
#pragma unroll
    for (int ii = 0; ii < 3; ii++) {
        float s = -F1[ii];
        ph -= F1[ii] * a[ii];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            s += F2[i2(ii, k)] * a[k];
            ph += 0.5f * F2[i2(ii, k)] * a[ii] * a[k];
#pragma unroll
            for (int m = 0; m < 3; m++) {
                s -= 0.5f * F3[i3(ii, k, m)] * a[k] * a[m];
                ph -= F3[i3(ii, k, m)] * a[ii] * a[k] * a[m] * (1.0f / 6.0f);
            }
        }
        g[ii] = s;
    }
    const double *q = A.acc + (size_t)i * 4;
    const uint32_t o = perm[i];
    ax[o] = G * (q[0] + (double)g[0]);
    ay[o] = G * (q[1] + (double)g[1]);
    az[o] = G * (q[2] + (double)g[2]);
    if (POT && pot) pot[o] = G * (q[3] - (double)ph);
}

// ------------------------------------------------------------------ host side
struct FmmLayout {
    size_t cnt, f0, f1, nkey, nkey2, nval, nval2, pkey, pkey2, pval, pval2, nstart, nend, pstart, pend, F, leafid,
        amin, sort_tmp, sort_bytes, total;
    uint32_t cap_pairs, cap_node, cap_part;
};

static int fmm_layout(int64_t n, int64_t cap_nodes, double factor, FmmLayout *L)
{
    const double f = factor > 0 ? factor : 1.0;
    L->cap_pairs = (uint32_t)std::min<double>(4.0e9, f * 48.0 * n + 4096);
    L->cap_node = (uint32_t)std::min<double>(4.0e9, f * 96.0 * n + 4096);
    L->cap_part = (uint32_t)std::min<double>(4.0e9, f * 160.0 * n + 4096);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += (b + 255) & ~(size_t)255;
        return o;
    };
    L->cnt = take(64);
    L->f0 = take((size_t)L->cap_pairs * 8);
    L->f1 = take((size_t)L->cap_pairs * 8);
    L->nkey = take((size_t)L->cap_node * 8);
    L->nkey2 = take((size_t)L->cap_node * 8);
    L->nval = take((size_t)L->cap_node * 4);
    L->nval2 = take((size_t)L->cap_node * 4);
    L->pkey = take((size_t)L->cap_part * 8);
    L->pkey2 = take((size_t)L->cap_part * 8);
    L->pval = take((size_t)L->cap_part * 4);
    L->pval2 = take((size_t)L->cap_part * 4);
    L->nstart = take((size_t)cap_nodes * 4);
    L->nend = take((size_t)cap_nodes * 4);
    L->pstart = take((size_t)n * 4);
    L->pend = take((size_t)n * 4);
    L->F = take((size_t)cap_nodes * 20 * 4);
    L->leafid = take((size_t)n * 4);
    L->amin = take((size_t)cap_nodes * 4);
    L->sort_bytes = g4_radix_sort_temp_bytes((int64_t)std::max(L->cap_node, L->cap_part));
    L->sort_tmp = take(L->sort_bytes);
    L->total = off;
    return G4_OK;
}

struct FastLayout {
    size_t cnt, f0, f1, ll, ln, pstart, cursor, bsum, plist, F, acc, leafid, amin, total;
    uint32_t cap_pairs, cap_ll, cap_ln;
};

static void fast_layout(int64_t n, int64_t cap_nodes, double factor, FastLayout *L)
{
    const double f = factor > 0 ? factor : 1.0;
    L->cap_pairs = (uint32_t)std::min<double>(2.0e9, f * 3.0 * n + 4096);
    L->cap_ll = (uint32_t)std::min<double>(2.0e9, f * 12.0 * n + 4096);
    L->cap_ln = (uint32_t)std::min<double>(2.0e9, f * 3.0 * n + 4096);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += (b + 255) & ~(size_t)255;
        return o;
    };
    L->cnt = take(64);
    L->f0 = take((size_t)L->cap_pairs * 8);
    L->f1 = take((size_t)L->cap_pairs * 8);
    L->ll = take((size_t)L->cap_ll * 8);
    L->ln = take((size_t)L->cap_ln * 8);
    L->pstart = take((size_t)(cap_nodes + 1) * 4);
    L->cursor = take((size_t)cap_nodes * 4);
    L->bsum = take((size_t)(cap_nodes / 1024 + 2) * 4);
    L->plist = take((size_t)L->cap_ll * 2 * 4);
    L->F = take((size_t)cap_nodes * 20 * 4);
    L->acc = take((size_t)n * 4 * 8);
    L->leafid = take((size_t)n * 4);
    L->amin = take((size_t)cap_nodes * 4);
    L->total = off;
}

int g4_fmm_layout_bytes(const g4_tree *t, const g4_fmm_params *fp, double factor, size_t *bytes)
{
    if (!fp->deterministic) {
        FastLayout F;
        fast_layout(t->n, t->cap, factor, &F);
        *bytes = F.total;
        return G4_OK;
    }
    FmmLayout L;
    int st = fmm_layout(t->n, t->cap, factor, &L);
    if (st) return st;
    *bytes = L.total;
    return G4_OK;
}

// Relative criterion: the caller's |a| in sorted order (the tree's seed
// buffer) and each node's minimum, levels from the deepest up.
static int fmm_seed_minima(g4_ctx *ctx, g4_tree *t, const g4_fmm_params *fp, float *amin)
{
    if (int st = g4_launch_gather_seed(ctx, t, fp->a_seed)) return st;
    t->seed_valid = 0;
    const int maxd = t->tp.max_depth;
    for (int l = maxd; l >= 0; l--) k_fmm_amin<<<256, 256, 0, ctx->stream>>>(t->ctr, t->wn, t->aseed, amin, l);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

template <int KER, bool POT>
// up to 4096 blocks of 4 wavefronts: the pairs of a leaf or of a leaf-node pair vary widely in cost,
// and with more, smaller static shares the last wavefronts finish sooner (measured against 1024,
// 2048 and 8192)
static void launch_fast_particles(const FastArgs &A, uint32_t nnodes, uint32_t nln, hipStream_t s)
{
    k_fast_pp<KER, POT><<<(unsigned)std::min<uint64_t>(4096, ((uint64_t)nnodes + 3) / 4), 256, 0, s>>>(A, nnodes);
    if (nln) k_fast_ln<KER, POT><<<(unsigned)std::min<uint64_t>(4096, ((uint64_t)nln + 3) / 4), 256, 0, s>>>(A, nln);
}

static int fmm_fast(g4_ctx *ctx, g4_tree *t, const g4_fmm_params *fp, double factor, void *ws, size_t ws_bytes,
                    double *ax, double *ay, double *az, double *pot, g4_stats *stats)
{
    FastLayout L;
    fast_layout(t->n, t->cap, factor, &L);
    if (ws_bytes < L.total) return g4_set_err(ctx, G4_ENOMEM, "fmm workspace too small");
    char *b = (char *)ws;
    hipStream_t s = ctx->stream;
    FastArgs A;
    A.wn = t->wn;
    A.parts = t->parts;
    A.q3 = t->q3;
    A.S = t->S;
    A.unit = (float)t->unit;
    A.box = (float)t->tp.box;
    const float th = (float)fp->theta;
    A.theta2 = th * th;
    const double h = 2.8 * fp->eps0;
    A.h2 = (float)(h * h);
    A.hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    A.asplit = fp->kernel == 1 ? (float)(0.5 / fp->r_s) : 0.f;
    A.rcut2 = (float)(fp->r_cut * fp->r_cut);
    A.kernel = fp->kernel;
    A.ew = static_cast<const float *>(fp->ewald_table);
    A.ew_n = fp->ewald_n;
    A.ew_h = fp->kernel == 2 ? (float)(0.5 * t->tp.box / fp->ewald_n) : 0.f;
    A.ew_hinv = fp->kernel == 2 ? (float)(2.0 * fp->ewald_n / t->tp.box) : 0.f;
    A.crit = fp->criterion;
    A.alpha = (float)fp->alpha;
    A.pseed = t->aseed;
    A.amin = (float *)(b + L.amin);
    if (A.crit)
        if (int st = fmm_seed_minima(ctx, t, fp, (float *)(b + L.amin))) return st;
    A.cnt = (uint32_t *)(b + L.cnt);
    A.cap_pairs = L.cap_pairs;
    A.ll = (uint2 *)(b + L.ll);
    A.ln = (uint2 *)(b + L.ln);
    A.cap_ll = L.cap_ll;
    A.cap_ln = L.cap_ln;
    A.pstart = (uint32_t *)(b + L.pstart);
    A.plist = (uint32_t *)(b + L.plist);
    A.F = (float *)(b + L.F);
    A.acc = (double *)(b + L.acc);
    A.stat = t->ctr->stat + 6;
    A.flags = &t->ctr->flags;
    uint2 *fr[2] = {(uint2 *)(b + L.f0), (uint2 *)(b + L.f1)};
    if ((uint64_t)t->nbox > L.cap_pairs) return g4_set_err(ctx, G4_ENOMEM, "fmm frontier smaller than the root count");
    if (int zst = g4_launch_zero(ctx, A.cnt, 64)) return zst;
    if (int zst = g4_launch_zero(ctx, A.stat, 3 * sizeof(unsigned long long))) return zst;
    if (int zst = g4_launch_zero(ctx, A.F, (size_t)t->cap * 20 * 4)) return zst;
    A.fin = fr[1];
    A.fout = fr[0];
    k_fast_init<<<(t->nbox + 255) / 256, 256, 0, s>>>(A, t->nbox);
    G4_HIP(ctx, hipGetLastError());
    // 1. node-level dual walk: one pass per level until the frontier is empty (1024 blocks of
    //    4 wavefronts grid-stride over a pass's pairs: measured faster than 512, 2048 or 4096)
    const bool P = pot != nullptr;
    int cur = 0;
    uint32_t h4[8];
    for (int pass = 0; pass < 64; pass++) {
        A.fin = fr[cur];
        A.fout = fr[cur ^ 1];
        if (fp->kernel == 2) {
            if (P) k_fast_open<true, true><<<1024, 256, 0, s>>>(A);
            else k_fast_open<false, true><<<1024, 256, 0, s>>>(A);
        } else {
            if (P) k_fast_open<true, false><<<1024, 256, 0, s>>>(A);
            else k_fast_open<false, false><<<1024, 256, 0, s>>>(A);
        }
        k_fmm_rotate<<<1, 64, 0, s>>>(A.cnt);
        cur ^= 1;
        if ((pass & 3) == 3) {
            G4_HIP(ctx, hipMemcpyAsync(h4, A.cnt, sizeof(h4), hipMemcpyDeviceToHost, s));
            G4_HIP(ctx, hipStreamSynchronize(s));
            if (h4[4]) return g4_set_err(ctx, G4_ENOMEM, "fmm lists exceed the workspace");
            if (h4[0] == 0) break;
        }
    }
    G4_HIP(ctx, hipGetLastError());
    uint32_t nnodes = 0;
    G4_HIP(ctx, hipMemcpyAsync(h4, A.cnt, sizeof(h4), hipMemcpyDeviceToHost, s));
    G4_HIP(ctx, hipMemcpyAsync(&nnodes, &t->ctr->node_count, 4, hipMemcpyDeviceToHost, s));
    G4_HIP(ctx, hipStreamSynchronize(s));
    if (h4[4]) return g4_set_err(ctx, G4_ENOMEM, "fmm lists exceed the workspace");
    if (h4[0] != 0) return g4_set_err(ctx, G4_EHIP, "fmm dual walk did not terminate");
    if (nnodes < 1 || (int64_t)nnodes > t->cap) return g4_set_err(ctx, G4_EHIP, "bad node count");
    const uint32_t nll = h4[2], nln = h4[3];
    // 2. partner lists of the leaf pairs (counting sort by leaf), then all particle pairs per leaf
    uint32_t *cursor = (uint32_t *)(b + L.cursor), *bsum = (uint32_t *)(b + L.bsum);
    if (int zst = g4_launch_zero(ctx, A.pstart, (size_t)(nnodes + 1) * 4)) return zst;
    if (nll) k_ll_count<<<2048, 256, 0, s>>>(A.ll, nll, A.pstart);
    const uint32_t nb = (nnodes + 1023) / 1024;
    k_scan_blocks<<<nb, 256, 0, s>>>(A.pstart, nnodes, bsum);
    k_scan_sums<<<1, 1024, 0, s>>>(bsum, nb, A.pstart + nnodes);
    k_scan_add<<<(unsigned)std::min<uint32_t>(4096, (nnodes + 255) / 256), 256, 0, s>>>(A.pstart, nnodes, bsum, cursor);
    if (nll) k_ll_scatter<<<2048, 256, 0, s>>>(A.ll, nll, cursor, A.plist);
    // 2 and 3: particle pairs per leaf (writes every particle's sums), then the leaf-node pairs (adds)
    if (fp->kernel == 1) {
        if (P) launch_fast_particles<1, true>(A, nnodes, nln, s);
        else launch_fast_particles<1, false>(A, nnodes, nln, s);
    } else if (fp->kernel == 2) {
        if (P) launch_fast_particles<2, true>(A, nnodes, nln, s);
        else launch_fast_particles<2, false>(A, nnodes, nln, s);
    } else {
        if (P) launch_fast_particles<0, true>(A, nnodes, nln, s);
        else launch_fast_particles<0, false>(A, nnodes, nln, s);
    }
    // 4. downward pass and evaluation at the particles
    FmmArgs D;
    D.wn = t->wn;
    D.ctr = t->ctr;
    D.parent = t->parent;
    D.unit = A.unit;
    const int maxd = t->tp.max_depth;
    for (int l = 1; l <= maxd; l++) k_fmm_l2l<<<1024, 256, 0, s>>>(D, l, A.F);
    uint32_t *leafid = (uint32_t *)(b + L.leafid);
    k_fmm_leafmap<<<(unsigned)std::min<uint32_t>(65535, (nnodes + 255) / 256), 256, 0, s>>>(t->ctr, t->wn, leafid);
    const unsigned pb = (unsigned)((t->n + 255) / 256);
    if (P) k_fast_finish<true><<<pb, 256, 0, s>>>(A, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
    else k_fast_finish<false><<<pb, 256, 0, s>>>(A, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
    G4_HIP(ctx, hipGetLastError());
    if (stats) {
        DevCounters hc;
        G4_HIP(ctx, hipMemcpyAsync(&hc, t->ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
        G4_HIP(ctx, hipStreamSynchronize(s));
        std::memset(stats, 0, sizeof(*stats));
        stats->n_pp = hc.stat[6];
        stats->n_pn = hc.stat[7];
        stats->n_nn = hc.stat[8];
        stats->n_nodes = hc.node_count;
        stats->flags = hc.flags;
    }
    return G4_OK;
}

static int bits_for(uint64_t v)
{
    int b = 1;
    while (b < 32 && (1ull << b) <= v) b++;
    return b;
}

int g4_launch_fmm(g4_ctx *ctx, g4_tree *t, const g4_fmm_params *fp, double factor, void *ws, size_t ws_bytes,
                  double *ax, double *ay, double *az, double *pot, g4_stats *stats)
{
    if (!fp->deterministic) return fmm_fast(ctx, t, fp, factor, ws, ws_bytes, ax, ay, az, pot, stats);
    FmmLayout L;
    int st = fmm_layout(t->n, t->cap, factor, &L);
    if (st) return g4_set_err(ctx, st, "fmm workspace layout failed");
    if (ws_bytes < L.total) return g4_set_err(ctx, G4_ENOMEM, "fmm workspace too small");
    char *b = (char *)ws;
    hipStream_t s = ctx->stream;
    FmmArgs A;
    A.wn = t->wn;
    A.parts = t->parts;
    A.q3 = t->q3;
    A.ctr = t->ctr;
    A.parent = t->parent;
    A.S = t->S;
    A.unit = (float)t->unit;
    A.box = (float)t->tp.box;
    A.theta = (float)fp->theta;
    const double h = 2.8 * fp->eps0;
    A.h2 = (float)(h * h);
    A.hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    A.asplit = fp->kernel == 1 ? (float)(0.5 / fp->r_s) : 0.f;
    A.rcut2 = (float)(fp->r_cut * fp->r_cut);
    A.kernel = fp->kernel;
    A.ew = static_cast<const float *>(fp->ewald_table);
    A.ew_n = fp->ewald_n;
    A.ew_h = fp->kernel == 2 ? (float)(0.5 * t->tp.box / fp->ewald_n) : 0.f;
    A.ew_hinv = fp->kernel == 2 ? (float)(2.0 * fp->ewald_n / t->tp.box) : 0.f;
    A.crit = fp->criterion;
    A.alpha = (float)fp->alpha;
    A.pseed = t->aseed;
    A.amin = (float *)(b + L.amin);
    if (A.crit)
        if (int st2 = fmm_seed_minima(ctx, t, fp, (float *)(b + L.amin))) return st2;
    A.cnt = (uint32_t *)(b + L.cnt);
    A.cap_pairs = L.cap_pairs;
    A.nkey = (uint64_t *)(b + L.nkey);
    A.nval = (uint32_t *)(b + L.nval);
    A.cap_node = L.cap_node;
    A.pkey = (uint64_t *)(b + L.pkey);
    A.pval = (uint32_t *)(b + L.pval);
    A.cap_part = L.cap_part;
    A.bfirst = t->bfirst;
    A.stat = t->ctr->stat + 6;
    uint2 *fr[2] = {(uint2 *)(b + L.f0), (uint2 *)(b + L.f1)};
    if ((uint64_t)t->nbox > L.cap_pairs) return g4_set_err(ctx, G4_ENOMEM, "fmm frontier smaller than the root count");
    k_fmm_init<<<(t->nbox + 255) / 256, 256, 0, s>>>(A.cnt, fr[0], A.stat, t->nbox);
    G4_HIP(ctx, hipGetLastError());
    // dual walk: passes until the frontier is empty (checked every 8 passes)
    int cur = 0;
    for (int pass = 0; pass < 512; pass++) {
        A.fin = fr[cur];
        A.fout = fr[cur ^ 1];
        k_fmm_traverse<<<2048, 256, 0, s>>>(A);
        k_fmm_rotate<<<1, 64, 0, s>>>(A.cnt);
        cur ^= 1;
        if ((pass & 7) == 7) {
            uint32_t h4[8];
            G4_HIP(ctx, hipMemcpyAsync(h4, A.cnt, sizeof(h4), hipMemcpyDeviceToHost, s));
            G4_HIP(ctx, hipStreamSynchronize(s));
            if (h4[4]) return g4_set_err(ctx, G4_ENOMEM, "fmm interaction lists exceed the workspace");
            if (h4[0] == 0) break;
        }
    }
    G4_HIP(ctx, hipGetLastError());
    uint32_t h4[8];
    G4_HIP(ctx, hipMemcpyAsync(h4, A.cnt, sizeof(h4), hipMemcpyDeviceToHost, s));
    G4_HIP(ctx, hipStreamSynchronize(s));
    if (h4[4]) return g4_set_err(ctx, G4_ENOMEM, "fmm interaction lists exceed the workspace");
    if (h4[0] != 0) return g4_set_err(ctx, G4_EHIP, "fmm dual walk did not terminate");
    const uint32_t n_node = h4[2], n_part = h4[3];
    int64_t nn_host = 0;
    {
        DevCounters hc;
        G4_HIP(ctx, hipMemcpyAsync(&hc, t->ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
        G4_HIP(ctx, hipStreamSynchronize(s));
        nn_host = hc.node_count;
    }
    // sort the entries by (target, source): each target's sum then runs in source order,
    // independent of the order in which the walk appended its entries
    uint64_t *nk2 = (uint64_t *)(b + L.nkey2), *pk2 = (uint64_t *)(b + L.pkey2);
    uint32_t *nv2 = (uint32_t *)(b + L.nval2), *pv2 = (uint32_t *)(b + L.pval2);
    int alt = 0;
    if (n_node) {
        if (int st = g4_radix_sort_u64(ctx, A.nkey, nk2, A.nval, nv2, n_node, 0, 32 + bits_for((uint64_t)nn_host),
                                       b + L.sort_tmp, L.sort_bytes, &alt))
            return st;
        if (!alt) {
            std::swap(A.nkey, nk2);
            std::swap(A.nval, nv2);
        }
    }
    if (n_part) {
        if (int st = g4_radix_sort_u64(ctx, A.pkey, pk2, A.pval, pv2, n_part, 0, 32 + bits_for((uint64_t)t->n),
                                       b + L.sort_tmp, L.sort_bytes, &alt))
            return st;
        if (!alt) {
            std::swap(A.pkey, pk2);
            std::swap(A.pval, pv2);
        }
    }
    // sorted entries: keys in nk2 / pk2, sources in nv2 / pv2
    uint32_t *nstart = (uint32_t *)(b + L.nstart), *nend = (uint32_t *)(b + L.nend);
    uint32_t *pstart = (uint32_t *)(b + L.pstart), *pend = (uint32_t *)(b + L.pend);
    if (int zst = g4_launch_zero(ctx, nstart, (size_t)t->cap * 4)) return zst;
    if (int zst = g4_launch_zero(ctx, nend, (size_t)t->cap * 4)) return zst;
    if (int zst = g4_launch_zero(ctx, pstart, (size_t)t->n * 4)) return zst;
    if (int zst = g4_launch_zero(ctx, pend, (size_t)t->n * 4)) return zst;
    if (n_node) k_fmm_csr<<<2048, 256, 0, s>>>(nk2, n_node, nstart, nend);
    if (n_part) k_fmm_csr<<<2048, 256, 0, s>>>(pk2, n_part, pstart, pend);
    A.nval = nv2;
    A.pval = pv2;
    float *F = (float *)(b + L.F);
    if (fp->kernel == 2) k_fmm_m2l<true><<<(unsigned)((nn_host + 255) / 256), 256, 0, s>>>(A, nstart, nend, F);
    else k_fmm_m2l<false><<<(unsigned)((nn_host + 255) / 256), 256, 0, s>>>(A, nstart, nend, F);
    const int maxd = t->tp.max_depth;
    for (int l = 1; l <= maxd; l++) k_fmm_l2l<<<1024, 256, 0, s>>>(A, l, F);
    uint32_t *leafid = (uint32_t *)(b + L.leafid);
    k_fmm_leafmap<<<(unsigned)((nn_host + 255) / 256), 256, 0, s>>>(t->ctr, t->wn, leafid);
    const unsigned pb = (unsigned)((t->n + 255) / 256);
    if (fp->kernel == 2) {
        if (pot) k_fmm_particles<2, true><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
        else k_fmm_particles<2, false><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
    } else if (fp->kernel == 1) {
        if (pot) k_fmm_particles<1, true><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
        else k_fmm_particles<1, false><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
    } else {
        if (pot) k_fmm_particles<0, true><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
        else k_fmm_particles<0, false><<<pb, 256, 0, s>>>(A, pstart, pend, F, leafid, t->perm1, t->n, fp->G, ax, ay, az, pot);
    }
    G4_HIP(ctx, hipGetLastError());
    if (stats) {
        DevCounters hc;
        G4_HIP(ctx, hipMemcpyAsync(&hc, t->ctr, sizeof(hc), hipMemcpyDeviceToHost, s));
        G4_HIP(ctx, hipStreamSynchronize(s));
        std::memset(stats, 0, sizeof(*stats));
        stats->n_pp = hc.stat[6];
        stats->n_pn = hc.stat[7];
        stats->n_nn = hc.stat[8];
        stats->n_nodes = hc.node_count;
        stats->flags = hc.flags;
    }
    return G4_OK;
}
