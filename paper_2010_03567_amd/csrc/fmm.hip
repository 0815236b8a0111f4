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

#include <rocprim/rocprim.hpp>

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
struct Ent {
    uint32_t gx, gy, gz;     // integer centre (position for a particle)
    uint32_t cx, cy, cz;     // integer centre of mass
    uint64_t half;           // integer half side (0 for a particle)
    float l;                 // side length (0 for a particle)
    float mass;
    bool part, leaf;
    uint32_t next, num;      // node: children or particle range
};

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
    const int64_t dc[3] = {(int32_t)(b.gx - a.gx), (int32_t)(b.gy - a.gy), (int32_t)(b.gz - a.gz)};
    const int64_t hs = (int64_t)(a.half + b.half);
    if (A.kernel == 1) {
        float g2 = 0.f;
        for (int k = 0; k < 3; k++) {
            const int64_t gap = (dc[k] < 0 ? -dc[k] : dc[k]) - hs;
            if (gap > 0) {
                const float gf = (float)gap * A.unit;
                g2 += gf * gf;
            }
        }
        if (g2 > A.rcut2) return X;  // nearest sides beyond r_cut: dropped
    }
    bool touching = true;
    for (int k = 0; k < 3; k++)
        if ((dc[k] < 0 ? -dc[k] : dc[k]) > hs) touching = false;
    const float rx = (float)(int32_t)(b.cx - a.cx) * A.unit, ry = (float)(int32_t)(b.cy - a.cy) * A.unit,
                rz = (float)(int32_t)(b.cz - a.cz) * A.unit;
    const float r2 = rx * rx + ry * ry + rz * rz;
    const float ls = a.l + b.l;
    if (!touching && ls * ls < A.theta * A.theta * r2 && r2 >= A.h2) {
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

// wavefront-aggregated append: returns this lane's base index
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, uint32_t n)
{
    const int lane = threadIdx.x & 63;
    uint32_t incl = n;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off);
        if (lane >= off) incl += v;
    }
    const uint32_t total = __shfl(incl, 63);
    uint32_t base = 0;
    if (lane == 63 && total) base = atomicAdd(counter, total);
    base = __shfl(base, 63);
    return base + incl - n;
}

__global__ __launch_bounds__(256) void k_fmm_traverse(FmmArgs A)
{
    // after an overflow the lists are incomplete: stop touching them
    if (A.cnt[4]) return;
    const uint32_t nin = min(A.cnt[0], A.cap_pairs);
    for (uint32_t base = blockIdx.x * blockDim.x; base < nin; base += gridDim.x * blockDim.x) {
        const uint32_t t = base + threadIdx.x;
        Act X;
        X.kind = ACT_NONE;
        X.n_pairs = X.n_node = X.n_part = 0;
        if (t < nin) {
            const uint2 pr = A.fin[t];
            X = classify(A, pr.x, pr.y);
        }
        const uint32_t op = wave_append(&A.cnt[1], X.n_pairs);
        const uint32_t on = wave_append(&A.cnt[2], X.n_node);
        const uint32_t ok = wave_append(&A.cnt[3], X.n_part);
        // interaction counters: particle pairs, particle-node, node-node (one atomic per wavefront)
        unsigned long long c_pp = 0, c_pn = 0, c_nn = 0;
        if (X.kind == ACT_PP) c_pp = 1;
        if (X.kind == ACT_OPEN_PP) c_pp = (unsigned long long)X.na * X.nb;
        if (X.kind == ACT_SELF_LEAF) c_pp = (unsigned long long)X.a.num * (X.a.num - 1) / 2;
        if (X.kind == ACT_PN) c_pn = 1;
        if (X.kind == ACT_NN) c_nn = 1;
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

// g0..g3 of the interaction kernel (Newtonian or short-range) at r
__device__ __forceinline__ void gfun_f(int kernel, float r2, float asplit, float &g0, float &g1, float &g2, float &g3)
{
    const float rinv = rsq(r2), ri2 = rinv * rinv;
    if (kernel == 0) {
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

// M2L / P2L: each node sums the fields of its sources
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
                pair_kernel<KER, POT>(sx * sx + sy * sy + sz * sz, A.asplit, A.h2, A.hinv, K, W);
                const float mk = __uint_as_float(p.w) * K;
                fx += mk * sx;
                fy += mk * sy;
                fz += mk * sz;
                if (POT) fp -= __uint_as_float(p.w) * W;
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

// ------------------------------------------------------------------ host side
struct FmmLayout {
    size_t cnt, f0, f1, nkey, nkey2, nval, nval2, pkey, pkey2, pval, pval2, nstart, nend, pstart, pend, F, leafid,
        sort_tmp, sort_bytes, total;
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
    size_t sb1 = 0, sb2 = 0;
    if (rocprim::radix_sort_pairs((void *)nullptr, sb1, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                  (uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)L->cap_node, 0, 64) != hipSuccess)
        return G4_EHIP;
    if (rocprim::radix_sort_pairs((void *)nullptr, sb2, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                  (uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)L->cap_part, 0, 64) != hipSuccess)
        return G4_EHIP;
    L->sort_bytes = std::max(sb1, sb2);
    L->sort_tmp = take(L->sort_bytes);
    L->total = off;
    return G4_OK;
}

int g4_fmm_layout_bytes(const g4_tree *t, double factor, size_t *bytes)
{
    FmmLayout L;
    int st = fmm_layout(t->n, t->cap, factor, &L);
    if (st) return st;
    *bytes = L.total;
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
    size_t sb = L.sort_bytes;
    if (n_node)
        G4_HIP(ctx, rocprim::radix_sort_pairs((void *)(b + L.sort_tmp), sb, A.nkey, nk2, A.nval, nv2, (size_t)n_node,
                                              0, 32 + bits_for((uint64_t)nn_host), s));
    sb = L.sort_bytes;
    if (n_part)
        G4_HIP(ctx, rocprim::radix_sort_pairs((void *)(b + L.sort_tmp), sb, A.pkey, pk2, A.pval, pv2, (size_t)n_part,
                                              0, 32 + bits_for((uint64_t)t->n), s));
    uint32_t *nstart = (uint32_t *)(b + L.nstart), *nend = (uint32_t *)(b + L.nend);
    uint32_t *pstart = (uint32_t *)(b + L.pstart), *pend = (uint32_t *)(b + L.pend);
    G4_HIP(ctx, hipMemsetAsync(nstart, 0, (size_t)t->cap * 4, s));
    G4_HIP(ctx, hipMemsetAsync(nend, 0, (size_t)t->cap * 4, s));
    G4_HIP(ctx, hipMemsetAsync(pstart, 0, (size_t)t->n * 4, s));
    G4_HIP(ctx, hipMemsetAsync(pend, 0, (size_t)t->n * 4, s));
    if (n_node) k_fmm_csr<<<2048, 256, 0, s>>>(nk2, n_node, nstart, nend);
    if (n_part) k_fmm_csr<<<2048, 256, 0, s>>>(pk2, n_part, pstart, pend);
    A.nval = nv2;
    A.pval = pv2;
    float *F = (float *)(b + L.F);
    k_fmm_m2l<<<(unsigned)((nn_host + 255) / 256), 256, 0, s>>>(A, nstart, nend, F);
    const int maxd = t->tp.max_depth;
    for (int l = 1; l <= maxd; l++) k_fmm_l2l<<<1024, 256, 0, s>>>(A, l, F);
    uint32_t *leafid = (uint32_t *)(b + L.leafid);
    k_fmm_leafmap<<<(unsigned)((nn_host + 255) / 256), 256, 0, s>>>(t->ctr, t->wn, leafid);
    const unsigned pb = (unsigned)((t->n + 255) / 256);
    if (fp->kernel == 1) {
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
