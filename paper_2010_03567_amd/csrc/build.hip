// build.hip -- integer mapping, Morton keys, radix sort, level-synchronous
// octree construction and the upward multipole pass on gfx950.
//
// Paper: Sec. "Integer coordinates" (fixed-point positions, two's-complement
// nearest image), Sec. "Non-periodic potentials" (isolated root mapped into a
// sub-range of the integer space), Sec. "Geometry of the tree" (nested cubes
// along a space-filling curve, node split only above B particles),
// Sec. "One-sided multipole expansion" (moments about the centre of mass),
// Sec. "Fast multipole method" first phase (moments from daughter moments).
//
// Design: every kernel is a grid-stride loop whose trip count is read from
// device counters, so the whole build is enqueued without a host round trip.
// Nodes of level l+1 are allocated by atomics while level l is processed;
// each level therefore occupies one contiguous index range.  Allocation order
// inside a level varies run to run, results do not: traversal and moment
// sums follow each node's own children in octant order.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "g4_internal.h"

#define TWO32 4294967296.0
#define TWO31 2147483648.0
#define TWO30 1073741824.0

static const int kBlock = 256;

static inline int grid_for(int64_t work, int max_blocks = 4096)
{
    int64_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

// ------------------------------------------------------------------ layout
int g4_layout(const g4_tree_params *tp, int64_t n, WsLayout *L)
{
    int B = tp->leaf_max < 1 ? 1 : tp->leaf_max;
    int maxd = tp->max_depth < 1 ? 1 : (tp->max_depth > G4_MAXLEV ? G4_MAXLEV : tp->max_depth);
    // every node is a leaf (disjoint, non-empty: <= n) or an internal node
    // (disjoint within a level, > B particles each: <= n/(B+1) per level)
    int64_t cap = n + (int64_t)maxd * (n / (B + 1)) + 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L->cap = cap;
    L->ctr = take(sizeof(DevCounters));
    L->keys0 = take((size_t)n * 8);
    L->keys1 = take((size_t)n * 8);
    L->perm0 = take((size_t)n * 4);
    L->perm1 = take((size_t)n * 4);
    L->parts = take((size_t)n * 16);
    L->bfirst = take((size_t)cap * 4);
    L->bcount = take((size_t)cap * 4);
    L->parent = take((size_t)cap * 4);
    L->wn = take((size_t)cap * sizeof(WNode));
    L->q3 = take((size_t)cap * 10 * 4);
    L->mom = take((size_t)cap * MOM_STRIDE * 8);
    L->aseed = take((size_t)n * 4);
    // a walk grid never has more wavefronts than work items (<= n), rounded up to whole blocks of 4
    int64_t waves = ((n > 0 ? n : 1) + 3) / 4 * 4;
    if (waves > G4_WALK_MAX_WAVES) waves = G4_WALK_MAX_WAVES;
    L->spill_waves = waves;
    L->spill = take((size_t)waves * G4_WALK_SPILL * 16);
    size_t sb = 0;
    if (rocprim::radix_sort_pairs((void *)nullptr, sb, (uint64_t *)nullptr, (uint64_t *)nullptr,
                                  (uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)(n > 0 ? n : 1), 0, 63) !=
        hipSuccess)
        return G4_EHIP;
    L->sort_bytes = sb;
    L->sort_tmp = take(sb);
    L->total = off;
    return G4_OK;
}

// ------------------------------------------------------------ quantisation
__global__ void k_quantize(const double *__restrict__ pos, int64_t n, int periodic, double inv, double ox,
                           double oy, double oz, uint32_t *__restrict__ X, uint32_t *__restrict__ Y,
                           uint32_t *__restrict__ Z, int32_t *flag)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double o[3] = {ox, oy, oz};
        uint32_t out[3];
        for (int k = 0; k < 3; k++) {
            double t = (pos[3 * i + k] - o[k]) * inv;
            double f = floor(t);
            if (periodic) {
                double w = f - TWO32 * floor(f * (1.0 / TWO32));
                out[k] = (uint32_t)(uint64_t)w;
            } else {
                if (f < 0.0 || f >= TWO31) {
                    atomicOr(flag, 1);
                    f = f < 0.0 ? 0.0 : TWO31 - 1.0;
                }
                out[k] = (uint32_t)(TWO30 + f);
            }
        }
        X[i] = out[0];
        Y[i] = out[1];
        Z[i] = out[2];
    }
}

int g4_launch_quantize(g4_ctx *ctx, const double *pos, int64_t n, const g4_tree_params *tp, uint32_t *x,
                       uint32_t *y, uint32_t *z, int32_t *flag)
{
    double inv = tp->periodic ? TWO32 / tp->box : TWO31 / tp->box;
    G4_HIP(ctx, hipMemsetAsync(flag, 0, 4, ctx->stream));
    if (n > 0)
        k_quantize<<<grid_for(n), kBlock, 0, ctx->stream>>>(pos, n, tp->periodic, inv, tp->origin[0], tp->origin[1],
                                                           tp->origin[2], x, y, z, flag);
    G4_HIP(ctx, hipGetLastError());
    int32_t h = 0;
    G4_HIP(ctx, hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, ctx->stream));
    G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (h) return g4_set_err(ctx, G4_EROOT, "particle outside the isolated root cube");
    return G4_OK;
}

// ------------------------------------------------------------------- keys
__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

// Morton key from the top 21 bits of each root-relative coordinate; the
// level-l octant digit (x<<2 | y<<1 | z) sits at bit 3 (21 - l).
__global__ void k_keys(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y,
                       const uint32_t *__restrict__ Z, int64_t n, int drop, uint32_t corner,
                       uint64_t *__restrict__ keys, uint32_t *__restrict__ perm)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t rx = (X[i] - corner) >> drop, ry = (Y[i] - corner) >> drop, rz = (Z[i] - corner) >> drop;
        keys[i] = (spread3(rx) << 2) | (spread3(ry) << 1) | spread3(rz);
        perm[i] = (uint32_t)i;
    }
}

__global__ void k_gather(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y,
                         const uint32_t *__restrict__ Z, const float *__restrict__ m,
                         const uint32_t *__restrict__ perm, int64_t n, uint4 *__restrict__ parts)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t p = perm[i];
        parts[i] = make_uint4(X[p], Y[p], Z[p], __float_as_uint(m[p]));
    }
}

__global__ void k_init(DevCounters *C, uint32_t *bfirst, uint32_t *bcount, uint32_t *parent, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        C->node_count = 1;
        C->flags = 0;
        for (int l = 0; l < G4_MAXLEV + 4; l++) {
            C->lvl_start[l] = 0;
            C->lvl_count[l] = 0;
        }
        C->lvl_start[0] = 0;
        C->lvl_count[0] = 1;
        for (int s = 0; s < 16; s++) C->stat[s] = 0;
        bfirst[0] = 0;
        bcount[0] = n;
        parent[0] = 0xffffffffu;
    }
}

// first index in keys[lo, hi) with key >= target
__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t *__restrict__ keys, uint32_t lo, uint32_t hi,
                                                    uint64_t target)
{
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Process the nodes of one level: a node with more than B particles (and
// above the depth cap) gets its non-empty octants as children, found by
// binary search for the octant digit boundaries in its sorted key range.
__global__ void k_split(DevCounters *C, const uint64_t *__restrict__ keys, const uint4 *__restrict__ parts,
                        uint32_t *__restrict__ bfirst, uint32_t *__restrict__ bcount, uint32_t *__restrict__ parent,
                        WNode *__restrict__ wn,
                        int level, int B, int maxd, int S, uint32_t corner, int64_t cap)
{
    // level l is complete (pass l-1 has finished); level l+1 starts right after it
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        C->lvl_start[level + 1] = end;
        if (level == maxd) C->node_count = end;
    }
    for (uint32_t q = beg + blockIdx.x * blockDim.x + threadIdx.x; q < end; q += gridDim.x * blockDim.x) {
        const uint32_t first = bfirst[q], count = bcount[q];
        const uint4 p0 = parts[first];
        const int sh = S - level;
        WNode w;
        uint32_t pc[3] = {p0.x, p0.y, p0.z}, g[3];
        for (int k = 0; k < 3; k++) {
            uint64_t rel = (uint64_t)(uint32_t)(pc[k] - corner);
            g[k] = (uint32_t)((uint64_t)corner + ((rel >> sh) << sh) + (1ull << (sh - 1)));
        }
        w.gx = g[0];
        w.gy = g[1];
        w.gz = g[2];
        w.cx = g[0];
        w.cy = g[1];
        w.cz = g[2];
        w.mass = 0.f;
        for (int k = 0; k < 6; k++) w.q[k] = 0.f;
        bool split = count > (uint32_t)B && level < maxd;
        if (split) {
            const int shift = 3 * (G4_MAXLEV - level - 1);
            const uint64_t base = (keys[first] >> (shift + 3)) << (shift + 3);
            uint32_t bnd[9];
            bnd[0] = first;
            bnd[8] = first + count;
            for (int d = 1; d < 8; d++)
                bnd[d] = lower_bound_u64(keys, bnd[d - 1], first + count, base | ((uint64_t)d << shift));
            uint32_t nch = 0;
            for (int d = 0; d < 8; d++) nch += bnd[d + 1] > bnd[d];
            uint32_t c0 = end + atomicAdd(&C->lvl_count[level + 1], nch);
            if ((int64_t)c0 + nch > cap) {
                atomicOr(&C->flags, 2u);
                split = false;
            } else {
                uint32_t c = c0;
                for (int d = 0; d < 8; d++) {
                    if (bnd[d + 1] > bnd[d]) {
                        bfirst[c] = bnd[d];
                        bcount[c] = bnd[d + 1] - bnd[d];
                        parent[c] = q;
                        c++;
                    }
                }
                w.next = c0;
                w.num = nch;
                w.meta = (uint32_t)level;
            }
        }
        if (!split) {
            w.next = first;
            w.num = count;
            w.meta = (uint32_t)level | WN_LEAF;
            if (count > (uint32_t)B) atomicOr(&C->flags, 1u);
        }
        wn[q] = w;
    }
}

int g4_launch_build(g4_ctx *ctx, g4_tree *t, const g4_particles *p)
{
    hipStream_t s = ctx->stream;
    const int64_t n = t->n;
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    k_keys<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, n, t->S - G4_MAXLEV, t->corner, t->keys0, t->perm0);
    G4_HIP(ctx, hipGetLastError());
    size_t sb = t->sort_tmp_bytes;
    G4_HIP(ctx, rocprim::radix_sort_pairs(t->sort_tmp, sb, t->keys0, t->keys1, t->perm0, t->perm1, (size_t)n, 0,
                                          63, s));
    // sorted keys now live in keys1; keep that name for the split kernels
    k_gather<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, p->mass, t->perm1, n, t->parts);
    k_init<<<1, 64, 0, s>>>(t->ctr, t->bfirst, t->bcount, t->parent, (uint32_t)n);
    G4_HIP(ctx, hipGetLastError());
    for (int l = 0; l <= maxd; l++) {
        // a fixed grid; the grid-stride loop reads the true range of the level
        k_split<<<grid_for(n, 1024), kBlock, 0, s>>>(t->ctr, t->keys1, t->parts, t->bfirst, t->bcount, t->parent, t->wn, l,
                                                      t->tp.leaf_max, maxd, t->S, t->corner, t->cap);
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ---------------------------------------------------------------- moments
// packed symmetric index tables
__constant__ int c_i3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};

__device__ __forceinline__ int p2i(int i, int j)
{
    // packed index of (i, j) in xx xy xz yy yz zz
    if (i > j) { int t = i; i = j; j = t; }
    return i == 0 ? j : (i == 1 ? 2 + j : 5);
}

// Upward pass for one level: leaves from their particles (P2M), internal
// nodes from their children (M2M by the parallel-axis shift):
//   Q2 = sum_c [Q2_c + M_c d d],
//   Q3 = sum_c [Q3_c + d(x)Q2_c (three placements) + M_c d d d],  d = s_c - s.
template <typename T>
__global__ void k_moments(const DevCounters *__restrict__ C, const uint4 *__restrict__ parts,
                          WNode *__restrict__ wn, double *__restrict__ mom, float *__restrict__ q3out, int level,
                          double unit_d)
{
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    const T unit = (T)unit_d;
    for (uint32_t q = beg + blockIdx.x * blockDim.x + threadIdx.x; q < end; q += gridDim.x * blockDim.x) {
        WNode w = wn[q];
        const uint32_t g[3] = {w.gx, w.gy, w.gz};
        T M = 0, c1[3] = {0, 0, 0}, s[3];
        T Q2[6] = {0, 0, 0, 0, 0, 0}, Q3[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (w.meta & WN_LEAF) {
            for (uint32_t j = w.next; j < w.next + w.num; j++) {
                uint4 p = parts[j];
                T m = (T)__uint_as_float(p.w);
                T d[3] = {(T)(int32_t)(p.x - g[0]) * unit, (T)(int32_t)(p.y - g[1]) * unit,
                          (T)(int32_t)(p.z - g[2]) * unit};
                M += m;
                for (int k = 0; k < 3; k++) c1[k] += m * d[k];
            }
            for (int k = 0; k < 3; k++) s[k] = M > 0 ? c1[k] / M : (T)0;
            for (uint32_t j = w.next; j < w.next + w.num; j++) {
                uint4 p = parts[j];
                T m = (T)__uint_as_float(p.w);
                T d[3] = {(T)(int32_t)(p.x - g[0]) * unit - s[0], (T)(int32_t)(p.y - g[1]) * unit - s[1],
                          (T)(int32_t)(p.z - g[2]) * unit - s[2]};
                Q2[0] += m * d[0] * d[0]; Q2[1] += m * d[0] * d[1]; Q2[2] += m * d[0] * d[2];
                Q2[3] += m * d[1] * d[1]; Q2[4] += m * d[1] * d[2]; Q2[5] += m * d[2] * d[2];
                for (int a = 0; a < 10; a++) Q3[a] += m * d[c_i3[a][0]] * d[c_i3[a][1]] * d[c_i3[a][2]];
            }
        } else {
            for (uint32_t c = w.next; c < w.next + w.num; c++) {
                const double *mc = mom + (size_t)c * MOM_STRIDE;
                const WNode &wc = wn[c];
                T Mc = (T)mc[0];
                T dl[3] = {(T)(int32_t)(wc.gx - g[0]) * unit + (T)mc[1], (T)(int32_t)(wc.gy - g[1]) * unit + (T)mc[2],
                           (T)(int32_t)(wc.gz - g[2]) * unit + (T)mc[3]};
                M += Mc;
                for (int k = 0; k < 3; k++) c1[k] += Mc * dl[k];
            }
            for (int k = 0; k < 3; k++) s[k] = M > 0 ? c1[k] / M : (T)0;
            for (uint32_t c = w.next; c < w.next + w.num; c++) {
                const double *mc = mom + (size_t)c * MOM_STRIDE;
                const WNode &wc = wn[c];
                T Mc = (T)mc[0];
                T d[3] = {(T)(int32_t)(wc.gx - g[0]) * unit + (T)mc[1] - s[0],
                          (T)(int32_t)(wc.gy - g[1]) * unit + (T)mc[2] - s[1],
                          (T)(int32_t)(wc.gz - g[2]) * unit + (T)mc[3] - s[2]};
                T q2c[6];
                for (int a = 0; a < 6; a++) q2c[a] = (T)mc[4 + a];
                Q2[0] += q2c[0] + Mc * d[0] * d[0]; Q2[1] += q2c[1] + Mc * d[0] * d[1];
                Q2[2] += q2c[2] + Mc * d[0] * d[2]; Q2[3] += q2c[3] + Mc * d[1] * d[1];
                Q2[4] += q2c[4] + Mc * d[1] * d[2]; Q2[5] += q2c[5] + Mc * d[2] * d[2];
                for (int a = 0; a < 10; a++) {
                    const int i = c_i3[a][0], j = c_i3[a][1], k = c_i3[a][2];
                    Q3[a] += (T)mc[10 + a] + d[i] * q2c[p2i(j, k)] + d[j] * q2c[p2i(i, k)] + d[k] * q2c[p2i(i, j)] +
                             Mc * d[i] * d[j] * d[k];
                }
            }
        }
        double *mo = mom + (size_t)q * MOM_STRIDE;
        mo[0] = (double)M;
        for (int k = 0; k < 3; k++) mo[1 + k] = (double)s[k];
        for (int a = 0; a < 6; a++) mo[4 + a] = (double)Q2[a];
        for (int a = 0; a < 10; a++) mo[10 + a] = (double)Q3[a];
        // walk record: COM on the integer grid, single-precision moments
        uint32_t cg[3];
        for (int k = 0; k < 3; k++) cg[k] = g[k] + (uint32_t)(int64_t)rint((double)s[k] / unit_d);
        w.cx = cg[0];
        w.cy = cg[1];
        w.cz = cg[2];
        w.mass = (float)M;
        for (int a = 0; a < 6; a++) w.q[a] = (float)Q2[a];
        wn[q] = w;
        for (int a = 0; a < 10; a++) q3out[(size_t)q * 10 + a] = (float)Q3[a];
    }
}

#define G4_FP64_LEVELS 8

int g4_launch_moments(g4_ctx *ctx, g4_tree *t)
{
    hipStream_t s = ctx->stream;
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    for (int l = maxd; l >= 0; l--) {
        if (l <= G4_FP64_LEVELS)
            k_moments<double><<<grid_for(t->n, 1024), kBlock, 0, s>>>(t->ctr, t->parts, t->wn, t->mom, t->q3, l,
                                                                     t->unit);
        else
            k_moments<float><<<grid_for(t->n, 1024), kBlock, 0, s>>>(t->ctr, t->parts, t->wn, t->mom, t->q3, l,
                                                                    t->unit);
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ export
__global__ void k_export(const DevCounters *__restrict__ C, const WNode *__restrict__ wn,
                         const uint32_t *__restrict__ bcount, const double *__restrict__ mom, int S, uint32_t corner,
                         double unit, int32_t *level, uint32_t *cell, int64_t *count, int32_t *leaf, double *mass,
                         double *com, double *q2, double *q3)
{
    const uint32_t nn = C->node_count;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += gridDim.x * blockDim.x) {
        const WNode w = wn[q];
        const int l = (int)(w.meta & 0xff);
        const uint32_t g[3] = {w.gx, w.gy, w.gz};
        if (level) level[q] = l;
        if (leaf) leaf[q] = (w.meta & WN_LEAF) ? 1 : 0;
        if (count) count[q] = bcount[q];
        for (int k = 0; k < 3; k++) {
            uint64_t rel = (uint64_t)(uint32_t)(g[k] - corner) - (1ull << (S - l - 1));
            if (cell) cell[3 * (size_t)q + k] = (uint32_t)(rel >> (S - l));
            if (com) com[3 * (size_t)q + k] = (double)(uint32_t)(g[k] - corner) * unit + mom[(size_t)q * MOM_STRIDE + 1 + k];
        }
        if (mass) mass[q] = mom[(size_t)q * MOM_STRIDE];
        if (q2)
            for (int a = 0; a < 6; a++) q2[6 * (size_t)q + a] = mom[(size_t)q * MOM_STRIDE + 4 + a];
        if (q3)
            for (int a = 0; a < 10; a++) q3[10 * (size_t)q + a] = mom[(size_t)q * MOM_STRIDE + 10 + a];
    }
}

int g4_launch_export(g4_ctx *ctx, const g4_tree *t, int32_t *level, uint32_t *cell, int64_t *count, int32_t *leaf,
                     double *mass, double *com, double *q2, double *q3)
{
    k_export<<<grid_for(t->cap), kBlock, 0, ctx->stream>>>(t->ctr, t->wn, t->bcount, t->mom, t->S, t->corner,
                                                           t->unit, level, cell, count, leaf, mass, com, q2, q3);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------- seed gather
__global__ void k_gather_seed(const float *__restrict__ a_caller, const uint32_t *__restrict__ perm, int64_t n,
                              float *__restrict__ a_sorted)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a_sorted[i] = a_caller[perm[i]];
}

int g4_launch_gather_seed(g4_ctx *ctx, g4_tree *t, const float *a_seed_caller)
{
    k_gather_seed<<<grid_for(t->n), kBlock, 0, ctx->stream>>>(a_seed_caller, t->perm1, t->n, t->aseed);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ forest
// Many independent boxes in one node array: particles sorted by (box, Morton
// key), one root per box at level 0 (nodes 0..nbox-1), then the same
// level-synchronous split and upward pass as a single tree.

// box of each Morton-sorted particle (caller index -> box by binary search)
__global__ void k_boxkey(const uint32_t *__restrict__ perm, int64_t n, const int64_t *__restrict__ off, int nbox,
                         uint32_t *__restrict__ bkey)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = perm[i];
        int lo = 0, hi = nbox - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        bkey[i] = (uint32_t)lo;
    }
}

// Morton keys in the final (box, key) order
__global__ void k_keys_perm(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y,
                            const uint32_t *__restrict__ Z, const uint32_t *__restrict__ perm, int64_t n, int drop,
                            uint32_t corner, uint64_t *__restrict__ keys)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = perm[i];
        const uint32_t rx = (X[p] - corner) >> drop, ry = (Y[p] - corner) >> drop, rz = (Z[p] - corner) >> drop;
        keys[i] = (spread3(rx) << 2) | (spread3(ry) << 1) | spread3(rz);
    }
}

__global__ void k_init_forest(DevCounters *C, uint32_t *bfirst, uint32_t *bcount, uint32_t *parent,
                              const int64_t *__restrict__ off, int nbox)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) {
        C->node_count = (uint32_t)nbox;
        C->flags = 0;
        for (int l = 0; l < G4_MAXLEV + 4; l++) {
            C->lvl_start[l] = 0;
            C->lvl_count[l] = 0;
        }
        C->lvl_count[0] = (uint32_t)nbox;
        for (int s = 0; s < 16; s++) C->stat[s] = 0;
    }
    if (b < nbox) {
        bfirst[b] = (uint32_t)off[b];
        bcount[b] = (uint32_t)(off[b + 1] - off[b]);
        parent[b] = 0xffffffffu;
    }
}

int g4_launch_build_forest(g4_ctx *ctx, g4_tree *t, const g4_particles *p, const int64_t *off_dev, uint32_t *bkey0,
                           uint32_t *bkey1)
{
    hipStream_t s = ctx->stream;
    const int64_t n = t->n;
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    k_keys<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, n, t->S - G4_MAXLEV, t->corner, t->keys0, t->perm0);
    G4_HIP(ctx, hipGetLastError());
    size_t sb = t->sort_tmp_bytes;
    G4_HIP(ctx, rocprim::radix_sort_pairs(t->sort_tmp, sb, t->keys0, t->keys1, t->perm0, t->perm1, (size_t)n, 0,
                                          63, s));
    k_boxkey<<<grid_for(n), kBlock, 0, s>>>(t->perm1, n, off_dev, t->nbox, bkey0);
    int bits = 1;
    while ((1 << bits) < t->nbox) bits++;
    sb = t->sort_tmp_bytes;
    // stable: particles of a box keep their Morton order
    G4_HIP(ctx, rocprim::radix_sort_pairs(t->sort_tmp, sb, bkey0, bkey1, t->perm1, t->perm0, (size_t)n, 0, bits, s));
    uint32_t *tmp = t->perm0;
    t->perm0 = t->perm1;
    t->perm1 = tmp;
    k_keys_perm<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, t->perm1, n, t->S - G4_MAXLEV, t->corner, t->keys1);
    k_gather<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, p->mass, t->perm1, n, t->parts);
    k_init_forest<<<(t->nbox + 255) / 256, 256, 0, s>>>(t->ctr, t->bfirst, t->bcount, t->parent, off_dev, t->nbox);
    G4_HIP(ctx, hipGetLastError());
    for (int l = 0; l <= maxd; l++)
        k_split<<<grid_for(n, 1024), kBlock, 0, s>>>(t->ctr, t->keys1, t->parts, t->bfirst, t->bcount, t->parent,
                                                      t->wn, l, t->tp.leaf_max, maxd, t->S, t->corner, t->cap);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
