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
#include <utility>

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
    L->leafof = take((size_t)n * 4);
    // a walk grid never has more wavefronts than work items (<= n), rounded up to whole blocks of 4
    int64_t waves = ((n > 0 ? n : 1) + 3) / 4 * 4;
    if (waves > G4_WALK_MAX_WAVES) waves = G4_WALK_MAX_WAVES;
    L->spill_waves = waves;
    L->spill = take((size_t)waves * G4_WALK_SPILL * 16);
    L->srtab = take((size_t)G4_SRTAB_FUNCS * G4_SRTAB_MAX * 16);
    // digit tables of the key sort and of the forest's sort by box
    L->sort_bytes = g4_radix_sort_temp_bytes(n > 0 ? n : 1);
    L->sort_tmp = take(L->sort_bytes);
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
    if (!tp->periodic)
        if (int st = g4_launch_zero(ctx, flag, 4)) return st;
    if (n > 0)
        k_quantize<<<grid_for(n), kBlock, 0, ctx->stream>>>(pos, n, tp->periodic, inv, tp->origin[0], tp->origin[1],
                                                           tp->origin[2], x, y, z, flag);
    G4_HIP(ctx, hipGetLastError());
    // the periodic map cannot fail: no read-back, so the host does not wait here
    if (tp->periodic) return G4_OK;
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

// Peano-Hilbert index of a cell of the 2^21 grid, from its 21-bit
// coordinates, by Skilling's method ("Programming the Hilbert curve", AIP
// Conf. Proc. 707, 2004): from the top bit down, the coordinates are reflected
// and exchanged so that each level's sub-cube is entered in the curve's own
// orientation, then Gray-decoded; the result interleaved x, y, z from the top
// bit is the index.  Its level-l digit (bits 3 (21 - l) .. +2) labels one
// octant of the level-(l - 1) cube, as the Morton digit does, so both keys
// cut the same nested cubes.
__device__ __forceinline__ uint64_t ph_key21(uint32_t x, uint32_t y, uint32_t z)
{
    uint32_t c[3] = {x, y, z};
    for (uint32_t q = 1u << 20; q > 1u; q >>= 1) {
        const uint32_t p = q - 1u;
        for (int i = 0; i < 3; i++) {
            if (c[i] & q) {
                c[0] ^= p;  // reflect the low bits of the first coordinate
            } else {
                const uint32_t t = (c[0] ^ c[i]) & p;  // exchange the low bits with coordinate i
                c[0] ^= t;
                c[i] ^= t;
            }
        }
    }
    c[1] ^= c[0];
    c[2] ^= c[1];
    uint32_t t = 0;
    for (uint32_t q = 1u << 20; q > 1u; q >>= 1)
        if (c[2] & q) t ^= q - 1u;
    return (spread3(c[0] ^ t) << 2) | (spread3(c[1] ^ t) << 1) | spread3(c[2] ^ t);
}

// Curve key from the top 21 bits of each root-relative coordinate: Morton
// (bit interleaving; the level-l octant digit (x<<2 | y<<1 | z) sits at bit
// 3 (21 - l)) or Peano-Hilbert.
__device__ __forceinline__ uint64_t curve_key(uint32_t x, uint32_t y, uint32_t z, int drop, uint32_t corner, int kind)
{
    const uint32_t rx = (x - corner) >> drop, ry = (y - corner) >> drop, rz = (z - corner) >> drop;
    return kind == 1 ? ph_key21(rx, ry, rz) : (spread3(rx) << 2) | (spread3(ry) << 1) | spread3(rz);
}

// Curve keys, the identity permutation, and the particles packed as one
// 16-byte record each in caller order (pk), so that the gather into key
// order reads one record per particle instead of four separate words.
__global__ void k_keys(const uint32_t *__restrict__ X, const uint32_t *__restrict__ Y,
                       const uint32_t *__restrict__ Z, const float *__restrict__ m, int64_t n, int drop,
                       uint32_t corner, int kind, uint64_t *__restrict__ keys, uint32_t *__restrict__ perm,
                       uint4 *__restrict__ pk)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = X[i], y = Y[i], z = Z[i];
        keys[i] = curve_key(x, y, z, drop, corner, kind);
        perm[i] = (uint32_t)i;
        pk[i] = make_uint4(x, y, z, __float_as_uint(m[i]));
    }
}

__global__ void k_gather(const uint4 *__restrict__ pk, const uint32_t *__restrict__ perm, int64_t n,
                         uint4 *__restrict__ parts)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        parts[i] = pk[perm[i]];
}

// the packed caller-order records live in the moments buffer, which is
// free from the key pass until the upward pass (it holds >= 160 bytes per
// particle, the records 16)
static inline uint4 *packed_staging(g4_tree *t) { return reinterpret_cast<uint4 *>(t->mom); }

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
        for (int s = 0; s < 18; s++) C->stat[s] = 0;
        bfirst[0] = 0;
        bcount[0] = n;
        parent[0] = 0xffffffffu;
    }
}

// sum over the eight lanes of a group; every lane ends with the same bits
template <typename T>
__device__ __forceinline__ T grp8_sum(T v)
{
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}

// nodes up to this many particles find their octant boundaries by one
// strided pass over their keys instead of a search
static constexpr uint32_t kScanMax = 256;
// blocks of the split passes: one per compute unit keeps the number of
// same-address atomics per level at most this
static constexpr int kSplitBlocks = 256;

// Process the nodes of one level: a node with more than B particles (and
// above the depth cap) gets its non-empty octants as children, delimited by
// the octant digit boundaries in its sorted key range.
//
// A block takes a slice of the level's nodes (the level spread evenly over
// the grid) and works in four steps, with block barriers between them:
//  1. one thread per node: leaf records are written, the nodes to split are
//     listed in LDS, small (<= kScanMax particles) and large apart;
//  2. octant starts: a small node by a group of eight lanes, which count its
//     octant digits in one strided pass (loads that do not wait on each
//     other); a large node by a whole wavefront, eight lanes per boundary
//     running a 9-ary search (log_9 of the size rounds of dependent loads
//     rather than log_2: the top levels hold nodes of millions of keys);
//  3. child counts, an exclusive scan over the block, and ONE atomic on the
//     level's counter for the block's children (same-address atomics are
//     serialised chip-wide, about 11 ns each, so one per node or per
//     wavefront would cost more than all the searches);
//  4. one thread per split node writes its children and its record.
// An empty level returns at once and writes nothing; the node count is
// summed from the level sizes after the last level.

// nodes a block takes per pass (LDS lists and octant starts are sized for it)
#define SPLIT_CHUNK 1024

__device__ __forceinline__ void node_record(DevCounters *C, const uint4 *__restrict__ parts, WNode *__restrict__ wn,
                                            uint32_t q, uint32_t first, uint32_t count, bool split, uint32_t c0,
                                            uint32_t nch, int level, int B, int S, uint32_t corner)
{
    // the geometric centre of the cube from any particle inside it
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
    if (split) {
        w.next = c0;
        w.num = nch;
        w.meta = (uint32_t)level;
    } else {
        w.next = first;
        w.num = count;
        w.meta = (uint32_t)level | WN_LEAF;
        if (count > (uint32_t)B) atomicOr(&C->flags, 1u);
    }
    wn[q] = w;
}

// Start of octant d = lane % 8 of a node of at most kScanMax particles, by
// the group of eight lanes holding `lane` (all eight call this): histogram of
// the octant digits over a strided pass (16-bit fields, two words), then
// prefix sums. The loads go out eight at a time (clamped indices, no
// branches), so a batch costs one trip to memory rather than eight.
__device__ __forceinline__ uint32_t group_octant_start(const uint64_t *__restrict__ keys, uint32_t first,
                                                       uint32_t count, uint32_t lane, int shift)
{
    const uint32_t d = lane & 7, stop = first + count;
    uint64_t h03 = 0, h47 = 0;
    for (uint32_t j0 = first + d; j0 < stop; j0 += 64) {
        uint64_t kv[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) {
            const uint32_t j = j0 + 8 * u;
            kv[u] = keys[j < stop ? j : stop - 1];
        }
#pragma unroll
        for (uint32_t u = 0; u < 8; u++) {
            const uint32_t e = (uint32_t)(kv[u] >> shift) & 7u;
            const uint64_t one = j0 + 8 * u < stop ? 1ull << (16 * (e & 3)) : 0ull;
            if (e < 4) h03 += one;
            else h47 += one;
        }
    }
    h03 = grp8_sum(h03);
    h47 = grp8_sum(h47);
    uint32_t lo = first;
    for (uint32_t e = 0; e < 8; e++) {
        const uint32_t he = (uint32_t)(((e < 4 ? h03 : h47) >> (16 * (e & 3))) & 0xffffu);
        if (e < d) lo += he;
    }
    return lo;
}

// Start of octant b = lane / 8 of a large node, by the whole wavefront (all
// 64 lanes call this). Lane (b, k) keeps the search range [lo, hi] of the
// first key with digit >= b and probes position k + 1 of 9 in it; the eight
// answers narrow the range to a ninth. Every lane of group b returns it.
__device__ __forceinline__ uint32_t wave_octant_start(const uint64_t *__restrict__ keys, uint32_t first,
                                                      uint32_t count, uint32_t lane, int shift)
{
    const uint32_t b = lane >> 3, k = lane & 7, stop = first + count;
    const uint64_t target = ((keys[first] >> (shift + 3)) << (shift + 3)) | ((uint64_t)b << shift);
    // octant 0 starts at the node's first key; the others are searched in [first, stop]
    uint32_t lo = first, hi = b == 0 ? first : stop;
    while (__ballot(hi > lo) != 0ull) {
        const uint32_t len = hi - lo;
        const uint32_t pos = lo + (uint32_t)(((uint64_t)len * (k + 1)) / 9u);
        const bool less = len > 0 && keys[pos] < target;
        const uint32_t c = __popc((uint32_t)(__ballot(less) >> (lane & 56)) & 0xffu);
        // the probes below target form a prefix; the boundary is in (probe c-1, probe c]
        const uint32_t p_lo = __shfl(pos, (int)((lane & 56) + (c > 0 ? c - 1 : 0)));
        const uint32_t p_hi = __shfl(pos, (int)((lane & 56) + (c < 8 ? c : 7)));
        if (len > 0) {
            if (c > 0) lo = p_lo + 1;
            if (c < 8) hi = p_hi;
        }
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_split(DevCounters *C, const uint64_t *__restrict__ keys,
                                               const uint4 *__restrict__ parts, uint32_t *__restrict__ bfirst,
                                               uint32_t *__restrict__ bcount, uint32_t *__restrict__ parent,
                                               WNode *__restrict__ wn, int level, int B, int maxd, int S,
                                               uint32_t corner, int64_t cap)
{
    // the pass's split nodes: small ones from the front, large ones from the back
    __shared__ uint32_t s_node[SPLIT_CHUNK];
    // entry i (small nodes first, then large): octant starts and end of the node
    __shared__ uint32_t s_start[SPLIT_CHUNK][8];
    __shared__ uint32_t s_stop[SPLIT_CHUNK];
    __shared__ uint32_t s_off[SPLIT_CHUNK];  // first child of entry i, relative to the block's base
    __shared__ uint32_t s_ctr[2], s_wsum[4], s_base;
    // level l is complete (pass l-1 has finished); level l+1 starts right after it
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    if (beg == end) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) C->lvl_start[level + 1] = end;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t cnt = end - beg;
    const int shift = 3 * (G4_MAXLEV - level - 1);
    uint32_t per = (cnt + gridDim.x - 1) / gridDim.x;
    if (per > SPLIT_CHUNK) per = SPLIT_CHUNK;
    for (uint64_t pass = blockIdx.x; pass * per < cnt; pass += gridDim.x) {
        const uint32_t cb = beg + (uint32_t)(pass * per), ce = min(cb + per, end);
        if (t < 2) s_ctr[t] = 0;
        __syncthreads();
        // 1. leaves and the list of nodes to split
        for (uint32_t q = cb + t; q < ce; q += 256) {
            const uint32_t first = bfirst[q], count = bcount[q];
            const bool split = count > (uint32_t)B && level < maxd;
            if (!split) node_record(C, parts, wn, q, first, count, false, 0, 0, level, B, S, corner);
            else if (count <= kScanMax) s_node[atomicAdd(&s_ctr[0], 1u)] = q;
            else s_node[SPLIT_CHUNK - 1 - atomicAdd(&s_ctr[1], 1u)] = q;
        }
        __syncthreads();
        const uint32_t ns = s_ctr[0], nl = s_ctr[1], nsplit = ns + nl;
        // 2. octant starts
        for (uint32_t i0 = 0; i0 < ns; i0 += 32) {
            const uint32_t i = i0 + (t >> 3);
            if (i < ns) {
                const uint32_t q = s_node[i], first = bfirst[q], count = bcount[q];
                s_start[i][lane & 7] = group_octant_start(keys, first, count, lane, shift);
                if ((lane & 7) == 0) s_stop[i] = first + count;
            }
        }
        for (uint32_t k = wv; k < nl; k += 4) {
            const uint32_t q = s_node[SPLIT_CHUNK - 1 - k], first = bfirst[q], count = bcount[q];
            const uint32_t lo = wave_octant_start(keys, first, count, lane, shift);
            if ((lane & 7) == 0) s_start[ns + k][lane >> 3] = lo;
            if (lane == 0) s_stop[ns + k] = first + count;
        }
        __syncthreads();
        // 3. child counts (four entries a thread), block scan, one atomic
        uint32_t nc[4], sum = 0;
#pragma unroll
        for (uint32_t u = 0; u < 4; u++) {
            const uint32_t i = 4 * t + u;
            nc[u] = 0;
            if (i < nsplit)
                for (uint32_t d = 0; d < 8; d++) nc[u] += (d < 7 ? s_start[i][d + 1] : s_stop[i]) > s_start[i][d];
            sum += nc[u];
        }
        uint32_t incl = sum;
#pragma unroll
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_wsum[wv] = incl;
        __syncthreads();
        uint32_t before = incl - sum, total = 0;
        for (uint32_t w = 0; w < 4; w++) {
            before += w < wv ? s_wsum[w] : 0u;
            total += s_wsum[w];
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; u++) {
            const uint32_t i = 4 * t + u;
            if (i < nsplit) s_off[i] = before;
            before += nc[u];
        }
        if (t == 0) s_base = total ? atomicAdd(&C->lvl_count[level + 1], total) : 0u;
        __syncthreads();
        // 4. children and records of the split nodes
        for (uint32_t i = t; i < nsplit; i += 256) {
            const uint32_t q = i < ns ? s_node[i] : s_node[SPLIT_CHUNK - 1 - (i - ns)];
            const uint32_t first = s_start[i][0], stop = s_stop[i];
            const uint32_t c0 = end + s_base + s_off[i];
            uint32_t nch = 0;
            for (uint32_t d = 0; d < 8; d++) nch += (d < 7 ? s_start[i][d + 1] : stop) > s_start[i][d];
            const bool fits = (int64_t)c0 + nch <= cap;
            if (fits) {
                uint32_t c = c0;
                for (uint32_t d = 0; d < 8; d++) {
                    const uint32_t lo = s_start[i][d], hi = d < 7 ? s_start[i][d + 1] : stop;
                    if (hi > lo) {
                        bfirst[c] = lo;
                        bcount[c] = hi - lo;
                        parent[c] = q;
                        c++;
                    }
                }
            } else {
                atomicOr(&C->flags, 2u);
            }
            node_record(C, parts, wn, q, first, stop - first, fits, c0, nch, level, B, S, corner);
        }
        __syncthreads();
    }
}

// node count = the sum of the level sizes (after the last split pass)
__global__ void k_count_nodes(DevCounters *C)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t s = 0;
        for (int l = 0; l < G4_MAXLEV + 1; l++) s += C->lvl_count[l];
        C->node_count = s;
    }
}

// stable sort of the 63-bit curve keys (keys0, values perm0); the result is
// left in keys1 / perm1 (the views are swapped when the passes end in the
// first pair)
static int sort_keys(g4_ctx *ctx, g4_tree *t)
{
    int alt = 0;
    if (int st = g4_radix_sort_u64(ctx, t->keys0, t->keys1, t->perm0, t->perm1, t->n, 0, 3 * G4_MAXLEV, t->sort_tmp,
                                   t->sort_tmp_bytes, &alt))
        return st;
    if (!alt) {
        std::swap(t->keys0, t->keys1);
        std::swap(t->perm0, t->perm1);
    }
    return G4_OK;
}

int g4_launch_build(g4_ctx *ctx, g4_tree *t, const g4_particles *p)
{
    hipStream_t s = ctx->stream;
    const int64_t n = t->n;
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    k_keys<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, p->mass, n, t->S - G4_MAXLEV, t->corner,
                                          t->tp.key_kind, t->keys0, t->perm0, packed_staging(t));
    G4_HIP(ctx, hipGetLastError());
    if (int st = sort_keys(ctx, t)) return st;
    // sorted keys now live in keys1, the permutation in perm1
    k_gather<<<grid_for(n), kBlock, 0, s>>>(packed_staging(t), t->perm1, n, t->parts);
    k_init<<<1, 64, 0, s>>>(t->ctr, t->bfirst, t->bcount, t->parent, (uint32_t)n);
    G4_HIP(ctx, hipGetLastError());
    for (int l = 0; l <= maxd; l++) {
        // a fixed grid; the kernel reads the true size of the level
        k_split<<<kSplitBlocks, kBlock, 0, s>>>(t->ctr, t->keys1, t->parts, t->bfirst, t->bcount, t->parent, t->wn, l,
                                                      t->tp.leaf_max, maxd, t->S, t->corner, t->cap);
    }
    k_count_nodes<<<1, 64, 0, s>>>(t->ctr);
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
// Eight lanes take one node: a leaf's particles go to the lanes in turn, an
// internal node's children one per lane; the sums close with a fixed
// butterfly over the group, so the result does not depend on timing.
template <typename T>
__global__ void k_moments(const DevCounters *__restrict__ C, const uint4 *__restrict__ parts,
                          WNode *__restrict__ wn, double *__restrict__ mom, float *__restrict__ q3out,
                          uint32_t *__restrict__ leafof, int level, double unit_d)
{
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    const T unit = (T)unit_d;
    const uint32_t d8 = threadIdx.x & 7;
    const uint32_t gid = (blockIdx.x * blockDim.x + threadIdx.x) >> 3, ngroups = (gridDim.x * blockDim.x) >> 3;
    for (uint32_t q = beg + gid; q < end; q += ngroups) {
        WNode w = wn[q];
        const uint32_t g[3] = {w.gx, w.gy, w.gz};
        T M = 0, c1[3] = {0, 0, 0}, s[3];
        T Q2[6] = {0, 0, 0, 0, 0, 0}, Q3[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (sizeof(T) == 4 && (w.meta & WN_LEAF) && w.num <= 32) {
            // up to four particles per lane, loaded together (clamped
            // indices) and kept in registers for both passes (measured
            // faster for the single-precision levels only)
            const uint32_t stop = w.next + w.num;
            uint4 pv[4];
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const uint32_t j = w.next + d8 + 8 * u;
                pv[u] = parts[j < stop ? j : stop - 1];
                if (j < stop) leafof[j] = q;
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const T m = w.next + d8 + 8 * u < stop ? (T)__uint_as_float(pv[u].w) : (T)0;
                const T d[3] = {(T)(int32_t)(pv[u].x - g[0]) * unit, (T)(int32_t)(pv[u].y - g[1]) * unit,
                                (T)(int32_t)(pv[u].z - g[2]) * unit};
                M += m;
                for (int k = 0; k < 3; k++) c1[k] += m * d[k];
            }
            M = grp8_sum(M);
            for (int k = 0; k < 3; k++) s[k] = M > 0 ? grp8_sum(c1[k]) / M : (T)0;
#pragma unroll
            for (uint32_t u = 0; u < 4; u++) {
                const T m = w.next + d8 + 8 * u < stop ? (T)__uint_as_float(pv[u].w) : (T)0;
                const T d[3] = {(T)(int32_t)(pv[u].x - g[0]) * unit - s[0], (T)(int32_t)(pv[u].y - g[1]) * unit - s[1],
                                (T)(int32_t)(pv[u].z - g[2]) * unit - s[2]};
                Q2[0] += m * d[0] * d[0]; Q2[1] += m * d[0] * d[1]; Q2[2] += m * d[0] * d[2];
                Q2[3] += m * d[1] * d[1]; Q2[4] += m * d[1] * d[2]; Q2[5] += m * d[2] * d[2];
                for (int a = 0; a < 10; a++) Q3[a] += m * d[c_i3[a][0]] * d[c_i3[a][1]] * d[c_i3[a][2]];
            }
        } else if (w.meta & WN_LEAF) {
            const uint32_t stop = w.next + w.num;
            for (uint32_t j = w.next + d8; j < stop; j += 8) {
                leafof[j] = q;
                uint4 p = parts[j];
                T m = (T)__uint_as_float(p.w);
                T d[3] = {(T)(int32_t)(p.x - g[0]) * unit, (T)(int32_t)(p.y - g[1]) * unit,
                          (T)(int32_t)(p.z - g[2]) * unit};
                M += m;
                for (int k = 0; k < 3; k++) c1[k] += m * d[k];
            }
            M = grp8_sum(M);
            for (int k = 0; k < 3; k++) s[k] = M > 0 ? grp8_sum(c1[k]) / M : (T)0;
            for (uint32_t j = w.next + d8; j < stop; j += 8) {
                uint4 p = parts[j];
                T m = (T)__uint_as_float(p.w);
                T d[3] = {(T)(int32_t)(p.x - g[0]) * unit - s[0], (T)(int32_t)(p.y - g[1]) * unit - s[1],
                          (T)(int32_t)(p.z - g[2]) * unit - s[2]};
                Q2[0] += m * d[0] * d[0]; Q2[1] += m * d[0] * d[1]; Q2[2] += m * d[0] * d[2];
                Q2[3] += m * d[1] * d[1]; Q2[4] += m * d[1] * d[2]; Q2[5] += m * d[2] * d[2];
                for (int a = 0; a < 10; a++) Q3[a] += m * d[c_i3[a][0]] * d[c_i3[a][1]] * d[c_i3[a][2]];
            }
        } else {
            const bool has = d8 < w.num;
            T Mc = 0, dl[3] = {0, 0, 0}, q2c[6] = {0, 0, 0, 0, 0, 0};
            const double *mc = mom + (size_t)(w.next + (has ? d8 : 0)) * MOM_STRIDE;
            if (has) {
                const WNode &wc = wn[w.next + d8];
                Mc = (T)mc[0];
                dl[0] = (T)(int32_t)(wc.gx - g[0]) * unit + (T)mc[1];
                dl[1] = (T)(int32_t)(wc.gy - g[1]) * unit + (T)mc[2];
                dl[2] = (T)(int32_t)(wc.gz - g[2]) * unit + (T)mc[3];
                for (int a = 0; a < 6; a++) q2c[a] = (T)mc[4 + a];
            }
            M = grp8_sum(Mc);
            for (int k = 0; k < 3; k++) s[k] = M > 0 ? grp8_sum(Mc * dl[k]) / M : (T)0;
            if (has) {
                const T d[3] = {dl[0] - s[0], dl[1] - s[1], dl[2] - s[2]};
                Q2[0] = q2c[0] + Mc * d[0] * d[0]; Q2[1] = q2c[1] + Mc * d[0] * d[1];
                Q2[2] = q2c[2] + Mc * d[0] * d[2]; Q2[3] = q2c[3] + Mc * d[1] * d[1];
                Q2[4] = q2c[4] + Mc * d[1] * d[2]; Q2[5] = q2c[5] + Mc * d[2] * d[2];
                for (int a = 0; a < 10; a++) {
                    const int i = c_i3[a][0], j = c_i3[a][1], k = c_i3[a][2];
                    Q3[a] = (T)mc[10 + a] + d[i] * q2c[p2i(j, k)] + d[j] * q2c[p2i(i, k)] + d[k] * q2c[p2i(i, j)] +
                            Mc * d[i] * d[j] * d[k];
                }
            }
        }
        for (int a = 0; a < 6; a++) Q2[a] = grp8_sum(Q2[a]);
        for (int a = 0; a < 10; a++) Q3[a] = grp8_sum(Q3[a]);
        if (d8 == 0) {
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
}

#define G4_FP64_LEVELS 8

int g4_launch_moments(g4_ctx *ctx, g4_tree *t)
{
    hipStream_t s = ctx->stream;
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    for (int l = maxd; l >= 0; l--) {
        if (l <= G4_FP64_LEVELS)
            k_moments<double><<<grid_for(t->n, 1024), kBlock, 0, s>>>(t->ctr, t->parts, t->wn, t->mom, t->q3, t->leafof, l,
                                                                     t->unit);
        else
            k_moments<float><<<grid_for(t->n, 1024), kBlock, 0, s>>>(t->ctr, t->parts, t->wn, t->mom, t->q3, t->leafof, l,
                                                                    t->unit);
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// Fourth moments Q4 (15 packed components, multi-index order xxxx xxxy ...
// zzzz) about every node's centre of mass, for the walk at p = 4, 5; FP64, one
// thread per node, levels from the deepest up.  A leaf sums m d^(a,b,c) over its
// particles; an internal node shifts its children's moments to its own centre
// of mass: for d = s_child - s,
//   Q4_alpha = sum_{beta <= alpha} C(alpha, beta) Qc_beta d^(alpha - beta),
// C the product of binomial coefficients per axis, Qc_beta the child's moment
// of order |beta| (its mass for 0, zero for 1 about its centre of mass).
__device__ __forceinline__ int m4_idx(int a, int b, int c)
{
    // position of a multi-index within its order: (b + c)(b + c + 1)/2 + c
    return (b + c) * (b + c + 1) / 2 + c;
}

__global__ __launch_bounds__(128) void k_moments4(const DevCounters *__restrict__ C, const uint4 *__restrict__ parts,
                                                  const WNode *__restrict__ wn, const double *__restrict__ mom,
                                                  double *__restrict__ q4, int level, double unit)
{
    const uint32_t beg = C->lvl_start[level], end = beg + C->lvl_count[level];
    constexpr double binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0}, {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
    for (uint32_t q = beg + blockIdx.x * blockDim.x + threadIdx.x; q < end; q += gridDim.x * blockDim.x) {
        const WNode w = wn[q];
        const double *mo = mom + (size_t)q * MOM_STRIDE;
        double Q[15];
#pragma unroll
        for (int k = 0; k < 15; k++) Q[k] = 0.0;
        if (w.meta & WN_LEAF) {
            for (uint32_t j = w.next; j < w.next + w.num; j++) {
                const uint4 p = parts[j];
                const double m = (double)__uint_as_float(p.w);
                const double d[3] = {(double)(int32_t)(p.x - w.gx) * unit - mo[1],
                                     (double)(int32_t)(p.y - w.gy) * unit - mo[2],
                                     (double)(int32_t)(p.z - w.gz) * unit - mo[3]};
                double pw[3][5];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    pw[k][0] = 1.0;
#pragma unroll
                    for (int e = 1; e < 5; e++) pw[k][e] = pw[k][e - 1] * d[k];
                }
#pragma unroll
                for (int a = 4; a >= 0; a--)
#pragma unroll
                    for (int b = 4 - a; b >= 0; b--) Q[m4_idx(a, b, 4 - a - b)] += m * pw[0][a] * pw[1][b] * pw[2][4 - a - b];
            }
        } else {
            for (uint32_t ch = w.next; ch < w.next + w.num; ch++) {
                const WNode wc = wn[ch];
                const double *mc = mom + (size_t)ch * MOM_STRIDE;
                const double *qc4 = q4 + (size_t)ch * 15;
                const double d[3] = {(double)(int32_t)(wc.gx - w.gx) * unit + mc[1] - mo[1],
                                     (double)(int32_t)(wc.gy - w.gy) * unit + mc[2] - mo[2],
                                     (double)(int32_t)(wc.gz - w.gz) * unit + mc[3] - mo[3]};
                double pw[3][5], qc[5][15];
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    pw[k][0] = 1.0;
#pragma unroll
                    for (int e = 1; e < 5; e++) pw[k][e] = pw[k][e - 1] * d[k];
                }
                // the child's moments by order: mass, (no dipole), Q2, Q3, Q4 (packed)
                qc[0][0] = mc[0];
#pragma unroll
                for (int k = 0; k < 6; k++) qc[2][k] = mc[4 + k];
#pragma unroll
                for (int k = 0; k < 10; k++) qc[3][k] = mc[10 + k];
#pragma unroll
                for (int k = 0; k < 15; k++) qc[4][k] = qc4[k];
#pragma unroll
                for (int a = 4; a >= 0; a--)
#pragma unroll
                    for (int b = 4 - a; b >= 0; b--) {
                        const int c = 4 - a - b;
                        double sum = 0.0;
#pragma unroll
                        for (int ba = 0; ba <= 4; ba++)
#pragma unroll
                            for (int bb = 0; bb <= 4; bb++)
#pragma unroll
                                for (int bc = 0; bc <= 4; bc++) {
                                    const int n = ba + bb + bc;
                                    if (ba > a || bb > b || bc > c || n == 1) continue;
                                    sum += binom[a][ba] * binom[b][bb] * binom[c][bc] * qc[n][m4_idx(ba, bb, bc)] *
                                           pw[0][a - ba] * pw[1][b - bb] * pw[2][c - bc];
                                }
                        Q[m4_idx(a, b, c)] += sum;
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < 15; k++) q4[(size_t)q * 15 + k] = Q[k];
    }
}

int g4_launch_moments4(g4_ctx *ctx, g4_tree *t, double *q4)
{
    const int maxd = t->tp.max_depth < 1 ? 1 : (t->tp.max_depth > G4_MAXLEV ? G4_MAXLEV : t->tp.max_depth);
    for (int l = maxd; l >= 0; l--)
        k_moments4<<<2048, 128, 0, ctx->stream>>>(t->ctr, t->parts, t->wn, t->mom, q4, l, t->unit);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ export
__global__ void k_export(const DevCounters *__restrict__ C, const WNode *__restrict__ wn,
                         const uint32_t *__restrict__ bfirst, const uint32_t *__restrict__ bcount,
                         const double *__restrict__ mom, int S, uint32_t corner, double unit, int32_t *level,
                         uint32_t *cell, int64_t *count, int64_t *first, int32_t *leaf, double *mass, double *com,
                         double *q2, double *q3)
{
    const uint32_t nn = C->node_count;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nn; q += gridDim.x * blockDim.x) {
        const WNode w = wn[q];
        const int l = (int)(w.meta & 0xff);
        const uint32_t g[3] = {w.gx, w.gy, w.gz};
        if (level) level[q] = l;
        if (leaf) leaf[q] = (w.meta & WN_LEAF) ? 1 : 0;
        if (count) count[q] = bcount[q];
        if (first) first[q] = bfirst[q];
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

int g4_launch_export(g4_ctx *ctx, const g4_tree *t, int32_t *level, uint32_t *cell, int64_t *count,
                     int64_t *first, int32_t *leaf, double *mass, double *com, double *q2, double *q3)
{
    k_export<<<grid_for(t->cap), kBlock, 0, ctx->stream>>>(t->ctr, t->wn, t->bfirst, t->bcount, t->mom, t->S,
                                                           t->corner, t->unit, level, cell, count, first, leaf, mass,
                                                           com, q2, q3);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

// ------------------------------------------------------------------ zeroing
__global__ void k_zero_words(uint32_t *__restrict__ p, size_t nwords)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int g4_launch_zero(g4_ctx *ctx, void *p, size_t bytes)
{
    const size_t nw = bytes / 4;
    if (nw == 0) return G4_OK;
    k_zero_words<<<grid_for((int64_t)nw), kBlock, 0, ctx->stream>>>(static_cast<uint32_t *>(p), nw);
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

// the particles and their curve keys in the final (box, key) order
__global__ void k_gather_keys(const uint4 *__restrict__ pk, const uint32_t *__restrict__ perm, int64_t n, int drop,
                              uint32_t corner, int kind, uint4 *__restrict__ parts, uint64_t *__restrict__ keys)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 q = pk[perm[i]];
        parts[i] = q;
        keys[i] = curve_key(q.x, q.y, q.z, drop, corner, kind);
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
        for (int s = 0; s < 18; s++) C->stat[s] = 0;
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
    k_keys<<<grid_for(n), kBlock, 0, s>>>(p->x, p->y, p->z, p->mass, n, t->S - G4_MAXLEV, t->corner,
                                          t->tp.key_kind, t->keys0, t->perm0, packed_staging(t));
    G4_HIP(ctx, hipGetLastError());
    if (int st = sort_keys(ctx, t)) return st;
    k_boxkey<<<grid_for(n), kBlock, 0, s>>>(t->perm1, n, off_dev, t->nbox, bkey0);
    int bits = 1;
    while ((1 << bits) < t->nbox) bits++;
    // stable: particles of a box keep their curve order
    int alt = 0;
    if (int st = g4_radix_sort_u32(ctx, bkey0, bkey1, t->perm1, t->perm0, n, 0, bits, t->sort_tmp, t->sort_tmp_bytes,
                                   &alt))
        return st;
    if (alt) std::swap(t->perm0, t->perm1);
    k_gather_keys<<<grid_for(n), kBlock, 0, s>>>(packed_staging(t), t->perm1, n, t->S - G4_MAXLEV, t->corner,
                                                  t->tp.key_kind, t->parts, t->keys1);
    k_init_forest<<<(t->nbox + 255) / 256, 256, 0, s>>>(t->ctr, t->bfirst, t->bcount, t->parent, off_dev, t->nbox);
    G4_HIP(ctx, hipGetLastError());
    for (int l = 0; l <= maxd; l++)
        k_split<<<kSplitBlocks, kBlock, 0, s>>>(t->ctr, t->keys1, t->parts, t->bfirst, t->bcount, t->parent,
                                                      t->wn, l, t->tp.leaf_max, maxd, t->S, t->corner, t->cap);
    k_count_nodes<<<1, 64, 0, s>>>(t->ctr);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
