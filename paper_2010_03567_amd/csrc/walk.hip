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
// 64 consecutive Morton-sorted particles, one particle per lane.  Traversal is
// wavefront-uniform: a small LDS stack holds (first sibling, sibling count,
// 64-bit lane mask) entries, so the node index is uniform and the 64-byte node
// record arrives through scalar loads (one read serves all lanes).  Every lane
// takes its own opening decision for its own particle, exactly as in the
// per-particle walk of the paper; __ballot turns the decisions into the masks
// of lanes that open the node (pushed with the children) or use its
// multipoles.  Interactions are FP32 arithmetic on int32 nearest-image
// differences; partial sums are flushed into per-lane FP64 accumulators.
#include <algorithm>
#include <new>
#include <vector>

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
    int exclusion;
    int order;
    float unit;       // physical length per integer step
    float box;        // physical root side
    float h, h2, hinv;
    float asplit;     // 1/(2 r_s)
    float rcut2;
    float theta2;
    float alpha;      // relative-criterion accuracy parameter
    double G;
    double *ax, *ay, *az, *pot;
    uint32_t *counts;
    float *aout_caller, *aout_sorted;
    unsigned long long *stat;   // 3 counters: p2p, p2m, visits
    unsigned long long *wstat;  // 3 counters: node pops, P2M passes, P2P source iterations (per wavefront)
    const uint4 *items;         // work items (first particle, count, root node), or null: groups of `group`
    uint32_t nitems;
    uint32_t *item_ctr;         // zeroed before the launch
};

// g1, g2, g3 (and g0) of the interaction kernel at r (r2, rinv given), r >= h.
template <int KER>
__device__ __forceinline__ void gfun(float r2, float rinv, const WalkArgs &A, float &g0, float &g1, float &g2,
                                     float &g3)
{
    float ri2 = rinv * rinv;
    if (KER == 0) {
        g0 = rinv;
        g1 = -rinv * ri2;
        g2 = -3.0f * g1 * ri2;
        g3 = -5.0f * g2 * ri2;
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

template <int KER, int CRIT, bool POT>
__global__ __launch_bounds__(256) void k_walk(const WalkArgs A)
{
    __shared__ uint4 stk[4][32];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    uint32_t t_pp = 0, t_pm = 0, t_visit = 0;  // per-lane totals over all items
    uint32_t w_pop = 0, w_pm = 0, w_pp = 0;    // wavefront-level work (uniform counters)

    // persistent wavefront: pull work items (a group of particles of one tree) until none are left
    for (;;) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(A.item_ctr, 1u);
    it = (uint32_t)__shfl((int)it, 0);
    if (it >= A.nitems) break;
    int64_t i0;
    uint32_t gcount, root;
    if (A.items) {
        const uint4 w = A.items[it];
        i0 = w.x;
        gcount = w.y;
        root = w.z;
    } else {
        i0 = (int64_t)it * A.group;
        gcount = (uint32_t)min((int64_t)A.group, A.n - i0);
        root = 0;
    }
    const int64_t i = i0 + lane;
    const bool act = (uint32_t)lane < gcount;
    const uint4 me = A.parts[act ? i : i0];
    const float arel = CRIT == 1 ? A.alpha * (act ? A.aseed[i] : 0.f) : 0.f;

    double dax = 0.0, day = 0.0, daz = 0.0, dpot = 0.0;
    float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
    uint32_t n_pp = 0, n_pm = 0, n_visit = 0;
    int pending = 0;

    const uint64_t amask = __ballot(act);
    int sp = 1;
    if (lane == 0) stk[wv][0] = make_uint4(root, 1u, (uint32_t)amask, (uint32_t)(amask >> 32));
    __builtin_amdgcn_wave_barrier();

    while (sp > 0) {
        const uint4 e = stk[wv][sp - 1];
        // readfirstlane returns int: go through uint32_t so no half of the mask sign-extends
        const uint32_t node = (uint32_t)__builtin_amdgcn_readfirstlane(e.x);
        const uint32_t cnt = (uint32_t)__builtin_amdgcn_readfirstlane(e.y);
        const uint64_t mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(e.w) << 32) |
                              (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(e.z);
        if (cnt > 1) {
            if (lane == 0) stk[wv][sp - 1] = make_uint4(node + 1, cnt - 1, e.z, e.w);
        } else {
            sp--;
        }
        const WNode nd = A.wn[node];
        w_pop++;
        const int level = (int)(nd.meta & 0xffu);
        const bool leaf = (nd.meta & WN_LEAF) != 0;
        bool mine = (mask >> lane) & 1ull;

        const float dx = (float)(int32_t)(nd.cx - me.x) * A.unit;
        const float dy = (float)(int32_t)(nd.cy - me.y) * A.unit;
        const float dz = (float)(int32_t)(nd.cz - me.z) * A.unit;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        const uint32_t ex = uabs((int32_t)(nd.gx - me.x));
        const uint32_t ey = uabs((int32_t)(nd.gy - me.y));
        const uint32_t ez = uabs((int32_t)(nd.gz - me.z));
        const float l = ldexpf(A.box, -level);
        if (KER == 1) {
            // nearest edge of the node's cube farther than r_cut: drop it
            const float hl = 0.5f * l;
            const float qx = fmaxf((float)ex * A.unit - hl, 0.f);
            const float qy = fmaxf((float)ey * A.unit - hl, 0.f);
            const float qz = fmaxf((float)ez * A.unit - hl, 0.f);
            mine = mine && (fmaf(qx, qx, fmaf(qy, qy, qz * qz)) <= A.rcut2);
        }
        bool inside = level == 0;
        if (A.exclusion && level > 0) {
            const uint32_t lint = 1u << (A.S - level);
            inside = ex < lint && ey < lint && ez < lint;
        }
        const float rinv = rsq(r2);
        bool accept = !inside && r2 >= A.h2;
        if (CRIT == 0) {
            accept = accept && (l * l < A.theta2 * r2);
        } else {
            // M (l/r)^p / r^2 < alpha |a|  <=>  M l^p < alpha |a| r^(p+2)
            const float lp = A.order >= 3 ? l * l * l : l * l;
            const float rp = A.order >= 3 ? r2 * r2 * r2 * rinv : r2 * r2;
            accept = accept && (nd.mass * lp < arel * rp);
        }
        n_visit += mine;
        const bool use = mine && accept;
        const uint64_t openm = __ballot(mine && !accept);
        if (__ballot(use)) {
            w_pm++;
            if (use) {
                float g0, g1, g2, g3;
                gfun<KER>(r2, rinv, A, g0, g1, g2, g3);
                if (A.order >= 3) {
                    const float qx = fmaf(nd.q[0], dx, fmaf(nd.q[1], dy, nd.q[2] * dz));
                    const float qy = fmaf(nd.q[1], dx, fmaf(nd.q[3], dy, nd.q[4] * dz));
                    const float qz = fmaf(nd.q[2], dx, fmaf(nd.q[4], dy, nd.q[5] * dz));
                    const float rqr = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
                    const float tr = nd.q[0] + nd.q[3] + nd.q[5];
                    const float fac = fmaf(nd.mass, g1, 0.5f * fmaf(g2, tr, g3 * rqr));
                    fx -= fmaf(fac, dx, g2 * qx);
                    fy -= fmaf(fac, dy, g2 * qy);
                    fz -= fmaf(fac, dz, g2 * qz);
                    if (POT) {
                        const float *o = A.q3 + (size_t)node * 10;
                        // Q3 . D3 = 3 g2 (t . r) + g3 Q3(r, r, r), t_k = sum_i Q3_iik
                        const float tx = o[0] + o[3] + o[5], ty = o[1] + o[6] + o[8], tz = o[2] + o[7] + o[9];
                        const float c3 = o[0] * dx * dx * dx + o[6] * dy * dy * dy + o[9] * dz * dz * dz +
                                         3.f * (o[1] * dx * dx * dy + o[2] * dx * dx * dz + o[3] * dx * dy * dy +
                                                o[5] * dx * dz * dz + o[7] * dy * dy * dz + o[8] * dy * dz * dz) +
                                         6.f * o[4] * dx * dy * dz;
                        const float q3d3 = 3.f * g2 * (tx * dx + ty * dy + tz * dz) + g3 * c3;
                        fp -= nd.mass * g0 + 0.5f * (g1 * tr + g2 * rqr) + q3d3 * (1.0f / 6.0f);
                    }
                } else {
                    const float fac = nd.mass * g1;
                    fx -= fac * dx;
                    fy -= fac * dy;
                    fz -= fac * dz;
                    if (POT) {
                        const float qx = fmaf(nd.q[0], dx, fmaf(nd.q[1], dy, nd.q[2] * dz));
                        const float qy = fmaf(nd.q[1], dx, fmaf(nd.q[3], dy, nd.q[4] * dz));
                        const float qz = fmaf(nd.q[2], dx, fmaf(nd.q[4], dy, nd.q[5] * dz));
                        const float rqr = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
                        const float tr = nd.q[0] + nd.q[3] + nd.q[5];
                        fp -= nd.mass * g0 + 0.5f * (g1 * tr + g2 * rqr);
                    }
                }
                n_pm++;
            }
            if (++pending >= 8) {
                dax += fx; day += fy; daz += fz;
                if (POT) dpot += fp;
                fx = fy = fz = fp = 0.f;
                pending = 0;
            }
        }
        if (openm) {
            if (leaf) {
                w_pp += nd.num;
                const bool op = (openm >> lane) & 1ull;
                for (uint32_t j = nd.next; j < nd.next + nd.num; j++) {
                    const uint4 src = A.parts[j];
                    const float mj = (op && (int64_t)j != i) ? __uint_as_float(src.w) : 0.f;
                    const float sx = (float)(int32_t)(src.x - me.x) * A.unit;
                    const float sy = (float)(int32_t)(src.y - me.y) * A.unit;
                    const float sz = (float)(int32_t)(src.z - me.z) * A.unit;
                    const float s2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
                    float K, W;
                    pair_kernel<KER, POT>(s2, A.asplit, A.h2, A.hinv, K, W);
                    const float mk = mj * K;
                    fx = fmaf(mk, sx, fx);
                    fy = fmaf(mk, sy, fy);
                    fz = fmaf(mk, sz, fz);
                    if (POT) fp = fmaf(-mj, W, fp);
                }
                if (op) n_pp += nd.num - ((i >= (int64_t)nd.next && i < (int64_t)(nd.next + nd.num)) ? 1u : 0u);
                dax += fx; day += fy; daz += fz;
                if (POT) dpot += fp;
                fx = fy = fz = fp = 0.f;
                pending = 0;
            } else {
                if (lane == 0) stk[wv][sp] = make_uint4(nd.next, nd.num, (uint32_t)openm, (uint32_t)(openm >> 32));
                sp++;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    dax += fx; day += fy; daz += fz;
    if (POT) dpot += fp;

    if (act) {
        const uint32_t o = A.perm[i];
        const double gx = A.G * dax, gy = A.G * day, gz = A.G * daz;
        A.ax[o] = gx;
        A.ay[o] = gy;
        A.az[o] = gz;
        if (POT && A.pot) A.pot[o] = A.G * dpot;
        const float amag = (float)sqrt(gx * gx + gy * gy + gz * gz);
        if (A.aout_sorted) A.aout_sorted[i] = amag;
        if (A.aout_caller) A.aout_caller[o] = amag;
        if (A.counts) {
            A.counts[2 * (size_t)o] = n_pp;
            A.counts[2 * (size_t)o + 1] = n_pm;
        }
    }
    t_pp += n_pp;
    t_pm += n_pm;
    t_visit += n_visit;
    }  // work items
    if (A.stat) {
        // wavefront sums of the interaction counters, one atomic per wavefront
        unsigned long long s0 = t_pp, s1 = t_pm, s2 = t_visit;
        for (int off = 32; off > 0; off >>= 1) {
            s0 += __shfl_xor(s0, off);
            s1 += __shfl_xor(s1, off);
            s2 += __shfl_xor(s2, off);
        }
        if (lane == 0) {
            atomicAdd(&A.stat[0], s0);
            atomicAdd(&A.stat[1], s1);
            atomicAdd(&A.stat[2], s2);
            // wavefront-level iterations (slots 9..11 of the counter block, walk call only)
            if (A.wstat) {
                atomicAdd(&A.wstat[0], (unsigned long long)w_pop);
                atomicAdd(&A.wstat[1], (unsigned long long)w_pm);
                atomicAdd(&A.wstat[2], (unsigned long long)w_pp);
            }
        }
    }
}

template <int KER, int CRIT, bool POT>
static void launch_walk(const WalkArgs &A, hipStream_t s)
{
    // persistent grid: 4 wavefronts per block, at most 8 resident wavefronts per SIMD
    int64_t blocks = ((int64_t)A.nitems + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    k_walk<KER, CRIT, POT><<<(unsigned)blocks, 256, 0, s>>>(A);
}

int g4_launch_walk(g4_ctx *ctx, g4_tree *t, const g4_walk_params *wp, int kernel, int criterion, double *ax,
                   double *ay, double *az, double *pot, uint32_t *counts, float *aout_caller, float *aout_sorted,
                   int stat_slot)
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
    A.exclusion = wp->exclusion;
    A.order = wp->order;
    A.unit = (float)t->unit;
    A.box = (float)t->tp.box;
    const double h = 2.8 * wp->eps0;
    A.h = (float)h;
    A.h2 = (float)(h * h);
    A.hinv = h > 0 ? (float)(1.0 / h) : 0.f;
    A.asplit = kernel == 1 ? (float)(0.5 / wp->r_s) : 0.f;
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
    A.stat = t->ctr->stat + stat_slot;
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
    G4_HIP(ctx, hipMemsetAsync(A.item_ctr, 0, sizeof(uint32_t), ctx->stream));
    A.wstat = stat_slot == 0 ? t->ctr->stat + 9 : nullptr;
    hipStream_t s = ctx->stream;
    const bool P = pot != nullptr;
    if (kernel == 0) {
        if (criterion == 0) { if (P) launch_walk<0, 0, true>(A, s); else launch_walk<0, 0, false>(A, s); }
        else { if (P) launch_walk<0, 1, true>(A, s); else launch_walk<0, 1, false>(A, s); }
    } else {
        if (criterion == 0) { if (P) launch_walk<1, 0, true>(A, s); else launch_walk<1, 0, false>(A, s); }
        else { if (P) launch_walk<1, 1, true>(A, s); else launch_walk<1, 1, false>(A, s); }
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
