// api.hip -- the extern "C" entry points of libg4hip.so declared in
// include/g4hip.h: argument checks, workspace carving, and the order of the
// kernel launches on the context's stream.
#include <cstdio>
#include <mutex>
#include <new>

#include "ewald.h"
#include "g4_internal.h"

// Static device scratch of the FMM entry point that allocates nothing
// (g4_fmm_force_noalloc).  Every device the library runs on holds one copy
// until the process ends.  In host code `scratch` is only a stand-in symbol:
// its device address comes from hipGetSymbolAddress, once per device.
#define G4_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
#define G4_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[G4_NOALLOC_SCRATCH_BYTES];
static void *g_scratch_ptr[G4_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of this context's device's scratch (looked up on the first
// call on that device, with that device current).
static int scratch_address(g4_ctx *ctx, void **out)
{
    if (ctx->device < 0 || ctx->device >= G4_MAX_DEVICES) return g4_set_err(ctx, G4_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        int cur = -1;
        G4_HIP(ctx, hipGetDevice(&cur));
        if (cur != ctx->device) G4_HIP(ctx, hipSetDevice(ctx->device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != ctx->device) hipSetDevice(cur);
        if (e != hipSuccess || !p) return g4_set_err(ctx, G4_EHIP, "hipGetSymbolAddress of the static scratch failed");
        g_scratch_ptr[ctx->device] = p;
    }
    *out = g_scratch_ptr[ctx->device];
    return G4_OK;
}

static int check_tp(g4_ctx *ctx, const g4_tree_params *tp)
{
    if (!tp) return g4_set_err(ctx, G4_EINVAL, "null tree params");
    if (!(tp->box > 0)) return g4_set_err(ctx, G4_EINVAL, "box must be positive");
    if (tp->leaf_max < 1) return g4_set_err(ctx, G4_EINVAL, "leaf_max must be >= 1");
    if (tp->max_depth < 1 || tp->max_depth > G4_MAXLEV)
        return g4_set_err(ctx, G4_EINVAL, "max_depth must be in [1, 21]");
    if (tp->key_kind != 0 && tp->key_kind != 1) return g4_set_err(ctx, G4_EINVAL, "key_kind must be 0 or 1");
    return G4_OK;
}

static int g4_build_tree_views(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, void *ws,
                               const WsLayout *Lp, g4_tree **out);

int g4_phase_begin(g4_ctx *ctx, g4_tree *t, int k)
{
    if (!t->ev_made) {
        for (int e = 0; e < 8; e++) G4_HIP(ctx, hipEventCreate(&t->ev[e]));
        t->ev_made = 1;
    }
    t->ev_rec &= ~(1 << k);
    G4_HIP(ctx, hipEventRecord(t->ev[2 * k], ctx->stream));
    return G4_OK;
}

int g4_phase_end(g4_ctx *ctx, g4_tree *t, int k)
{
    G4_HIP(ctx, hipEventRecord(t->ev[2 * k + 1], ctx->stream));
    t->ev_rec |= 1 << k;
    return G4_OK;
}

double g4_phase_seconds(const g4_tree *t, int k)
{
    if (!t->ev_made || !(t->ev_rec & (1 << k))) return 0.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t->ev[2 * k], t->ev[2 * k + 1]) != hipSuccess) return 0.0;
    return 1e-3 * (double)ms;
}

// fill the phase times of stats (the stream has been synchronised)
static void fill_times(const g4_tree *t, g4_stats *stats, bool seeded)
{
    stats->t_build = g4_phase_seconds(t, 0);
    stats->t_moments = g4_phase_seconds(t, 1);
    stats->t_seed = seeded ? g4_phase_seconds(t, 2) : 0.0;
    stats->t_walk = g4_phase_seconds(t, 3);
}

extern "C" {

int g4_ctx_create(int device, void *hip_stream, g4_ctx **out)
{
    if (!out) return G4_EINVAL;
    g4_ctx *c = new (std::nothrow) g4_ctx;
    if (!c) return G4_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->err[0] = 0;
    *out = c;
    return G4_OK;
}

int g4_ctx_destroy(g4_ctx *ctx)
{
    delete ctx;
    return G4_OK;
}

const char *g4_last_error(const g4_ctx *ctx) { return ctx ? ctx->err : "null context"; }

int g4_quantize(g4_ctx *ctx, const double *pos, int64_t n, const g4_tree_params *tp, uint32_t *x, uint32_t *y,
                uint32_t *z, int32_t *flag)
{
    if (!ctx) return G4_EINVAL;
    int st = check_tp(ctx, tp);
    if (st) return st;
    if (n < 0 || (n > 0 && (!pos || !x || !y || !z)) || !flag) return g4_set_err(ctx, G4_EINVAL, "bad quantize args");
    return g4_launch_quantize(ctx, pos, n, tp, x, y, z, flag);
}

int g4_workspace_bytes(const g4_tree_params *tp, int64_t n, size_t *bytes)
{
    if (!tp || !bytes || n < 1 || n > 0xFFFFFFF0ll) return G4_EINVAL;
    if (check_tp(nullptr, tp)) return G4_EINVAL;
    WsLayout L;
    int st = g4_layout(tp, n, &L);
    if (st) return st;
    *bytes = L.total;
    return G4_OK;
}

int g4_build_tree(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, void *ws, size_t ws_bytes,
                  g4_tree **out)
{
    if (!ctx) return G4_EINVAL;
    int st = check_tp(ctx, tp);
    if (st) return st;
    if (!p || !out || !ws) return g4_set_err(ctx, G4_EINVAL, "null argument");
    if (p->n < 1 || p->n > 0xFFFFFFF0ll) return g4_set_err(ctx, G4_EINVAL, "particle count out of range");
    if (!p->x || !p->y || !p->z || !p->mass) return g4_set_err(ctx, G4_EINVAL, "null particle array");
    if (((uintptr_t)ws & 255) != 0) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    WsLayout L;
    st = g4_layout(tp, p->n, &L);
    if (st) return g4_set_err(ctx, st, "workspace layout failed");
    if (ws_bytes < L.total) return g4_set_err(ctx, G4_ENOMEM, "workspace too small");
    g4_tree *t = nullptr;
    st = g4_build_tree_views(ctx, p, tp, ws, &L, &t);
    if (st) return st;
    st = g4_phase_begin(ctx, t, 0);
    if (!st) st = g4_launch_build(ctx, t, p);
    if (!st) st = g4_phase_end(ctx, t, 0);
    if (st) {
        g4_tree_free(ctx, t);
        return st;
    }
    *out = t;
    return G4_OK;
}

// host handle with views into a workspace laid out by L
static int g4_build_tree_views(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, void *ws,
                               const WsLayout *Lp, g4_tree **out)
{
    const WsLayout &L = *Lp;
    g4_tree *t = new (std::nothrow) g4_tree;
    if (!t) return g4_set_err(ctx, G4_ENOMEM, "host allocation failed");
    char *b = (char *)ws;
    t->n = p->n;
    t->tp = *tp;
    t->S = tp->periodic ? 32 : 31;
    t->corner = tp->periodic ? 0u : (1u << 30);
    t->unit = tp->box / (tp->periodic ? 4294967296.0 : 2147483648.0);
    t->cap = L.cap;
    t->moments_order = 0;
    t->q4d = nullptr;
    t->seed_valid = 0;
    t->nbox = 1;
    t->items = nullptr;
    t->nitems = 0;
    t->items_group = 0;
    t->box_off = nullptr;
    t->items_host = nullptr;
    t->items_cap = 0;
    t->ctr = (DevCounters *)(b + L.ctr);
    t->keys0 = (uint64_t *)(b + L.keys0);
    t->keys1 = (uint64_t *)(b + L.keys1);
    t->perm0 = (uint32_t *)(b + L.perm0);
    t->perm1 = (uint32_t *)(b + L.perm1);
    t->parts = (uint4 *)(b + L.parts);
    t->bfirst = (uint32_t *)(b + L.bfirst);
    t->bcount = (uint32_t *)(b + L.bcount);
    t->parent = (uint32_t *)(b + L.parent);
    t->wn = (WNode *)(b + L.wn);
    t->q3 = (float *)(b + L.q3);
    t->mom = (double *)(b + L.mom);
    t->aseed = (float *)(b + L.aseed);
    t->leafof = (uint32_t *)(b + L.leafof);
    t->walk_spill = (uint4 *)(b + L.spill);
    t->srtab = (float4 *)(b + L.srtab);
    t->tab_n = 0;
    t->walk_spill_waves = L.spill_waves;
    t->sort_tmp = b + L.sort_tmp;
    t->sort_tmp_bytes = L.sort_bytes;
    t->ev_made = 0;
    t->ev_rec = 0;
    *out = t;
    return G4_OK;
}

int g4_compute_multipoles(g4_ctx *ctx, g4_tree *tree, int order)
{
    if (!ctx || !tree) return G4_EINVAL;
    if (order != 2 && order != 3) return g4_set_err(ctx, G4_EINVAL, "order must be 2 or 3");
    int st = g4_phase_begin(ctx, tree, 1);
    if (!st) st = g4_launch_moments(ctx, tree);
    if (!st) st = g4_phase_end(ctx, tree, 1);
    if (st) return st;
    tree->moments_order = order;
    tree->q4d = nullptr;
    tree->seed_valid = 0;
    return G4_OK;
}

size_t g4_moments4_bytes(const g4_tree *tree)
{
    return tree ? (size_t)tree->cap * 15 * sizeof(double) : 0;
}

int g4_compute_moments4(g4_ctx *ctx, g4_tree *tree, void *ws, size_t bytes)
{
    if (!ctx || !tree) return G4_EINVAL;
    if (tree->moments_order < 3) return g4_set_err(ctx, G4_ESTATE, "compute the multipoles to order 3 first");
    if (!ws || ((uintptr_t)ws & 255)) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < g4_moments4_bytes(tree)) return g4_set_err(ctx, G4_EINVAL, "workspace too small");
    int st = g4_launch_moments4(ctx, tree, static_cast<double *>(ws));
    if (st) return st;
    tree->q4d = static_cast<double *>(ws);
    tree->moments_order = 5;
    return G4_OK;
}

int g4_tree_info(g4_ctx *ctx, const g4_tree *tree, int64_t *nnodes, int64_t *level_start)
{
    if (!ctx || !tree) return G4_EINVAL;
    DevCounters h;
    G4_HIP(ctx, hipMemcpyAsync(&h, tree->ctr, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (nnodes) *nnodes = h.node_count;
    if (level_start) {
        // levels are stored one after another, so the starts are the running
        // sums of the level sizes (the device keeps starts only for non-empty levels)
        const int maxd = tree->tp.max_depth;
        level_start[0] = 0;
        for (int l = 0; l <= maxd; l++) level_start[l + 1] = level_start[l] + h.lvl_count[l];
    }
    if (h.flags & 2u) return g4_set_err(ctx, G4_ENOMEM, "node capacity exceeded");
    if (h.flags & G4_FLAG_WALK_STACK) return g4_set_err(ctx, G4_ENOMEM, "walk traversal stack overflowed");
    if (h.flags & G4_FLAG_FMM_STACK) return g4_set_err(ctx, G4_ENOMEM, "FMM leaf-node stack overflowed");
    return G4_OK;
}

int g4_tree_export(g4_ctx *ctx, const g4_tree *tree, int32_t *level, uint32_t *cell, int64_t *count,
                   int64_t *first, int32_t *leaf, double *mass, double *com, double *q2, double *q3)
{
    if (!ctx || !tree) return G4_EINVAL;
    if ((mass || com || q2 || q3) && !tree->moments_order)
        return g4_set_err(ctx, G4_ESTATE, "moments not computed");
    return g4_launch_export(ctx, tree, level, cell, count, first, leaf, mass, com, q2, q3);
}

int g4_tree_free(g4_ctx *ctx, g4_tree *tree)
{
    if (tree) {
        // the items may still be in flight to the device: wait before releasing their host copy
        if (ctx && tree->items_host) hipStreamSynchronize(ctx->stream);
        if (tree->ev_made)
            for (int e = 0; e < 8; e++) hipEventDestroy(tree->ev[e]);
        delete[] tree->box_off;
        delete[] tree->items_host;
    }
    delete tree;
    return G4_OK;
}

int g4_forest_workspace_bytes(const g4_tree_params *tp, int nbox, int64_t n, size_t *bytes)
{
    if (!tp || !bytes || nbox < 1 || n < nbox) return G4_EINVAL;
    size_t b = 0;
    int st = g4_workspace_bytes(tp, n, &b);
    if (st) return st;
    // box offsets, two box-key arrays, work items (one per particle at worst)
    b += (((size_t)(nbox + 1) * 8 + 255) & ~(size_t)255) + 2 * (((size_t)n * 4 + 255) & ~(size_t)255) +
         (((size_t)(n + nbox) * 16 + 255) & ~(size_t)255);
    *bytes = b;
    return G4_OK;
}

int g4_build_forest(g4_ctx *ctx, int nbox, const int64_t *box_offsets, const g4_particles *p,
                    const g4_tree_params *tp, void *ws, size_t ws_bytes, g4_tree **out)
{
    if (!ctx) return G4_EINVAL;
    int st = check_tp(ctx, tp);
    if (st) return st;
    if (!tp->periodic && nbox > 1) return g4_set_err(ctx, G4_EINVAL, "a forest needs periodic boxes");
    if (nbox < 1 || !box_offsets || !p || !out || !ws) return g4_set_err(ctx, G4_EINVAL, "bad forest args");
    if (box_offsets[0] != 0 || box_offsets[nbox] != p->n) return g4_set_err(ctx, G4_EINVAL, "offsets must span [0, n]");
    for (int b = 0; b < nbox; b++)
        if (box_offsets[b + 1] <= box_offsets[b]) return g4_set_err(ctx, G4_EINVAL, "every box needs a particle");
    size_t need = 0;
    st = g4_forest_workspace_bytes(tp, nbox, p->n, &need);
    if (st) return g4_set_err(ctx, st, "forest layout failed");
    if (ws_bytes < need) return g4_set_err(ctx, G4_ENOMEM, "workspace too small");
    if (((uintptr_t)ws & 255) != 0) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    WsLayout L;
    g4_layout(tp, p->n, &L);
    g4_tree *t = nullptr;
    // carve the single-tree part, then the forest extras behind it
    st = g4_build_tree_views(ctx, p, tp, ws, &L, &t);
    if (st) return st;
    char *extra = (char *)ws + L.total;
    int64_t *off_dev = (int64_t *)extra;
    extra += (((size_t)(nbox + 1) * 8 + 255) & ~(size_t)255);
    uint32_t *bkey0 = (uint32_t *)extra;
    extra += (((size_t)p->n * 4 + 255) & ~(size_t)255);
    uint32_t *bkey1 = (uint32_t *)extra;
    extra += (((size_t)p->n * 4 + 255) & ~(size_t)255);
    t->items = (uint4 *)extra;
    t->items_cap = p->n + nbox;
    t->nbox = nbox;
    t->box_off = new (std::nothrow) int64_t[nbox + 1];
    if (!t->box_off) {
        delete t;
        return g4_set_err(ctx, G4_ENOMEM, "host allocation failed");
    }
    for (int b = 0; b <= nbox; b++) t->box_off[b] = box_offsets[b];
    st = g4_phase_begin(ctx, t, 0);
    if (st) {
        g4_tree_free(ctx, t);
        return st;
    }
    G4_HIP(ctx, hipMemcpyAsync(off_dev, t->box_off, (size_t)(nbox + 1) * 8, hipMemcpyHostToDevice, ctx->stream));
    st = g4_launch_build_forest(ctx, t, p, off_dev, bkey0, bkey1);
    if (!st) st = g4_phase_end(ctx, t, 0);
    if (st) {
        g4_tree_free(ctx, t);
        return st;
    }
    // the offsets copy reads host memory owned by the tree; it completes before any later call returns
    *out = t;
    return G4_OK;
}

static int tree_force_impl(g4_ctx *ctx, g4_tree *tree, const g4_walk_params *wp, int kernel, double *ax,
                           double *ay, double *az, double *pot, uint32_t *counts, float *a_out, g4_stats *stats)
{
    if (!ctx || !tree || !wp) return G4_EINVAL;
    if (!ax || !ay || !az) return g4_set_err(ctx, G4_EINVAL, "null output");
    if (!tree->moments_order) return g4_set_err(ctx, G4_ESTATE, "moments not computed");
    if (wp->order < 2 || wp->order > 5) return g4_set_err(ctx, G4_EINVAL, "order must be 2..5");
    if (wp->order > tree->moments_order) return g4_set_err(ctx, G4_ESTATE, "moments computed at a lower order");
    if (wp->order >= 4 && (kernel == 2 || (kernel == 1 && wp->sr_table > 0)))
        return g4_set_err(ctx, G4_EINVAL, "orders 4 and 5 take the evaluated Newtonian or short-range kernel");
    if (wp->criterion != 0 && wp->criterion != 1) return g4_set_err(ctx, G4_EINVAL, "criterion must be 0 or 1");
    if (kernel == 1 && !(wp->r_s > 0)) return g4_set_err(ctx, G4_EINVAL, "r_s must be positive");
    if (kernel == 1 && !(wp->r_cut > 0)) return g4_set_err(ctx, G4_EINVAL, "r_cut must be positive");
    if (wp->eps0 < 0) return g4_set_err(ctx, G4_EINVAL, "eps0 must be >= 0");
    if (wp->group_size < 0 || wp->group_size > 64) return g4_set_err(ctx, G4_EINVAL, "group_size must be 0..64");
    if (wp->sr_table != 0 && (wp->sr_table < 8 || wp->sr_table > G4_SRTAB_MAX))
        return g4_set_err(ctx, G4_EINVAL, "sr_table must be 0 or 8..512");
    if (!tree->tp.periodic && kernel == 1) return g4_set_err(ctx, G4_EINVAL, "short-range kernel needs a periodic box");
    if (kernel == 2) {
        if (!tree->tp.periodic) return g4_set_err(ctx, G4_EINVAL, "the Ewald-corrected kernel needs a periodic box");
        if (!wp->ewald_table) return g4_set_err(ctx, G4_EINVAL, "kernel 2 needs ewald_table");
        if (wp->ewald_n < G4_EWALD_NE_MIN || wp->ewald_n > G4_EWALD_NE_MAX)
            return g4_set_err(ctx, G4_EINVAL, "ewald_n must be 4..128");
    }
    if (stats) {
        const int zs = g4_launch_zero(ctx, tree->ctr->stat, sizeof(tree->ctr->stat));
        if (zs) return zs;
    }
    int st;
    bool seeded = false;
    if (wp->criterion == 1) {
        if (wp->seed_from_tree && !wp->a_seed && !tree->seed_valid)
            return g4_set_err(ctx, G4_ESTATE, "no geometric walk has left |a| in this tree");
        if (!wp->a_seed && !wp->seed_from_tree && !(wp->theta_seed > 0))
            return g4_set_err(ctx, G4_EINVAL, "theta_seed must be positive");
        if (wp->a_seed || !wp->seed_from_tree) {
            seeded = true;
            st = g4_phase_begin(ctx, tree, 2);
            if (st) return st;
        }
        if (wp->a_seed) {
            st = g4_launch_gather_seed(ctx, tree, wp->a_seed);
        } else if (wp->seed_from_tree) {
            st = G4_OK;
        } else {
            // geometric pre-walk (first-force footnote of eq. eqnrelcriterion): |a| estimate
            // written into the tree's sorted seed buffer; its forces are scratch and go to ax..az
            st = g4_launch_walk(ctx, tree, wp, kernel, 0, ax, ay, az, nullptr, nullptr, nullptr, tree->aseed, 3,
                                stats != nullptr);
        }
        if (st) return st;
        if (seeded && (st = g4_phase_end(ctx, tree, 2))) return st;
    }
    if ((st = g4_phase_begin(ctx, tree, 3))) return st;
    st = g4_launch_walk(ctx, tree, wp, kernel, wp->criterion, ax, ay, az, pot, counts, a_out,
                        wp->criterion == 0 ? tree->aseed : nullptr, 0, stats != nullptr);
    if (st) return st;
    if ((st = g4_phase_end(ctx, tree, 3))) return st;
    if (wp->criterion == 0) tree->seed_valid = 1;
    if (stats) {
        DevCounters h;
        G4_HIP(ctx, hipMemcpyAsync(&h, tree->ctr, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
        G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
        fill_times(tree, stats, seeded);
        stats->n_p2p = h.stat[0];
        stats->n_p2m = h.stat[1];
        stats->n_visit = h.stat[2];
        stats->n_seed_p2p = h.stat[3];
        stats->n_seed_p2m = h.stat[4];
        stats->n_seed_visit = h.stat[5];
        stats->n_pp = stats->n_pn = stats->n_nn = 0;
        stats->n_nodes = h.node_count;
        stats->w_pop = h.stat[9];
        stats->w_p2m = h.stat[10];
        stats->w_p2p = h.stat[11];
        stats->flags = h.flags;
        stats->max_stack = (uint32_t)h.stat[12];
        stats->w_entry = h.stat[13];
        stats->w_leaf = h.stat[14];
        stats->w_chunk = h.stat[15];
        stats->n_group_use = h.stat[16];
        stats->n_group_drop = h.stat[17];
        if (h.flags & G4_FLAG_WALK_STACK) return g4_set_err(ctx, G4_ENOMEM, "walk traversal stack overflowed");
    }
    return G4_OK;
}

int g4_tree_force(g4_ctx *ctx, g4_tree *tree, const g4_walk_params *wp, double *ax, double *ay, double *az,
                  double *pot, uint32_t *counts, float *a_out, g4_stats *stats)
{
    if (!wp) return G4_EINVAL;
    if (wp->kernel < 0 || wp->kernel > 2) return g4_set_err(ctx, G4_EINVAL, "kernel must be 0, 1 or 2");
    return tree_force_impl(ctx, tree, wp, wp->kernel, ax, ay, az, pot, counts, a_out, stats);
}

int g4_treepm_shortrange(g4_ctx *ctx, g4_tree *tree, const g4_walk_params *wp, double *ax, double *ay, double *az,
                         double *pot, uint32_t *counts, float *a_out, g4_stats *stats)
{
    if (!wp) return G4_EINVAL;
    g4_walk_params w = *wp;
    w.kernel = 1;
    return tree_force_impl(ctx, tree, &w, 1, ax, ay, az, pot, counts, a_out, stats);
}

size_t g4_ewald_table_bytes(int ne)
{
    if (ne < G4_EWALD_NE_MIN || ne > G4_EWALD_NE_MAX) return 0;
    return g4_ewald_layout_bytes(ne);
}

int g4_ewald_table(g4_ctx *ctx, double box, int ne, void *table, size_t bytes)
{
    if (!ctx) return G4_EINVAL;
    if (!(box > 0)) return g4_set_err(ctx, G4_EINVAL, "box must be positive");
    if (ne < G4_EWALD_NE_MIN || ne > G4_EWALD_NE_MAX) return g4_set_err(ctx, G4_EINVAL, "ne must be 4..128");
    if (!table || ((uintptr_t)table & 255)) return g4_set_err(ctx, G4_EINVAL, "table must be 256-byte aligned");
    if (bytes < g4_ewald_layout_bytes(ne)) return g4_set_err(ctx, G4_EINVAL, "table too small");
    return g4_launch_ewald_table(ctx, box, ne, static_cast<float *>(table));
}

int g4_ewald_eval(g4_ctx *ctx, const void *table, int ne, double box, int64_t n, const double *dx, const double *dy,
                  const double *dz, double *psi, double *gx, double *gy, double *gz)
{
    if (!ctx) return G4_EINVAL;
    if (!table || !(box > 0) || ne < G4_EWALD_NE_MIN || ne > G4_EWALD_NE_MAX || n < 0)
        return g4_set_err(ctx, G4_EINVAL, "bad table, box, ne or n");
    if (n > 0 && (!dx || !dy || !dz || !psi || !gx || !gy || !gz)) return g4_set_err(ctx, G4_EINVAL, "null array");
    return g4_launch_ewald_eval(ctx, static_cast<const float *>(table), ne, box, n, dx, dy, dz, psi, gx, gy, gz);
}

int g4_pm_workspace_bytes(int ng, size_t *bytes)
{
    if (!bytes) return G4_EINVAL;
    return g4_pm_layout_bytes(ng, bytes);
}

int g4_pm_longrange(g4_ctx *ctx, const g4_tree *tree, const g4_pm_params *pp, void *ws, size_t ws_bytes,
                    int accumulate, double *ax, double *ay, double *az, double *pot)
{
    if (!ctx || !tree || !pp || !ws) return G4_EINVAL;
    if (!ax || !ay || !az) return g4_set_err(ctx, G4_EINVAL, "null output");
    if (!tree->tp.periodic) return g4_set_err(ctx, G4_EINVAL, "the PM force needs a periodic box");
    if (tree->nbox != 1) return g4_set_err(ctx, G4_EINVAL, "the PM force takes one box, not a forest");
    if (!(pp->r_s > 0)) return g4_set_err(ctx, G4_EINVAL, "r_s must be positive");
    if (((uintptr_t)ws & 255) != 0) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    return g4_launch_pm(ctx, tree, pp, ws, ws_bytes, accumulate ? 1 : 0, ax, ay, az, pot);
}

static int check_kdk(g4_ctx *ctx, const g4_kdk_params *kp)
{
    if (!kp) return g4_set_err(ctx, G4_EINVAL, "null kdk params");
    if (check_tp(ctx, &kp->tp)) return G4_EINVAL;
    if (kp->solver < 0 || kp->solver > 2) return g4_set_err(ctx, G4_EINVAL, "solver must be 0, 1 or 2");
    if (kp->max_level < 0 || kp->max_level > G4_KDK_MAX_LEVEL) return g4_set_err(ctx, G4_EINVAL, "max_level out of range");
    if (!(kp->eta > 0) || !(kp->eps > 0)) return g4_set_err(ctx, G4_EINVAL, "eta and eps must be positive");
    const int kernel = kp->solver == 2 ? kp->fp.kernel : kp->wp.kernel;
    if (kernel >= 1 && !kp->tp.periodic) return g4_set_err(ctx, G4_EINVAL, "this kernel needs a periodic box");
    // every force call acts on a subset: seeds given per particle of the whole set cannot be used
    if ((kp->solver == 1 && kp->wp.a_seed) || (kp->solver == 2 && kp->fp.criterion != 0))
        return g4_set_err(ctx, G4_EINVAL, "per-particle seeds are not supported by the hierarchical step");
    return G4_OK;
}

int g4_kdk_workspace_bytes(const g4_kdk_params *kp, int64_t n, size_t *bytes)
{
    if (!kp || !bytes || n < 1 || n > 0xFFFFFFF0ll) return G4_EINVAL;
    if (check_kdk(nullptr, kp)) return G4_EINVAL;
    return g4_kdk_layout_bytes(kp, n, bytes);
}

int g4_kdk_step(g4_ctx *ctx, const g4_kdk_params *kp, int64_t n, double *pos, double *vel, const float *mass,
                double dt, double *ax, double *ay, double *az, int have_acc, void *ws, size_t ws_bytes,
                g4_kdk_stats *stats)
{
    if (!ctx) return G4_EINVAL;
    int st = check_kdk(ctx, kp);
    if (st) return st;
    if (n < 1 || n > 0xFFFFFFF0ll) return g4_set_err(ctx, G4_EINVAL, "particle count out of range");
    if (!pos || !vel || !mass || !ax || !ay || !az || !ws) return g4_set_err(ctx, G4_EINVAL, "null argument");
    if (!(dt > 0)) return g4_set_err(ctx, G4_EINVAL, "dt must be positive");
    if (((uintptr_t)ws & 255) != 0) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    return g4_launch_kdk(ctx, kp, n, pos, vel, mass, dt, ax, ay, az, have_acc, ws, ws_bytes, stats);
}

int g4_direct_force(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, const g4_walk_params *wp,
                    int truncate, const int64_t *targets, int64_t ntargets, double *ax, double *ay, double *az,
                    double *pot)
{
    if (!ctx) return G4_EINVAL;
    int st = check_tp(ctx, tp);
    if (st) return st;
    if (!p || !wp || !ax || !ay || !az) return g4_set_err(ctx, G4_EINVAL, "null argument");
    if (p->n < 1 || !p->x || !p->y || !p->z || !p->mass) return g4_set_err(ctx, G4_EINVAL, "bad particles");
    if (targets && ntargets < 0) return g4_set_err(ctx, G4_EINVAL, "negative target count");
    if (wp->kernel < 0 || wp->kernel > 2) return g4_set_err(ctx, G4_EINVAL, "kernel must be 0, 1 or 2");
    if (wp->kernel == 1 && !(wp->r_s > 0)) return g4_set_err(ctx, G4_EINVAL, "r_s must be positive");
    if (wp->kernel >= 1 && !tp->periodic) return g4_set_err(ctx, G4_EINVAL, "this kernel needs a periodic box");
    return g4_launch_direct(ctx, p, tp, wp, truncate, targets, ntargets, ax, ay, az, pot);
}

int g4_fmm_workspace_bytes(const g4_tree *tree, const g4_fmm_params *fp, double list_factor, size_t *bytes)
{
    if (!tree || !fp || !bytes) return G4_EINVAL;
    return g4_fmm_layout_bytes(tree, fp, list_factor, bytes);
}

static int fmm_checks(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double *ax, double *ay, double *az)
{
    if (!ax || !ay || !az) return g4_set_err(ctx, G4_EINVAL, "null output");
    if (tree->moments_order < 3) return g4_set_err(ctx, G4_ESTATE, "FMM needs moments to order 3");
    if (fp->kernel < 0 || fp->kernel > 2) return g4_set_err(ctx, G4_EINVAL, "kernel must be 0, 1 or 2");
    if (fp->kernel == 2) {
        if (!tree->tp.periodic) return g4_set_err(ctx, G4_EINVAL, "the Ewald-corrected kernel needs a periodic box");
        if (!fp->ewald_table || fp->ewald_n < G4_EWALD_NE_MIN || fp->ewald_n > G4_EWALD_NE_MAX)
            return g4_set_err(ctx, G4_EINVAL, "kernel 2 needs ewald_table and ewald_n in 4..128");
    }
    if (fp->criterion != 0 && fp->criterion != 1) return g4_set_err(ctx, G4_EINVAL, "criterion must be 0 or 1");
    if (fp->criterion == 1 && (!fp->a_seed || !(fp->alpha > 0)))
        return g4_set_err(ctx, G4_EINVAL, "the relative criterion needs a_seed and alpha > 0");
    if (fp->kernel == 1 && (!(fp->r_s > 0) || !(fp->r_cut > 0)))
        return g4_set_err(ctx, G4_EINVAL, "r_s and r_cut must be positive");
    if (fp->kernel == 1 && !tree->tp.periodic) return g4_set_err(ctx, G4_EINVAL, "short-range kernel needs a periodic box");
    if (!(fp->theta > 0) || fp->eps0 < 0) return g4_set_err(ctx, G4_EINVAL, "bad theta or eps0");
    if (tree->n >= (1ll << 27)) return g4_set_err(ctx, G4_EINVAL, "FMM supports up to 2^27 particles per call");
    return G4_OK;
}

static int fmm_run(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double list_factor, void *ws,
                   size_t ws_bytes, double *ax, double *ay, double *az, double *pot, g4_stats *stats)
{
    int st = g4_phase_begin(ctx, tree, 3);
    if (st) return st;
    st = g4_launch_fmm(ctx, tree, fp, list_factor, ws, ws_bytes, ax, ay, az, pot, stats);
    if (st) return st;
    if ((st = g4_phase_end(ctx, tree, 3))) return st;
    // the FMM synchronises anyway (list sizes): its overflow flag is always checked
    uint32_t flags = 0;
    G4_HIP(ctx, hipMemcpyAsync(&flags, &tree->ctr->flags, 4, hipMemcpyDeviceToHost, ctx->stream));
    G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (stats) {
        fill_times(tree, stats, false);
        stats->flags = flags;
    }
    if (flags & G4_FLAG_FMM_STACK) return g4_set_err(ctx, G4_ENOMEM, "FMM leaf-node stack overflowed");
    return G4_OK;
}

int g4_fmm_force(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double list_factor, void *ws, size_t ws_bytes,
                 double *ax, double *ay, double *az, double *pot, g4_stats *stats)
{
    if (!ctx || !tree || !fp || !ws) return G4_EINVAL;
    int st = fmm_checks(ctx, tree, fp, ax, ay, az);
    if (st) return st;
    if (((uintptr_t)ws & 255) != 0) return g4_set_err(ctx, G4_EINVAL, "workspace must be 256-byte aligned");
    return fmm_run(ctx, tree, fp, list_factor, ws, ws_bytes, ax, ay, az, pot, stats);
}

int g4_fmm_force_noalloc(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double *ax, double *ay, double *az,
                         double *pot, g4_stats *stats)
{
    if (!ctx || !tree || !fp) return G4_EINVAL;
    int st = fmm_checks(ctx, tree, fp, ax, ay, az);
    if (st) return st;
    // the largest list factor (4, 2 or 1) whose workspace fits in the scratch
    double factor = 0.0;
    size_t need1 = 0;
    for (double f : {4.0, 2.0, 1.0}) {
        size_t b = 0;
        if ((st = g4_fmm_layout_bytes(tree, fp, f, &b))) return g4_set_err(ctx, st, "fmm workspace layout failed");
        if (f == 1.0) need1 = b;
        if (b <= G4_NOALLOC_SCRATCH_BYTES) {
            factor = f;
            break;
        }
    }
    if (factor == 0.0) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "tree too large for the static FMM scratch: %zu bytes needed at list factor 1, %zu available",
                 need1, G4_NOALLOC_SCRATCH_BYTES);
        return g4_set_err(ctx, G4_EINVAL, msg);
    }
    void *ws = nullptr;
    if ((st = scratch_address(ctx, &ws))) return st;
    return fmm_run(ctx, tree, fp, factor, ws, G4_NOALLOC_SCRATCH_BYTES, ax, ay, az, pot, stats);
}

int g4_mlp_features(g4_ctx *ctx, const g4_tree *tree, const g4_walk_params *wp, const float *norm, float *feat)
{
    if (!ctx || !tree || !feat || !wp) return G4_EINVAL;
    if (!tree->moments_order) return g4_set_err(ctx, G4_ESTATE, "moments not computed");
    if (wp->kernel == 1 && !(wp->r_s > 0)) return g4_set_err(ctx, G4_EINVAL, "r_s must be positive");
    return g4_launch_mlp_features(ctx, tree, wp, norm, feat);
}

int g4_mlp_forward(g4_ctx *ctx, const void *w_bf16, const float *feat, int64_t n, float *out, float shift, int mode)
{
    if (!ctx) return G4_EINVAL;
    if (!w_bf16 || !feat || !out || n < 0) return g4_set_err(ctx, G4_EINVAL, "bad mlp_forward args");
    if (((uintptr_t)feat & 15) != 0) return g4_set_err(ctx, G4_EINVAL, "feat must be 16-byte aligned");
    return g4_launch_mlp_forward(ctx, (const uint16_t *)w_bf16, feat, n, out, shift, mode ? 1 : 0);
}

int g4_mlp_grad(g4_ctx *ctx, const void *w_bf16, const float *feat, const float *target, int64_t n, float tau,
                float *grad, float *loss)
{
    if (!ctx) return G4_EINVAL;
    if (!w_bf16 || !feat || !target || !grad || !loss || n < 1) return g4_set_err(ctx, G4_EINVAL, "bad mlp_grad args");
    if (!(tau < 1.0f)) return g4_set_err(ctx, G4_EINVAL, "tau must be < 1");
    return g4_launch_mlp_grad(ctx, (const uint16_t *)w_bf16, feat, target, n, tau, grad, loss);
}

int g4_mlp_adam(g4_ctx *ctx, void *w_bf16, float *w_master, float *m, float *v, const float *grad, float lr,
                float beta1, float beta2, float eps, int64_t step)
{
    if (!ctx) return G4_EINVAL;
    if (!w_bf16 || !w_master || !m || !v || !grad || step < 1) return g4_set_err(ctx, G4_EINVAL, "bad adam args");
    return g4_launch_mlp_adam(ctx, (uint16_t *)w_bf16, w_master, m, v, grad, lr, beta1, beta2, eps, step);
}

int g4_mlp_train_step(g4_ctx *ctx, void *w_bf16, float *w_master, float *adam_state, float *grad, const float *feat,
                      const float *target, int64_t n, float tau, float lr, int64_t step, float *loss)
{
    if (!ctx || !adam_state) return G4_EINVAL;
    int st = g4_mlp_grad(ctx, w_bf16, feat, target, n, tau, grad, loss);
    if (st) return st;
    return g4_mlp_adam(ctx, w_bf16, w_master, adam_state, adam_state + 4801, grad, lr, 0.9f, 0.999f, 1e-8f, step);
}

}  // extern "C"
