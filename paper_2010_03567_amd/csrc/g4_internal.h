// g4_internal.h -- device data layout and launch helpers shared by the HIP
// sources of libg4hip.so (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/g4hip.h"

#define G4_MAXLEV 21  // 63-bit Morton keys: 21 bits per axis

// Traversal stack of the walk: entries needed at most, entries kept in LDS
// (fewer with the diagnostic G4_WALK_LDS_STACK environment variable), the
// device spill area per wavefront (room for the whole stack, so any LDS share
// is safe), and the wavefront cap of the persistent walk grid.
#define G4_WALK_STACK (1 + 7 * (G4_MAXLEV - 1) + 8)
#define G4_WALK_LDS_STACK 32
#define G4_WALK_SPILL G4_WALK_STACK
#define G4_WALK_MAX_WAVES 8192

struct g4_ctx {
    int device;
    hipStream_t stream;
    char err[512];
};

// Walk record of one node, 64 bytes, read by a whole wavefront through the
// scalar cache (the node index is wave-uniform during traversal).
struct __attribute__((aligned(16))) WNode {
    uint32_t cx, cy, cz;   // centre of mass on the integer grid (nearest point)
    float mass;
    float q[6];            // Q2 about the centre of mass: xx xy xz yy yz zz (physical units)
    uint32_t gx, gy, gz;   // integer geometric centre of the node's cube
    uint32_t next;         // internal: first child node; leaf: first particle (sorted order)
    uint32_t num;          // internal: number of children; leaf: number of particles
    uint32_t meta;         // bits 0-7 level, bit 8 leaf
};
static_assert(sizeof(WNode) == 64, "WNode must be 64 bytes");

#define WN_LEAF (1u << 8)

// Full-precision moments of one node (double storage for the upward pass):
// [0] mass, [1..3] centre of mass minus geometric centre (physical),
// [4..9] Q2 packed, [10..19] Q3 packed (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
#define MOM_STRIDE 20

// Short-range factor table: S_0..S_3 (erfc-type factors of g_0..g_3), up to
// G4_SRTAB_MAX intervals over x = alpha_split r in [0, G4_SRTAB_XMAX].
#define G4_SRTAB_FUNCS 4
#define G4_SRTAB_MAX 512
#define G4_SRTAB_XMAX 6.0

// Device counters at the head of the tree workspace.
struct DevCounters {
    uint32_t node_count;      // total nodes (the level sizes summed after the split passes)
    uint32_t item_ctr;        // work-item counter of the persistent walk
    uint32_t flags;           // bit 0: depth-capped leaf above leaf_max; bit 1: node overflow;
                              // bit 2: walk stack overflow; bit 3: FMM leaf-node stack overflow
    uint32_t pad;
    uint32_t lvl_start[G4_MAXLEV + 4];  // first node of each level
    uint32_t lvl_count[G4_MAXLEV + 4];  // nodes of each level (children allocated by atomics)
    unsigned long long stat[16];  // [0..2] walk p2p/p2m/visits, [3..5] seed walk, [6..8] FMM pp/pn/nn,
                                  // [9..15] walk passes, deepest stack, entries, leaves, chunks
};

struct g4_tree {
    int64_t n;
    g4_tree_params tp;
    int S;              // bits spanned by the root: 32 periodic, 31 isolated
    uint32_t corner;    // integer lower corner of the root
    double unit;        // physical length of one integer step
    int64_t cap;        // node capacity
    int moments_order;  // 0 until g4_compute_multipoles
    int seed_valid;     // aseed holds |a| of a geometric walk over this tree
    // workspace views
    DevCounters *ctr;
    uint64_t *keys0, *keys1;
    uint32_t *perm0, *perm1;  // perm1[i] = caller index of sorted particle i
    uint4 *parts;             // sorted particles: x, y, z, mass bits
    uint32_t *bfirst, *bcount;
    uint32_t *parent;         // parent node (0xffffffff for the root)
    WNode *wn;
    float *q3;                // 10 floats per node (potential only)
    double *mom;              // MOM_STRIDE doubles per node
    float *aseed;             // n floats, sorted order
    uint32_t *leafof;         // n: the leaf holding each particle (sorted order), set with the moments
    uint4 *walk_spill;        // G4_WALK_SPILL stack entries per wavefront of the walk
    float4 *srtab;            // short-range factor table: G4_SRTAB_FUNCS x tab_n cubic pieces
    int tab_n;                // intervals it holds (0: not built); it is in units of alpha_split r
    int64_t walk_spill_waves; // wavefronts with a spill area (multiple of 4)
    // forest of independent boxes: one root per box (nodes 0..nbox-1)
    int nbox;
    uint4 *items;             // device work items of the walk (first, count, root), 0 for a single tree
    uint32_t nitems;
    int items_group;          // group size the items were made for
    int64_t *box_off;         // host copy of the box offsets (nbox + 1)
    uint4 *items_host;        // host staging of the items
    int64_t items_cap;
    void *sort_tmp;
    size_t sort_tmp_bytes;
    // phase timers on the context's stream: build, moments, seed, walk (start, end)
    hipEvent_t ev[8];
    int ev_made;              // events created
    int ev_rec;               // bit k: pair k (build, moments, seed, walk) recorded
};

#define G4_FLAG_WALK_STACK 4u
#define G4_FLAG_FMM_STACK 8u
#define G4_FLAG_FATAL (2u | G4_FLAG_WALK_STACK | G4_FLAG_FMM_STACK)

// phase k of the timers: 0 build, 1 moments, 2 seed, 3 walk
int g4_phase_begin(g4_ctx *ctx, g4_tree *t, int k);
int g4_phase_end(g4_ctx *ctx, g4_tree *t, int k);
// seconds between the recorded events of phase k (0 if not recorded); the
// events must be complete (the caller has synchronised the stream)
double g4_phase_seconds(const g4_tree *t, int k);

// Layout of a tree workspace (byte offsets).
struct WsLayout {
    size_t ctr, keys0, keys1, perm0, perm1, parts, bfirst, bcount, parent, wn, q3, mom, aseed, leafof, spill,
        srtab, sort_tmp, sort_bytes, total;
    int64_t cap;
    int64_t spill_waves;
};

int g4_layout(const g4_tree_params *tp, int64_t n, WsLayout *L);

static inline int g4_set_err(g4_ctx *ctx, int code, const char *msg)
{
    if (ctx) {
        int i = 0;
        for (; msg[i] && i < 511; i++) ctx->err[i] = msg[i];
        ctx->err[i] = 0;
    }
    return code;
}

#define G4_HIP(ctx, call)                                                       \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return g4_set_err((ctx), G4_EHIP, hipGetErrorString(e_)); \
    } while (0)

// host launchers implemented in the .hip files
int g4_launch_build(g4_ctx *ctx, g4_tree *t, const g4_particles *p);
int g4_launch_moments(g4_ctx *ctx, g4_tree *t);
int g4_launch_build_forest(g4_ctx *ctx, g4_tree *t, const g4_particles *p, const int64_t *off_dev, uint32_t *bkey0,
                           uint32_t *bkey1);
int g4_launch_walk(g4_ctx *ctx, g4_tree *t, const g4_walk_params *wp, int kernel, int criterion,
                   double *ax, double *ay, double *az, double *pot, uint32_t *counts, float *aout_caller,
                   float *aout_sorted, int stat_slot);
int g4_launch_export(g4_ctx *ctx, const g4_tree *t, int32_t *level, uint32_t *cell, int64_t *count,
                     int64_t *first, int32_t *leaf, double *mass, double *com, double *q2, double *q3);
int g4_launch_direct(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, const g4_walk_params *wp,
                     int truncate, const int64_t *targets, int64_t ntargets, double *ax, double *ay, double *az,
                     double *pot);
int g4_launch_quantize(g4_ctx *ctx, const double *pos, int64_t n, const g4_tree_params *tp, uint32_t *x,
                       uint32_t *y, uint32_t *z, int32_t *flag);
int g4_launch_gather_seed(g4_ctx *ctx, g4_tree *t, const float *a_seed_caller);
// stable LSD radix sort of (key, value) pairs over bits [bit_lo, bit_hi) in
// 8-bit digits, ping-ponging between (k0, v0) and (k1, v1); *in_alt = 1 when
// the sorted pairs end in (k1, v1), 0 when in (k0, v0).  temp: device bytes of
// g4_radix_sort_temp_bytes(n).  Enqueued on the context's stream.
size_t g4_radix_sort_temp_bytes(int64_t n);
int g4_radix_sort_u64(g4_ctx *ctx, uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt);
int g4_radix_sort_u32(g4_ctx *ctx, uint32_t *k0, uint32_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt);
// zero `bytes` (a multiple of 4) of device memory with a kernel, so that the
// calls stay valid under stream capture (no memset nodes in a graph)
int g4_launch_zero(g4_ctx *ctx, void *p, size_t bytes);
int g4_launch_mlp_features(g4_ctx *ctx, const g4_tree *t, const g4_walk_params *wp, const float *norm,
                           float *feat);
int g4_launch_mlp_forward(g4_ctx *ctx, const uint16_t *w, const float *feat, int64_t n, float *out, float shift,
                          int mode);
int g4_launch_mlp_grad(g4_ctx *ctx, const uint16_t *w, const float *feat, const float *target, int64_t n,
                       float tau, float *grad, float *loss);
int g4_fmm_layout_bytes(const g4_tree *t, const g4_fmm_params *fp, double factor, size_t *bytes);
int g4_launch_fmm(g4_ctx *ctx, g4_tree *t, const g4_fmm_params *fp, double factor, void *ws, size_t ws_bytes,
                  double *ax, double *ay, double *az, double *pot, g4_stats *stats);
int g4_launch_mlp_adam(g4_ctx *ctx, uint16_t *w, float *master, float *m, float *v, const float *grad, float lr,
                       float b1, float b2, float eps, int64_t step);
