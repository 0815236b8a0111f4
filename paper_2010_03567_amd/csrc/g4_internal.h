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
#define G4_WALK_LDS_STACK 30
#define G4_WALK_SPILL G4_WALK_STACK
#define G4_WALK_MAX_WAVES 8192

// levels of the hierarchical time integration (index lists kept per level)
#define G4_KDK_LEVELS (G4_KDK_MAX_LEVEL + 1)

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
    unsigned long long stat[18];  // [0..2] walk p2p/p2m/visits, [3..5] seed walk, [6..8] FMM pp/pn/nn,
                                  // [9..15] walk passes, deepest stack, entries, leaves, chunks,
                                  // [16..17] walk pairs used / dropped by a decision for the whole group
};

struct g4_tree {
    int64_t n;
    g4_tree_params tp;
    int S;              // bits spanned by the root: 32 periodic, 31 isolated
    uint32_t corner;    // integer lower corner of the root
    double unit;        // physical length of one integer step
    int64_t cap;        // node capacity
    int moments_order;  // 0 until g4_compute_multipoles; 5 once g4_compute_moments4 has run
    double *q4d;        // fourth moments, 15 per node (caller's buffer, g4_compute_moments4), or null
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

// host launchers of every kernel file
#include "g4_launch.h"
