/*
 * g4hip.h -- C ABI of libg4hip.so, the MI355X (gfx950) gravity hot path of
 * Springel, Pakmor, Zier & Reinecke, "Simulating cosmic structure formation
 * with the GADGET-4 code" (arXiv:2010.03567).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller unless a comment
 *    says "host".  The library never allocates device memory: the caller
 *    queries a workspace size and passes the buffer in.
 *  - Work is enqueued on the stream bound to the context and is asynchronous
 *    unless the call returns host-side results (stats, counts, status of a
 *    device-side check), in which case it synchronises that stream.
 *  - Return value: G4_OK (0) or a negative g4_status; g4_last_error() gives a
 *    message.  No C++ exception crosses the ABI.
 *  - Particles are given in the caller's order; outputs are written in the
 *    caller's order.  Positions are the integer fixed-point coordinates of the
 *    paper's Sec. "Integer coordinates" (see g4_quantize).
 *  - One context is bound to one stream and one device and is not re-entrant.
 */
#ifndef G4HIP_H
#define G4HIP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct g4_ctx g4_ctx;
typedef struct g4_tree g4_tree;

typedef enum {
    G4_OK = 0,
    G4_EINVAL = -1,  /* invalid argument */
    G4_ENOMEM = -2,  /* workspace too small */
    G4_EHIP = -3,    /* HIP runtime error */
    G4_ESTATE = -4,  /* call out of order (e.g. moments not computed) */
    G4_EROOT = -5    /* a particle lies outside an isolated root cube */
} g4_status;

/* Root geometry and tree shape (paper Sec. "Geometry of the tree").
 * periodic = 1: cube [origin, origin+box)^3 with periodic wrap; integer
 *               coordinates span the full 2^32 range (one step = box/2^32).
 * periodic = 0: isolated; the root cube [origin, origin+box)^3 maps onto
 *               [2^30, 3*2^30) so coordinate differences never wrap
 *               (Sec. "Non-periodic potentials"); one step = box/2^31.
 * leaf_max  = B: a node is split only while it holds more than B particles.
 * max_depth: deepest level (<= 21); leaves there may hold more than B.
 * key_kind:  order of the particles along a space-filling curve through the
 *            top 21 bits of each coordinate: 0 Morton (bit interleaving),
 *            1 Peano-Hilbert (the paper's curve).  Both cut into the same
 *            nested cubes, so the node set, the decisions and the forces are
 *            the same; only the particle and node order change. */
typedef struct {
    int periodic;
    double box;
    double origin[3];
    int leaf_max;
    int max_depth;
    int key_kind;
} g4_tree_params;

/* Particle set in the caller's order: integer coordinates and masses. */
typedef struct {
    int64_t n;
    const uint32_t *x, *y, *z;
    const float *mass;
} g4_particles;

/* One-sided walk (Sec. "One-sided multipole expansion", "Tree walk and
 * opening criterion", "TreePM approach", "Periodic boundary conditions").
 * kernel:    0 softened Newtonian, 1 TreePM short-range (eq. eqnpo4 force),
 *            2 periodic Newtonian: every node and particle at its nearest
 *            image with the softened Newtonian kernel, plus the correction
 *            potential psi of the other images (eq. eqnpo1) expanded to the
 *            same order, its derivatives from ewald_table (periodic trees).
 * criterion: 0 geometric l/r < theta; 1 relative M l^p < alpha |a| r^(p+2)
 *            (eq. eqnrelcriterion) with |a| from a_seed, or, when a_seed is
 *            NULL, from a geometric pre-walk with theta_seed.
 * order:     p = 2 (monopole force) or 3 (monopole + quadrupole force;
 *            octupole enters the potential); 4 and 5 (kernels 0 and 1
 *            evaluated, after g4_compute_moments4) add the octupole and
 *            hexadecapole force terms; the criterion takes l^p / r^(p+2).
 * exclusion: 1 = never accept a node whose cube of side 2l centred on the
 *            node holds the target.  Nodes closer than h = 2.8 eps0 are
 *            always opened.  TreePM drops nodes whose nearest edge is farther
 *            than r_cut.  alpha_split = 1/(2 r_s).
 * group_size: particles per 64-lane wavefront group (1..64).
 * a_seed:    device, caller order, |a| per particle (nullable).
 * seed_from_tree: with a_seed NULL, 1 = use the |a| that the previous
 *            geometric (criterion 0) call left in this tree instead of
 *            running a pre-walk (lets a caller time the two walks apart).
 * sr_table:  kernel 1 only.  0 = evaluate the short-range factors with erfc
 *            and exp per interaction; 8..512 = interpolate them from a
 *            one-dimensional look-up table of that many intervals over
 *            alpha_split r in [0, 6] (Sec. "TreePM approach": the paper
 *            interpolates linearly in a table of 48 to 256 entries; here
 *            each interval holds a cubic Hermite piece, max. error about
 *            4e-6 of the Newtonian factor at 64 intervals).  Pairs beyond
 *            alpha_split r = 6 (factor < 2e-15) get the value at 6.  The
 *            table lives in the tree workspace and is rebuilt when its
 *            length changes.  Node decisions and interaction counts do not
 *            depend on it.
 * ewald_table, ewald_n: kernel 2 only: a table that g4_ewald_table built for
 *            the tree's box side with ewald_n intervals (device, read only). */
typedef struct {
    int kernel;
    int criterion;
    int order;
    int exclusion;
    double G, eps0, r_s, r_cut, theta, alpha, theta_seed;
    const float *a_seed;
    int group_size;
    int seed_from_tree;
    int sr_table;
    const void *ewald_table;
    int ewald_n;
} g4_walk_params;

/* FMM (Sec. "Fast multipole method", "The FMM-PM approach"), p = 3.
 * Node pairs interact when the opening criterion holds, the cubes do not
 * touch and r >= h; kernel 1 drops pairs whose nearest sides are farther
 * apart than r_cut.  criterion 0: (l_A + l_B)/r < theta (eq. eqnNodeDec);
 * criterion 1: (M_max / r^2)(l_max / r)^(p-1) < alpha |a|_min, M_max and
 * l_max the larger mass and side of the two, |a|_min the smallest |a| of any
 * particle in either (a particle counts with l = 0, its own mass and |a|);
 * a_seed: device, caller order, |a| per particle (needed by criterion 1; the
 * per-node minima are formed in the call; it uses the tree's seed buffer, so
 * a later walk with seed_from_tree needs a new geometric call first).
 * deterministic = 1 sums every target's sources in a fixed order (bitwise
 * reproducible, slower: per-interaction lists are sorted); 0 gives the same
 * interactions with sums accumulated by atomics (round-off may differ from
 * run to run; the section on deterministic outcomes allows giving up binary
 * invariance for speed).
 * kernel 2 (periodic trees): Newtonian between the nearest images of the two
 * sides plus the correction potential psi of the other images in every
 * interaction's expansion (Sec. "Fast multipole method", periodic case), its
 * derivatives from ewald_table (built by g4_ewald_table for the tree's box
 * side with ewald_n intervals); no r_cut. */
typedef struct {
    int kernel;
    double G, eps0, r_s, r_cut, theta;
    int deterministic;
    int criterion;
    double alpha;
    const float *a_seed;
    const void *ewald_table;
    int ewald_n;
} g4_fmm_params;

/* Long-range (particle-mesh) part of the TreePM split (Sec. "TreePM
 * approach"): ng^3 mesh over the periodic box, split scale r_s (the same as
 * the short-range walk's), G. */
typedef struct {
    int ng;
    double r_s, G;
} g4_pm_params;

/* Hierarchical time integration (Sec. "Hierarchical time integration"). */
#define G4_KDK_MAX_LEVEL 30
typedef struct {
    int solver;          /* force of a set sourced by itself: 0 FP64 direct sum (wp: kernel, G, eps0, r_s),
                            1 tree walk (wp), 2 FMM (fp) */
    g4_tree_params tp;   /* root of every force calculation: a periodic box (positions are wrapped into it),
                            or an isolated root cube that must hold every position during the step */
    g4_walk_params wp;
    g4_fmm_params fp;
    double eta, eps;     /* step criterion sqrt(2 eta eps / |a|) */
    int max_level;       /* deepest level of the step hierarchy, 0..G4_KDK_MAX_LEVEL */
} g4_kdk_params;

typedef struct {
    uint64_t force_evals;          /* particles that received a force (the paper's force computations) */
    uint32_t force_calls;          /* force calculations (one tree per call) */
    uint32_t deepest_level;        /* deepest level entered */
    uint64_t evals_per_level[32];  /* force evaluations by the level of the set */
} g4_kdk_stats;

/* Counters and phase times filled by the force calls (host struct).
 * t_build, t_moments: duration of the tree's last g4_build_tree /
 * g4_build_forest and g4_compute_multipoles (HIP events on the context's
 * stream); t_seed: the geometric pre-walk, or the gather of a caller's
 * a_seed, of this call (0 for a geometric call); t_walk: this call's walk, or
 * the whole FMM of g4_fmm_force.  Seconds. */
typedef struct {
    double t_build, t_moments, t_seed, t_walk;
    uint64_t n_p2p;      /* particle-particle interactions */
    uint64_t n_p2m;      /* particle-node (one-sided) interactions */
    uint64_t n_visit;    /* node visits by active lanes (criterion evaluations) */
    uint64_t n_seed_p2p, n_seed_p2m, n_seed_visit;  /* same, geometric pre-walk (if run) */
    uint64_t n_pp, n_pn, n_nn;   /* FMM interaction counts */
    uint64_t n_nodes;    /* nodes in the tree */
    /* 64-lane steps of the walk: node visits, particle-node interactions,
     * particle-particle interactions; lane utilisation = count / (64 x steps) */
    uint64_t w_pop, w_p2m, w_p2p;
    /* bit 0: a leaf at max_depth holds more than leaf_max particles;
     * bit 1: node capacity exceeded (cannot happen within the documented sizes);
     * bit 2: a walk's traversal stack overflowed, forces incomplete;
     * bit 3: an FMM leaf-node stack overflowed, forces incomplete.
     * Bits 2 and 3 stay set until the tree is rebuilt and make the force call
     * that reads them (any call with stats, every g4_fmm_force) and
     * g4_tree_info return G4_ENOMEM. */
    uint32_t flags;
    uint32_t max_stack;  /* deepest traversal stack of the walk (entries; the first 30 are kept in LDS) */
    /* walk bookkeeping: sibling sets popped, (opened leaf, target) items,
     * particle-pair phases of the lane queue */
    uint64_t w_entry, w_leaf, w_chunk;
    /* (node, target) pairs of the walk decided once for the whole group of
     * targets: used by every target (included in n_p2m and n_visit), dropped
     * beyond r_cut by every target (not in n_visit) */
    uint64_t n_group_use, n_group_drop;
} g4_stats;

/* ---------------------------------------------------------------- context */
/* Bind a context to device `device` and HIP stream `hip_stream` (a
 * hipStream_t, or NULL for the default stream).  Host allocation only. */
int g4_ctx_create(int device, void *hip_stream, g4_ctx **out);
int g4_ctx_destroy(g4_ctx *ctx);
/* Message of the last error on this context (static storage of the ctx). */
const char *g4_last_error(const g4_ctx *ctx);

/* ---------------------------------------------------------- integer mapping */
/* pos: device, n x 3 float64 row-major (physical).  Writes x, y, z (device,
 * n uint32 each) per the mapping of g4_tree_params (periodic: floor(x/L 2^32)
 * mod 2^32; isolated: 2^30 + floor((x-origin)/box 2^31)).  Isolated root:
 * synchronises and returns G4_EROOT if a particle lies outside the root cube
 * (coordinates are then clamped to the root).  Periodic: cannot fail, returns
 * without synchronising.  `flag` is a device int32 scratch word supplied by
 * the caller (written only for an isolated root). */
int g4_quantize(g4_ctx *ctx, const double *pos, int64_t n, const g4_tree_params *tp,
                uint32_t *x, uint32_t *y, uint32_t *z, int32_t *flag);

/* ---------------------------------------------------------------- tree */
/* Workspace bytes for a tree over n particles (node storage sized for the
 * worst case N + max_depth * N/(B+1) nodes, key sort buffers, moments). */
int g4_workspace_bytes(const g4_tree_params *tp, int64_t n, size_t *bytes);

/* Build the octree over Morton-sorted particles (Sec. "Geometry of the
 * tree"): quantised coordinates -> 63-bit Morton keys -> stable radix sort ->
 * level-synchronous node splitting.  ws: device buffer of ws_bytes (kept by
 * the tree until g4_tree_free; the particle arrays are copied into it).
 * *out receives a host handle. */
int g4_build_tree(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, void *ws, size_t ws_bytes,
                  g4_tree **out);

/* Forest of nbox independent periodic boxes of side tp->box (batching):
 * box b holds the caller's particles [box_offsets[b], box_offsets[b+1])
 * (host array of nbox + 1, starting at 0 and ending at n, every box
 * non-empty).  One node array with one root per box (nodes 0..nbox-1);
 * multipoles and walks work on it as on a single tree, the walk running as
 * one persistent launch over (box, particle group) work items, largest boxes
 * first.  Workspace from g4_forest_workspace_bytes. */
int g4_forest_workspace_bytes(const g4_tree_params *tp, int nbox, int64_t n, size_t *bytes);
int g4_build_forest(g4_ctx *ctx, int nbox, const int64_t *box_offsets, const g4_particles *p,
                    const g4_tree_params *tp, void *ws, size_t ws_bytes, g4_tree **out);

/* Multipole moments up to octupole about each node's centre of mass
 * (Sec. "One-sided multipole expansion"; upward pass as in the first FMM
 * phase): leaves from their particles, parents from their children by the
 * parallel-axis shift.  FP64 accumulation at levels <= 8, FP32 below. */
int g4_compute_multipoles(g4_ctx *ctx, g4_tree *tree, int order);

/* Fourth moments (15 per node, FP64) about each node's centre of mass, for
 * walks at p = 4 and 5 (Appendix A, "Multipole extensions at different
 * order"): leaves from their particles, parents from their children's
 * moments of orders 0..4 shifted to the parent's centre of mass.  Needs
 * g4_compute_multipoles(order 3) of the same tree; ws: device, 256-byte
 * aligned, at least g4_moments4_bytes(tree) bytes, owned by the caller and kept
 * by the tree (until the next g4_compute_multipoles) for its walks.  Then
 * walks may take order 4 (force with the octupole term, potential to the
 * fourth moments) or 5 (force with the hexadecapole term as well; the
 * potential's fifth-moment term is left out, as in the paper's practice).
 * Asynchronous. */
size_t g4_moments4_bytes(const g4_tree *tree);
int g4_compute_moments4(g4_ctx *ctx, g4_tree *tree, void *ws, size_t bytes);

/* Node count and level ranges of a built tree (host outputs; synchronises).
 * level_start: host array of max_depth + 2 int64 (may be NULL). */
int g4_tree_info(g4_ctx *ctx, const g4_tree *tree, int64_t *nnodes, int64_t *level_start);

/* Copy node data to caller device buffers (any pointer may be NULL):
 * level (int32), cell (3 x uint32 per node: integer cube index at its level),
 * count (int64 particles), first (int64: the node's first particle in curve
 * order; its particles are the next count), leaf (int32), mass (f64), com (3 x f64 physical,
 * relative to the root's lower corner), q2 (6 x f64: xx xy xz yy yz zz), q3 (10 x f64:
 * xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).  Moments need g4_compute_multipoles. */
int g4_tree_export(g4_ctx *ctx, const g4_tree *tree, int32_t *level, uint32_t *cell, int64_t *count,
                   int64_t *first, int32_t *leaf, double *mass, double *com, double *q2, double *q3);

int g4_tree_free(g4_ctx *ctx, g4_tree *tree);

/* --------------------------------------------------------------- forces */
/* One-sided tree walk (kernel per params).  ax, ay, az: device, n float64,
 * caller order.  pot: device n float64 or NULL.  counts: device n x 2 uint32
 * (particle-particle, particle-node per particle) or NULL.  a_out: device n
 * float32 |a| (caller order) or NULL.  stats: host or NULL (synchronises);
 * the walk counts interactions and passes only when it is given, so a call
 * without it runs slightly less work.  A geometric call (criterion 0) also
 * keeps |a| inside the tree for a later relative call with seed_from_tree = 1. */
int g4_tree_force(g4_ctx *ctx, g4_tree *tree, const g4_walk_params *wp, double *ax, double *ay, double *az,
                  double *pot, uint32_t *counts, float *a_out, g4_stats *stats);

/* The TreePM short-range force (kernel forced to 1). */
int g4_treepm_shortrange(g4_ctx *ctx, g4_tree *tree, const g4_walk_params *wp, double *ax, double *ay,
                         double *az, double *pot, uint32_t *counts, float *a_out, g4_stats *stats);

/* Table of the periodic correction potential psi for kernel 2 of the walk
 * (Sec. "Periodic boundary conditions", eqs. eqnpo2 and eqnewal):
 *   psi(x) = 1/|x| + pi/(alpha^2 V) - sum_n erfc(alpha|x + q_n|)/|x + q_n|
 *            - (4 pi/V) sum_{k != 0} exp(-k^2/(4 alpha^2))/k^2 cos(k.x),
 * the potential of a unit mass's periodic images other than the nearest one
 * (with the sign of eq. eqnpo1: phi = -m/r + m psi).  psi is even in every
 * coordinate, so one octant is stored: the derivatives D^(a,b,c) psi of
 * orders 0..6 (84 FP32 values) at the (ne + 1)^3 points (i, j, k) box/(2 ne),
 * i, j, k = 0..ne, each computed in FP64 from the Ewald sums (alpha = 2/box).
 * The walk evaluates psi's derivatives of order n at an offset d from the
 * nearest grid point d0 by the third-order Taylor expansion
 * D_n(d) = sum_{|b| <= 3} D_{n+b}(d0) (d - d0)^b / b! that the paper uses in
 * place of trilinear interpolation.  ne: 4..128 (error of the expansion about
 * (box / 4 ne)^4 relative; 32 keeps it near FP32 round-off).  table: device,
 * 256-byte aligned, at least g4_ewald_table_bytes(ne) bytes (12 MB at ne 32),
 * owned by the caller.  Asynchronous. */
size_t g4_ewald_table_bytes(int ne);
int g4_ewald_table(g4_ctx *ctx, double box, int ne, void *table, size_t bytes);

/* psi and grad psi at n offsets through the table's Taylor expansion (the
 * lookup the walk uses for a single particle).  dx, dy, dz: device float64,
 * each component in [-box/2, box/2]; psi, gx, gy, gz: device float64 outputs.
 * Asynchronous. */
int g4_ewald_eval(g4_ctx *ctx, const void *table, int ne, double box, int64_t n, const double *dx, const double *dy,
                  const double *dz, double *psi, double *gx, double *gy, double *gz);

/* Workspace bytes of g4_pm_longrange for an ng^3 mesh (12 bytes per mesh
 * point: the complex FP32 mesh and the real potential). */
int g4_pm_workspace_bytes(int ng, size_t *bytes);

/* Long-range TreePM force and potential of every particle of a built
 * periodic tree (Sec. "TreePM approach"): clouds-in-cell assignment of the
 * masses to the mesh (mesh point c at c L/ng), FFT, multiplication with the
 * Green's function -G (4 pi / V) exp(-k^2 r_s^2) / k^2 divided twice by the
 * CIC window prod_d sinc^2(pi n_d / ng) (deconvolution of assignment and
 * interpolation; zero at k = 0), inverse FFT, 4th-order central differences
 * for the gradient, CIC interpolation.  ng: power of two in [8, 1024].
 * ax, ay, az (pot nullable): device n float64, caller order; accumulate = 0
 * writes them, 1 adds to them (e.g. to the short-range walk's output, giving
 * the total TreePM force).  FP32 mesh arithmetic, FP64 outputs.  Needs no
 * moments; a forest (several boxes) is refused.  Asynchronous. */
int g4_pm_longrange(g4_ctx *ctx, const g4_tree *tree, const g4_pm_params *pp, void *ws, size_t ws_bytes,
                    int accumulate, double *ax, double *ay, double *az, double *pot);

/* Workspace bytes of g4_kdk_step for n particles (index lists and forces of
 * every level, one tree workspace, the FMM's lists for solver 2). */
int g4_kdk_workspace_bytes(const g4_kdk_params *kp, int64_t n, size_t *bytes);

/* One step dt of the hierarchical time integration of n particles: a set P
 * whose forces (sourced by P) are known is advanced by
 * K_P^P(dt/2) K_F^F(-dt/2) E(H_F, dt/2) D_S(dt) E(H_F, dt/2) K_F^F(-dt/2) K_P^P(dt/2),
 * F the particles whose step sqrt(2 eta eps / |a|) is below dt, S the rest,
 * E(H_F, dt/2) the same step applied to F alone with dt/2 (its first forces
 * are the F-sourced forces computed to split it), and a plain kick-drift-kick
 * when F is empty or the level is max_level.  Every force is sourced by the
 * set it acts on, so momentum is conserved to round-off by the FMM (solver 2)
 * and by direct sums.
 * pos, vel: device n x 3 float64 (row-major, physical), updated in place;
 * mass: device n float32; ax, ay, az: device n float64: the forces of all
 * particles at the start (have_acc = 1) -- else computed first -- and at the
 * end on return.  Synchronises (the size of every fast set is read back).
 * Returns G4_EROOT when an isolated root no longer holds a particle. */
int g4_kdk_step(g4_ctx *ctx, const g4_kdk_params *kp, int64_t n, double *pos, double *vel, const float *mass,
                double dt, double *ax, double *ay, double *az, int have_acc, void *ws, size_t ws_bytes,
                g4_kdk_stats *stats);

/* Direct summation on the device (the exact reference of Sec. "Softened
 * potential in periodic systems"): forces on `ntargets` particles (device
 * int64 indices into the caller order, or NULL for all) from all n particles,
 * FP64 arithmetic.  kernel/eps0/r_s from wp; r_cut used only if truncate.
 * kernel 2 (periodic): the softened nearest image plus psi of the other
 * images by exact Ewald sums per pair (Sec. "Periodic boundary conditions";
 * ~10^3 terms per pair, meant for sampled targets).  Kernels 1 and 2 need a
 * periodic tp. */
int g4_direct_force(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, const g4_walk_params *wp,
                    int truncate, const int64_t *targets, int64_t ntargets, double *ax, double *ay, double *az,
                    double *pot);

/* ------------------------------------------------------- learned |a| seed */
/* The relative criterion needs |a| before the first force; the paper gets it
 * from a geometric pre-walk (footnote to eq. eqnrelcriterion).  These calls
 * predict log10 |a| instead with a perceptron 8 -> 64 -> 64 -> 1 (SiLU), BF16
 * weights (4801 values, layout W1[64][8], b1[64], W2[64][64], b2[64], w3[64],
 * b3), FP32 arithmetic. */

/* Per-particle features from the particle's leaf L, its parent P and its
 * grandparent (caller order, n x 8 float): log10 M_L, log10 l_L, level of L,
 * log10(|x - s_L|/l_L + 1e-3), log10(|x - s_P|/l_P + 1e-3), log10 M_P,
 * log10 M_grandparent, log10 |a_near| (pair forces of the other particles of
 * L plus monopoles of the siblings of L and of P, with the softened kernel of
 * wp: kernel, eps0, r_s).  norm: device 16 floats (mean[8], 1/std[8]) applied
 * as (f - mean) / std, or NULL for raw features.  Needs
 * g4_compute_multipoles. */
int g4_mlp_features(g4_ctx *ctx, const g4_tree *tree, const g4_walk_params *wp, const float *norm, float *feat);

/* out[i] = y_i (mode 0) or 10^(y_i + shift) (mode 1, directly usable as
 * g4_walk_params.a_seed); w_bf16: device 4801 bf16; feat: device n x 8. */
int g4_mlp_forward(g4_ctx *ctx, const void *w_bf16, const float *feat, int64_t n, float *out, float shift, int mode);

/* Gradient of the loss with respect to the 4801 parameters (device float
 * grad[4801], overwritten) and the loss itself (device float).  tau <= 0:
 * L = (1/n) sum (y_i - target_i)^2; 0 < tau < 1: pinball loss
 * L = (1/n) sum rho_tau(target_i - y_i), rho_tau(u) = u (tau - [u < 0]),
 * which fits the tau-quantile (a conservative, low seed for small tau). */
int g4_mlp_grad(g4_ctx *ctx, const void *w_bf16, const float *feat, const float *target, int64_t n, float tau,
                float *grad, float *loss);

/* One Adam step (Kingma & Ba 2015) on FP32 master weights with moment buffers
 * m, v (device float[4801] each); rewrites w_bf16 as the rounded master
 * weights.  step counts from 1. */
int g4_mlp_adam(g4_ctx *ctx, void *w_bf16, float *w_master, float *m, float *v, const float *grad, float lr,
                float beta1, float beta2, float eps, int64_t step);

/* grad + Adam in one call: adam_state = m[4801] followed by v[4801]; grad is
 * caller scratch of 4801 floats; loss receives L before the update. */
int g4_mlp_train_step(g4_ctx *ctx, void *w_bf16, float *w_master, float *adam_state, float *grad,
                      const float *feat, const float *target, int64_t n, float tau, float lr, int64_t step,
                      float *loss);

/* ------------------------------------------------------------------ FMM */
/* Workspace for g4_fmm_force on this tree with these parameters: field
 * expansions (20 floats per node) and, for deterministic = 1, a pair frontier
 * and interaction lists of list_factor x (48, 96, 160) x n entries plus sort
 * scratch; for deterministic = 0, a frontier of node pairs and a task list of
 * list_factor x 2n entries each and FP64 accumulators (32 bytes per
 * particle).  list_factor <= 0 means 1. */
int g4_fmm_workspace_bytes(const g4_tree *tree, const g4_fmm_params *fp, double list_factor, size_t *bytes);

/* Symmetric FMM at p = 3 (Sec. "Fast multipole method"): dual walk from
 * (root, root), field expansions in both nodes of every accepted pair,
 * particle-node and particle-particle interactions, downward shift and
 * evaluation at the particles.  Needs g4_compute_multipoles(order 3).
 * ax, ay, az (pot nullable): device n float64, caller order.  Synchronises
 * (list sizes are read back); returns G4_ENOMEM when the lists exceed the
 * workspace of list_factor (retry with a larger factor).  With deterministic
 * = 1 each target sums its sources in the order of their first particle and
 * level, so results do not depend on list construction or node numbering.
 * n < 2^27. */
int g4_fmm_force(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double list_factor, void *ws, size_t ws_bytes,
                 double *ax, double *ay, double *az, double *pot, g4_stats *stats);

/* g4_fmm_force without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The FMM's lists, field expansions and
 * accumulators live in a static 64 MiB device array that the library holds
 * on every device it runs on until the process ends; the call itself
 * allocates nothing.  It uses the largest list factor (4, 2 or 1) whose
 * workspace fits and returns G4_EINVAL with the sizes in the message when
 * even factor 1 does not (about 500 bytes per particle at leaf 16: trees up
 * to roughly 10^5 particles), G4_ENOMEM when the interaction lists outgrow
 * the chosen factor.  All calls on one device share that device's array:
 * calls that overlap on one device (two streams, two host threads) race and
 * must be serialised by the caller.  Same results as g4_fmm_force: bitwise
 * for deterministic = 1, to round-off for deterministic = 0. */
int g4_fmm_force_noalloc(g4_ctx *ctx, g4_tree *tree, const g4_fmm_params *fp, double *ax, double *ay, double *az,
                         double *pot, g4_stats *stats);

#ifdef __cplusplus
}
#endif
#endif
