/*
 * g4oracle.h -- interface of the plain FP64 CPU oracle (test infrastructure
 * only; never linked by the HIP library).  Arrays are host memory owned by
 * the caller unless stated otherwise; positions are the integer fixed-point
 * coordinates of the paper's Sec. "Integer coordinates".
 */
#ifndef G4ORACLE_H
#define G4ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_tree orc_tree;

typedef struct {
    int kernel;      /* 0 softened Newtonian, 1 TreePM short-range (eq. eqnpo4),
                        2 periodic softened Newtonian + Ewald correction (eq. eqnpo1) */
    int criterion;   /* 0 geometric l/r < theta, 1 relative (eq. eqnrelcriterion) */
    int order;       /* expansion order p (2..5; 4 and 5 need orc_moments4) */
    int exclusion;   /* 1: never accept a node whose 2l-cube holds the target */
    double G, eps0, r_s, r_cut, theta, alpha;
} orc_walk_params;

typedef struct {
    int kernel;      /* 0 Newtonian (isolated), 1 short-range (FMM-PM short-range pass),
                        2 periodic Newtonian + Ewald correction */
    double G, eps0, r_s, r_cut, theta;
    int criterion;   /* 0 geometric (l_A + l_B)/r < theta, 1 relative (M_max/r^2)(l_max/r)^2 < alpha |a|_min */
    double alpha;
} orc_fmm_params;

/* softening and kernels (scalar closed forms) */
double orc_soft_K(double r, double h);
double orc_soft_W(double r, double h);
double orc_sr_K(double r, double h, double alpha);
double orc_sr_W(double r, double h, double alpha);
void orc_gn(int kernel, double r, double alpha, double g[4]);
void orc_Dn(int kernel, const double rv[3], double alpha, double *D0, double D1[3], double D2[9], double D3[27]);
/* g_0..g_nmax (nmax <= 7) and the full tensor D_n (3^n values) from them */
void orc_gn_ext(int kernel, double r, double alpha, int nmax, double *g);
void orc_Dfull(const double *g, const double r[3], int n, double *D);
/* periodic correction potential psi of a cube of side L and its derivative
 * tensors (full 3, 3x3, 3x3x3 arrays), exact Ewald sums; alpha <= 0: 2/L */
void orc_ewald_psi(const double x[3], double L, double alpha, double *D0, double D1[3], double D2[9], double D3[27]);

/* integer mapping: pos is n x 3 row-major; returns 0 or -5 (outside root) */
int orc_quantize(int64_t n, const double *pos, int periodic, double box, const double origin[3],
                 uint32_t *X, uint32_t *Y, uint32_t *Z);

/* tree (recursive partition), moments (direct sums) */
orc_tree *orc_build(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                    int periodic, double box, int leaf_max, int max_depth);
void orc_free(orc_tree *t);
int64_t orc_tree_nnodes(const orc_tree *t);
void orc_tree_nodes(const orc_tree *t, int32_t *level, uint32_t *cell3, int64_t *count, int32_t *leaf);
void orc_moments(orc_tree *t);
/* fourth moments (81 per node) for walks at p = 4, 5 */
void orc_moments4(orc_tree *t);
/* the same, with the work shared out to nthreads threads (the serial code
 * above for nthreads <= 1; the threaded build numbers the nodes differently) */
orc_tree *orc_build_mt(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                       int periodic, double box, int leaf_max, int max_depth, int nthreads);
void orc_moments_mt(orc_tree *t, int nthreads);
void orc_tree_moments(const orc_tree *t, double *mass, double *com3, double *q2p, double *q3p);

/* one-sided walk; aseed (|a| per particle, caller order) needed for criterion 1.
 * targets: optional list of particle indices (NULL = all).  acc: ntargets x 3.
 * counts: optional ntargets x 2 (particle-particle, particle-node). */
int orc_walk(const orc_tree *t, const orc_walk_params *P, const double *aseed, const int64_t *targets,
             int64_t ntargets, double *acc, double *pot, int64_t *counts, int nthreads);

/* direct summation; unit = physical length of one integer step */
void orc_direct(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                double unit, const orc_walk_params *P, int truncate, const int64_t *targets, int64_t ntargets,
                double *acc, double *pot, int nthreads);

/* FMM, p = 3; acc n x 3 (caller order); stats: pp, pn, nn interaction counts;
 * aseed: |a| per particle (caller order), needed by criterion 1 */
int orc_fmm(const orc_tree *t, const orc_fmm_params *P, const double *aseed, double *acc, double *pot,
            int64_t stats[3]);

/* MLP 8 -> 64 -> 64 -> 1 (SiLU), 4801 parameters */
void orc_mlp_forward(const double *w, const double *feat, int64_t n, double *out);
double orc_mlp_loss_grad(const double *w, const double *feat, const double *target, int64_t n, double tau,
                         double *grad);
void orc_adam(double *w, const double *g, double *m, double *v, int64_t np, double lr, double b1, double b2,
              double eps, int64_t step);

/* two isolated groups (physical positions, G = 1, Newtonian): forces on the
 * particles of each group from the other, FMM (p = 3) and one-sided tree */
void orc_two_groups(int64_t nA, const double *posA, const double *mA, int64_t nB, const double *posB,
                    const double *mB, double *accA_fmm, double *accB_fmm, double *accA_tree, double *accB_tree);

/* learned-seed features of every particle (n x 8, caller order); P gives
 * the pair kernel (kernel, eps0, r_s) of the near-field force feature */
int orc_features(const orc_tree *t, const orc_walk_params *P, double *feat);

#ifdef __cplusplus
}
#endif
#endif
