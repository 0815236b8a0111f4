/*
 * g4oracle.c -- plain FP64 CPU oracle for the gravity hot path of
 * Springel, Pakmor, Zier & Reinecke (2021), "Simulating cosmic structure
 * formation with the GADGET-4 code" (arXiv:2010.03567).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this
 * code; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no source, header or table with the
 * HIP library: it is written independently from the paper's formulas.
 *
 * Everything is double precision and written for a reader to check
 * against the paper by eye: recursive index partition for the tree,
 * direct per-node sums for the moments, full 3x3 / 3x3x3 tensors for the
 * multipole algebra, a recursive walk per particle, a recursive dual-tree
 * interaction routine for FMM.
 *
 * Paper passages followed (section / equation names of the paper):
 *   softening law ............ Sec. "Softened potential in periodic systems",
 *                              eq. (eqnsoft) + the cubic spline kernel of
 *                              the SPH section (Sec. "SPH kernels")
 *   nearest image / integers . Sec. "Integer coordinates"; Sec.
 *                              "Non-periodic potentials"
 *   tree geometry ............ Sec. "Geometry of the tree"
 *   one-sided expansion ...... Sec. "One-sided multipole expansion",
 *                              eqs. (eqonesidetreepotential), (eqonesidetreeacc)
 *   opening criteria ......... Sec. "Tree walk and opening criterion",
 *                              eq. (eqnrelcriterion), exclusion zone
 *   short-range kernel ....... Sec. "TreePM approach", eq. (eqnpo4);
 *                              r_s = 1/(2 alpha) from eq. (eqnewal)
 *   derivative tensors ....... Sec. "Fast multipole method", eqs.
 *                              (eqngderiv0)-(eqngderiv); Appendix A g_n
 *   FMM ...................... Sec. "Fast multipole method" (symmetric
 *                              expansion, node-node criterion eq.
 *                              (eqnNodeDec), no-touching rule, three
 *                              phases); Sec. "The FMM-PM approach"
 *
 * Readings where the paper is silent are listed in the design notes; the
 * ones that matter here: node opened when r < h = 2.8 eps0 (GADGET-3
 * rule for softened nodes), relative criterion M l^3 < alpha |a| r^5 with
 * strict "<", exclusion zone = cube of side 2l centred on the node, TreePM
 * node dropped when its nearest edge is farther than r_cut (strict ">").
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "g4oracle.h"

#define TWO32 4294967296.0
#define TWO31 2147483648.0
#define TWO30 1073741824.0
#define SQRTPI 1.77245385090551602729816748334

/* ======================================================================
 * 1. Softening: cubic-spline (M4) mass distribution of radius h = 2.8 eps0
 * ====================================================================== */

/* Force factor K(r): a_i = G m_j (x_j - x_i) K(r).  Enclosed mass of the
 * M4 density (8 m / pi h^3) w(r/h), divided by m r^3. */
double orc_soft_K(double r, double h)
{
    if (r >= h) return 1.0 / (r * r * r);
    double u = r / h, h3 = h * h * h;
    if (u < 0.5) return (32.0 / 3.0 - 192.0 / 5.0 * u * u + 32.0 * u * u * u) / h3;
    return (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u * u - 32.0 / 3.0 * u * u * u - 1.0 / (15.0 * u * u * u)) / h3;
}

/* Potential factor W(r): phi_i = -G m_j W(r); W(0) = 2.8/h = 1/eps0. */
double orc_soft_W(double r, double h)
{
    if (r >= h) return 1.0 / r;
    double u = r / h, u2 = u * u;
    if (u < 0.5) return (14.0 / 5.0 - 16.0 / 3.0 * u2 + 48.0 / 5.0 * u2 * u2 - 32.0 / 5.0 * u2 * u2 * u) / h;
    return (16.0 / 5.0 - 1.0 / (15.0 * u) - 32.0 / 3.0 * u2 + 16.0 * u2 * u - 48.0 / 5.0 * u2 * u2
            + 32.0 / 15.0 * u2 * u2 * u) / h;
}

/* ======================================================================
 * 2. Short-range (TreePM) kernel, g(r) = erfc(alpha r)/r, alpha = 1/(2 r_s)
 * ====================================================================== */

/* f(x)/x^3 with f(x) = erf(x) - (2x/sqrt(pi)) exp(-x^2): the long-range
 * pair factor is alpha^3 f(x)/x^3.  f' = (4/sqrt(pi)) x^2 exp(-x^2), so
 * f(x)/x^3 = (4/sqrt(pi)) sum_k (-1)^k x^(2k) / (k! (2k+3)). */
static double lr_force_over_x3(double x)
{
    if (x < 0.5) {
        double s = 0.0, t = 1.0, x2 = x * x;
        for (int k = 0; k < 30; k++) {
            s += t / (2.0 * k + 3.0);
            t *= -x2 / (k + 1.0);
        }
        return 4.0 / SQRTPI * s;
    }
    return (erf(x) - 2.0 * x / SQRTPI * exp(-x * x)) / (x * x * x);
}

/* erf(x)/x via its Taylor series near 0. */
static double erf_over_x(double x)
{
    if (x < 0.5) {
        double s = 0.0, t = 1.0, x2 = x * x;
        for (int k = 0; k < 30; k++) {
            s += t / (2.0 * k + 1.0);
            t *= -x2 / (k + 1.0);
        }
        return 2.0 / SQRTPI * s;
    }
    return erf(x) / x;
}

/* Short-range pair force factor: softened Newtonian minus the long-range
 * (erf) part, i.e. the gradient of eq. (eqnpo4) for one source. */
double orc_sr_K(double r, double h, double alpha)
{
    double x = alpha * r;
    if (r >= h) {
        return (erfc(x) + 2.0 * x / SQRTPI * exp(-x * x)) / (r * r * r);
    }
    return orc_soft_K(r, h) - alpha * alpha * alpha * lr_force_over_x3(x);
}

/* Short-range potential factor (phi_i = -G m_j W_sr), eq. (eqnpo4) without
 * the constant pi/(alpha^2 V). */
double orc_sr_W(double r, double h, double alpha)
{
    double x = alpha * r;
    if (r >= h) return erfc(x) / r;
    return orc_soft_W(r, h) - alpha * erf_over_x(x);
}

/* g_n(r) = (r^-1 d/dr)^n g(r), n = 0..3.
 * kernel 0: Newtonian g = 1/r (Appendix A values).
 * kernel 1: g = erfc(alpha r)/r (closed forms from the recursion). */
void orc_gn(int kernel, double r, double alpha, double g[4])
{
    double ri = 1.0 / r, ri2 = ri * ri;
    if (kernel == 0) {
        g[0] = ri;
        g[1] = -ri * ri2;
        g[2] = 3.0 * ri * ri2 * ri2;
        g[3] = -15.0 * ri * ri2 * ri2 * ri2;
        return;
    }
    double x = alpha * r, ec = erfc(x);
    double E = 2.0 * alpha / SQRTPI * exp(-x * x);
    double a2 = alpha * alpha;
    g[0] = ec * ri;
    g[1] = -(ec * ri * ri2 + E * ri2);
    g[2] = 3.0 * ec * ri * ri2 * ri2 + E * (3.0 * ri2 * ri2 + 2.0 * a2 * ri2);
    g[3] = -(15.0 * ec * ri * ri2 * ri2 * ri2 + E * (15.0 * ri2 * ri2 * ri2 + 10.0 * a2 * ri2 * ri2
                                                      + 4.0 * a2 * a2 * ri2));
}

/* Derivative tensors D_0..D_3 as full arrays, eqs. (eqngderiv0)-(eqngderiv):
 * D1_i = g1 r_i, D2_ij = g1 d_ij + g2 r_i r_j,
 * D3_ijk = g2 (d_ij r_k + d_jk r_i + d_ik r_j) + g3 r_i r_j r_k. */
void orc_Dn(int kernel, const double rv[3], double alpha, double *D0, double D1[3], double D2[9], double D3[27])
{
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double g[4];
    orc_gn(kernel, r, alpha, g);
    *D0 = g[0];
    for (int i = 0; i < 3; i++) {
        D1[i] = g[1] * rv[i];
        for (int j = 0; j < 3; j++) {
            D2[i * 3 + j] = (i == j ? g[1] : 0.0) + g[2] * rv[i] * rv[j];
            for (int k = 0; k < 3; k++) {
                double t = 0.0;
                if (i == j) t += rv[k];
                if (j == k) t += rv[i];
                if (i == k) t += rv[j];
                D3[(i * 3 + j) * 3 + k] = g[2] * t + g[3] * rv[i] * rv[j] * rv[k];
            }
        }
    }
}

/* g_0..g_nmax (nmax <= 7) of the Newtonian kernel (Appendix A: g_n =
 * (-1)^n (2n-1)!! / r^(2n+1)) or of erfc(alpha r)/r, whose g_n follow from
 * the recursion g_{n+1} = r^-1 d g_n/dr with
 * g_n = A_n erfc(alpha r) r^-(2n+1) + E sum_j b_nj r^-2j,
 * E = (2 alpha/sqrt(pi)) exp(-alpha^2 r^2), A_{n+1} = -(2n+1) A_n,
 * b_{n+1,j} += -2 alpha^2 b_nj, b_{n+1,j+1} += -2j b_nj, b_{n+1,n+1} += -A_n. */
void orc_gn_ext(int kernel, double r, double alpha, int nmax, double *g)
{
    double ri2 = 1.0 / (r * r), rp = 1.0 / r, A = 1.0;
    if (kernel == 0) {
        for (int n = 0; n <= nmax; n++) {
            g[n] = A * rp;
            A *= -(2.0 * n + 1.0);
            rp *= ri2;
        }
        return;
    }
    double ec = erfc(alpha * r), E = 2.0 * alpha / SQRTPI * exp(-alpha * alpha * r * r), a2 = alpha * alpha;
    double b[9] = {0}, nb[9];
    for (int n = 0; n <= nmax; n++) {
        double sum = 0.0, rj = 1.0;
        for (int j = 1; j <= n; j++) {
            rj *= ri2;
            sum += b[j] * rj;
        }
        g[n] = A * ec * rp + E * sum;
        for (int j = 0; j <= n + 1; j++) nb[j] = 0.0;
        for (int j = 1; j <= n; j++) {
            nb[j] += -2.0 * a2 * b[j];
            nb[j + 1] += -2.0 * j * b[j];
        }
        nb[n + 1] += -A;
        memcpy(b, nb, sizeof(double) * (size_t)(n + 2));
        A *= -(2.0 * n + 1.0);
        rp *= ri2;
    }
}

/* sum over the ways to pair up some of the indices idx[k..n-1] that are not
 * yet used: each pair gives a Kronecker delta, each index left alone gives
 * the component of r; a term with m pairs carries g_{n-m} */
static double pairings_sum(const int *idx, int n, unsigned used, int npairs, const double *r, const double *g)
{
    int k = 0;
    while (k < n && (used >> k & 1u)) k++;
    if (k == n) return g[n - npairs];
    used |= 1u << k;
    double s = r[idx[k]] * pairings_sum(idx, n, used, npairs, r, g);   /* idx[k] alone */
    for (int l = k + 1; l < n; l++)
        if (!(used >> l & 1u) && idx[l] == idx[k]) s += pairings_sum(idx, n, used | 1u << l, npairs + 1, r, g);
    return s;
}

/* the full derivative tensor D_n (3^n components, row-major) of a radial
 * kernel with scalars g at offset r:  d^n g / dx_i1 .. dx_in =
 * sum over pairings of Kronecker deltas and r-components, times g_{n - #pairs} */
void orc_Dfull(const double *g, const double r[3], int n, double *D)
{
    int total = 1;
    for (int k = 0; k < n; k++) total *= 3;
    for (int c = 0; c < total; c++) {
        int idx[8], v = c;
        for (int k = n - 1; k >= 0; k--) {
            idx[k] = v % 3;
            v /= 3;
        }
        D[c] = pairings_sum(idx, n, 0u, 0, r, g);
    }
}

/* ======================================================================
 * 2b. Periodic correction potential psi (Sec. "Periodic boundary
 *     conditions", eqs. (eqnpo1), (eqnpo2), (eqnewal))
 * ====================================================================== */

/* For a cube of side L, V = L^3:
 *   psi(x) = 1/|x| + pi/(alpha^2 V) - sum_n erfc(alpha |x + q_n|)/|x + q_n|
 *            - (4 pi / V) sum_{k != 0} exp(-k^2/(4 alpha^2))/k^2 cos(k.x),
 * q_n = L n, k = 2 pi n / L.  The n = 0 image and 1/|x| combine into
 * erf(alpha r)/r, which is regular at r = 0.  The result does not depend on
 * alpha (a pin); the sums stop where their terms fall below ~1e-22 of the
 * leading ones: real images with (NR + 1/2) alpha L >= 7, wave vectors with
 * pi (NK + 1)/(alpha L) >= 7.5.  A periodic mass distribution then has the
 * potential phi(x) = -sum_j m_j [1/|d_j| - psi(d_j)] with d_j = x_j - x
 * reduced to the nearest image (eq. eqnpo1, softening of the nearest image
 * aside), and the force a = sum_j m_j [d_j/|d_j|^3 + grad psi(d_j)].       */

/* g_k = (r^-1 d/dr)^k of erf(alpha r)/r, k = 0..3: the series
 * erf(ar)/r = (2a/sqrt(pi)) sum_m (-a^2)^m r^(2m) / (m! (2m+1)) for small
 * alpha r, Newtonian minus the erfc closed forms otherwise. */
static void erf_over_r_gn(double r, double alpha, double g[4])
{
    if (alpha * r < 0.5) {
        /* with u = r^2, r^-1 d/dr = 2 d/du: g_k = (2a/sqrt(pi)) 2^k sum_{m>=k} (-a^2)^m u^(m-k) / ((m-k)! (2m+1)) */
        double u = r * r, a2 = alpha * alpha;
        for (int k = 0; k < 4; k++) {
            double sum = 0.0, am = 1.0;              /* (-a^2)^m */
            for (int m = 0; m < k; m++) am *= -a2;
            double um = 1.0, fact = 1.0;            /* u^(m-k), (m-k)! */
            for (int m = k; m < k + 30; m++) {
                sum += am * um / (fact * (2.0 * m + 1.0));
                am *= -a2;
                um *= u;
                fact *= (double)(m - k + 1);
            }
            g[k] = 2.0 * alpha / SQRTPI * ldexp(sum, k);
        }
        return;
    }
    double gn[4], ge[4];
    orc_gn(0, r, alpha, gn);
    orc_gn(1, r, alpha, ge);
    for (int k = 0; k < 4; k++) g[k] = gn[k] - ge[k];
}

/* add c * (D0..D3 of a radial function with scalars g at offset rv) */
static void add_radial(const double g[4], const double rv[3], double c, double *D0, double D1[3], double D2[9],
                       double D3[27])
{
    *D0 += c * g[0];
    for (int i = 0; i < 3; i++) {
        D1[i] += c * g[1] * rv[i];
        for (int j = 0; j < 3; j++) {
            D2[i * 3 + j] += c * ((i == j ? g[1] : 0.0) + g[2] * rv[i] * rv[j]);
            for (int k = 0; k < 3; k++) {
                double t = 0.0;
                if (i == j) t += rv[k];
                if (j == k) t += rv[i];
                if (i == k) t += rv[j];
                D3[(i * 3 + j) * 3 + k] += c * (g[2] * t + g[3] * rv[i] * rv[j] * rv[k]);
            }
        }
    }
}

/* psi and its derivative tensors D1_i = d_i psi, D2_ij, D3_ijk at x (any x;
 * alpha <= 0 selects alpha = 2/L). */
void orc_ewald_psi(const double x[3], double L, double alpha, double *D0, double D1[3], double D2[9], double D3[27])
{
    if (alpha <= 0.0) alpha = 2.0 / L;
    double V = L * L * L;
    int NR = (int)ceil(7.0 / (alpha * L) - 0.5), NK = (int)ceil(7.5 * alpha * L / M_PI - 1.0);
    if (NR < 1) NR = 1;
    if (NK < 1) NK = 1;
    *D0 = M_PI / (alpha * alpha * V);
    memset(D1, 0, 3 * sizeof(double));
    memset(D2, 0, 9 * sizeof(double));
    memset(D3, 0, 27 * sizeof(double));
    double g[4];
    /* n = 0: 1/|x| - erfc(alpha r)/r = erf(alpha r)/r */
    erf_over_r_gn(sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]), alpha, g);
    add_radial(g, x, 1.0, D0, D1, D2, D3);
    /* the other real-space images */
    for (int nx = -NR; nx <= NR; nx++)
        for (int ny = -NR; ny <= NR; ny++)
            for (int nz = -NR; nz <= NR; nz++) {
                if (!nx && !ny && !nz) continue;
                double rv[3] = {x[0] + nx * L, x[1] + ny * L, x[2] + nz * L};
                double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                orc_gn(1, r, alpha, g);
                add_radial(g, rv, -1.0, D0, D1, D2, D3);
            }
    /* Fourier space: d/dx_i cos(k.x) = -k_i sin(k.x), and so on */
    for (int nx = -NK; nx <= NK; nx++)
        for (int ny = -NK; ny <= NK; ny++)
            for (int nz = -NK; nz <= NK; nz++) {
                if (!nx && !ny && !nz) continue;
                double k[3] = {2.0 * M_PI * nx / L, 2.0 * M_PI * ny / L, 2.0 * M_PI * nz / L};
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                double w = 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                double th = k[0] * x[0] + k[1] * x[1] + k[2] * x[2], c = cos(th), sn = sin(th);
                *D0 -= w * c;
                for (int i = 0; i < 3; i++) {
                    D1[i] += w * sn * k[i];
                    for (int j = 0; j < 3; j++) {
                        D2[i * 3 + j] += w * c * k[i] * k[j];
                        for (int l = 0; l < 3; l++) D3[(i * 3 + j) * 3 + l] -= w * sn * k[i] * k[j] * k[l];
                    }
                }
            }
}

/* ======================================================================
 * 3. Integer coordinates
 * ====================================================================== */

/* Periodic: X = floor(x/L * 2^32) mod 2^32 (two's-complement wrap).
 * Isolated: the root cube [origin, origin+D) maps onto [2^30, 3*2^30) so
 * that differences of two coordinates never wrap.  Returns 0, or -5 if an
 * isolated particle lies outside the root cube. */
int orc_quantize(int64_t n, const double *pos, int periodic, double box, const double origin[3],
                 uint32_t *X, uint32_t *Y, uint32_t *Z)
{
    uint32_t *out[3] = {X, Y, Z};
    double inv = periodic ? TWO32 / box : TWO31 / box;
    int status = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int k = 0; k < 3; k++) {
            double t = (pos[3 * i + k] - origin[k]) * inv;
            double f = floor(t);
            if (periodic) {
                /* reduce into [0, 2^32) first so the conversion is exact */
                double w = f - TWO32 * floor(f / TWO32);
                out[k][i] = (uint32_t)(uint64_t)w;
            } else {
                if (f < 0.0 || f >= TWO31) {
                    status = -5;
                    f = f < 0.0 ? 0.0 : TWO31 - 1.0;
                }
                out[k][i] = (uint32_t)(TWO30 + f);
            }
        }
    }
    return status;
}

/* ======================================================================
 * 4. Octree by recursive index partition
 * ====================================================================== */

typedef struct {
    int level;
    uint32_t cell[3];      /* cell coordinates at this level */
    uint32_t gc[3];        /* integer geometric centre */
    int64_t first, count;  /* range into tree->idx */
    int64_t child0;        /* first child (children contiguous), -1 for a leaf */
    int nchild;
    int leaf;
    double mass;
    double dcom[3];        /* centre of mass minus geometric centre (physical) */
    double q2[9], q3[27];  /* full symmetric tensors about the centre of mass */
} onode;

struct orc_tree {
    int64_t n;
    int periodic, S, leaf_max, max_depth;
    double box, unit;      /* unit = physical length of one integer step */
    uint32_t corner;       /* integer lower corner of the root */
    uint32_t *X, *Y, *Z;
    double *m;
    int64_t *idx;          /* particle indices grouped by node */
    onode *nodes;
    int64_t nnodes, cap;
    int has_moments;
    double *q4;            /* 81 per node: fourth moments about the centre of mass (orc_moments4) */
};

/* Node storage: the tree's own array, or a private buffer of one thread. */
typedef struct {
    onode *nodes;
    int64_t nnodes, cap;
} node_store;

static int64_t new_nodes(node_store *st, int k)
{
    if (st->nnodes + k > st->cap) {
        st->cap = 2 * (st->nnodes + k) + 64;
        st->nodes = (onode *)realloc(st->nodes, (size_t)st->cap * sizeof(onode));
    }
    int64_t first = st->nnodes;
    memset(st->nodes + first, 0, (size_t)k * sizeof(onode));
    st->nnodes += k;
    return first;
}

static uint32_t rel_coord(const orc_tree *t, uint32_t X) { return X - t->corner; }

/* Split node `ni` of store `st` into its occupied octants if it holds more
 * than B particles and lies above the depth cap (the particle indices of the
 * node are regrouped by octant, stably).  Returns the number of children. */
static int split_one(const orc_tree *t, node_store *st, int64_t ni)
{
    onode nd = st->nodes[ni];
    if (nd.count <= t->leaf_max || nd.level >= t->max_depth) {
        st->nodes[ni].leaf = 1;
        st->nodes[ni].child0 = -1;
        return 0;
    }
    int bit = t->S - nd.level - 1;  /* bit selecting the child half */
    int64_t cnt[8] = {0};
    int64_t *tmp = (int64_t *)malloc((size_t)nd.count * sizeof(int64_t));
    int *oct = (int *)malloc((size_t)nd.count * sizeof(int));
    for (int64_t q = 0; q < nd.count; q++) {
        int64_t p = t->idx[nd.first + q];
        int bx = (rel_coord(t, t->X[p]) >> bit) & 1;
        int by = (rel_coord(t, t->Y[p]) >> bit) & 1;
        int bz = (rel_coord(t, t->Z[p]) >> bit) & 1;
        oct[q] = (bx << 2) | (by << 1) | bz;
        cnt[oct[q]]++;
    }
    int64_t off[8], o = 0;
    for (int c = 0; c < 8; c++) { off[c] = o; o += cnt[c]; }
    int64_t pos[8];
    memcpy(pos, off, sizeof(pos));
    for (int64_t q = 0; q < nd.count; q++) tmp[pos[oct[q]]++] = t->idx[nd.first + q];  /* stable */
    memcpy(t->idx + nd.first, tmp, (size_t)nd.count * sizeof(int64_t));
    free(tmp);
    free(oct);

    int nch = 0;
    for (int c = 0; c < 8; c++) nch += cnt[c] > 0;
    int64_t c0 = new_nodes(st, nch);
    onode *parent = &st->nodes[ni];
    parent->child0 = c0;
    parent->nchild = nch;
    parent->leaf = 0;
    int k = 0;
    for (int c = 0; c < 8; c++) {
        if (!cnt[c]) continue;
        onode *ch = &st->nodes[c0 + k++];
        ch->level = nd.level + 1;
        ch->cell[0] = 2 * nd.cell[0] + ((c >> 2) & 1);
        ch->cell[1] = 2 * nd.cell[1] + ((c >> 1) & 1);
        ch->cell[2] = 2 * nd.cell[2] + (c & 1);
        ch->first = nd.first + off[c];
        ch->count = cnt[c];
    }
    return nch;
}

/* Split recursively, depth first. */
static void split_node(const orc_tree *t, node_store *st, int64_t ni)
{
    int nch = split_one(t, st, ni);
    int64_t c0 = st->nodes[ni].child0;
    for (int q = 0; q < nch; q++) split_node(t, st, c0 + q);
}

/* Parallel build: the top levels are split in order on one thread; each
 * node left unsplit there roots a subtree that one thread builds into its
 * own store (the subtrees own disjoint ranges of t->idx); the subtrees are
 * then appended to the tree's array with their child indices shifted.  The
 * node set and every node's particles are those of the serial build; only
 * the numbering of the nodes differs. */
typedef struct {
    const orc_tree *t;
    int64_t *roots;        /* main-store indices of the subtree roots */
    node_store *stores;    /* one per root */
    int64_t nroots;
    int64_t next;          /* shared work counter */
} sub_job;

static void *subtree_thread(void *arg)
{
    sub_job *J = (sub_job *)arg;
    for (;;) {
        int64_t k = __sync_fetch_and_add(&J->next, 1);
        if (k >= J->nroots) break;
        split_node(J->t, &J->stores[k], 0);
    }
    return NULL;
}

static void build_parallel(orc_tree *t, node_store *main, int nthreads)
{
    /* breadth-first split of the top until there are enough subtrees */
    int64_t lo = 0, hi = main->nnodes;
    while (hi - lo < 8 * (int64_t)nthreads && hi > lo) {
        for (int64_t q = lo; q < hi; q++) split_one(t, main, q);
        lo = hi;
        hi = main->nnodes;
    }
    int64_t nr = hi - lo;
    sub_job J;
    J.t = t;
    J.nroots = nr;
    J.next = 0;
    J.roots = (int64_t *)malloc((size_t)(nr > 0 ? nr : 1) * sizeof(int64_t));
    J.stores = (node_store *)calloc((size_t)(nr > 0 ? nr : 1), sizeof(node_store));
    for (int64_t k = 0; k < nr; k++) {
        J.roots[k] = lo + k;
        new_nodes(&J.stores[k], 1);
        J.stores[k].nodes[0] = main->nodes[lo + k];
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    for (int k = 0; k < nthreads; k++) pthread_create(&th[k], NULL, subtree_thread, &J);
    for (int k = 0; k < nthreads; k++) pthread_join(th[k], NULL);
    free(th);
    for (int64_t k = 0; k < nr; k++) {
        node_store *sb = &J.stores[k];
        int64_t base = main->nnodes - 1;  /* local index i >= 1 goes to base + i */
        if (main->nnodes + sb->nnodes - 1 > main->cap) {
            main->cap = main->nnodes + sb->nnodes + 64;
            main->nodes = (onode *)realloc(main->nodes, (size_t)main->cap * sizeof(onode));
        }
        for (int64_t i = 0; i < sb->nnodes; i++) {
            onode nd = sb->nodes[i];
            if (!nd.leaf) nd.child0 += base;
            if (i == 0) main->nodes[J.roots[k]] = nd;
            else main->nodes[base + i] = nd;
        }
        main->nnodes += sb->nnodes - 1;
        free(sb->nodes);
    }
    free(J.roots);
    free(J.stores);
}

orc_tree *orc_build(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                    int periodic, double box, int leaf_max, int max_depth)
{
    return orc_build_mt(n, X, Y, Z, mass, periodic, box, leaf_max, max_depth, 1);
}

orc_tree *orc_build_mt(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                       int periodic, double box, int leaf_max, int max_depth, int nthreads)
{
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->n = n;
    t->periodic = periodic;
    t->S = periodic ? 32 : 31;
    t->corner = periodic ? 0u : (uint32_t)TWO30;
    t->box = box;
    t->unit = box / (periodic ? TWO32 : TWO31);
    t->leaf_max = leaf_max;
    t->max_depth = max_depth > 21 ? 21 : max_depth;
    t->X = (uint32_t *)malloc((size_t)n * 4);
    t->Y = (uint32_t *)malloc((size_t)n * 4);
    t->Z = (uint32_t *)malloc((size_t)n * 4);
    t->m = (double *)malloc((size_t)n * 8);
    t->idx = (int64_t *)malloc((size_t)n * 8);
    memcpy(t->X, X, (size_t)n * 4);
    memcpy(t->Y, Y, (size_t)n * 4);
    memcpy(t->Z, Z, (size_t)n * 4);
    memcpy(t->m, mass, (size_t)n * 8);
    for (int64_t i = 0; i < n; i++) t->idx[i] = i;
    node_store st = {NULL, 0, 0};
    int64_t r = new_nodes(&st, 1);
    st.nodes[r].first = 0;
    st.nodes[r].count = n;
    if (nthreads > 1) build_parallel(t, &st, nthreads);
    else split_node(t, &st, r);
    t->nodes = st.nodes;
    t->nnodes = st.nnodes;
    t->cap = st.cap;
    /* geometric centres */
    for (int64_t q = 0; q < t->nnodes; q++) {
        onode *nd = &t->nodes[q];
        int sh = t->S - nd->level;
        for (int k = 0; k < 3; k++) {
            uint64_t c = (uint64_t)t->corner + ((uint64_t)nd->cell[k] << sh) + (1ull << (sh - 1));
            nd->gc[k] = (uint32_t)c;
        }
    }
    return t;
}

void orc_free(orc_tree *t)
{
    if (!t) return;
    free(t->X); free(t->Y); free(t->Z); free(t->m); free(t->idx); free(t->nodes); free(t->q4);
    free(t);
}

int64_t orc_tree_nnodes(const orc_tree *t) { return t->nnodes; }

/* Export node geometry: level, cell coords, particle count, leaf flag. */
void orc_tree_nodes(const orc_tree *t, int32_t *level, uint32_t *cell3, int64_t *count, int32_t *leaf)
{
    for (int64_t q = 0; q < t->nnodes; q++) {
        const onode *nd = &t->nodes[q];
        level[q] = nd->level;
        for (int k = 0; k < 3; k++) cell3[3 * q + k] = nd->cell[k];
        count[q] = nd->count;
        leaf[q] = nd->leaf;
    }
}

/* Physical length of a node side at a given level. */
static double node_side(const orc_tree *t, int level) { return ldexp(t->box, -level); }

/* Integer half side of a node (0 for a particle entity, level < 0). */
static uint64_t half_side_int(const orc_tree *t, int level)
{
    return level < 0 ? 0 : (1ull << (t->S - level - 1));
}

/* ======================================================================
 * 5. Multipole moments by direct sums over each node's particles
 * ====================================================================== */

static void node_moments(orc_tree *t, int64_t q)
{
    {
        onode *nd = &t->nodes[q];
        double M = 0.0, c[3] = {0, 0, 0};
        for (int64_t a = 0; a < nd->count; a++) {
            int64_t p = t->idx[nd->first + a];
            double d[3] = {(double)(int32_t)(t->X[p] - nd->gc[0]) * t->unit,
                           (double)(int32_t)(t->Y[p] - nd->gc[1]) * t->unit,
                           (double)(int32_t)(t->Z[p] - nd->gc[2]) * t->unit};
            M += t->m[p];
            for (int k = 0; k < 3; k++) c[k] += t->m[p] * d[k];
        }
        nd->mass = M;
        for (int k = 0; k < 3; k++) nd->dcom[k] = M > 0 ? c[k] / M : 0.0;
        memset(nd->q2, 0, sizeof(nd->q2));
        memset(nd->q3, 0, sizeof(nd->q3));
        for (int64_t a = 0; a < nd->count; a++) {
            int64_t p = t->idx[nd->first + a];
            double d[3] = {(double)(int32_t)(t->X[p] - nd->gc[0]) * t->unit - nd->dcom[0],
                           (double)(int32_t)(t->Y[p] - nd->gc[1]) * t->unit - nd->dcom[1],
                           (double)(int32_t)(t->Z[p] - nd->gc[2]) * t->unit - nd->dcom[2]};
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    nd->q2[i * 3 + j] += t->m[p] * d[i] * d[j];
                    for (int k = 0; k < 3; k++) nd->q3[(i * 3 + j) * 3 + k] += t->m[p] * d[i] * d[j] * d[k];
                }
        }
    }
}

/* fourth moments Q4_ijkl = sum m d_i d_j d_k d_l about each node's centre of
 * mass (direct sums; needed from p = 4 on) */
void orc_moments4(orc_tree *t)
{
    free(t->q4);
    t->q4 = (double *)calloc((size_t)t->nnodes * 81, sizeof(double));
    for (int64_t q = 0; q < t->nnodes; q++) {
        const onode *nd = &t->nodes[q];
        double *Q = t->q4 + (size_t)q * 81;
        for (int64_t a = 0; a < nd->count; a++) {
            int64_t p = t->idx[nd->first + a];
            double d[3] = {(double)(int32_t)(t->X[p] - nd->gc[0]) * t->unit - nd->dcom[0],
                           (double)(int32_t)(t->Y[p] - nd->gc[1]) * t->unit - nd->dcom[1],
                           (double)(int32_t)(t->Z[p] - nd->gc[2]) * t->unit - nd->dcom[2]};
            for (int c = 0; c < 81; c++) Q[c] += t->m[p] * d[c / 27] * d[(c / 9) % 3] * d[(c / 3) % 3] * d[c % 3];
        }
    }
}

void orc_moments(orc_tree *t)
{
    for (int64_t q = 0; q < t->nnodes; q++) node_moments(t, q);
    t->has_moments = 1;
}

/* The same direct sums with the nodes shared out to threads (each node's
 * sums are independent of every other node's). */
typedef struct { orc_tree *t; int64_t next; } mom_job;

static void *moments_thread(void *arg)
{
    mom_job *J = (mom_job *)arg;
    for (;;) {
        int64_t q = __sync_fetch_and_add(&J->next, 1);
        if (q >= J->t->nnodes) break;
        node_moments(J->t, q);
    }
    return NULL;
}

void orc_moments_mt(orc_tree *t, int nthreads)
{
    if (nthreads <= 1) {
        orc_moments(t);
        return;
    }
    mom_job J = {t, 0};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    for (int k = 0; k < nthreads; k++) pthread_create(&th[k], NULL, moments_thread, &J);
    for (int k = 0; k < nthreads; k++) pthread_join(th[k], NULL);
    free(th);
    t->has_moments = 1;
}

/* Export moments: mass, COM (physical, relative to the root's lower corner),
 * Q2 packed (xx,xy,xz,yy,yz,zz), Q3 packed (xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz). */
void orc_tree_moments(const orc_tree *t, double *mass, double *com3, double *q2p, double *q3p)
{
    static const int i2[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    static const int i3[10][3] = {{0, 0, 0}, {0, 0, 1}, {0, 0, 2}, {0, 1, 1}, {0, 1, 2},
                                  {0, 2, 2}, {1, 1, 1}, {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
    for (int64_t q = 0; q < t->nnodes; q++) {
        const onode *nd = &t->nodes[q];
        mass[q] = nd->mass;
        for (int k = 0; k < 3; k++)
            com3[3 * q + k] = (double)(nd->gc[k] - t->corner) * t->unit + nd->dcom[k];
        for (int a = 0; a < 6; a++) q2p[6 * q + a] = nd->q2[i2[a][0] * 3 + i2[a][1]];
        for (int a = 0; a < 10; a++) q3p[10 * q + a] = nd->q3[(i3[a][0] * 3 + i3[a][1]) * 3 + i3[a][2]];
    }
}

/* ======================================================================
 * 6. One-sided tree walk, per particle
 * ====================================================================== */

typedef struct {
    const orc_tree *t;
    orc_walk_params P;
    const double *aseed;   /* |a| per particle (caller order) for the relative criterion */
    const int64_t *targets;
    int64_t ntargets;
    double *acc, *pot;     /* ntargets x 3, ntargets */
    int64_t *counts;       /* ntargets x 2: particle-particle, particle-node */
} walk_job;

/* P2P contribution of source j on target i: r = x_j - x_i (nearest image). */
static void p2p_one(const orc_tree *t, const orc_walk_params *P, int64_t i, int64_t j, double a[3], double *phi)
{
    double d[3] = {(double)(int32_t)(t->X[j] - t->X[i]) * t->unit,
                   (double)(int32_t)(t->Y[j] - t->Y[i]) * t->unit,
                   (double)(int32_t)(t->Z[j] - t->Z[i]) * t->unit};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double h = 2.8 * P->eps0;
    double K, W;
    if (P->kernel != 1) {
        K = orc_soft_K(r, h);
        W = (r > 0.0 || h > 0.0) ? orc_soft_W(r, h) : 0.0;
    } else {
        double alpha = 0.5 / P->r_s;
        K = orc_sr_K(r, h, alpha);
        W = orc_sr_W(r, h, alpha);
    }
    for (int k = 0; k < 3; k++) a[k] += t->m[j] * d[k] * K;
    *phi -= t->m[j] * W;
    if (P->kernel == 2) {
        /* the other images: + m grad psi(d), potential + m psi(d) (eq. eqnpo1) */
        double D0, D1[3], D2[9], D3[27];
        orc_ewald_psi(d, t->box, 0.0, &D0, D1, D2, D3);
        for (int k = 0; k < 3; k++) a[k] += t->m[j] * D1[k];
        *phi += t->m[j] * D0;
    }
}

/* Accepted node: eqs. (eqonesidetreeacc) and (eqonesidetreepotential) with
 * p = 3 and vanishing dipole: a = -[M D1 + Q2:D3 / 2],
 * phi = -[M D0 + Q2:D2 / 2 + Q3.D3 / 6], D evaluated at r = s - x. */
/* Accepted node at p = 4 or 5 (Appendix A): the force
 * a = -[M D1 + Q2:D3/2 + Q3:D4/6 (+ Q4:D5/24 at p = 5)] and the potential
 * phi = -[M D0 + Q2:D2/2 + Q3:D3/6 + Q4:D4/24] (the p = 5 term Q5:D5/120 is
 * left out, as the paper does in practice: it is constant over the target's
 * neighbourhood and adds no force), full tensors at r = s - x. */
static void p2m_high(const orc_walk_params *P, const onode *nd, const double *q4, const double rv[3], double a[3],
                     double *phi)
{
    double g[8], r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    orc_gn_ext(P->kernel == 1, r, P->kernel == 1 ? 0.5 / P->r_s : 0.0, 6, g);
    static __thread double D[6][243];
    for (int n = 0; n <= 5; n++) orc_Dfull(g, rv, n, D[n]);
    for (int i = 0; i < 3; i++) {
        double s = nd->mass * D[1][i];
        for (int c = 0; c < 9; c++) s += 0.5 * nd->q2[c] * D[3][i * 9 + c];
        for (int c = 0; c < 27; c++) s += nd->q3[c] * D[4][i * 27 + c] / 6.0;
        if (P->order >= 5)
            for (int c = 0; c < 81; c++) s += q4[c] * D[5][i * 81 + c] / 24.0;
        a[i] -= s;
    }
    double ph = nd->mass * D[0][0];
    for (int c = 0; c < 9; c++) ph += 0.5 * nd->q2[c] * D[2][c];
    for (int c = 0; c < 27; c++) ph += nd->q3[c] * D[3][c] / 6.0;
    for (int c = 0; c < 81; c++) ph += q4[c] * D[4][c] / 24.0;
    *phi -= ph;
}

static void p2m_one(const orc_walk_params *P, const onode *nd, const double rv[3], double box, double a[3],
                    double *phi)
{
    double D0, D1[3], D2[9], D3[27];
    orc_Dn(P->kernel == 1, rv, 0.5 / (P->kernel == 1 ? P->r_s : 1.0), &D0, D1, D2, D3);
    if (P->kernel == 2) {
        /* periodic: g = 1/r - psi, so D_n(g) = D_n(1/r) - D_n(psi) (eqs. eqnpo1, eqnpo2) */
        double E0, E1[3], E2[9], E3[27];
        orc_ewald_psi(rv, box, 0.0, &E0, E1, E2, E3);
        D0 -= E0;
        for (int i = 0; i < 3; i++) D1[i] -= E1[i];
        for (int i = 0; i < 9; i++) D2[i] -= E2[i];
        for (int i = 0; i < 27; i++) D3[i] -= E3[i];
    }
    for (int i = 0; i < 3; i++) {
        double s = nd->mass * D1[i];
        if (P->order >= 3)
            for (int j = 0; j < 3; j++)
                for (int k = 0; k < 3; k++) s += 0.5 * nd->q2[j * 3 + k] * D3[(i * 3 + j) * 3 + k];
        a[i] -= s;
    }
    /* potential to order p: the octupole term only at p = 3 */
    double ph = nd->mass * D0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            ph += 0.5 * nd->q2[i * 3 + j] * D2[i * 3 + j];
            if (P->order >= 3)
                for (int k = 0; k < 3; k++) ph += nd->q3[(i * 3 + j) * 3 + k] * D3[(i * 3 + j) * 3 + k] / 6.0;
        }
    *phi -= ph;
}

static void walk_node(const walk_job *J, int64_t i, double aseed, int64_t q, double a[3], double *phi, int64_t cnt[2])
{
    const orc_tree *t = J->t;
    const orc_walk_params *P = &J->P;
    const onode *nd = &t->nodes[q];
    double l = node_side(t, nd->level);
    int32_t dc[3] = {(int32_t)(nd->gc[0] - t->X[i]), (int32_t)(nd->gc[1] - t->Y[i]), (int32_t)(nd->gc[2] - t->Z[i])};

    /* TreePM: drop the node when its nearest edge lies beyond r_cut */
    if (P->kernel == 1) {
        double e2 = 0.0;
        for (int k = 0; k < 3; k++) {
            double e = fabs((double)dc[k]) * t->unit - 0.5 * l;
            if (e > 0.0) e2 += e * e;
        }
        if (e2 > P->r_cut * P->r_cut) return;
    }
    /* the node's centre of mass, the point its expansion is about, taken at
     * its nearest periodic image (Sec. "Periodic boundary conditions"); it can
     * lie on the other side of the half-box plane than the geometric centre */
    double rv[3], r2 = 0.0;
    for (int k = 0; k < 3; k++) {
        rv[k] = (double)dc[k] * t->unit + nd->dcom[k];
        if (t->periodic) {
            if (rv[k] >= 0.5 * t->box) rv[k] -= t->box;
            else if (rv[k] < -0.5 * t->box) rv[k] += t->box;
        }
        r2 += rv[k] * rv[k];
    }
    /* exclusion zone: cube of side 2l centred on the node's geometric centre */
    int inside = 1;
    if (P->exclusion) {
        uint64_t lint = 2 * half_side_int(t, nd->level);
        inside = 0;
        if ((uint64_t)llabs((long long)dc[0]) < lint && (uint64_t)llabs((long long)dc[1]) < lint &&
            (uint64_t)llabs((long long)dc[2]) < lint)
            inside = 1;
        if (nd->level == 0) inside = 1;
    } else {
        inside = (nd->level == 0);  /* the root always holds the target */
    }
    double h = 2.8 * P->eps0;
    int accept = 0;
    if (!inside && r2 >= h * h) {
        double r = sqrt(r2);
        if (P->criterion == 0)
            accept = l < P->theta * r;
        else
            /* M l^p < alpha |a| r^(p+2) (eq. eqnrelcriterion) */
            accept = nd->mass * pow(l, P->order) < P->alpha * aseed * pow(r, P->order + 2);
    }
    if (accept) {
        if (P->order >= 4) p2m_high(P, nd, t->q4 + (size_t)q * 81, rv, a, phi);
        else p2m_one(P, nd, rv, t->box, a, phi);
        cnt[1]++;
        return;
    }
    if (nd->leaf) {
        for (int64_t s = 0; s < nd->count; s++) {
            int64_t j = t->idx[nd->first + s];
            if (j == i) continue;
            p2p_one(t, P, i, j, a, phi);
            cnt[0]++;
        }
        return;
    }
    for (int c = 0; c < nd->nchild; c++) walk_node(J, i, aseed, nd->child0 + c, a, phi, cnt);
}

typedef struct { walk_job *J; int64_t lo, hi; } walk_chunk;

static void *walk_thread(void *arg)
{
    walk_chunk *C = (walk_chunk *)arg;
    walk_job *J = C->J;
    for (int64_t q = C->lo; q < C->hi; q++) {
        int64_t i = J->targets ? J->targets[q] : q;
        double a[3] = {0, 0, 0}, phi = 0.0;
        int64_t cnt[2] = {0, 0};
        double as = J->aseed ? J->aseed[i] : 0.0;
        walk_node(J, i, as, 0, a, &phi, cnt);
        for (int k = 0; k < 3; k++) J->acc[3 * q + k] = J->P.G * a[k];
        if (J->pot) J->pot[q] = J->P.G * phi;
        if (J->counts) { J->counts[2 * q] = cnt[0]; J->counts[2 * q + 1] = cnt[1]; }
    }
    return NULL;
}

static void run_chunks(void *(*fn)(void *), void *job, size_t chunk_size, int64_t ntot, int nthreads,
                       void (*init)(void *chunk, void *job, int64_t lo, int64_t hi))
{
    if (nthreads < 1) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    char *chunks = (char *)malloc(chunk_size * nthreads);
    for (int k = 0; k < nthreads; k++) {
        int64_t lo = ntot * k / nthreads, hi = ntot * (k + 1) / nthreads;
        init(chunks + k * chunk_size, job, lo, hi);
        if (nthreads > 1) pthread_create(&th[k], NULL, fn, chunks + k * chunk_size);
        else fn(chunks);
    }
    if (nthreads > 1)
        for (int k = 0; k < nthreads; k++) pthread_join(th[k], NULL);
    free(th);
    free(chunks);
}

static void walk_chunk_init(void *c, void *job, int64_t lo, int64_t hi)
{
    walk_chunk *C = (walk_chunk *)c;
    C->J = (walk_job *)job; C->lo = lo; C->hi = hi;
}

int orc_walk(const orc_tree *t, const orc_walk_params *P, const double *aseed, const int64_t *targets,
             int64_t ntargets, double *acc, double *pot, int64_t *counts, int nthreads)
{
    if (P->order >= 4 && (!t->q4 || P->kernel == 2)) return -4;  /* fourth moments needed; no Ewald beyond p = 3 */
    if (!t->has_moments) return -4;
    if (P->criterion == 1 && !aseed) return -1;
    walk_job J = {t, *P, aseed, targets, targets ? ntargets : t->n, acc, pot, counts};
    run_chunks(walk_thread, &J, sizeof(walk_chunk), J.ntargets, nthreads, walk_chunk_init);
    return 0;
}

/* ======================================================================
 * 7. Direct summation (the exact reference)
 * ====================================================================== */

typedef struct {
    int64_t n; const uint32_t *X, *Y, *Z; const double *m; double unit;
    orc_walk_params P; int truncate;
    const int64_t *targets; int64_t ntargets; double *acc, *pot;
} direct_job;
typedef struct { direct_job *J; int64_t lo, hi; } direct_chunk;

static void *direct_thread(void *arg)
{
    direct_chunk *C = (direct_chunk *)arg;
    direct_job *J = C->J;
    const orc_walk_params *P = &J->P;
    double h = 2.8 * P->eps0, alpha = P->kernel == 1 ? 0.5 / P->r_s : 0.0;
    /* beyond x = alpha r = 6 erfc(x) < 3e-17: such sources add nothing in FP64 */
    double rskip2 = P->kernel == 1 ? (6.0 / alpha) * (6.0 / alpha) : INFINITY;
    double rc2 = P->r_cut * P->r_cut;
    for (int64_t q = C->lo; q < C->hi; q++) {
        int64_t i = J->targets ? J->targets[q] : q;
        double a[3] = {0, 0, 0}, phi = 0.0;
        for (int64_t j = 0; j < J->n; j++) {
            if (j == i) continue;
            double d[3] = {(double)(int32_t)(J->X[j] - J->X[i]) * J->unit,
                           (double)(int32_t)(J->Y[j] - J->Y[i]) * J->unit,
                           (double)(int32_t)(J->Z[j] - J->Z[i]) * J->unit};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 > rskip2) continue;
            if (J->truncate && r2 > rc2) continue;
            double r = sqrt(r2), K, W;
            if (P->kernel != 1) { K = orc_soft_K(r, h); W = orc_soft_W(r, h); }
            else { K = orc_sr_K(r, h, alpha); W = orc_sr_W(r, h, alpha); }
            for (int k = 0; k < 3; k++) a[k] += J->m[j] * d[k] * K;
            phi -= J->m[j] * W;
            if (P->kernel == 2) {
                double D0, D1[3], D2[9], D3[27];
                orc_ewald_psi(d, J->unit * TWO32, 0.0, &D0, D1, D2, D3);
                for (int k = 0; k < 3; k++) a[k] += J->m[j] * D1[k];
                phi += J->m[j] * D0;
            }
        }
        for (int k = 0; k < 3; k++) J->acc[3 * q + k] = P->G * a[k];
        if (J->pot) J->pot[q] = P->G * phi;
    }
    return NULL;
}

static void direct_chunk_init(void *c, void *job, int64_t lo, int64_t hi)
{
    direct_chunk *C = (direct_chunk *)c;
    C->J = (direct_job *)job; C->lo = lo; C->hi = hi;
}

/* a_i = G sum_{j != i} m_j (x_j - x_i) K(|x_j - x_i|), nearest image for a
 * periodic box.  kernel 0: softened Newtonian (isolated); kernel 1:
 * short-range q=0 sum of eq. (eqnpo4), optionally truncated at r_cut. */
void orc_direct(int64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z, const double *mass,
                double unit, const orc_walk_params *P, int truncate, const int64_t *targets, int64_t ntargets,
                double *acc, double *pot, int nthreads)
{
    direct_job J = {n, X, Y, Z, mass, unit, *P, truncate, targets, targets ? ntargets : n, acc, pot};
    run_chunks(direct_thread, &J, sizeof(direct_chunk), J.ntargets, nthreads, direct_chunk_init);
}

/* ======================================================================
 * 8. Fast multipole method, p = 3, symmetric expansion
 * ====================================================================== */

typedef struct {
    double F0, F1[3], F2[9], F3[27];
} field;

typedef struct {
    const orc_tree *t;
    orc_fmm_params P;
    field *F;              /* per node */
    double *acc, *pot;     /* per particle (caller order), unscaled by G */
    const double *aseed;   /* |a| per particle (caller order), relative criterion */
    double *amin;          /* smallest |a| among each node's particles */
    int64_t n_pp, n_pn, n_nn;
} fmm_ctx;

/* |a|_min of every node: the smallest seed among its particles */
static double node_amin(fmm_ctx *C, int64_t q)
{
    const onode *nd = &C->t->nodes[q];
    double m = INFINITY;
    if (nd->leaf) {
        for (int64_t s = 0; s < nd->count; s++) m = fmin(m, C->aseed[C->t->idx[nd->first + s]]);
    } else {
        for (int c = 0; c < nd->nchild; c++) m = fmin(m, node_amin(C, nd->child0 + c));
    }
    C->amin[q] = m;
    return m;
}

/* Entity: node q >= 0, particle j encoded as -(j+1). */
typedef struct {
    int level;             /* -1 for a particle */
    uint32_t gc[3];        /* integer centre (position for a particle) */
    double dcom[3];        /* COM minus centre */
    double mass, q2[9], q3[27];
    double amin;           /* smallest |a| of its particles (relative criterion) */
} entity;

static void get_entity(const fmm_ctx *C, int64_t e, entity *E)
{
    const orc_tree *t = C->t;
    if (e >= 0) {
        const onode *nd = &t->nodes[e];
        E->level = nd->level;
        memcpy(E->gc, nd->gc, sizeof(E->gc));
        memcpy(E->dcom, nd->dcom, sizeof(E->dcom));
        E->mass = nd->mass;
        memcpy(E->q2, nd->q2, sizeof(E->q2));
        memcpy(E->q3, nd->q3, sizeof(E->q3));
        E->amin = C->amin ? C->amin[e] : 0.0;
    } else {
        int64_t j = -e - 1;
        E->level = -1;
        E->gc[0] = t->X[j]; E->gc[1] = t->Y[j]; E->gc[2] = t->Z[j];
        memset(E->dcom, 0, sizeof(E->dcom));
        E->mass = t->m[j];
        memset(E->q2, 0, sizeof(E->q2));
        memset(E->q3, 0, sizeof(E->q3));
        E->amin = C->aseed ? C->aseed[j] : 0.0;
    }
}

/* Field expansion at sink A due to source moments (mass, Q2, Q3) seen at
 * r = s_source - s_sink:  F_k = sum_{n=0}^{p-k} D_{n+k} . Q_n / n!
 * (p = 3, Q1 = 0).  sgn = -1 evaluates the mirrored expansion
 * F_k = sum_n (-1)^(n+k) D_{n+k} . Q_n / n! used for the B side. */
static void add_field(field *F, const double D[4][27], const entity *src, double sgn)
{
    /* D[0][0]=D0, D[1][0..2]=D1, D[2][0..8]=D2, D[3][0..26]=D3 */
    double s1 = sgn, s2 = 1.0, s3 = sgn;  /* (-1)^k for k=1,2,3 when mirrored */
    double q2d2 = 0.0, q3d3 = 0.0;
    for (int a = 0; a < 9; a++) q2d2 += src->q2[a] * D[2][a];
    for (int a = 0; a < 27; a++) q3d3 += src->q3[a] * D[3][a];
    /* F0: n=0,2,3  -> (-1)^n for the mirrored expansion: +, +, sgn */
    F->F0 += src->mass * D[0][0] + 0.5 * q2d2 + sgn * q3d3 / 6.0;
    for (int i = 0; i < 3; i++) {
        double q2d3 = 0.0;
        for (int j = 0; j < 3; j++)
            for (int k = 0; k < 3; k++) q2d3 += src->q2[j * 3 + k] * D[3][(i * 3 + j) * 3 + k];
        F->F1[i] += s1 * (src->mass * D[1][i] + 0.5 * q2d3);
    }
    for (int a = 0; a < 9; a++) F->F2[a] += s2 * src->mass * D[2][a];
    for (int a = 0; a < 27; a++) F->F3[a] += s3 * src->mass * D[3][a];
}

static void fmm_p2p(fmm_ctx *C, int64_t i, int64_t j)
{
    const orc_tree *t = C->t;
    orc_walk_params W = {0};
    W.kernel = C->P.kernel; W.eps0 = C->P.eps0; W.r_s = C->P.r_s;
    double ai[3] = {0, 0, 0}, aj[3] = {0, 0, 0}, pi = 0.0, pj = 0.0;
    p2p_one(t, &W, i, j, ai, &pi);
    p2p_one(t, &W, j, i, aj, &pj);
    for (int k = 0; k < 3; k++) { C->acc[3 * i + k] += ai[k]; C->acc[3 * j + k] += aj[k]; }
    C->pot[i] += pi;
    C->pot[j] += pj;
    C->n_pp++;
}

static void entity_children(const fmm_ctx *C, int64_t e, int64_t **list, int64_t *nl)
{
    const orc_tree *t = C->t;
    if (e < 0) { *nl = 1; *list = (int64_t *)malloc(8); (*list)[0] = e; return; }
    const onode *nd = &t->nodes[e];
    if (nd->leaf) {
        *nl = nd->count;
        *list = (int64_t *)malloc((size_t)nd->count * 8);
        for (int64_t s = 0; s < nd->count; s++) (*list)[s] = -(t->idx[nd->first + s] + 1);
    } else {
        *nl = nd->nchild;
        *list = (int64_t *)malloc((size_t)nd->nchild * 8);
        for (int c = 0; c < nd->nchild; c++) (*list)[c] = nd->child0 + c;
    }
}

static void fmm_interact(fmm_ctx *C, int64_t A, int64_t B)
{
    const orc_tree *t = C->t;
    const orc_fmm_params *P = &C->P;
    if (A == B) {
        if (A < 0) return;
        const onode *nd = &t->nodes[A];
        if (nd->leaf) {
            for (int64_t a = 0; a < nd->count; a++)
                for (int64_t b = a + 1; b < nd->count; b++) fmm_p2p(C, t->idx[nd->first + a], t->idx[nd->first + b]);
        } else {
            for (int c1 = 0; c1 < nd->nchild; c1++)
                for (int c2 = c1; c2 < nd->nchild; c2++) fmm_interact(C, nd->child0 + c1, nd->child0 + c2);
        }
        return;
    }
    if (A < 0 && B < 0) { fmm_p2p(C, -A - 1, -B - 1); return; }

    entity EA, EB;
    get_entity(C, A, &EA);
    get_entity(C, B, &EB);
    int64_t dc[3];
    for (int k = 0; k < 3; k++) dc[k] = (int32_t)(EB.gc[k] - EA.gc[k]);
    uint64_t hsum = half_side_int(t, EA.level) + half_side_int(t, EB.level);
    /* TreePM / FMM-PM: drop pairs whose nearest sides are farther apart than r_cut */
    if (P->kernel == 1) {
        double g2 = 0.0;
        for (int k = 0; k < 3; k++) {
            int64_t g = llabs(dc[k]) - (int64_t)hsum;
            if (g > 0) g2 += ((double)g * t->unit) * ((double)g * t->unit);
        }
        if (g2 > P->r_cut * P->r_cut) return;
    }
    int touching = 1;
    for (int k = 0; k < 3; k++)
        if ((uint64_t)llabs(dc[k]) > hsum) touching = 0;
    /* the offset of the two centres of mass, at its nearest periodic image */
    double rv[3], r2 = 0.0;
    for (int k = 0; k < 3; k++) {
        rv[k] = (double)dc[k] * t->unit + EB.dcom[k] - EA.dcom[k];
        if (t->periodic) {
            if (rv[k] >= 0.5 * t->box) rv[k] -= t->box;
            else if (rv[k] < -0.5 * t->box) rv[k] += t->box;
        }
        r2 += rv[k] * rv[k];
    }
    double r = sqrt(r2);
    double lA = EA.level < 0 ? 0.0 : node_side(t, EA.level), lB = EB.level < 0 ? 0.0 : node_side(t, EB.level);
    double h = 2.8 * P->eps0;
    int accept;
    if (P->criterion == 0) {
        accept = lA + lB < P->theta * r;                               /* eq. (eqnNodeDec) */
    } else {
        /* relative: (M_max / r^2)(l_max / r)^(p-1) < alpha |a|_min, p = 3 */
        double Mmax = fmax(EA.mass, EB.mass), lmax = fmax(lA, lB), amin = fmin(EA.amin, EB.amin);
        accept = Mmax * lmax * lmax < P->alpha * amin * r2 * r2;
    }
    if (!touching && accept && r >= h) {
        double D0, D1[3], D2[9], D3[27], D[4][27];
        orc_Dn(P->kernel == 1, rv, P->kernel == 1 ? 0.5 / P->r_s : 0.0, &D0, D1, D2, D3);
        if (P->kernel == 2) {
            /* periodic: the Green's function 1/r - psi (eqs. eqnpo1, eqnpo2) */
            double E0, E1[3], E2[9], E3[27];
            orc_ewald_psi(rv, t->box, 0.0, &E0, E1, E2, E3);
            D0 -= E0;
            for (int i = 0; i < 3; i++) D1[i] -= E1[i];
            for (int i = 0; i < 9; i++) D2[i] -= E2[i];
            for (int i = 0; i < 27; i++) D3[i] -= E3[i];
        }
        memset(D, 0, sizeof(D));
        D[0][0] = D0;
        memcpy(D[1], D1, sizeof(D1));
        memcpy(D[2], D2, sizeof(D2));
        memcpy(D[3], D3, sizeof(D3));
        /* sink A sees source B at +r; sink B sees source A (mirrored) */
        field FA = {0}, FB = {0};
        add_field(&FA, D, &EB, +1.0);
        add_field(&FB, D, &EA, -1.0);
        /* particles evaluate their field at their own position (a = 0):
         * acceleration -F1, potential F0 (times -G); nodes store the field */
        if (A >= 0) {
            field *T = &C->F[A];
            T->F0 += FA.F0;
            for (int a = 0; a < 3; a++) T->F1[a] += FA.F1[a];
            for (int a = 0; a < 9; a++) T->F2[a] += FA.F2[a];
            for (int a = 0; a < 27; a++) T->F3[a] += FA.F3[a];
        } else {
            int64_t j = -A - 1;
            for (int k = 0; k < 3; k++) C->acc[3 * j + k] -= FA.F1[k];
            C->pot[j] -= FA.F0;
        }
        if (B >= 0) {
            field *T = &C->F[B];
            T->F0 += FB.F0;
            for (int a = 0; a < 3; a++) T->F1[a] += FB.F1[a];
            for (int a = 0; a < 9; a++) T->F2[a] += FB.F2[a];
            for (int a = 0; a < 27; a++) T->F3[a] += FB.F3[a];
        } else {
            int64_t j = -B - 1;
            for (int k = 0; k < 3; k++) C->acc[3 * j + k] -= FB.F1[k];
            C->pot[j] -= FB.F0;
        }
        if (A >= 0 && B >= 0) C->n_nn++;
        else C->n_pn++;
        return;
    }
    /* open every side that is not a single particle */
    int64_t *LA, *LB, nA, nB;
    entity_children(C, A, &LA, &nA);
    entity_children(C, B, &LB, &nB);
    for (int64_t a = 0; a < nA; a++)
        for (int64_t b = 0; b < nB; b++) fmm_interact(C, LA[a], LB[b]);
    free(LA);
    free(LB);
}

/* Phase 3: shift parent fields to the children (exact re-centring of the
 * cubic polynomial), then evaluate at the particles of each leaf. */
static void fmm_down(fmm_ctx *C, int64_t q)
{
    const orc_tree *t = C->t;
    const onode *nd = &t->nodes[q];
    field *Fp = &C->F[q];
    if (!nd->leaf) {
        for (int c = 0; c < nd->nchild; c++) {
            int64_t ch = nd->child0 + c;
            const onode *cn = &t->nodes[ch];
            double d[3];
            for (int k = 0; k < 3; k++)
                d[k] = (double)(int32_t)(cn->gc[k] - nd->gc[k]) * t->unit + cn->dcom[k] - nd->dcom[k];
            field *Fc = &C->F[ch];
            /* F'_k = sum_j (-1)^j F_{k+j} . d^(j) / j! */
            double f0 = Fp->F0;
            for (int i = 0; i < 3; i++) f0 -= Fp->F1[i] * d[i];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) f0 += 0.5 * Fp->F2[i * 3 + j] * d[i] * d[j];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++)
                    for (int k = 0; k < 3; k++) f0 -= Fp->F3[(i * 3 + j) * 3 + k] * d[i] * d[j] * d[k] / 6.0;
            Fc->F0 += f0;
            for (int i = 0; i < 3; i++) {
                double f1 = Fp->F1[i];
                for (int j = 0; j < 3; j++) f1 -= Fp->F2[i * 3 + j] * d[j];
                for (int j = 0; j < 3; j++)
                    for (int k = 0; k < 3; k++) f1 += 0.5 * Fp->F3[(i * 3 + j) * 3 + k] * d[j] * d[k];
                Fc->F1[i] += f1;
            }
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    double f2 = Fp->F2[i * 3 + j];
                    for (int k = 0; k < 3; k++) f2 -= Fp->F3[(i * 3 + j) * 3 + k] * d[k];
                    Fc->F2[i * 3 + j] += f2;
                }
            for (int a = 0; a < 27; a++) Fc->F3[a] += Fp->F3[a];
            fmm_down(C, ch);
        }
        return;
    }
    /* L2P: phi = -G[F0 - F1.a + F2:a^2/2 - F3.a^3/6], acc = G[-F1 + F2.a - F3:a^2/2] */
    for (int64_t s = 0; s < nd->count; s++) {
        int64_t j = t->idx[nd->first + s];
        double a[3] = {(double)(int32_t)(t->X[j] - nd->gc[0]) * t->unit - nd->dcom[0],
                       (double)(int32_t)(t->Y[j] - nd->gc[1]) * t->unit - nd->dcom[1],
                       (double)(int32_t)(t->Z[j] - nd->gc[2]) * t->unit - nd->dcom[2]};
        double phi = Fp->F0;
        for (int i = 0; i < 3; i++) phi -= Fp->F1[i] * a[i];
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) phi += 0.5 * Fp->F2[i * 3 + k] * a[i] * a[k];
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++)
                for (int m = 0; m < 3; m++) phi -= Fp->F3[(i * 3 + k) * 3 + m] * a[i] * a[k] * a[m] / 6.0;
        C->pot[j] -= phi;
        for (int i = 0; i < 3; i++) {
            double g = -Fp->F1[i];
            for (int k = 0; k < 3; k++) g += Fp->F2[i * 3 + k] * a[k];
            for (int k = 0; k < 3; k++)
                for (int m = 0; m < 3; m++) g -= 0.5 * Fp->F3[(i * 3 + k) * 3 + m] * a[k] * a[m];
            C->acc[3 * j + i] += g;
        }
    }
}

int orc_fmm(const orc_tree *t, const orc_fmm_params *P, const double *aseed, double *acc, double *pot,
            int64_t stats[3])
{
    if (!t->has_moments) return -4;
    if (P->criterion == 1 && !aseed) return -1;
    fmm_ctx C;
    C.t = t;
    C.P = *P;
    C.F = (field *)calloc((size_t)t->nnodes, sizeof(field));
    C.acc = (double *)calloc((size_t)t->n * 3, sizeof(double));
    C.pot = (double *)calloc((size_t)t->n, sizeof(double));
    C.aseed = P->criterion == 1 ? aseed : NULL;
    C.amin = NULL;
    if (C.aseed) {
        C.amin = (double *)malloc((size_t)t->nnodes * sizeof(double));
        node_amin(&C, 0);
    }
    C.n_pp = C.n_pn = C.n_nn = 0;
    fmm_interact(&C, 0, 0);
    fmm_down(&C, 0);
    for (int64_t i = 0; i < t->n; i++) {
        for (int k = 0; k < 3; k++) acc[3 * i + k] = P->G * C.acc[3 * i + k];
        if (pot) pot[i] = P->G * C.pot[i];
    }
    if (stats) { stats[0] = C.n_pp; stats[1] = C.n_pn; stats[2] = C.n_nn; }
    free(C.F);
    free(C.acc);
    free(C.pot);
    free(C.amin);
    return 0;
}

/* ======================================================================
 * 9. Learned |a| seed: MLP 8 -> 64 -> 64 -> 1 with SiLU, in FP64
 * ====================================================================== */

/* Parameter layout (4801 values): W1[64][8], b1[64], W2[64][64], b2[64],
 * w3[64], b3[1].  The weights given are already rounded to the storage
 * precision; this code computes in double. */
static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

void orc_mlp_forward(const double *w, const double *feat, int64_t n, double *out)
{
    const double *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *w3 = w + 4736, *b3 = w + 4800;
    for (int64_t p = 0; p < n; p++) {
        double h1[64], h2[64];
        for (int o = 0; o < 64; o++) {
            double z = b1[o];
            for (int i = 0; i < 8; i++) z += W1[o * 8 + i] * feat[p * 8 + i];
            h1[o] = silu(z);
        }
        for (int o = 0; o < 64; o++) {
            double z = b2[o];
            for (int i = 0; i < 64; i++) z += W2[o * 64 + i] * h1[i];
            h2[o] = silu(z);
        }
        double y = b3[0];
        for (int i = 0; i < 64; i++) y += w3[i] * h2[i];
        out[p] = y;
    }
}

/* Loss and its gradient with respect to all 4801 parameters
 * (backpropagation).  tau <= 0: mean squared error L = (1/n) sum (y - t)^2;
 * 0 < tau < 1: pinball loss L = (1/n) sum rho(t - y), rho(u) = u (tau - [u<0]). */
double orc_mlp_loss_grad(const double *w, const double *feat, const double *target, int64_t n, double tau,
                         double *grad)
{
    const double *W1 = w, *b1 = w + 512, *W2 = w + 576, *b2 = w + 4672, *w3 = w + 4736, *b3 = w + 4800;
    double *gW1 = grad, *gb1 = grad + 512, *gW2 = grad + 576, *gb2 = grad + 4672, *gw3 = grad + 4736,
           *gb3 = grad + 4800;
    memset(grad, 0, sizeof(double) * 4801);
    double loss = 0.0;
    for (int64_t p = 0; p < n; p++) {
        double z1[64], h1[64], z2[64], h2[64];
        for (int o = 0; o < 64; o++) {
            double z = b1[o];
            for (int i = 0; i < 8; i++) z += W1[o * 8 + i] * feat[p * 8 + i];
            z1[o] = z;
            h1[o] = silu(z);
        }
        for (int o = 0; o < 64; o++) {
            double z = b2[o];
            for (int i = 0; i < 64; i++) z += W2[o * 64 + i] * h1[i];
            z2[o] = z;
            h2[o] = silu(z);
        }
        double y = b3[0];
        for (int i = 0; i < 64; i++) y += w3[i] * h2[i];
        double e = y - target[p], dy;
        if (tau > 0.0) {
            double u = -e;  /* target - y */
            loss += u >= 0.0 ? tau * u : (tau - 1.0) * u;
            dy = (u >= 0.0 ? -tau : 1.0 - tau) / (double)n;
        } else {
            loss += e * e;
            dy = 2.0 * e / (double)n;
        }
        gb3[0] += dy;
        double dz2[64], dh1[64];
        for (int i = 0; i < 64; i++) {
            gw3[i] += dy * h2[i];
            dz2[i] = dy * w3[i] * dsilu(z2[i]);
        }
        for (int i = 0; i < 64; i++) dh1[i] = 0.0;
        for (int o = 0; o < 64; o++) {
            gb2[o] += dz2[o];
            for (int i = 0; i < 64; i++) {
                gW2[o * 64 + i] += dz2[o] * h1[i];
                dh1[i] += dz2[o] * W2[o * 64 + i];
            }
        }
        for (int o = 0; o < 64; o++) {
            double dz1 = dh1[o] * dsilu(z1[o]);
            gb1[o] += dz1;
            for (int i = 0; i < 8; i++) gW1[o * 8 + i] += dz1 * feat[p * 8 + i];
        }
    }
    return loss / (double)n;
}

/* One Adam step (Kingma & Ba 2015) on master weights w, moments m, v;
 * step is the 1-based step count. */
void orc_adam(double *w, const double *g, double *m, double *v, int64_t np, double lr, double b1, double b2,
              double eps, int64_t step)
{
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < np; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ======================================================================
 * 10. Two isolated particle groups A and B (Sec. "The FMM force accuracy
 *     between two interacting nodes"): forces on each group's particles
 *     from the other group, by the symmetric FMM expansion (p = 3) and by
 *     the one-sided expansion of the source group at each particle.
 *     Positions are physical (n x 3), Newtonian, G = 1, no softening.
 * ====================================================================== */

static void group_moments(int64_t n, const double *pos, const double *m, entity *E, double s[3])
{
    double M = 0.0, c[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        M += m[i];
        for (int k = 0; k < 3; k++) c[k] += m[i] * pos[3 * i + k];
    }
    for (int k = 0; k < 3; k++) s[k] = c[k] / M;
    E->level = 0;
    memset(E->gc, 0, sizeof(E->gc));
    memset(E->dcom, 0, sizeof(E->dcom));
    E->mass = M;
    memset(E->q2, 0, sizeof(E->q2));
    memset(E->q3, 0, sizeof(E->q3));
    for (int64_t p = 0; p < n; p++) {
        double d[3] = {pos[3 * p] - s[0], pos[3 * p + 1] - s[1], pos[3 * p + 2] - s[2]};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                E->q2[i * 3 + j] += m[p] * d[i] * d[j];
                for (int k = 0; k < 3; k++) E->q3[(i * 3 + j) * 3 + k] += m[p] * d[i] * d[j] * d[k];
            }
    }
}

/* evaluate a stored field expansion at offset a from its centre: acceleration (G = 1) */
static void field_acc(const field *F, const double a[3], double out[3])
{
    for (int i = 0; i < 3; i++) {
        double g = -F->F1[i];
        for (int k = 0; k < 3; k++) g += F->F2[i * 3 + k] * a[k];
        for (int k = 0; k < 3; k++)
            for (int m = 0; m < 3; m++) g -= 0.5 * F->F3[(i * 3 + k) * 3 + m] * a[k] * a[m];
        out[i] = g;
    }
}

void orc_two_groups(int64_t nA, const double *posA, const double *mA, int64_t nB, const double *posB,
                    const double *mB, double *accA_fmm, double *accB_fmm, double *accA_tree, double *accB_tree)
{
    entity EA, EB;
    double sA[3], sB[3];
    group_moments(nA, posA, mA, &EA, sA);
    group_moments(nB, posB, mB, &EB, sB);
    double rv[3] = {sB[0] - sA[0], sB[1] - sA[1], sB[2] - sA[2]};
    double D0, D1[3], D2[9], D3[27], D[4][27];
    orc_Dn(0, rv, 0.0, &D0, D1, D2, D3);
    memset(D, 0, sizeof(D));
    D[0][0] = D0;
    memcpy(D[1], D1, sizeof(D1));
    memcpy(D[2], D2, sizeof(D2));
    memcpy(D[3], D3, sizeof(D3));
    field FA = {0}, FB = {0};
    add_field(&FA, D, &EB, +1.0);
    add_field(&FB, D, &EA, -1.0);
    orc_walk_params P = {0};
    P.order = 3;
    onode nA_ = {0}, nB_ = {0};
    nA_.mass = EA.mass; memcpy(nA_.q2, EA.q2, sizeof(EA.q2)); memcpy(nA_.q3, EA.q3, sizeof(EA.q3));
    nB_.mass = EB.mass; memcpy(nB_.q2, EB.q2, sizeof(EB.q2)); memcpy(nB_.q3, EB.q3, sizeof(EB.q3));
    for (int64_t i = 0; i < nA; i++) {
        double a[3] = {posA[3 * i] - sA[0], posA[3 * i + 1] - sA[1], posA[3 * i + 2] - sA[2]};
        field_acc(&FA, a, accA_fmm + 3 * i);
        double r[3] = {sB[0] - posA[3 * i], sB[1] - posA[3 * i + 1], sB[2] - posA[3 * i + 2]};
        double acc[3] = {0, 0, 0}, phi = 0.0;
        p2m_one(&P, &nB_, r, 0.0, acc, &phi);
        memcpy(accA_tree + 3 * i, acc, sizeof(acc));
    }
    for (int64_t i = 0; i < nB; i++) {
        double a[3] = {posB[3 * i] - sB[0], posB[3 * i + 1] - sB[1], posB[3 * i + 2] - sB[2]};
        field_acc(&FB, a, accB_fmm + 3 * i);
        double r[3] = {sA[0] - posB[3 * i], sA[1] - posB[3 * i + 1], sA[2] - posB[3 * i + 2]};
        double acc[3] = {0, 0, 0}, phi = 0.0;
        p2m_one(&P, &nA_, r, 0.0, acc, &phi);
        memcpy(accB_tree + 3 * i, acc, sizeof(acc));
    }
}

/* ======================================================================
 * 11. Features of the learned |a| seed, per particle, from the leaf L that
 *     holds it, its parent P and grandparent Q (a missing ancestor is
 *     replaced by the node itself):
 *       log10 M_L, log10 l_L, level of L,
 *       log10(|x - s_L|/l_L + 1e-3), log10(|x - s_P|/l_P + 1e-3),
 *       log10 M_P, log10 M_Q,
 *       log10 |a_near|, a_near = pair forces of the other particles of L
 *       + point-mass forces of the siblings of L (other children of P) and
 *       of the siblings of P (other children of Q), with the pair kernel
 *       of the walk (softened, short-range for kernel 1).
 *     feat: n x 8, caller order.
 * ====================================================================== */

/* force factor of a point mass at distance r, as in p2p_one */
static double pair_K(const orc_walk_params *P, double r)
{
    double h = 2.8 * P->eps0;
    if (P->kernel == 0) return orc_soft_K(r, h);
    return orc_sr_K(r, h, 0.5 / P->r_s);
}

static void features_rec(const orc_tree *t, const orc_walk_params *P, int64_t q, int64_t par, int64_t gpar,
                         double *feat)
{
    const onode *nd = &t->nodes[q];
    if (!nd->leaf) {
        for (int c = 0; c < nd->nchild; c++) features_rec(t, P, nd->child0 + c, q, par, feat);
        return;
    }
    const onode *np = &t->nodes[par >= 0 ? par : q];
    const onode *ng = gpar >= 0 ? &t->nodes[gpar] : np;
    double l = node_side(t, nd->level), lp = node_side(t, np->level);
    for (int64_t s = 0; s < nd->count; s++) {
        int64_t j = t->idx[nd->first + s];
        double *f = feat + 8 * j;
        uint32_t xj[3] = {t->X[j], t->Y[j], t->Z[j]};
        double dL = 0.0, dP = 0.0;
        for (int k = 0; k < 3; k++) {
            double a = (double)(int32_t)(xj[k] - nd->gc[k]) * t->unit - nd->dcom[k];
            double b = (double)(int32_t)(xj[k] - np->gc[k]) * t->unit - np->dcom[k];
            dL += a * a;
            dP += b * b;
        }
        double acc[3] = {0, 0, 0};
        for (int64_t u = 0; u < nd->count; u++) {
            int64_t k = t->idx[nd->first + u];
            if (k == j) continue;
            double d[3] = {(double)(int32_t)(t->X[k] - xj[0]) * t->unit, (double)(int32_t)(t->Y[k] - xj[1]) * t->unit,
                           (double)(int32_t)(t->Z[k] - xj[2]) * t->unit};
            double K = pair_K(P, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
            for (int c = 0; c < 3; c++) acc[c] += t->m[k] * d[c] * K;
        }
        int64_t selfs[2] = {q, par}, ups[2] = {par, gpar};
        for (int lev = 0; lev < 2; lev++) {
            if (selfs[lev] < 0 || ups[lev] < 0) break;
            const onode *up = &t->nodes[ups[lev]];
            for (int c = 0; c < up->nchild; c++) {
                int64_t sib = up->child0 + c;
                if (sib == selfs[lev]) continue;
                const onode *sn = &t->nodes[sib];
                double d[3];
                for (int k = 0; k < 3; k++) d[k] = (double)(int32_t)(sn->gc[k] - xj[k]) * t->unit + sn->dcom[k];
                double K = pair_K(P, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
                for (int k = 0; k < 3; k++) acc[k] += sn->mass * d[k] * K;
            }
        }
        double am = sqrt(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
        f[0] = log10(nd->mass);
        f[1] = log10(l);
        f[2] = nd->level;
        f[3] = log10(sqrt(dL) / l + 1e-3);
        f[4] = log10(sqrt(dP) / lp + 1e-3);
        f[5] = log10(np->mass);
        f[6] = log10(ng->mass);
        f[7] = log10(am > 1e-30 ? am : 1e-30);
    }
}

int orc_features(const orc_tree *t, const orc_walk_params *P, double *feat)
{
    if (!t->has_moments) return -4;
    features_rec(t, P, 0, -1, -1, feat);
    return 0;
}
