// direct.hip -- direct summation on the device, FP64 throughout: the exact
// reference against which the paper measures every force algorithm (Sec.
// "Softened potential in periodic systems").  Kernel 0: spline-softened
// Newtonian; kernel 1: the short-range force of eq. (eqnpo4) over the nearest
// image only, optionally truncated at r_cut; kernel 2: periodic gravity, the
// softened nearest image plus the correction psi of the other images summed
// exactly by Ewald's method for every pair (Sec. "Periodic boundary
// conditions", eqs. eqnpo1, eqnewal) -- about a thousand terms per pair, for
// sampled targets.  One thread per target; source particles are staged
// through LDS tiles shared by the block.
#include "g4_internal.h"

#define DT 256

struct DirectArgs {
    const uint32_t *x, *y, *z;
    const float *m;
    int64_t n;
    const int64_t *targets;
    int64_t nt;
    double unit, h, hinv, asplit, rskip2, rcut2, G, L;
    int kernel, truncate;
    double *ax, *ay, *az, *pot;
};

__device__ __forceinline__ void soft_kw(double u, double hinv, double &K, double &W)
{
    double h3 = hinv * hinv * hinv, u2 = u * u;
    if (u < 0.5) {
        K = h3 * (32.0 / 3.0 + u2 * (-192.0 / 5.0 + 32.0 * u));
        W = hinv * (14.0 / 5.0 + u2 * (-16.0 / 3.0 + u2 * (48.0 / 5.0 - 32.0 / 5.0 * u)));
    } else {
        K = h3 * (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u2 - 32.0 / 3.0 * u2 * u - 1.0 / (15.0 * u2 * u));
        W = hinv * (16.0 / 5.0 - 1.0 / (15.0 * u) + u2 * (-32.0 / 3.0 + u * (16.0 + u * (-48.0 / 5.0 + 32.0 / 15.0 * u))));
    }
}

// (erf x - 2x e^{-x^2}/sqrt(pi)) / x^3 and erf(x)/x, series below x = 0.5
__device__ __forceinline__ double lrf(double x)
{
    if (x < 0.5) {
        double s = 0, t = 1, x2 = x * x;
        for (int k = 0; k < 14; k++) { s += t / (2 * k + 3); t *= -x2 / (k + 1); }
        return 4.0 / 1.7724538509055160273 * s;
    }
    return (erf(x) - 2.0 * x / 1.7724538509055160273 * exp(-x * x)) / (x * x * x);
}
__device__ __forceinline__ double erfx(double x)
{
    if (x < 0.5) {
        double s = 0, t = 1, x2 = x * x;
        for (int k = 0; k < 14; k++) { s += t / (2 * k + 1); t *= -x2 / (k + 1); }
        return 2.0 / 1.7724538509055160273 * s;
    }
    return erf(x) / x;
}

// psi(d) and grad psi(d) of a cube of side L by the Ewald sums with alpha = 2/L:
// the n = 0 image combined with 1/|d| as erf(alpha r)/r, 342 further real
// images (|n_i| <= 3) and 728 wave vectors (|n_i| <= 4).
__device__ void ewald_exact(double dx, double dy, double dz, double L, double &psi, double &gx, double &gy,
                            double &gz)
{
    const double alpha = 2.0 / L, V = L * L * L, c2 = 2.0 * alpha / 1.7724538509055160273;
    const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    // erf(alpha r)/r and its r^-1 d/dr = -(erf(ar) - 2ar e^{-a^2 r^2}/sqrt(pi))/r^3
    psi = alpha * erfx(alpha * r) + M_PI / (alpha * alpha * V);
    double g1 = -alpha * alpha * alpha * lrf(alpha * r);
    gx = g1 * dx;
    gy = g1 * dy;
    gz = g1 * dz;
    for (int nx = -3; nx <= 3; nx++)
        for (int ny = -3; ny <= 3; ny++)
            for (int nz = -3; nz <= 3; nz++) {
                if (!nx && !ny && !nz) continue;
                const double px = dx + nx * L, py = dy + ny * L, pz = dz + nz * L;
                const double q2 = px * px + py * py + pz * pz, q = sqrt(q2), x = alpha * q;
                const double ec = erfc(x);
                psi -= ec / q;
                // d/dx_i [erfc(alpha q)/q] = -(erfc + 2 x e^{-x^2}/sqrt(pi)) x_i / q^3
                const double f = (ec + c2 * q * exp(-x * x)) / (q2 * q);
                gx += f * px;
                gy += f * py;
                gz += f * pz;
            }
    const double tp = 2.0 * M_PI / L;
    for (int nx = -4; nx <= 4; nx++)
        for (int ny = -4; ny <= 4; ny++)
            for (int nz = -4; nz <= 4; nz++) {
                if (!nx && !ny && !nz) continue;
                const double kx = tp * nx, ky = tp * ny, kz = tp * nz, k2 = kx * kx + ky * ky + kz * kz;
                const double w = 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                double sn, cs;
                sincos(kx * dx + ky * dy + kz * dz, &sn, &cs);
                psi -= w * cs;
                gx += w * sn * kx;
                gy += w * sn * ky;
                gz += w * sn * kz;
            }
}

__global__ __launch_bounds__(DT) void k_direct(const DirectArgs A)
{
    __shared__ uint4 tile[DT];
    const int64_t q = blockIdx.x * (int64_t)DT + threadIdx.x;
    const bool act = q < A.nt;
    const int64_t i = act ? (A.targets ? A.targets[q] : q) : 0;
    const uint32_t xi = A.x[i], yi = A.y[i], zi = A.z[i];
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int64_t base = 0; base < A.n; base += DT) {
        const int64_t j = base + threadIdx.x;
        __syncthreads();
        tile[threadIdx.x] = j < A.n ? make_uint4(A.x[j], A.y[j], A.z[j], __float_as_uint(A.m[j])) : make_uint4(0, 0, 0, 0);
        __syncthreads();
        const int cnt = (int)min((int64_t)DT, A.n - base);
        for (int k = 0; k < cnt; k++) {
            const uint4 s = tile[k];
            if (base + k == i) continue;
            const double dx = (double)(int32_t)(s.x - xi) * A.unit;
            const double dy = (double)(int32_t)(s.y - yi) * A.unit;
            const double dz = (double)(int32_t)(s.z - zi) * A.unit;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 > A.rskip2 || (A.truncate && r2 > A.rcut2)) continue;
            const double m = (double)__uint_as_float(s.w);
            const double r = sqrt(r2);
            double K, W;
            if (r >= A.h) {
                if (A.kernel == 0) { K = 1.0 / (r2 * r); W = 1.0 / r; }
                else {
                    const double x = A.asplit * r, ec = erfc(x);
                    K = (ec + 2.0 * x / 1.7724538509055160273 * exp(-x * x)) / (r2 * r);
                    W = ec / r;
                }
            } else {
                soft_kw(r * A.hinv, A.hinv, K, W);
                if (A.kernel == 1) {
                    const double x = A.asplit * r;
                    K -= A.asplit * A.asplit * A.asplit * lrf(x);
                    W -= A.asplit * erfx(x);
                }
            }
            ax += m * K * dx;
            ay += m * K * dy;
            az += m * K * dz;
            ph -= m * W;
        }
    }
    if (act) {
        A.ax[q] = A.G * ax;
        A.ay[q] = A.G * ay;
        A.az[q] = A.G * az;
        if (A.pot) A.pot[q] = A.G * ph;
    }
}

// Kernel 2 costs about a thousand terms per pair, so a target gets a whole
// block: its threads split the sources and their FP64 sums are reduced in LDS.
__global__ __launch_bounds__(DT) void k_direct_ewald(const DirectArgs A)
{
    __shared__ double red[4][DT];
    const int64_t q = blockIdx.x;
    const int64_t i = A.targets ? A.targets[q] : q;
    const uint32_t xi = A.x[i], yi = A.y[i], zi = A.z[i];
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int64_t j = threadIdx.x; j < A.n; j += DT) {
        if (j == i) continue;
        const double dx = (double)(int32_t)(A.x[j] - xi) * A.unit;
        const double dy = (double)(int32_t)(A.y[j] - yi) * A.unit;
        const double dz = (double)(int32_t)(A.z[j] - zi) * A.unit;
        const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
        const double m = (double)A.m[j];
        double K, W;
        if (r >= A.h) {
            K = 1.0 / (r2 * r);
            W = 1.0 / r;
        } else {
            soft_kw(r * A.hinv, A.hinv, K, W);
        }
        double ps, gx, gy, gz;
        ewald_exact(dx, dy, dz, A.L, ps, gx, gy, gz);
        ax += m * (K * dx + gx);
        ay += m * (K * dy + gy);
        az += m * (K * dz + gz);
        ph += m * (ps - W);
    }
    red[0][threadIdx.x] = ax;
    red[1][threadIdx.x] = ay;
    red[2][threadIdx.x] = az;
    red[3][threadIdx.x] = ph;
    __syncthreads();
    for (int s = DT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 4; c++) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A.ax[q] = A.G * red[0][0];
        A.ay[q] = A.G * red[1][0];
        A.az[q] = A.G * red[2][0];
        if (A.pot) A.pot[q] = A.G * red[3][0];
    }
}

int g4_launch_direct(g4_ctx *ctx, const g4_particles *p, const g4_tree_params *tp, const g4_walk_params *wp,
                     int truncate, const int64_t *targets, int64_t ntargets, double *ax, double *ay, double *az,
                     double *pot)
{
    DirectArgs A;
    A.x = p->x; A.y = p->y; A.z = p->z; A.m = p->mass; A.n = p->n;
    A.targets = targets;
    A.nt = targets ? ntargets : p->n;
    A.unit = tp->box / (tp->periodic ? 4294967296.0 : 2147483648.0);
    A.L = tp->box;
    A.h = 2.8 * wp->eps0;
    A.hinv = A.h > 0 ? 1.0 / A.h : 0.0;
    A.kernel = wp->kernel;
    A.asplit = wp->kernel == 1 ? 0.5 / wp->r_s : 0.0;
    // beyond alpha r = 6, erfc < 3e-17: such sources add nothing in FP64
    A.rskip2 = wp->kernel == 1 ? (6.0 / A.asplit) * (6.0 / A.asplit) : 1e300;
    A.truncate = truncate;
    A.rcut2 = wp->r_cut * wp->r_cut;
    A.G = wp->G;
    A.ax = ax; A.ay = ay; A.az = az; A.pot = pot;
    if (A.nt > 0 && A.kernel == 2) k_direct_ewald<<<(unsigned)A.nt, DT, 0, ctx->stream>>>(A);
    else if (A.nt > 0) k_direct<<<(unsigned)((A.nt + DT - 1) / DT), DT, 0, ctx->stream>>>(A);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
