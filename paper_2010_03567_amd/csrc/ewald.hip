// ewald.hip -- table of the periodic correction potential psi and its
// derivatives, and a point evaluation through the same Taylor lookup that
// the walk uses.
//
// Paper: Sec. "Periodic boundary conditions", eq. (eqnewal):
//   psi(x) = 1/|x| + pi/(alpha^2 V) - sum_n erfc(alpha |x + q_n|)/|x + q_n|
//            - (4 pi / V) sum_{k != 0} exp(-k^2/(4 alpha^2))/k^2 cos(k.x),
// tabulated with the derivatives of orders 0..6 so that the walk's
// third-order Taylor expansion reaches the third derivatives its quadrupole
// force needs.  Every table entry is one FP64 thread: the real-space images
// and wave vectors are summed for one derivative component D^(a,b,c) psi at
// one grid point, from the closed forms of the radial derivatives.
#include "g4_internal.h"
#include "ewald.h"

#define EW_T 128
#define EW_SQRTPI 1.7724538509055160273

namespace {

// alpha = 2/L: the nearest real image left out lies 3.5 L away or more
// (erfc(7) ~ 4e-23); the smallest wave vector left out has |n| = 5, whose
// factor exp(-k^2 / (4 alpha^2)) = exp(-(5 pi / 2)^2) ~ 2e-27.
constexpr int EW_NR = 3;
constexpr int EW_NK = 4;
constexpr int EW_ORD = 6;

__device__ double dpow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

// a! / (2^i i! (a - 2i)!): the number of ways to pair 2i of a equal indices
__device__ double pairings(int a, int i)
{
    double r = 1.0;
    for (int t = a - 2 * i + 1; t <= a; t++) r *= t;   // a! / (a - 2i)!
    for (int t = 1; t <= i; t++) r /= 2.0 * t;           // / (2^i i!)
    return r;
}

// g_k = (r^-1 d/dr)^k f for f = erfc(alpha r)/r, k = 0..o:
//   g_k = A_k erfc(alpha r) r^-(2k+1) + E sum_j b_kj r^-2j,  E = (2 alpha / sqrt(pi)) exp(-alpha^2 r^2),
// A_{k+1} = -(2k+1) A_k, and b follows from d/dr E = -2 alpha^2 r E.
__device__ void erfc_g(double r, double alpha, int o, double *g)
{
    const double ec = erfc(alpha * r), E = 2.0 * alpha / EW_SQRTPI * exp(-alpha * alpha * r * r);
    const double ri2 = 1.0 / (r * r), a2 = alpha * alpha;
    double b[EW_ORD + 2] = {0}, nb[EW_ORD + 2];
    double A = 1.0, rp = 1.0 / r;                          // A_k, r^-(2k+1)
    for (int k = 0; k <= o; k++) {
        double s = 0.0, rj = 1.0;
        for (int j = 1; j <= k; j++) {
            rj *= ri2;
            s += b[j] * rj;
        }
        g[k] = A * ec * rp + E * s;
        for (int j = 0; j <= k + 1; j++) nb[j] = 0.0;
        for (int j = 1; j <= k; j++) {
            nb[j] += -2.0 * a2 * b[j];
            nb[j + 1] += -2.0 * j * b[j];
        }
        nb[k + 1] += -A;
        for (int j = 0; j <= k + 1; j++) b[j] = nb[j];
        A *= -(2.0 * k + 1.0);
        rp *= ri2;
    }
}

// g_k of erf(alpha r)/r = 1/r - erfc(alpha r)/r (the n = 0 image with 1/|x|),
// regular at r = 0: with u = r^2, r^-1 d/dr = 2 d/du and
// erf(alpha r)/r = (2 alpha / sqrt(pi)) sum_m (-alpha^2 u)^m / (m! (2m + 1)).
__device__ void erf_g(double r, double alpha, int o, double *g)
{
    if (alpha * r < 0.5) {
        const double u = r * r, a2 = alpha * alpha;
        for (int k = 0; k <= o; k++) {
            double am = 1.0;
            for (int m = 0; m < k; m++) am *= -a2;
            double s = 0.0, um = 1.0, f = 1.0;
            for (int m = k; m < k + 24; m++) {
                s += am * um / (f * (2.0 * m + 1.0));
                am *= -a2;
                um *= u;
                f *= (double)(m - k + 1);
            }
            g[k] = 2.0 * alpha / EW_SQRTPI * ldexp(s, k);
        }
        return;
    }
    erfc_g(r, alpha, o, g);
    double A = 1.0, rp = 1.0 / r;
    const double ri2 = 1.0 / (r * r);
    for (int k = 0; k <= o; k++) {
        g[k] = A * rp - g[k];     // Newtonian g_k = A_k r^-(2k+1)
        A *= -(2.0 * k + 1.0);
        rp *= ri2;
    }
}

// D^(a,b,c) of a radial function with scalars g at x:
//   sum_{i,j,l} P(a,i) P(b,j) P(c,l) x^(a-2i) y^(b-2j) z^(c-2l) g_{a+b+c-i-j-l}
__device__ double radial_deriv(const double *g, double x, double y, double z, int a, int b, int c)
{
    double s = 0.0;
    for (int i = 0; 2 * i <= a; i++)
        for (int j = 0; 2 * j <= b; j++)
            for (int l = 0; 2 * l <= c; l++)
                s += pairings(a, i) * pairings(b, j) * pairings(c, l) * dpow(x, a - 2 * i) * dpow(y, b - 2 * j) *
                     dpow(z, c - 2 * l) * g[a + b + c - i - j - l];
    return s;
}

__global__ __launch_bounds__(EW_T) void k_ewald_table(float *tab, int ne, double L)
{
    const int64_t npts = (int64_t)(ne + 1) * (ne + 1) * (ne + 1);
    const int64_t t = (int64_t)blockIdx.x * EW_T + threadIdx.x;
    if (t >= npts * G4_EWALD_NCOMP) return;
    const int comp = (int)(t % G4_EWALD_NCOMP);
    const int64_t pt = t / G4_EWALD_NCOMP;
    // component -> (a, b, c): order o, then s = b + c with s (s + 1)/2 <= rest
    int o = 0;
    while ((o + 1) * (o + 2) * (o + 3) / 6 <= comp) o++;
    const int rest = comp - o * (o + 1) * (o + 2) / 6;
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= rest) s++;
    const int c = rest - s * (s + 1) / 2, b = s - c, a = o - s;
    const double h = 0.5 * L / ne;
    const double x = (double)(pt / ((int64_t)(ne + 1) * (ne + 1))) * h;
    const double y = (double)((pt / (ne + 1)) % (ne + 1)) * h;
    const double z = (double)(pt % (ne + 1)) * h;
    const double alpha = 2.0 / L, V = L * L * L;
    double g[EW_ORD + 1];
    // n = 0: 1/|x| - erfc(alpha r)/r
    erf_g(sqrt(x * x + y * y + z * z), alpha, o, g);
    double sum = radial_deriv(g, x, y, z, a, b, c);
    // the other real-space images
    for (int nx = -EW_NR; nx <= EW_NR; nx++)
        for (int ny = -EW_NR; ny <= EW_NR; ny++)
            for (int nz = -EW_NR; nz <= EW_NR; nz++) {
                if (!nx && !ny && !nz) continue;
                const double px = x + nx * L, py = y + ny * L, pz = z + nz * L;
                erfc_g(sqrt(px * px + py * py + pz * pz), alpha, o, g);
                sum -= radial_deriv(g, px, py, pz, a, b, c);
            }
    // wave vectors: d^o/dtheta^o cos(theta) = cos(theta + o pi / 2)
    const double tp = 2.0 * M_PI / L;
    for (int nx = -EW_NK; nx <= EW_NK; nx++)
        for (int ny = -EW_NK; ny <= EW_NK; ny++)
            for (int nz = -EW_NK; nz <= EW_NK; nz++) {
                if (!nx && !ny && !nz) continue;
                const double kx = tp * nx, ky = tp * ny, kz = tp * nz;
                const double k2 = kx * kx + ky * ky + kz * kz;
                const double w = 4.0 * M_PI / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                const double th = kx * x + ky * y + kz * z;
                double cs;
                switch (o & 3) {
                case 0: cs = cos(th); break;
                case 1: cs = -sin(th); break;
                case 2: cs = -cos(th); break;
                default: cs = sin(th); break;
                }
                sum -= w * dpow(kx, a) * dpow(ky, b) * dpow(kz, c) * cs;
            }
    if (o == 0) sum += M_PI / (alpha * alpha * V);
    tab[pt * G4_EWALD_NCOMP + comp] = (float)sum;
}

__global__ __launch_bounds__(EW_T) void k_ewald_eval(const float *__restrict__ tab, int ne, float h, float hinv,
                                                     int64_t n, const double *dx, const double *dy, const double *dz,
                                                     double *psi, double *gx, double *gy, double *gz)
{
    const int64_t i = (int64_t)blockIdx.x * EW_T + threadIdx.x;
    if (i >= n) return;
    float fx, fy, fz, fp;
    ew_grad<true>(tab, ne, h, hinv, (float)dx[i], (float)dy[i], (float)dz[i], fx, fy, fz, fp);
    psi[i] = fp;
    gx[i] = fx;
    gy[i] = fy;
    gz[i] = fz;
}

}  // namespace

size_t g4_ewald_layout_bytes(int ne)
{
    return (size_t)(ne + 1) * (ne + 1) * (ne + 1) * G4_EWALD_NCOMP * sizeof(float);
}

int g4_launch_ewald_table(g4_ctx *ctx, double box, int ne, float *tab)
{
    const int64_t tot = (int64_t)(ne + 1) * (ne + 1) * (ne + 1) * G4_EWALD_NCOMP;
    k_ewald_table<<<(unsigned)((tot + EW_T - 1) / EW_T), EW_T, 0, ctx->stream>>>(tab, ne, box);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

int g4_launch_ewald_eval(g4_ctx *ctx, const float *tab, int ne, double box, int64_t n, const double *dx,
                         const double *dy, const double *dz, double *psi, double *gx, double *gy, double *gz)
{
    if (n <= 0) return G4_OK;
    const double h = 0.5 * box / ne;
    k_ewald_eval<<<(unsigned)((n + EW_T - 1) / EW_T), EW_T, 0, ctx->stream>>>(tab, ne, (float)h, (float)(1.0 / h), n,
                                                                                dx, dy, dz, psi, gx, gy, gz);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
