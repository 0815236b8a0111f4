// pm.hip -- long-range force of the TreePM split on a periodic mesh (gfx950).
//
// Paper: Sec. "TreePM approach": the long-range potential is the k-space
// sum of the Ewald decomposition with the Green's function
// exp(-k^2 r_s^2) / k^2, evaluated with a particle-mesh method -- clouds-in-
// cell assignment, FFT, multiplication with the Green's function, inverse
// FFT, a 4th-order finite-difference gradient on the mesh and CIC
// interpolation to the particles, the smoothing of assignment and
// interpolation deconvolved by dividing by the CIC window (a squared sinc per
// axis) once for each.  The potential carries the sign of the Newtonian one
// (attractive): phi_lr = -G (4 pi / V) sum_{k != 0} exp(-k^2 r_s^2)/k^2 ...
//
// Layout: an ng^3 mesh of complex FP32 (z fastest), mesh point c at c h,
// h = L / ng.  The particles come from a built tree in curve order (so that
// neighbouring threads touch neighbouring cells) with 32-bit integer
// coordinates: for ng = 2^g the cell is the top g bits and the CIC weight
// the remaining bits, both exact.
//
// Steps: k_pm_deposit (8 float atomics per particle) -> three passes of
// k_pm_fft (ng-point radix-2 transforms of tiles of lines staged in LDS, one
// pass per axis; the tiles of the strided axes take consecutive lines so
// every load and store is a run of consecutive cells) -> k_pm_green -> three
// inverse passes, the last one keeping only the real part -> k_pm_interp
// (gradient and interpolation fused: each particle reads the potential around
// its 8 CIC points).
#include <cmath>

#include "g4_internal.h"

#define PM_THREADS 256
#define PM_TILE_CELLS 4096  // complex cells per FFT tile (32 KiB of LDS, plus the twiddles)

__global__ void k_pm_twiddle(float2 *__restrict__ tw, int ng)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ng / 2) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)ng, &s, &c);  // exp(-2 pi i k / ng)
    tw[k] = make_float2((float)c, (float)s);
}

__global__ void k_pm_clear(float2 *__restrict__ m, size_t ncell)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x)
        m[i] = make_float2(0.f, 0.f);
}

// CIC cell and upper weight of one coordinate: top g bits, remaining bits / 2^(32-g)
__device__ __forceinline__ void pm_cell(uint32_t X, int shift, float wscale, int &i, float &f)
{
    i = (int)(X >> shift);
    f = (float)(X & ((1u << shift) - 1u)) * wscale;
}

// Particles arrive in curve order, so particles that share a mesh cell sit
// in consecutive lanes (the cell index is a prefix of the curve key; each CIC
// corner is the same shift of it).  Every corner's contributions are summed
// over such runs by a segmented scan across the wavefront and the last lane
// of a run issues the one atomic: in haloes most atomics disappear.
__global__ void k_pm_deposit(const uint4 *__restrict__ parts, int64_t n, int ng, int shift, float wscale,
                             float2 *__restrict__ mesh)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
        const int64_t p = base + threadIdx.x;
        const bool act = p < n;
        const uint4 q = act ? parts[p] : make_uint4(0u, 0u, 0u, 0u);
        const float m = act ? __uint_as_float(q.w) : 0.f;
        int ix, iy, iz;
        float fx, fy, fz;
        pm_cell(q.x, shift, wscale, ix, fx);
        pm_cell(q.y, shift, wscale, iy, fy);
        pm_cell(q.z, shift, wscale, iz, fz);
        const int mask = ng - 1;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c >> 2, dy = (c >> 1) & 1, dz = c & 1;
            float v = m * (dx ? fx : 1.f - fx) * (dy ? fy : 1.f - fy) * (dz ? fz : 1.f - fz);
            const uint32_t key = act ? (uint32_t)((((ix + dx) & mask) * ng + ((iy + dy) & mask)) * ng + ((iz + dz) & mask))
                                     : 0xffffffffu;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t ku = (uint32_t)__shfl_up((int)key, off);
                const float vu = __shfl_up(v, off);
                if (lane >= off && ku == key) v += vu;
            }
            const uint32_t kd = (uint32_t)__shfl_down((int)key, 1);
            if (act && (lane == 63 || kd != key)) atomicAdd(&mesh[key].x, v);
        }
    }
}

// One pass of ng-point transforms along `axis` (0 x, 1 y, 2 z) over every
// line of the mesh.  A block takes tl lines: for z, tl consecutive lines
// (one contiguous run of tl ng cells); for y and x, tl lines that are
// neighbours in z, so each of the ng rows of the tile is a run of tl cells.
// In LDS: bit-reversed load, lg in-place radix-2 stages, natural-order store.
// sign -1: forward (exp(-i k x)); +1: inverse, unnormalised.  real_out, if
// given, receives the real part instead of the complex result.
__global__ __launch_bounds__(PM_THREADS) void k_pm_fft(float2 *__restrict__ data, const float2 *__restrict__ tw,
                                                        int ng, int lg, int tl, int axis, float sign,
                                                        float *__restrict__ real_out)
{
    extern __shared__ float2 sm[];
    const int tid = threadIdx.x;
    const int cells = tl * ng;
    float2 *tws = sm + cells;  // twiddles of this direction: exp(sign 2 pi i k / ng), k < ng/2
    for (int k = tid; k < ng / 2; k += PM_THREADS) {
        const float2 w = tw[k];
        tws[k] = make_float2(w.x, -sign * w.y);
    }
    size_t base;
    size_t estride;  // distance between consecutive points of one line
    size_t lstride;  // distance between the tile's lines
    if (axis == 2) {
        base = (size_t)blockIdx.x * cells;
        estride = 1;
        lstride = ng;
    } else {
        const int per = ng / tl;  // tiles per outer index
        const size_t outer = blockIdx.x / per, z0 = (size_t)(blockIdx.x % per) * tl;
        estride = axis == 1 ? (size_t)ng : (size_t)ng * ng;
        base = (axis == 1 ? outer * ng * ng : outer * ng) + z0;
        lstride = 1;
    }
    // load: consecutive threads take consecutive addresses
    for (int e = tid; e < cells; e += PM_THREADS) {
        int t, k;
        if (axis == 2) {
            t = e / ng;
            k = e - t * ng;
        } else {
            k = e / tl;
            t = e - k * tl;
        }
        const int kr = (int)(__brev((unsigned)k) >> (32 - lg));
        sm[t * ng + kr] = data[base + (size_t)t * lstride + (size_t)k * estride];
    }
    __syncthreads();
    auto cmul = [](float2 a, float2 w) { return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x); };
    // radix-2 stages s and s + 1 fused: each thread takes the 4 points
    // i0, i0 + h, i0 + 2h, i0 + 3h (h = 2^s) through both stages in registers
    const int qb = ng >> 2;
    int s = 0;
    for (; s + 1 < lg; s += 2) {
        const int half = 1 << s;
        for (int b = tid; b < tl * qb; b += PM_THREADS) {
            const int t = b / qb, j = b - t * qb;
            const int grp = j >> s, pos = j & (half - 1);
            const int i0 = t * ng + (grp << (s + 2)) + pos;
            const float2 a0 = sm[i0], a1 = sm[i0 + half], a2 = sm[i0 + 2 * half], a3 = sm[i0 + 3 * half];
            const float2 w1 = tws[pos << (lg - s - 1)];
            const float2 b1 = cmul(a1, w1), b3 = cmul(a3, w1);
            const float2 c0 = make_float2(a0.x + b1.x, a0.y + b1.y), c1 = make_float2(a0.x - b1.x, a0.y - b1.y);
            const float2 c2 = make_float2(a2.x + b3.x, a2.y + b3.y), c3 = make_float2(a2.x - b3.x, a2.y - b3.y);
            const float2 d2 = cmul(c2, tws[pos << (lg - s - 2)]), d3 = cmul(c3, tws[(pos + half) << (lg - s - 2)]);
            sm[i0] = make_float2(c0.x + d2.x, c0.y + d2.y);
            sm[i0 + 2 * half] = make_float2(c0.x - d2.x, c0.y - d2.y);
            sm[i0 + half] = make_float2(c1.x + d3.x, c1.y + d3.y);
            sm[i0 + 3 * half] = make_float2(c1.x - d3.x, c1.y - d3.y);
        }
        __syncthreads();
    }
    if (s < lg) {  // odd lg: one radix-2 stage left
        const int half = 1 << s, hb = ng >> 1;
        for (int b = tid; b < tl * hb; b += PM_THREADS) {
            const int t = b / hb, j = b - t * hb;
            const int grp = j >> s, pos = j & (half - 1);
            const int i0 = t * ng + (grp << (s + 1)) + pos, i1 = i0 + half;
            const float2 a = sm[i0], bw = cmul(sm[i1], tws[pos << (lg - s - 1)]);
            sm[i0] = make_float2(a.x + bw.x, a.y + bw.y);
            sm[i1] = make_float2(a.x - bw.x, a.y - bw.y);
        }
        __syncthreads();
    }
    for (int e = tid; e < cells; e += PM_THREADS) {
        int t, k;
        if (axis == 2) {
            t = e / ng;
            k = e - t * ng;
        } else {
            k = e / tl;
            t = e - k * tl;
        }
        const size_t o = base + (size_t)t * lstride + (size_t)k * estride;
        const float2 v = sm[t * ng + k];
        if (real_out) real_out[o] = v.x;
        else data[o] = v;
    }
}

// the Green's function with the CIC window deconvolved twice:
// F(k) = -G (4 pi / V) exp(-k^2 r_s^2) / k^2 / W(k)^2, W = prod_d sinc^2(pi n_d / ng); F(0) = 0
__global__ void k_pm_green(float2 *__restrict__ mesh, int ng, int lg, double box, double r_s, double G)
{
    const size_t ncell = (size_t)ng * ng * ng;
    const float kf = (float)(2.0 * M_PI / box);
    const float rs2 = (float)(r_s * r_s);
    const float pref = (float)(-G * 4.0 * M_PI / (box * box * box));
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
        const int iz = (int)(i & (size_t)(ng - 1)), iy = (int)((i >> lg) & (size_t)(ng - 1)), ix = (int)(i >> (2 * lg));
        const int nx = ix < ng / 2 ? ix : ix - ng, ny = iy < ng / 2 ? iy : iy - ng, nz = iz < ng / 2 ? iz : iz - ng;
        if (nx == 0 && ny == 0 && nz == 0) {
            mesh[i] = make_float2(0.f, 0.f);
            continue;
        }
        const float kx = kf * nx, ky = kf * ny, kz = kf * nz;
        const float k2 = kx * kx + ky * ky + kz * kz;
        float W = 1.f;
        const int nn[3] = {nx, ny, nz};
#pragma unroll
        for (int d = 0; d < 3; d++) {
            if (nn[d]) {
                const float u = (float)M_PI * (float)nn[d] / (float)ng;
                const float sc = sinf(u) / u;
                W *= sc * sc;
            }
        }
        const float f = pref * expf(-k2 * rs2) / (k2 * W * W);
        const float2 v = mesh[i];
        mesh[i] = make_float2(v.x * f, v.y * f);
    }
}

// gradient (4th-order differences) and CIC interpolation, one particle per thread
__global__ void k_pm_interp(const uint4 *__restrict__ parts, const uint32_t *__restrict__ perm, int64_t n,
                            const float *__restrict__ phi, int ng, int lg, int shift, float wscale, float inv_h,
                            int accumulate, double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az,
                            double *__restrict__ pot)
{
    const int mask = ng - 1;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint4 q = parts[p];
        int ix, iy, iz;
        float fx, fy, fz;
        pm_cell(q.x, shift, wscale, ix, fx);
        pm_cell(q.y, shift, wscale, iy, fy);
        pm_cell(q.z, shift, wscale, iz, fz);
        auto at = [&](int x, int y, int z) {
            return phi[((size_t)(x & mask) << (2 * lg)) + ((size_t)(y & mask) << lg) + (size_t)(z & mask)];
        };
        float gx = 0.f, gy = 0.f, gz = 0.f, ph = 0.f;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const int dx = c >> 2, dy = (c >> 1) & 1, dz = c & 1;
            const float w = (dx ? fx : 1.f - fx) * (dy ? fy : 1.f - fy) * (dz ? fz : 1.f - fz);
            const int x = ix + dx, y = iy + dy, z = iz + dz;
            const float d1x = at(x + 1, y, z) - at(x - 1, y, z), d2x = at(x + 2, y, z) - at(x - 2, y, z);
            const float d1y = at(x, y + 1, z) - at(x, y - 1, z), d2y = at(x, y + 2, z) - at(x, y - 2, z);
            const float d1z = at(x, y, z + 1) - at(x, y, z - 1), d2z = at(x, y, z + 2) - at(x, y, z - 2);
            gx = fmaf(w, (2.f / 3.f) * d1x - (1.f / 12.f) * d2x, gx);
            gy = fmaf(w, (2.f / 3.f) * d1y - (1.f / 12.f) * d2y, gy);
            gz = fmaf(w, (2.f / 3.f) * d1z - (1.f / 12.f) * d2z, gz);
            if (pot) ph = fmaf(w, at(x, y, z), ph);
        }
        const uint32_t o = perm[p];
        const double a0 = -(double)gx * inv_h, a1 = -(double)gy * inv_h, a2 = -(double)gz * inv_h;
        if (accumulate) {
            ax[o] += a0;
            ay[o] += a1;
            az[o] += a2;
            if (pot) pot[o] += (double)ph;
        } else {
            ax[o] = a0;
            ay[o] = a1;
            az[o] = a2;
            if (pot) pot[o] = (double)ph;
        }
    }
}

static int ilog2(int v)
{
    int g = 0;
    while ((1 << g) < v) g++;
    return g;
}

int g4_pm_layout_bytes(int ng, size_t *bytes)
{
    if (ng < 8 || ng > 1024 || (ng & (ng - 1))) return G4_EINVAL;
    const size_t ncell = (size_t)ng * ng * ng;
    *bytes = ((size_t)ng / 2 * 8 + 255) / 256 * 256 + (ncell * 8 + 255) / 256 * 256 + (ncell * 4 + 255) / 256 * 256;
    return G4_OK;
}

int g4_launch_pm(g4_ctx *ctx, const g4_tree *t, const g4_pm_params *pp, void *ws, size_t ws_bytes, int accumulate,
                 double *ax, double *ay, double *az, double *pot)
{
    const int ng = pp->ng, lg = ilog2(ng);
    size_t need = 0;
    if (g4_pm_layout_bytes(ng, &need)) return g4_set_err(ctx, G4_EINVAL, "ng must be a power of two in [8, 1024]");
    if (ws_bytes < need) return g4_set_err(ctx, G4_ENOMEM, "pm workspace too small");
    char *b = (char *)ws;
    const size_t ncell = (size_t)ng * ng * ng;
    float2 *tw = (float2 *)b;
    b += ((size_t)ng / 2 * 8 + 255) / 256 * 256;
    float2 *mesh = (float2 *)b;
    b += (ncell * 8 + 255) / 256 * 256;
    float *phi = (float *)b;
    hipStream_t s = ctx->stream;
    const int shift = 32 - lg;
    const float wscale = ldexpf(1.f, -shift);
    k_pm_twiddle<<<(ng / 2 + 255) / 256, 256, 0, s>>>(tw, ng);
    k_pm_clear<<<4096, 256, 0, s>>>(mesh, ncell);
    const int64_t n = t->n;
    const unsigned pblocks = (unsigned)std::min<int64_t>(8192, (n + 255) / 256);
    k_pm_deposit<<<pblocks, 256, 0, s>>>(t->parts, n, ng, shift, wscale, mesh);
    const int tl = std::min(ng, std::max(1, PM_TILE_CELLS / ng));
    const unsigned tiles = (unsigned)((size_t)ng * ng / tl);
    const size_t lds = ((size_t)tl * ng + ng / 2) * sizeof(float2);
    for (int axis = 2; axis >= 0; axis--)
        k_pm_fft<<<tiles, PM_THREADS, lds, s>>>(mesh, tw, ng, lg, tl, axis, -1.f, nullptr);
    k_pm_green<<<4096, 256, 0, s>>>(mesh, ng, lg, t->tp.box, pp->r_s, pp->G);
    for (int axis = 0; axis <= 2; axis++)
        k_pm_fft<<<tiles, PM_THREADS, lds, s>>>(mesh, tw, ng, lg, tl, axis, 1.f, axis == 2 ? phi : nullptr);
    const float inv_h = (float)(ng / t->tp.box);
    k_pm_interp<<<pblocks, 256, 0, s>>>(t->parts, t->perm1, n, phi, ng, lg, shift, wscale, inv_h, accumulate, ax,
                                        ay, az, pot);
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}
