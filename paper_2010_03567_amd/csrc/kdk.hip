// kdk.hip -- hierarchical time integration driver (gfx950 kernels, host
// recursion).
//
// Paper: Sec. "Hierarchical time integration".  A set P whose forces, sourced
// by P itself, are known is advanced over dt by
//     K_P^P(dt/2) K_F^F(-dt/2) E(H_F, dt/2) D_S(dt) E(H_F, dt/2) K_F^F(-dt/2) K_P^P(dt/2),
// where F are the particles whose criterion step sqrt(2 eta eps / |a|) is
// below dt (S the rest), E(H_F, dt/2) the same step applied to F alone with
// half the step size (F's forces sourced by F, computed to split it, start
// that recursion), and the step is a plain kick-drift-kick when F is empty.
// Every force is sourced by the set it acts on, so with the symmetric FMM
// the scheme conserves momentum to round-off.
//
// Device side: the active set of each level is an index list into the
// caller's arrays; its positions are gathered and mapped to integer
// coordinates, a tree over those particles alone is built in one shared
// workspace and the chosen solver gives their forces (in list order).
// Kicks, drifts, the split and the list compaction (stable: block counts,
// scan, ordered write) are kernels; the host holds the recursion and reads
// back only the size of each fast set.
#include <cmath>
#include <cstring>
#include <vector>

#include "g4_internal.h"

#define KDK_T 256
#define KDK_CHUNK 1024  // list elements per compaction block

__global__ void k_kdk_iota(uint32_t *__restrict__ idx, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = (uint32_t)i;
}

__global__ void k_kdk_gather(const double *__restrict__ pos, const float *__restrict__ mass,
                             const uint32_t *__restrict__ idx, int64_t m, double *__restrict__ sp,
                             float *__restrict__ sm)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = idx[j];
        sp[3 * j] = pos[3 * (size_t)i];
        sp[3 * j + 1] = pos[3 * (size_t)i + 1];
        sp[3 * j + 2] = pos[3 * (size_t)i + 2];
        sm[j] = mass[i];
    }
}

// vel[idx[j]] += c a[j]
__global__ void k_kdk_kick(double *__restrict__ vel, const uint32_t *__restrict__ idx, int64_t m,
                           const double *__restrict__ ax, const double *__restrict__ ay,
                           const double *__restrict__ az, double c)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const size_t i = idx[j];
        vel[3 * i] += c * ax[j];
        vel[3 * i + 1] += c * ay[j];
        vel[3 * i + 2] += c * az[j];
    }
}

// pos[idx[j]] += dt vel[idx[j]] for the list entries not flagged fast (all if
// fast is null); periodic boxes wrap into [origin, origin + box)
__global__ void k_kdk_drift(double *__restrict__ pos, const double *__restrict__ vel, const uint32_t *__restrict__ idx,
                            int64_t m, const uint8_t *__restrict__ fast, double dt, int periodic, double box,
                            double ox, double oy, double oz)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        if (fast && fast[j]) continue;
        const size_t i = idx[j];
        const double o[3] = {ox, oy, oz};
        for (int k = 0; k < 3; k++) {
            double x = pos[3 * i + k] + dt * vel[3 * i + k];
            if (periodic) {
                x -= box * floor((x - o[k]) / box);
                if (x >= o[k] + box) x -= box;  // rounding at the upper edge
            }
            pos[3 * i + k] = x;
        }
    }
}

// fast[j] = 1 iff the criterion step sqrt(2 eta eps / |a_j|) is below dt,
// i.e. |a_j| > thr = 2 eta eps / dt^2
__global__ void k_kdk_split(const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ az,
                            int64_t m, double thr, uint8_t *__restrict__ fast)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        const double a2 = ax[j] * ax[j] + ay[j] * ay[j] + az[j] * az[j];
        fast[j] = a2 > thr * thr ? 1 : 0;
    }
}

// stable compaction of the flagged list entries: counts per chunk, then an
// ordered write with each chunk's offset
__global__ __launch_bounds__(KDK_T) void k_kdk_count(const uint8_t *__restrict__ fast, int64_t m,
                                                     uint32_t *__restrict__ cnt)
{
    __shared__ uint32_t s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    uint32_t c = 0;
    const int64_t b0 = (int64_t)blockIdx.x * KDK_CHUNK;
    for (int k = threadIdx.x; k < KDK_CHUNK; k += KDK_T) c += (b0 + k < m && fast[b0 + k]) ? 1u : 0u;
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = s;
}

// exclusive scan of nb chunk counts in one block; total to cnt[nb]
__global__ __launch_bounds__(1024) void k_kdk_scan(uint32_t *__restrict__ cnt, uint32_t nb)
{
    __shared__ uint32_t part[1024];
    const uint32_t per = (nb + 1023) / 1024, lo = threadIdx.x * per, hi = min(nb, lo + per);
    uint32_t s = 0;
    for (uint32_t k = lo; k < hi; k++) s += cnt[k];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t k = lo; k < hi; k++) {
        const uint32_t v = cnt[k];
        cnt[k] = run;
        run += v;
    }
    if (threadIdx.x == 1023) cnt[nb] = part[1023];
}

__global__ __launch_bounds__(KDK_T) void k_kdk_compact(const uint8_t *__restrict__ fast, const uint32_t *__restrict__ idx,
                                                       int64_t m, const uint32_t *__restrict__ off,
                                                       uint32_t *__restrict__ out)
{
    __shared__ uint32_t wsum[KDK_T / 64];
    __shared__ uint32_t base;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) base = off[blockIdx.x];
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * KDK_CHUNK;
    for (int r = 0; r < KDK_CHUNK; r += KDK_T) {
        const int64_t j = b0 + r + threadIdx.x;
        const bool f = j < m && fast[j];
        const uint64_t bal = __builtin_amdgcn_ballot_w64(f);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (lane == 0) wsum[w] = (uint32_t)__builtin_popcountll(bal);
        __syncthreads();
        uint32_t pre = base;
        for (int k = 0; k < w; k++) pre += wsum[k];
        if (f) out[pre + below] = idx[j];
        __syncthreads();
        if (threadIdx.x == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

static inline unsigned kdk_grid(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (m + KDK_T - 1) / KDK_T)); }

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct KdkLayout {
    size_t idx[G4_KDK_LEVELS + 1], acc[G4_KDK_LEVELS + 1], fast[G4_KDK_LEVELS + 1];
    size_t subpos, submass, X, Y, Z, flag, cnt, tree, solver, total;
    size_t tree_bytes, solver_bytes;
};

static int kdk_layout(const g4_kdk_params *kp, int64_t n, KdkLayout *L)
{
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += al256(b);
        return o;
    };
    for (int k = 0; k <= kp->max_level && k <= G4_KDK_LEVELS; k++) {
        L->idx[k] = take((size_t)n * 4);
        L->acc[k] = k == 0 ? 0 : take((size_t)n * 24);  // level 0 uses the caller's arrays
        L->fast[k] = take((size_t)n);
    }
    L->subpos = take((size_t)n * 24);
    L->submass = take((size_t)n * 4);
    L->X = take((size_t)n * 4);
    L->Y = take((size_t)n * 4);
    L->Z = take((size_t)n * 4);
    L->flag = take(4);
    L->cnt = take(((size_t)(n + KDK_CHUNK - 1) / KDK_CHUNK + 2) * 4);
    size_t tb = 0;
    if (kp->solver != 0) {
        if (g4_workspace_bytes(&kp->tp, n, &tb) != G4_OK) return G4_EINVAL;
    }
    L->tree_bytes = tb;
    L->tree = take(tb);
    size_t sb = 0;
    if (kp->solver == 2) {
        WsLayout W;
        if (g4_layout(&kp->tp, n, &W) != G4_OK) return G4_EINVAL;
        g4_tree t;
        std::memset(&t, 0, sizeof(t));
        t.n = n;
        t.cap = W.cap;
        if (g4_fmm_layout_bytes(&t, &kp->fp, 2.0, &sb) != G4_OK) return G4_EINVAL;
    }
    L->solver_bytes = sb;
    L->solver = take(sb);
    L->total = off;
    return G4_OK;
}

int g4_kdk_layout_bytes(const g4_kdk_params *kp, int64_t n, size_t *bytes)
{
    KdkLayout L;
    const int st = kdk_layout(kp, n, &L);
    if (st == G4_OK) *bytes = L.total;
    return st;
}

namespace {

struct Kdk {
    g4_ctx *ctx;
    const g4_kdk_params *kp;
    int64_t n;
    double *pos, *vel;
    const float *mass;
    char *ws;
    KdkLayout L;
    double *ax0, *ay0, *az0;
    g4_kdk_stats *stats;

    uint32_t *idx(int k) { return (uint32_t *)(ws + L.idx[k]); }
    uint8_t *fast(int k) { return (uint8_t *)(ws + L.fast[k]); }
    void acc(int k, double **a, double **b, double **c)
    {
        if (k == 0) {
            *a = ax0, *b = ay0, *c = az0;
            return;
        }
        double *base = (double *)(ws + L.acc[k]);
        *a = base, *b = base + n, *c = base + 2 * n;
    }

    // forces on the m particles of list k sourced by the same particles, into acc(k)
    int force(int k, int64_t m)
    {
        if (m == 0) return G4_OK;
        hipStream_t s = ctx->stream;
        double *sp = (double *)(ws + L.subpos);
        float *sm = (float *)(ws + L.submass);
        uint32_t *X = (uint32_t *)(ws + L.X), *Y = (uint32_t *)(ws + L.Y), *Z = (uint32_t *)(ws + L.Z);
        k_kdk_gather<<<kdk_grid(m), KDK_T, 0, s>>>(pos, mass, idx(k), m, sp, sm);
        G4_HIP(ctx, hipGetLastError());
        int st = g4_launch_quantize(ctx, sp, m, &kp->tp, X, Y, Z, (int32_t *)(ws + L.flag));
        if (st) return st;
        g4_particles p{m, X, Y, Z, sm};
        double *a, *b, *c;
        acc(k, &a, &b, &c);
        if (kp->solver == 0) {
            st = g4_direct_force(ctx, &p, &kp->tp, &kp->wp, 0, nullptr, m, a, b, c, nullptr);
        } else {
            g4_tree *t = nullptr;
            st = g4_build_tree(ctx, &p, &kp->tp, ws + L.tree, L.tree_bytes, &t);
            if (st) return st;
            st = g4_compute_multipoles(ctx, t, kp->solver == 2 ? 3 : kp->wp.order);
            if (!st) {
                if (kp->solver == 1) st = g4_tree_force(ctx, t, &kp->wp, a, b, c, nullptr, nullptr, nullptr, nullptr);
                else st = g4_fmm_force(ctx, t, &kp->fp, 2.0, ws + L.solver, L.solver_bytes, a, b, c, nullptr, nullptr);
            }
            g4_tree_free(ctx, t);
            if (st) return st;
        }
        if (st) return st;
        stats->force_evals += (uint64_t)m;
        stats->force_calls++;
        if (k < 32) stats->evals_per_level[k] += (uint64_t)m;
        return G4_OK;
    }

    void kick(int k, int64_t m, double c)
    {
        if (m == 0) return;
        double *a, *b, *cc;
        acc(k, &a, &b, &cc);
        k_kdk_kick<<<kdk_grid(m), KDK_T, 0, ctx->stream>>>(vel, idx(k), m, a, b, cc, c);
    }

    void drift(int k, int64_t m, const uint8_t *skip_fast, double dt)
    {
        if (m == 0) return;
        const g4_tree_params &tp = kp->tp;
        k_kdk_drift<<<kdk_grid(m), KDK_T, 0, ctx->stream>>>(pos, vel, idx(k), m, skip_fast, dt, tp.periodic, tp.box,
                                                             tp.origin[0], tp.origin[1], tp.origin[2]);
    }

    // list k + 1 = the fast entries of list k; returns their number
    int split(int k, int64_t m, double dt, int64_t *mf)
    {
        hipStream_t s = ctx->stream;
        double *a, *b, *c;
        acc(k, &a, &b, &c);
        const double thr = 2.0 * kp->eta * kp->eps / (dt * dt);
        k_kdk_split<<<kdk_grid(m), KDK_T, 0, s>>>(a, b, c, m, thr, fast(k));
        const uint32_t nb = (uint32_t)((m + KDK_CHUNK - 1) / KDK_CHUNK);
        uint32_t *cnt = (uint32_t *)(ws + L.cnt);
        k_kdk_count<<<nb, KDK_T, 0, s>>>(fast(k), m, cnt);
        k_kdk_scan<<<1, 1024, 0, s>>>(cnt, nb);
        k_kdk_compact<<<nb, KDK_T, 0, s>>>(fast(k), idx(k), m, cnt, idx(k + 1));
        G4_HIP(ctx, hipGetLastError());
        uint32_t h = 0;
        G4_HIP(ctx, hipMemcpyAsync(&h, cnt + nb, 4, hipMemcpyDeviceToHost, s));
        G4_HIP(ctx, hipStreamSynchronize(s));
        *mf = h;
        return G4_OK;
    }

    // advance list k (m entries, forces in acc(k)) by dt; forces at the end in acc(k)
    int step(int k, int64_t m, double dt)
    {
        if (m == 0) return G4_OK;
        int64_t mf = 0;
        if (k < kp->max_level) {
            const int st = split(k, m, dt, &mf);
            if (st) return st;
        }
        if ((uint32_t)k > stats->deepest_level) stats->deepest_level = (uint32_t)k;
        kick(k, m, 0.5 * dt);                       // K_P^P(dt/2)
        if (mf == 0) {
            drift(k, m, nullptr, dt);               // D_P(dt)
            int st = force(k, m);
            if (st) return st;
            kick(k, m, 0.5 * dt);                   // K_P^P(dt/2)
            return G4_OK;
        }
        int st = force(k + 1, mf);
        if (st) return st;
        kick(k + 1, mf, -0.5 * dt);                 // K_F^F(-dt/2)
        if ((st = step(k + 1, mf, 0.5 * dt))) return st;
        drift(k, m, fast(k), dt);                   // D_S(dt)
        if ((st = step(k + 1, mf, 0.5 * dt))) return st;
        kick(k + 1, mf, -0.5 * dt);                 // K_F^F(-dt/2)
        if ((st = force(k, m))) return st;
        kick(k, m, 0.5 * dt);                       // K_P^P(dt/2)
        return G4_OK;
    }
};

}  // namespace

int g4_launch_kdk(g4_ctx *ctx, const g4_kdk_params *kp, int64_t n, double *pos, double *vel, const float *mass,
                  double dt, double *ax, double *ay, double *az, int have_acc, void *ws, size_t ws_bytes,
                  g4_kdk_stats *stats)
{
    Kdk K;
    K.ctx = ctx;
    K.kp = kp;
    K.n = n;
    K.pos = pos;
    K.vel = vel;
    K.mass = mass;
    K.ws = (char *)ws;
    K.ax0 = ax;
    K.ay0 = ay;
    K.az0 = az;
    g4_kdk_stats local;
    K.stats = stats ? stats : &local;
    std::memset(K.stats, 0, sizeof(g4_kdk_stats));
    int st = kdk_layout(kp, n, &K.L);
    if (st) return g4_set_err(ctx, st, "kdk workspace layout failed");
    if (ws_bytes < K.L.total) return g4_set_err(ctx, G4_ENOMEM, "kdk workspace too small");
    k_kdk_iota<<<kdk_grid(n), KDK_T, 0, ctx->stream>>>(K.idx(0), n);
    G4_HIP(ctx, hipGetLastError());
    if (!have_acc && (st = K.force(0, n))) return st;
    st = K.step(0, n, dt);
    if (st) return st;
    G4_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return G4_OK;
}
