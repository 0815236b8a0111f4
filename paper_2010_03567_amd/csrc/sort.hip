// sort.hip -- stable least-significant-digit radix sort of (key, value)
// pairs on gfx950: the ordering of the particles along the space-filling
// curve (Sec. "Geometry of the tree": particles sorted by their curve key) and
// the regrouping of a forest's particles by box.
//
// One pass per 8-bit digit, three steps each:
//   1. k_rs_hist:    every block counts the digits of its tile of RS_TILE keys
//                    (LDS atomics) into hist[digit][block];
//   2. k_rs_scan_*:  the table is scanned digit-major (one block per digit row,
//                    then the 256 row totals), so hist[d][b] becomes the first
//                    output slot of block b's keys with digit d;
//   3. k_rs_scatter: every block ranks its tile stably -- each wavefront
//                    takes its quarter in chunks of 64 keys in order; lanes
//                    with equal digits find each other with 8 ballots, rank by
//                    the lanes below them and by a per-wavefront running count
//                    -- then places the tile in LDS in digit order and writes
//                    it out so that consecutive threads write consecutive
//                    slots of each digit's run.
// Equal keys keep their input order (every rank follows chunk, wavefront and
// block order), which the tree build relies on for ties.
#include <algorithm>

#include "g4_internal.h"

#define RS_BITS 8
#define RS_BINS 256
#define RS_THREADS 256
#define RS_ITEMS 8                         // keys per lane and wavefront chunk count
#define RS_TILE (RS_THREADS * RS_ITEMS)    // 2048 keys per block
#define RS_WTILE (RS_TILE / 4)             // 512 keys per wavefront

__device__ __forceinline__ uint64_t rs_ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ uint32_t rs_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ void rs_wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <typename K>
__device__ __forceinline__ uint32_t rs_digit(K k, int shift)
{
    return (uint32_t)(k >> shift) & (RS_BINS - 1);
}

template <typename K>
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                        uint32_t *__restrict__ hist, uint32_t nb)
{
    __shared__ uint32_t h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + c * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[rs_digit(keys[i], shift)], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of one digit row hist[d][0..nb) in place; the row total to tot[d]
__global__ __launch_bounds__(RS_THREADS) void k_rs_scan_rows(uint32_t *__restrict__ hist, uint32_t nb,
                                                             uint32_t *__restrict__ tot)
{
    __shared__ uint32_t part[RS_THREADS];
    uint32_t *row = hist + (size_t)blockIdx.x * nb;
    const uint32_t per = (nb + RS_THREADS - 1) / RS_THREADS;
    const uint32_t lo = threadIdx.x * per, hi = min(nb, lo + per);
    uint32_t s = 0;
    for (uint32_t k = lo; k < hi; k++) s += row[k];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 256 partial sums
    for (int off = 1; off < RS_THREADS; off <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t k = lo; k < hi; k++) {
        const uint32_t v = row[k];
        row[k] = run;
        run += v;
    }
    if (threadIdx.x == RS_THREADS - 1) tot[blockIdx.x] = part[RS_THREADS - 1];
}

// exclusive scan of the 256 digit totals: the first output slot of each digit
__global__ __launch_bounds__(RS_BINS) void k_rs_scan_digits(const uint32_t *__restrict__ tot,
                                                            uint32_t *__restrict__ dbase)
{
    __shared__ uint32_t v[RS_BINS];
    const uint32_t own = tot[threadIdx.x];
    v[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < RS_BINS; off <<= 1) {
        const uint32_t a = threadIdx.x >= (unsigned)off ? v[threadIdx.x - off] : 0u;
        __syncthreads();
        v[threadIdx.x] += a;
        __syncthreads();
    }
    dbase[threadIdx.x] = v[threadIdx.x] - own;
}

template <typename K>
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                           K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                           int64_t n, int shift, const uint32_t *__restrict__ hist,
                                                           uint32_t nb, const uint32_t *__restrict__ dbase)
{
    __shared__ uint32_t cnt[4][RS_BINS];  // per wavefront: running count, then the wavefront's base
    __shared__ uint32_t bpre[RS_BINS];    // block-local first slot of each digit
    __shared__ uint32_t gpos[RS_BINS];    // global first slot of this block's run of each digit
    __shared__ K skey[RS_TILE];
    __shared__ uint32_t sval[RS_TILE];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < 4 * RS_BINS; k += RS_THREADS) (&cnt[0][0])[k] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_WTILE;
    K key[RS_ITEMS];
    uint32_t val[RS_ITEMS], rank[RS_ITEMS];
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + c * 64 + lane;
        const bool valid = i < n;
        key[c] = valid ? kin[i] : (K)0;
        val[c] = valid ? vin[i] : 0u;
        const uint32_t d = rs_digit(key[c], shift);
        // lanes of this chunk with the same digit
        uint64_t m = rs_ballot(valid);
#pragma unroll
        for (int b = 0; b < RS_BITS; b++) {
            const uint64_t bal = rs_ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = cnt[w][d];
        rank[c] = before + rs_below(m);
        rs_wave_fence();
        if (valid && (uint32_t)lane == (uint32_t)__builtin_ctzll(m)) cnt[w][d] = before + (uint32_t)__builtin_popcountll(m);
        rs_wave_fence();
    }
    __syncthreads();
    {
        // one thread per digit: wavefront bases, the block's digit prefix, the global start
        const int d = threadIdx.x;
        const uint32_t c0 = cnt[0][d], c1 = cnt[1][d], c2 = cnt[2][d], c3 = cnt[3][d];
        const uint32_t total = c0 + c1 + c2 + c3;
        cnt[0][d] = 0u;
        cnt[1][d] = c0;
        cnt[2][d] = c0 + c1;
        cnt[3][d] = c0 + c1 + c2;
        gpos[d] = hist[(size_t)d * nb + blockIdx.x] + dbase[d];
        bpre[d] = total;
    }
    __syncthreads();
    {
        // exclusive scan of the block's digit totals (in place, Hillis-Steele)
        const uint32_t own = bpre[threadIdx.x];
        for (int off = 1; off < RS_BINS; off <<= 1) {
            const uint32_t a = threadIdx.x >= (unsigned)off ? bpre[threadIdx.x - off] : 0u;
            __syncthreads();
            bpre[threadIdx.x] += a;
            __syncthreads();
        }
        bpre[threadIdx.x] -= own;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < RS_ITEMS; c++) {
        const int64_t i = base + c * 64 + lane;
        if (i < n) {
            const uint32_t d = rs_digit(key[c], shift);
            const uint32_t lp = bpre[d] + cnt[w][d] + rank[c];
            skey[lp] = key[c];
            sval[lp] = val[c];
        }
    }
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * RS_TILE;
    const uint32_t valid_n = (uint32_t)std::min<int64_t>(RS_TILE, n - b0);
    for (uint32_t j = threadIdx.x; j < valid_n; j += RS_THREADS) {
        const K k = skey[j];
        const uint32_t d = rs_digit(k, shift);
        const uint32_t o = gpos[d] + (j - bpre[d]);
        kout[o] = k;
        vout[o] = sval[j];
    }
}

size_t g4_radix_sort_temp_bytes(int64_t n)
{
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    return ((size_t)RS_BINS * (size_t)(nb > 0 ? nb : 1) * 4 + 2 * RS_BINS * 4 + 255) & ~(size_t)255;
}

template <typename K>
static int radix_sort(g4_ctx *ctx, K *k0, K *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo, int bit_hi,
                      void *temp, size_t temp_bytes, int *in_alt)
{
    *in_alt = 0;
    if (n <= 1 || bit_hi <= bit_lo) return G4_OK;
    if (n > 0xFFFFFFFFll) return g4_set_err(ctx, G4_EINVAL, "radix sort: more than 2^32 - 1 keys");
    if (temp_bytes < g4_radix_sort_temp_bytes(n)) return g4_set_err(ctx, G4_ENOMEM, "radix sort: temp too small");
    const uint32_t nb = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *tot = hist + (size_t)RS_BINS * nb;
    uint32_t *dbase = tot + RS_BINS;
    hipStream_t s = ctx->stream;
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int shift = bit_lo; shift < bit_hi; shift += RS_BITS) {
        k_rs_hist<K><<<nb, RS_THREADS, 0, s>>>(ki, n, shift, hist, nb);
        k_rs_scan_rows<<<RS_BINS, RS_THREADS, 0, s>>>(hist, nb, tot);
        k_rs_scan_digits<<<1, RS_BINS, 0, s>>>(tot, dbase);
        k_rs_scatter<K><<<nb, RS_THREADS, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nb, dbase);
        std::swap(ki, ko);
        std::swap(vi, vo);
        *in_alt ^= 1;
    }
    G4_HIP(ctx, hipGetLastError());
    return G4_OK;
}

int g4_radix_sort_u64(g4_ctx *ctx, uint64_t *k0, uint64_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt)
{
    return radix_sort<uint64_t>(ctx, k0, k1, v0, v1, n, bit_lo, bit_hi, temp, temp_bytes, in_alt);
}

int g4_radix_sort_u32(g4_ctx *ctx, uint32_t *k0, uint32_t *k1, uint32_t *v0, uint32_t *v1, int64_t n, int bit_lo,
                      int bit_hi, void *temp, size_t temp_bytes, int *in_alt)
{
    return radix_sort<uint32_t>(ctx, k0, k1, v0, v1, n, bit_lo, bit_hi, temp, temp_bytes, in_alt);
}
