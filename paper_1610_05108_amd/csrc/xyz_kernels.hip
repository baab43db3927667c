// xyz_kernels.hip -- gfx950 kernels of the xyz interaction search.
//
// Data layout in HBM (per resident X):
//   XC [p][W32p] u32  column-major bits, bit (i % 32) of word i / 32 = [X_ij = -1] (sign of real X),
//                     W32p = ceil(n/32) rounded up to a multiple of 4 (16-byte rows), zero padded.
//   XR [n][P64]   u64 row-major bits, bit (j % 64) of word j / 64 = [X_ij = -1].
//   XF [p][nF]    f32 values of real X, nF = n rounded up to 32, zero padded.
// Per search: yb [W32p] bits of Y (sign for real Y), yd [nF] values of Y.
//
// Paper mapping (Thanei, Meinshausen & Shah):
//   k_pack_*       term (i) of eq. (8), forming the data Z is reduced to one XOR per word;
//   k_sample       eq. (6) with tau = 0 (minimal subsampling, Section 2.1), |Y|-weighted for real Y (Section 3.1);
//   k_hash         Algorithm 2's projection x = X^T R, z = Z^T R: with tau = 0 a column's projection is
//                  determined by its entries on the sampled rows, packed here into an m-bit key;
//                  z_k's key equals x_k's key XOR the bits of Y on the sampled rows (Z = Y o X);
//   k_bucket       the equal-pairs search of Section 2.2 (Figure 2), as a counting sort of the p keys;
//   k_tiles        E_l as a union of Cartesian products of a bucket b and its partner b ^ c;
//   k_verify_*     the strength check of Algorithm 2 / eq. (1), term (iv) of eq. (8);
//   k_rs_*, dedup  "add to I": the union over repetitions.
#include "xyz_internal.h"

#include <algorithm>
#include <cstring>
#include <type_traits>

namespace xyz {

#define XYZ_DEV __device__ __forceinline__

XYZ_DEV unsigned lane_id() { return threadIdx.x & 63u; }

XYZ_DEV unsigned long long lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// v_bcnt_u32_b32 with accumulate: popcount(x) + acc in one VALU op.
XYZ_DEV uint32_t bcnt_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

XYZ_DEV uint64_t cdiv_u64(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every outstanding global load (its fence covers all address
// spaces), which would drain the prefetches issued ahead of the barrier.
XYZ_DEV void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exclusive scan of one value per thread over a block of NT threads.
template <int NT>
XYZ_DEV unsigned long long block_scan_excl(unsigned long long v, unsigned long long *shm, unsigned long long *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned long long y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) shm[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long acc = 0;
        for (int i = 0; i < NT / 64; ++i) {
            unsigned long long t = shm[i];
            shm[i] = acc;
            acc += t;
        }
        shm[NT / 64] = acc;
    }
    __syncthreads();
    unsigned long long res = shm[w] + x - v;
    *total = shm[NT / 64];
    __syncthreads();
    return res;
}

template <int NT>
XYZ_DEV unsigned long long block_sum(unsigned long long v, unsigned long long *shm)
{
    unsigned long long t;
    block_scan_excl<NT>(v, shm, &t);
    return t;
}

template <int NT>
XYZ_DEV unsigned block_max(unsigned v, unsigned *shm)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (unsigned)__shfl_xor(v, d, 64));
    if (lane == 0) shm[w] = v;
    __syncthreads();
    unsigned r = 0;
    for (int i = 0; i < NT / 64; ++i) r = max(r, shm[i]);
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- packing --

// One wave per column: each lane reads one entry of 64 consecutive rows, a
// ballot forms the 64-bit word; lane c keeps word c of a group of 64 words.
__global__ __launch_bounds__(256) void k_pack_x_i8(const int8_t *__restrict__ X, int64_t ld, int64_t n, int64_t p,
                                                   int W32p, uint32_t *__restrict__ XC, int *__restrict__ err)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= p) return;
    const unsigned lane = lane_id();
    const int W64p = W32p / 2;
    const int8_t *col = X + j * ld;
    uint64_t *dst = reinterpret_cast<uint64_t *>(XC + j * (int64_t)W32p);
    bool bad = false;
    for (int g = 0; g < W64p; g += 64) {
        uint64_t mine = 0;
        const int gend = min(W64p, g + 64);
        for (int c = g; c < gend; ++c) {
            const int64_t i = (int64_t)c * 64 + lane;
            int8_t v = 1;
            if (i < n) {
                v = col[i];
                bad |= (v != 1 && v != -1);
            }
            unsigned long long w = __ballot(v == -1);
            if ((int)lane == c - g) mine = w;
        }
        if (g + (int)lane < W64p) dst[g + lane] = mine;
    }
    if (__ballot(bad) && lane == 0) atomicOr(err, 1);
}

// Row-major int8 X: one wave per (row i, group g of 64 columns); lane l reads
// entry (i, 64g + l) (64 contiguous bytes per wave) and a ballot forms the
// row-major word XR[i][g] directly.  Columns past p read as +1 (bit 0).
__global__ __launch_bounds__(256) void k_pack_x_i8_rows(const int8_t *__restrict__ X, int64_t ld, int64_t n,
                                                        int64_t p, uint64_t *__restrict__ XR, int64_t P64,
                                                        int *__restrict__ err)
{
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= n * P64) return;
    const int64_t i = wave / P64, g = wave % P64;
    const unsigned lane = lane_id();
    const int64_t j = g * 64 + lane;
    int8_t v = 1;
    if (j < p) v = X[i * ld + j];
    const bool bad = v != 1 && v != -1;
    const unsigned long long w = __ballot(v == -1);
    if (lane == 0) XR[i * P64 + g] = w;
    if (__ballot(bad) && lane == 0) atomicOr(err, 1);
}

// Bit transpose XR -> XC (the inverse of k_transpose).  One wave takes 64
// columns (row word g) and 128 rows (quad q of every column): lane l loads the
// words of rows 128q + l and 128q + 64 + l; 128 ballots give each column's 128
// bits, and lane c writes the quad of column 64g + c as one 16-byte store.
// Rows past n read as 0.
__global__ __launch_bounds__(256) void k_transpose_rc(const uint64_t *__restrict__ XR, int64_t n, int64_t p,
                                                      int64_t P64, int W32p, uint32_t *__restrict__ XC)
{
    const int W4 = W32p / 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= P64 * W4) return;
    const int64_t g = wave / W4;
    const int q = (int)(wave % W4);
    const unsigned lane = lane_id();
    const int64_t r0 = (int64_t)q * 128 + lane;
    const uint64_t lo = r0 < n ? XR[r0 * P64 + g] : 0ull;
    const uint64_t hi = r0 + 64 < n ? XR[(r0 + 64) * P64 + g] : 0ull;
    uint4 out = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        const unsigned long long a = __ballot((lo >> c) & 1ull);   // rows 128q .. 128q + 63 of column 64g + c
        const unsigned long long b = __ballot((hi >> c) & 1ull);   // rows 128q + 64 .. 128q + 127
        if ((int)lane == c) out = make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    }
    const int64_t j = g * 64 + lane;
    if (j < p) reinterpret_cast<uint4 *>(XC + j * (int64_t)W32p)[q] = out;
}

__global__ __launch_bounds__(256) void k_pack_x_f32(const float *__restrict__ X, int64_t ld, int64_t n, int64_t p,
                                                    int W32p, uint32_t *__restrict__ XC, float *__restrict__ XF,
                                                    int64_t nF, int *__restrict__ err)
{
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= p) return;
    const unsigned lane = lane_id();
    const int W64p = W32p / 2;
    const float *col = X + j * ld;
    uint64_t *dst = reinterpret_cast<uint64_t *>(XC + j * (int64_t)W32p);
    float *fdst = XF + j * nF;
    bool bad = false;
    for (int g = 0; g < W64p; g += 64) {
        uint64_t mine = 0;
        const int gend = min(W64p, g + 64);
        for (int c = g; c < gend; ++c) {
            const int64_t i = (int64_t)c * 64 + lane;
            float v = 0.0f;
            if (i < n) {
                v = col[i];
                bad |= !isfinite(v);
            }
            if (i < nF) fdst[i] = v;
            unsigned long long w = __ballot(v < 0.0f);
            if ((int)lane == c - g) mine = w;
        }
        if (g + (int)lane < W64p) dst[g + lane] = mine;
    }
    for (int64_t i = (int64_t)W64p * 64 + lane; i < nF; i += 64) fdst[i] = 0.0f;
    if (__ballot(bad) && lane == 0) atomicOr(err, 2);
}

__global__ __launch_bounds__(256) void k_pack_x_bits(const uint64_t *__restrict__ X, int64_t ld, int64_t n,
                                                     int64_t p, int W32p, uint32_t *__restrict__ XC)
{
    const int W64p = W32p / 2;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= p * W64p) return;
    const int64_t j = gid / W64p;
    const int w = (int)(gid % W64p);
    const int64_t nw = (n + 63) / 64;
    uint64_t v = 0;
    if (w < nw) {
        v = X[j * ld + w];
        const int64_t tail = n - (int64_t)w * 64;
        if (tail < 64) v &= (1ull << tail) - 1ull;
    }
    reinterpret_cast<uint64_t *>(XC)[j * W64p + w] = v;
}

// Bit transpose XC -> XR.  One wave takes 64 columns and 4 words (128 rows):
// lane l holds 4 words of column 64g + l; 128 ballots produce the 64-column
// words of 128 rows; lane l writes rows l and l + 64.
__global__ __launch_bounds__(256) void k_transpose(const uint32_t *__restrict__ XC, int64_t n, int64_t p, int W32p,
                                                   uint64_t *__restrict__ XR, int64_t P64)
{
    const int W4 = W32p / 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ngroups = (p + 63) / 64;
    if (wave >= ngroups * W4) return;
    const int64_t g = wave / W4;
    const int q = (int)(wave % W4);
    const unsigned lane = lane_id();
    const int64_t j = g * 64 + lane;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (j < p) v = reinterpret_cast<const uint4 *>(XC + j * (int64_t)W32p)[q];
    uint64_t lo = 0, hi = 0;
    const uint32_t words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < 32; ++b) {
            unsigned long long m = __ballot((words[e] >> b) & 1u);
            const int row = e * 32 + b;
            if (row < 64) {
                if ((int)lane == row) lo = m;
            } else {
                if ((int)lane == row - 64) hi = m;
            }
        }
    }
    const int64_t r0 = (int64_t)q * 128 + lane;
    if (r0 < n) XR[r0 * P64 + g] = lo;
    if (r0 + 64 < n) XR[(r0 + 64) * P64 + g] = hi;
}

__global__ __launch_bounds__(256) void k_pack_y(const void *__restrict__ Y, int yfmt, int64_t n, int W32p,
                                                uint32_t *__restrict__ yb, double *__restrict__ yd, int64_t nF,
                                                int *__restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)W32p * 32;
    const int64_t lim = nb > nF ? nb : nF;
    if (i >= lim) return;
    double v = 0.0;
    bool bad = false;
    if (i < n) {
        if (yfmt == 0) {
            const int8_t y = static_cast<const int8_t *>(Y)[i];
            bad = (y != 1 && y != -1);
            v = (double)y;
        } else if (yfmt == 1) {
            v = (double)static_cast<const float *>(Y)[i];
            bad = !isfinite(v);
        } else {
            v = static_cast<const double *>(Y)[i];
            bad = !isfinite(v);
        }
    }
    if (i < nF) yd[i] = v;
    const unsigned long long m = __ballot(v < 0.0);
    const unsigned lane = lane_id();
    if (i < nb && (lane & 31) == 0) yb[i >> 5] = (lane == 0) ? (uint32_t)m : (uint32_t)(m >> 32);
    if (__ballot(bad) && lane == 0) atomicOr(err, 4);
}

// Running sum of |Y_i| in binary64, in the order i = 0, 1, ..., n-1.
__global__ void k_cdf(const double *__restrict__ yd, int64_t n, double *__restrict__ cdf, int64_t *__restrict__ last,
                      int *__restrict__ err)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    int64_t lst = -1;
    for (int64_t i = 0; i < n; ++i) {
        const double y = yd[i];
        acc = __dadd_rn(acc, fabs(y));
        cdf[i] = acc;
        if (y != 0.0) lst = i;
    }
    *last = lst;
    if (!(acc > 0.0)) atomicOr(err, 8);
}

// ------------------------------------------------------ unbiased transform --
//
// Section 3.2, Proposition 4: with rows scaled by nu_i = max_j |X_ij| (and Y_i by
// nu_i^2), a sampled entry becomes +1 with probability (1 + X_ij / nu_i) / 2,
// independently for every repetition, draw and column.

// nu_i as float bits: non-negative floats order like their bit patterns, so an
// integer atomic max over |x| bits is the float max.  Entries capped at +-cap
// (+inf: none) count as capped.  Thread (i, column slice).
__global__ __launch_bounds__(256) void k_row_absmax(const float *__restrict__ XF, int64_t nF, int64_t n, int64_t p,
                                                    int64_t cols_per, uint32_t capb, uint32_t *__restrict__ nu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j0 = (int64_t)blockIdx.y * cols_per, j1 = min(p, j0 + cols_per);
    uint32_t mb = 0;
    for (int64_t j = j0; j < j1; ++j) mb = max(mb, __float_as_uint(XF[j * nF + i]) & 0x7FFFFFFFu);
    mb = min(mb, capb);
    if (mb) atomicMax(&nu[i], mb);
}

// Running sum of the row weights |Y_i| * (nu_i * nu_i), binary64, i = 0, 1, ..., n-1.
__global__ void k_cdf_unbiased(const double *__restrict__ yd, const uint32_t *__restrict__ nu, int64_t n,
                               double *__restrict__ cdf, int64_t *__restrict__ last, int *__restrict__ err)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    int64_t lst = -1;
    for (int64_t i = 0; i < n; ++i) {
        const double v = (double)__uint_as_float(nu[i]);
        const double w = __dmul_rn(fabs(yd[i]), __dmul_rn(v, v));
        acc = __dadd_rn(acc, w);
        cdf[i] = acc;
        if (w != 0.0) lst = i;
    }
    *last = lst;
    if (!(acc > 0.0)) atomicOr(err, 8);
}

// ----------------------------------------------------------------- sampler --

// SplitMix64 (Steele, Lea & Flood 2014): output number k of the generator seeded with `seed`.
XYZ_DEV uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Row draw t of repetition l is output 1 + l * 2^16 + t.  Uniform rows map u to
// floor(u n / 2^64); weighted rows take the first i with cdf[i] > (u >> 11) 2^-53 cdf[n-1].
__global__ __launch_bounds__(256) void k_sample(uint64_t seed, int64_t rep0, int nrep, int m, int64_t n,
                                                int weighted, const double *__restrict__ cdf,
                                                const int64_t *__restrict__ last, int32_t *__restrict__ rows)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nrep * m) return;
    const int64_t r = gid / m;
    const int t = (int)(gid % m);
    const uint64_t l = (uint64_t)(rep0 + r);
    const uint64_t u = splitmix64_at(seed, 1ull + l * 65536ull + (uint64_t)t);
    int64_t row;
    if (!weighted) {
        row = (int64_t)__umul64hi(u, (uint64_t)n);
    } else {
        const double v = __dmul_rn((double)(u >> 11) * 0x1p-53, cdf[n - 1]);
        int64_t lo = 0, hi = n;   // first i in [lo, hi) with cdf[i] > v; n if none
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (cdf[mid] > v) hi = mid; else lo = mid + 1;
        }
        row = lo < n ? lo : *last;
    }
    rows[gid] = (int32_t)row;
}

__global__ __launch_bounds__(256) void k_cmask(const int32_t *__restrict__ rows, int nrep, int m, int nys,
                                               const uint32_t *__restrict__ yb, int yb_stride,
                                               RepInfo *__restrict__ info)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nrep * nys) return;
    const int64_t r = gid / nys;
    const int y = (int)(gid % nys);
    const uint32_t *yy = yb + (int64_t)y * yb_stride;
    unsigned long long c = 0;
    for (int t = 0; t < m; ++t) {
        const int32_t i = rows[r * m + t];
        c |= (unsigned long long)((yy[i >> 5] >> (i & 31)) & 1u) << t;
    }
    info[gid].cmask = c;
}

// ------------------------------------------------------------------- hash --

// key_j = sum_t bit(X_{r_t, j}) << t.  Four consecutive columns per thread, so
// that a workgroup reads whole 128-byte lines of every sampled row (1024
// columns) and writes its keys as 16-byte stores.
constexpr int HASH_COLS = 4;

__global__ __launch_bounds__(256) void k_hash(const uint64_t *__restrict__ XR, int64_t P64, int64_t p, int m,
                                              const int32_t *__restrict__ rows, uint32_t *__restrict__ keys)
{
    const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * HASH_COLS;
    const int r = blockIdx.y;
    __shared__ int32_t rr[32];
    if (threadIdx.x < (unsigned)m) rr[threadIdx.x] = rows[(int64_t)r * m + threadIdx.x];
    __syncthreads();
    if (j0 >= p) return;
    const int64_t w = j0 >> 6;
    const unsigned sh = (unsigned)(j0 & 63);          // the four columns share one word
    uint32_t k[HASH_COLS] = {0, 0, 0, 0};
    for (int t = 0; t < m; ++t) {
        const uint32_t nib = (uint32_t)(XR[(int64_t)rr[t] * P64 + w] >> sh);
#pragma unroll
        for (int i = 0; i < HASH_COLS; ++i) k[i] |= ((nib >> i) & 1u) << t;
    }
    uint32_t *kr = keys + (int64_t)r * p;
    if ((p & 3) == 0) {
        *reinterpret_cast<uint4 *>(kr + j0) = make_uint4(k[0], k[1], k[2], k[3]);
    } else {
#pragma unroll
        for (int i = 0; i < HASH_COLS; ++i)
            if (j0 + i < p) kr[j0 + i] = k[i];
    }
}

// Keys under the unbiased transform: thread (column j, repetition r); bit t is
// [X~ = -1] for sampled row r_t.  Draw t of repetition l seeds a SplitMix64
// stream (output 1 + l*2^16 + t of the generator seeded with seed ^ UNB_STREAM);
// column j takes the top 24 bits u of the stream's output 1 + j, and X~ = +1
// exactly when (u * 2) * nu < (nu + x) * 2^24 in binary64 (u / 2^24 < (1 + x/nu) / 2
// without a division; every product is exact), or u < 2^23 on an all-zero row.
constexpr uint64_t UNB_STREAM = 0x2545F4914F6CDD1Dull;

__global__ __launch_bounds__(256) void k_hash_unbiased(const float *__restrict__ XF, int64_t nF, int64_t p, int m,
                                                       const int32_t *__restrict__ rows,
                                                       const uint32_t *__restrict__ nu, float cap, uint64_t seed,
                                                       int64_t rep0, uint32_t *__restrict__ keys)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    __shared__ int32_t rr[32];
    __shared__ float nus[32];
    __shared__ uint64_t ss[32];
    if (threadIdx.x < (unsigned)m) {
        const int t = (int)threadIdx.x;
        const int32_t row = rows[(int64_t)r * m + t];
        rr[t] = row;
        nus[t] = __uint_as_float(nu[row]);
        ss[t] = splitmix64_at(seed ^ UNB_STREAM, 1ull + (uint64_t)(rep0 + r) * 65536ull + (uint64_t)t);
    }
    __syncthreads();
    if (j >= p) return;
    uint32_t key = 0;
    for (int t = 0; t < m; ++t) {
        const double x = (double)fminf(fmaxf(XF[j * nF + rr[t]], -cap), cap);
        const double v = (double)nus[t];
        const uint64_t u = splitmix64_at(ss[t], 1ull + (uint64_t)j) >> 40;
        const bool plus = v > 0.0 ? __dmul_rn(__dmul_rn((double)u, 2.0), v) < __dmul_rn(__dadd_rn(v, x), 16777216.0)
                                  : u < 8388608ull;
        key |= (plus ? 0u : 1u) << t;
    }
    keys[(int64_t)r * p + j] = key;
}

// ----------------------------------------------------------------- bucket --

// Bucket pair (b, b2) of a repetition: b < b2 -> all pairs of the two buckets;
// b == b2 (partner mask 0) -> pairs inside the bucket.  Returns the candidate
// count and sorts the product into one of three tile lists:
//   kind 1: one TILE x TILE tile with at most SMALL_TILE_PAIRS pairs (small list),
//   kind 2: T tiles of TILE x TILE (popcount list),
//   kind 3: T tiles of MTILE x MTILE for the matrix cores (mfma = 1, +-1 data with
//           n < 2^24: both sides at least MTILE_MIN columns, and a product within
//           MTILE x MTILE_WIDE is one tile; mfma = 2, real data: both sides at least
//           MTILE_MIN_REAL),
//   kind 4: T block pairs of at most BIG_TILE x BIG_TILE staged through LDS (mfma = 1: a
//           larger product whose shorter side has at least BIG_MIN_SHORT columns, or a
//           bucket's own pairs past MTILE columns).
// A product of two different buckets that is one matrix-core tile (+-1 data): one side of
// at most MTILE columns, the other of at most MTILE_WIDE.
XYZ_DEV bool mfma_single(uint32_t a, uint32_t a2, int mfma)
{
    return mfma == 1 && ((a <= (uint32_t)MTILE && a2 <= MTILE_WIDE) || (a <= MTILE_WIDE && a2 <= (uint32_t)MTILE));
}

// Thin strips of a big product of two buckets: a side past BIG_TILE columns whose remainder
// after its full blocks is shorter than THIN_MAX leaves that remainder to matrix-core tiles
// (MTILE wide) instead of block pairs of its own, which would keep most of a workgroup idle.
constexpr uint32_t THIN_MAX = 64;

XYZ_DEV uint32_t thin_cols(uint32_t s)
{
    const uint32_t r = s % (uint32_t)BIG_TILE;
    return (s > (uint32_t)BIG_TILE && r < THIN_MAX) ? r : 0u;
}

// Matrix-core tiles of the thin strips of a big product (a x a2): A's remainder against all of
// B, then B's remainder against A's blocks.
XYZ_DEV unsigned long long thin_tiles(uint32_t a, uint32_t a2)
{
    const uint32_t ra = thin_cols(a), rb = thin_cols(a2);
    return (ra ? cdiv_u64(a2, MTILE) : 0) + (rb ? cdiv_u64(a - ra, MTILE) : 0);
}

// Candidate pairs of a big product that its block pairs hold.
XYZ_DEV unsigned long long big_block_pairs(uint32_t a, uint32_t a2)
{
    return (unsigned long long)(a - thin_cols(a)) * (a2 - thin_cols(a2));
}

XYZ_DEV unsigned long long product_tiles(uint32_t b, uint32_t b2, uint32_t a, uint32_t a2, int mfma, int &kind,
                                         unsigned long long &T)
{
    kind = 0;
    T = 0;
    if (b < b2) {
        const unsigned long long c = (unsigned long long)a * a2;
        if (c == 0) return 0;
        const uint32_t mmin = mfma == 2 ? MTILE_MIN_REAL : MTILE_MIN;
        if (mfma == 1 && min(a, a2) >= BIG_MIN_SHORT && !mfma_single(a, a2, mfma)) {
            kind = 4;      // block pairs here; the thin strips' tiles (thin_tiles) join the matrix-core list
            T = cdiv_u64(a - thin_cols(a), BIG_TILE) * cdiv_u64(a2 - thin_cols(a2), BIG_TILE);
        } else if (mfma && a >= mmin && a2 >= mmin) {
            kind = 3;
            T = mfma_single(a, a2, mfma) ? 1 : cdiv_u64(a, MTILE) * cdiv_u64(a2, MTILE);
        } else if (a <= (uint32_t)TILE && a2 <= (uint32_t)TILE && c <= SMALL_TILE_PAIRS) {
            kind = 1;
            T = 1;
        } else {
            kind = 2;
            T = cdiv_u64(a, TILE) * cdiv_u64(a2, TILE);
        }
        return c;
    }
    if (b == b2 && a >= 2) {
        const unsigned long long c = (unsigned long long)a * (a - 1) / 2;
        if (mfma == 1 && a > (uint32_t)MTILE) {
            kind = 4;
            const unsigned long long n = cdiv_u64(a, BIG_TILE);
            T = n * (n + 1) / 2;
        } else if (mfma && a >= (mfma == 2 ? MTILE_MIN_REAL : MTILE_MIN_DIAG)) {
            kind = 3;
            const unsigned long long n = cdiv_u64(a, MTILE);
            T = n * (n + 1) / 2;
        } else if (a <= (uint32_t)TILE && c <= SMALL_TILE_PAIRS) {
            kind = 1;
            T = 1;
        } else {
            kind = 2;
            const unsigned long long n = cdiv_u64(a, TILE);
            T = n * (n + 1) / 2;
        }
        return c;
    }
    return 0;
}

constexpr int BKU = 8;       // keys per thread and round in k_bucket
constexpr size_t BUCKET_LDS = (size_t)148 << 10;   // dynamic LDS of k_bucket's chunked scatter (of 160 KiB)

// k_bucket's scatter in chunks of `ch` keys (a multiple of 1024 BKU, 0: direct scatter):
// the chunk is counting-sorted by key in LDS first, so that the ids of one bucket leave
// as one contiguous run instead of one 4-byte write each.
__global__ __launch_bounds__(1024) void k_bucket(const uint32_t *__restrict__ keys, int64_t p, int m, int nys,
                                                 RepInfo *__restrict__ info, int two_sided, int mfma,
                                                 uint32_t *__restrict__ offs, uint32_t *__restrict__ perm, int ch)
{
    extern __shared__ uint32_t cnt[];
    __shared__ unsigned long long shm[17];
    __shared__ unsigned shmax[16];
    const int nb = 1 << m;
    const uint32_t mask = (uint32_t)(nb - 1);
    const int r = blockIdx.x;
    const uint32_t *kr = keys + (int64_t)r * p;
    for (int b = threadIdx.x; b < nb; b += 1024) cnt[b] = 0;
    __syncthreads();
    // the key loads of BKU iterations go out together (the loop is latency-bound otherwise)
    for (int64_t j0 = threadIdx.x; j0 < p; j0 += 1024 * BKU) {
        uint32_t kv[BKU];
#pragma unroll
        for (int u = 0; u < BKU; ++u) kv[u] = j0 + u * 1024 < p ? kr[j0 + u * 1024] : ~0u;
#pragma unroll
        for (int u = 0; u < BKU; ++u)
            if (kv[u] != ~0u) atomicAdd(&cnt[kv[u]], 1u);
    }
    __syncthreads();
    for (int y = 0; y < nys; ++y) {
        RepInfo *inf = info + (int64_t)r * nys + y;
        const uint32_t c = (uint32_t)inf->cmask & mask;
        const uint32_t cn = (~c) & mask;
        unsigned long long cand = 0, cnts[5] = {0, 0, 0, 0, 0}, bigc = 0;
        unsigned mx = 0;
        for (int b = threadIdx.x; b < nb; b += 1024) {
            const uint32_t a = cnt[b];
            mx = max(mx, a);
            for (int side = 0; side < ((two_sided && cn != c) ? 2 : 1); ++side) {
                const uint32_t b2 = (uint32_t)b ^ (side ? cn : c);
                unsigned long long T;
                int kind;
                const unsigned long long c = product_tiles((uint32_t)b, b2, a, cnt[b2], mfma, kind, T);
                cand += c;
                cnts[kind] += T;
                if (kind == 4) {
                    if (b2 != (uint32_t)b) {
                        cnts[3] += thin_tiles(a, cnt[b2]);
                        bigc += big_block_pairs(a, cnt[b2]);
                    } else {
                        bigc += c;
                    }
                }
            }
        }
        cand = block_sum<1024>(cand, shm);
        const unsigned long long tiles = block_sum<1024>(cnts[2], shm);
        const unsigned long long small = block_sum<1024>(cnts[1], shm);
        const unsigned long long mtiles = block_sum<1024>(cnts[3], shm);
        const unsigned long long btiles = block_sum<1024>(cnts[4], shm);
        const unsigned long long bpairs = block_sum<1024>(bigc, shm);
        mx = block_max<1024>(mx, shmax);
        if (threadIdx.x == 0) {
            inf->candidates = cand;
            inf->tiles = tiles;
            inf->small_tiles = (unsigned)small;
            inf->mfma_tiles = mtiles;
            inf->big_tiles = btiles;
            inf->big_pairs = bpairs;
            inf->max_bucket = mx;
            inf->passed = 0;
            inf->fresh = 0;
        }
    }
    // exclusive scan of the histogram: each thread owns a contiguous segment
    const int seg = (nb + 1023) / 1024;
    const int b0 = min(nb, (int)threadIdx.x * seg), b1 = min(nb, b0 + seg);
    unsigned long long loc = 0;
    for (int b = b0; b < b1; ++b) loc += cnt[b];
    unsigned long long tot;
    unsigned long long pre = block_scan_excl<1024>(loc, shm, &tot);
    uint32_t *of = offs + (int64_t)r * (nb + 1);
    for (int b = b0; b < b1; ++b) {
        const uint32_t c0 = cnt[b];
        cnt[b] = (uint32_t)pre;
        of[b] = (uint32_t)pre;
        pre += c0;
    }
    if (threadIdx.x == 0) of[nb] = (uint32_t)p;
    __syncthreads();
    uint32_t *pr = perm + (int64_t)r * p;
    if (ch > 0) {
        // cnt: next free position of every bucket; lo: the chunk's exclusive prefix of counts (lo[nb]:
        // the chunk's length); cur: placement cursors; sid / skey: the chunk's ids and keys in key
        // order; kin: the chunk's keys as read
        uint32_t *lo = cnt + nb, *cur = lo + nb + 1, *sid = cur + nb;
        uint16_t *skey = reinterpret_cast<uint16_t *>(sid + ch), *kin = skey + ch;
        for (int64_t c0 = 0; c0 < p; c0 += ch) {
            const int len = (int)(p - c0 < ch ? p - c0 : (int64_t)ch);
            const uint32_t *kc = kr + c0;
            for (int b = threadIdx.x; b < nb; b += 1024) cur[b] = 0;
            __syncthreads();
            for (int i0 = threadIdx.x; i0 < len; i0 += 1024 * BKU) {
                uint32_t kv[BKU];
#pragma unroll
                for (int u = 0; u < BKU; ++u) kv[u] = i0 + u * 1024 < len ? kc[i0 + u * 1024] : ~0u;
#pragma unroll
                for (int u = 0; u < BKU; ++u)
                    if (kv[u] != ~0u) {
                        atomicAdd(&cur[kv[u]], 1u);
                        kin[i0 + u * 1024] = (uint16_t)kv[u];
                    }
            }
            __syncthreads();
            unsigned long long lloc = 0;
            for (int b = b0; b < b1; ++b) lloc += cur[b];
            unsigned long long ltot;
            unsigned long long lpre = block_scan_excl<1024>(lloc, shm, &ltot);
            for (int b = b0; b < b1; ++b) {
                const uint32_t c1 = cur[b];
                lo[b] = (uint32_t)lpre;
                cur[b] = (uint32_t)lpre;
                lpre += c1;
            }
            if (threadIdx.x == 0) lo[nb] = (uint32_t)len;
            __syncthreads();
            // each key placed at its bucket's cursor
            for (int i = threadIdx.x; i < len; i += 1024) {
                const uint32_t key = kin[i];
                const uint32_t slot = atomicAdd(&cur[key], 1u);
                sid[slot] = (uint32_t)(c0 + i);
                skey[slot] = (uint16_t)key;
            }
            __syncthreads();
            // consecutive slots of a bucket go to consecutive positions of its range
            for (int s = threadIdx.x; s < len; s += 1024) {
                const uint32_t b = skey[s];
                pr[cnt[b] + (uint32_t)s - lo[b]] = sid[s];
            }
            __syncthreads();
            for (int b = threadIdx.x; b < nb; b += 1024) cnt[b] += lo[b + 1] - lo[b];
            __syncthreads();
        }
    }
    for (int64_t j0 = threadIdx.x; ch == 0 && j0 < p; j0 += 1024 * BKU) {
        uint32_t kv[BKU];
#pragma unroll
        for (int u = 0; u < BKU; ++u) kv[u] = j0 + u * 1024 < p ? kr[j0 + u * 1024] : ~0u;
#pragma unroll
        for (int u = 0; u < BKU; ++u)
            if (kv[u] != ~0u) pr[atomicAdd(&cnt[kv[u]], 1u)] = (uint32_t)(j0 + u * 1024);
    }
}

__global__ __launch_bounds__(1024) void k_tile_scan(const RepInfo *__restrict__ info, int count,
                                                    unsigned long long *__restrict__ base,
                                                    unsigned long long *__restrict__ totals)
{
    __shared__ unsigned long long shm[17];
    const int seg = (count + 1023) / 1024;
    const int i0 = min(count, (int)threadIdx.x * seg), i1 = min(count, i0 + seg);
    auto tiles_of = [&](int list, int i) -> unsigned long long {
        return list == 0 ? info[i].tiles
                         : (list == 1 ? (unsigned long long)info[i].small_tiles
                                      : (list == 2 ? info[i].mfma_tiles : info[i].big_tiles));
    };
    for (int list = 0; list < NLISTS; ++list) {
        unsigned long long *bs = base + list * (count + 1);
        unsigned long long loc = 0;
        for (int i = i0; i < i1; ++i) loc += tiles_of(list, i);
        unsigned long long tot;
        unsigned long long pre = block_scan_excl<1024>(loc, shm, &tot);
        for (int i = i0; i < i1; ++i) {
            bs[i] = pre;
            pre += tiles_of(list, i);
        }
        if (threadIdx.x == 0) {
            bs[count] = tot;
            if (totals) totals[list] = tot;
        }
        __syncthreads();
    }
}

// Tile (ia, ib) number t of a bucket's own product (ia <= ib < T), in row order:
// row ia starts at S(ia) = ia T - ia (ia - 1) / 2.
XYZ_DEV void tri_index(uint64_t t, uint64_t T, uint32_t &ia, uint32_t &ib)
{
    const double b = 2.0 * (double)T + 1.0;
    double r = 0.5 * (b - sqrt(b * b - 8.0 * (double)t));
    int64_t i = (int64_t)r;
    if (i < 0) i = 0;
    if (i > (int64_t)T - 1) i = (int64_t)T - 1;
    auto S = [T](int64_t q) { return (uint64_t)q * T - (uint64_t)q * (uint64_t)(q - 1) / 2; };
    while (i > 0 && S(i) > t) --i;
    while (i + 1 < (int64_t)T && S(i + 1) <= t) ++i;
    ia = (uint32_t)i;
    ib = (uint32_t)(i + (int64_t)(t - S(i)));
}

XYZ_DEV Tile make_tile(uint32_t ts, uint32_t r, uint32_t ysel, uint32_t pbase, uint32_t o1, uint32_t a, uint32_t o2,
                       uint32_t a2, uint32_t ia, uint32_t ib, uint8_t diag)
{
    Tile t;
    t.rep = r;
    t.a0 = pbase + o1 + ia * ts;
    t.b0 = pbase + o2 + ib * ts;
    t.na = (uint8_t)min(ts, a - ia * ts);
    t.nb = (uint8_t)min(ts, a2 - ib * ts);
    t.diag = diag;
    t.ysel = (uint8_t)ysel;
    return t;
}

// The product of two different buckets as one matrix-core tile (mfma_single).
XYZ_DEV Tile single_tile(uint32_t r, uint32_t ysel, uint32_t pbase, uint32_t o1, uint32_t a, uint32_t o2, uint32_t a2)
{
    Tile t;
    t.rep = r;
    t.a0 = pbase + o1;
    t.b0 = pbase + o2;
    t.na = (uint8_t)a;
    t.nb = (uint8_t)a2;
    t.diag = 0;
    t.ysel = (uint8_t)ysel;
    return t;
}

// Block pair (ia, ib) of BIG_TILE columns per side; the sides are stored minus one.
XYZ_DEV Tile big_tile(uint32_t r, uint32_t ysel, uint32_t pbase, uint32_t o1, uint32_t a, uint32_t o2, uint32_t a2,
                      uint32_t ia, uint32_t ib, uint8_t diag)
{
    Tile t;
    t.rep = r;
    t.a0 = pbase + o1 + ia * BIG_TILE;
    t.b0 = pbase + o2 + ib * BIG_TILE;
    t.na = (uint8_t)(min((uint32_t)BIG_TILE, a - ia * BIG_TILE) - 1);
    t.nb = (uint8_t)(min((uint32_t)BIG_TILE, a2 - ib * BIG_TILE) - 1);
    t.diag = diag;
    t.ysel = (uint8_t)ysel;
    return t;
}

// Tile number t of the product of bucket b (o1, a) and its partner b2 (o2, a2): a big block
// pair (ts = BIG_TILE), a tile of ts x ts, or the one tile of mfma_single.
XYZ_DEV Tile product_tile(uint32_t ts, uint64_t t, uint32_t r, uint32_t ysel, uint32_t pbase, bool own, uint32_t o1,
                          uint32_t a, uint32_t o2, uint32_t a2, int mfma)
{
    if (ts == (uint32_t)BIG_TILE) {
        uint32_t ia, ib;
        if (own) {
            tri_index(t, (a + BIG_TILE - 1) / BIG_TILE, ia, ib);
            return big_tile(r, ysel, pbase, o1, a, o1, a, ia, ib, (uint8_t)(ia == ib));
        }
        const uint32_t ea = a - thin_cols(a), eb = a2 - thin_cols(a2);   // sides without thin strips
        const uint32_t nB = (eb + BIG_TILE - 1) / BIG_TILE;
        return big_tile(r, ysel, pbase, o1, ea, o2, eb, (uint32_t)(t / nB), (uint32_t)(t % nB), 0);
    }
    if (!own) {
        if (ts == (uint32_t)MTILE && mfma_single(a, a2, mfma)) return single_tile(r, ysel, pbase, o1, a, o2, a2);
        const uint32_t nB = (a2 + ts - 1) / ts;
        return make_tile(ts, r, ysel, pbase, o1, a, o2, a2, (uint32_t)(t / nB), (uint32_t)(t % nB), 0);
    }
    const uint32_t T = (a + ts - 1) / ts;
    uint32_t ia, ib;
    tri_index(t, T, ia, ib);
    return make_tile(ts, r, ysel, pbase, o1, a, o1, a, ia, ib, (uint8_t)(ia == ib));
}

// Thin-strip tile number t of the big product of (o1, a) and (o2, a2) (see thin_tiles).
XYZ_DEV Tile thin_tile(uint64_t t, uint32_t r, uint32_t ysel, uint32_t pbase, uint32_t o1, uint32_t a, uint32_t o2,
                       uint32_t a2)
{
    const uint32_t ra = thin_cols(a), rb = thin_cols(a2);
    const uint64_t ta = ra ? cdiv_u64(a2, MTILE) : 0;
    Tile tl;
    tl.rep = r;
    tl.diag = 0;
    tl.ysel = (uint8_t)ysel;
    if (t < ta) {
        const uint32_t j = (uint32_t)t * MTILE;
        tl.a0 = pbase + o1 + (a - ra);
        tl.na = (uint8_t)ra;
        tl.b0 = pbase + o2 + j;
        tl.nb = (uint8_t)min((uint32_t)MTILE, a2 - j);
    } else {
        const uint32_t i = (uint32_t)(t - ta) * MTILE;
        tl.a0 = pbase + o1 + i;
        tl.na = (uint8_t)min((uint32_t)MTILE, a - ra - i);
        tl.b0 = pbase + o2 + (a2 - rb);
        tl.nb = (uint8_t)rb;
    }
    return tl;
}

// Tile number t of the product of bucket b and its partner b2 (offsets of).
XYZ_DEV Tile pair_tile(uint32_t ts, uint64_t t, uint32_t r, uint32_t ysel, uint32_t pbase, uint32_t b, uint32_t b2,
                       const uint32_t *of, int mfma)
{
    const uint32_t o1 = of[b], a = of[b + 1] - o1;
    const uint32_t o2 = of[b2], a2 = of[b2 + 1] - o2;
    return product_tile(ts, t, r, ysel, pbase, b == b2, o1, a, o2, a2, mfma);
}

XYZ_DEV uint32_t kind_tile(int kind)
{
    return kind == 4 ? (uint32_t)BIG_TILE : (kind == 3 ? (uint32_t)MTILE : (uint32_t)TILE);
}

// Bucket products with more tiles than this are emitted by the whole block.
constexpr unsigned HEAVY_TILES = 64;
constexpr int HEAVY_CAP = 512;

// Tiles of every (repetition, response) into four regions of one array: the
// popcount tiles (TILE) at base0[ry], the small tiles after all popcount tiles
// at base0[count] + base1[ry], the matrix-core tiles (MTILE) after those at
// base0[count] + base1[count] + base2[ry], the big tiles (BIG_TILE) last
// (baseK = base + K (count + 1)).
__global__ __launch_bounds__(256) void k_tiles(const uint32_t *__restrict__ offs, int64_t p, int m, int nys,
                                               const RepInfo *__restrict__ info, int two_sided, int mfma,
                                               const unsigned long long *__restrict__ base, Tile *__restrict__ tiles,
                                               uint64_t cap)
{
    __shared__ unsigned long long shm[5];
    __shared__ uint32_t hb[HEAVY_CAP], hb2[HEAVY_CAP], hts[HEAVY_CAP];
    __shared__ unsigned long long hpos[HEAVY_CAP], hcnt_t[HEAVY_CAP];
    __shared__ int hcnt;
    const int ry = blockIdx.x, count = gridDim.x;
    const unsigned long long *base0 = base, *base1 = base + (count + 1), *base2 = base + 2 * (count + 1),
                             *base3 = base + 3 * (count + 1);
    const int r = ry / nys, y = ry % nys;
    const int nb = 1 << m;
    const uint32_t mask = (uint32_t)(nb - 1);
    const uint32_t *of = offs + (int64_t)r * (nb + 1);
    const uint32_t c = (uint32_t)info[ry].cmask & mask;
    const uint32_t cn = (~c) & mask;
    const bool second = two_sided && cn != c;
    if (threadIdx.x == 0) hcnt = 0;
    const int seg = (nb + 255) / 256;
    const int b0 = min(nb, (int)threadIdx.x * seg), b1 = min(nb, b0 + seg);
    unsigned long long loc[5] = {0, 0, 0, 0, 0};
    for (int b = b0; b < b1; ++b) {
        const uint32_t a = of[b + 1] - of[b];
        for (int side = 0; side < (second ? 2 : 1); ++side) {
            const uint32_t b2 = (uint32_t)b ^ (side ? cn : c);
            unsigned long long T;
            int kind;
            const uint32_t a2 = of[b2 + 1] - of[b2];
            product_tiles(b, b2, a, a2, mfma, kind, T);
            loc[kind] += T;
            if (kind == 4 && b2 != (uint32_t)b) loc[3] += thin_tiles(a, a2);
        }
    }
    unsigned long long tot, pos[5];
    pos[2] = base0[ry] + block_scan_excl<256>(loc[2], shm, &tot);
    pos[1] = base0[count] + base1[ry] + block_scan_excl<256>(loc[1], shm, &tot);
    pos[3] = base0[count] + base1[count] + base2[ry] + block_scan_excl<256>(loc[3], shm, &tot);
    pos[4] = base0[count] + base1[count] + base2[count] + base3[ry] + block_scan_excl<256>(loc[4], shm, &tot);
    const uint32_t pbase = (uint32_t)((int64_t)r * p);
    for (int b = b0; b < b1; ++b) {
        for (int side = 0; side < (second ? 2 : 1); ++side) {
            const uint32_t b2 = (uint32_t)b ^ (side ? cn : c);
            unsigned long long T;
            int kind;
            product_tiles(b, b2, of[b + 1] - of[b], of[b2 + 1] - of[b2], mfma, kind, T);
            if (kind == 0) continue;
            const uint32_t ts = kind_tile(kind);
            int h = -1;
            if (T > HEAVY_TILES) {
                h = atomicAdd(&hcnt, 1);
                if (h < HEAVY_CAP) {
                    hb[h] = b;
                    hb2[h] = b2;
                    hts[h] = ts;
                    hpos[h] = pos[kind];
                    hcnt_t[h] = T;
                }
            }
            if (h < 0 || h >= HEAVY_CAP)
                for (unsigned long long t = 0; t < T && pos[kind] + t < cap; ++t)
                    tiles[pos[kind] + t] = pair_tile(ts, t, r, y, pbase, b, b2, of, mfma);
            pos[kind] += T;
            if (kind == 4 && b2 != (uint32_t)b) {
                const uint32_t a = of[b + 1] - of[b], a2 = of[b2 + 1] - of[b2];
                const unsigned long long Tt = thin_tiles(a, a2);
                for (unsigned long long t = 0; t < Tt && pos[3] + t < cap; ++t)
                    tiles[pos[3] + t] = thin_tile(t, r, y, pbase, of[b], a, of[b2], a2);
                pos[3] += Tt;
            }
        }
    }
    __syncthreads();
    const int nh = min(hcnt, HEAVY_CAP);
    for (int h = 0; h < nh; ++h) {
        const unsigned long long T = hcnt_t[h], p0 = hpos[h];
        for (unsigned long long t = threadIdx.x; t < T && p0 + t < cap; t += 256)
            tiles[p0 + t] = pair_tile(hts[h], t, r, y, pbase, hb[h], hb2[h], of, mfma);
    }
}

// ------------------------------------------------ bucket sort for m > 15 --
//
// With more than MAX_M_LDS key bits the 2^m counters do not fit in LDS.  The
// keys of every repetition of a chunk are then sorted by (repetition, key)
// with the LSD radix sort below, equal keys form runs (the non-empty buckets),
// and the partner of run b, the bucket b ^ c of the same repetition (Section
// 2.2), is found by binary search among the sorted run keys.  The tile lists
// are the same as on the LDS path.

__global__ __launch_bounds__(256) void k_sk_init(const uint32_t *__restrict__ keys, uint64_t S, int64_t p, int m,
                                                 uint64_t *__restrict__ K, uint32_t *__restrict__ V)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= S) return;
    const uint64_t r = i / (uint64_t)p;
    K[i] = (r << m) | keys[i];
    V[i] = (uint32_t)(i - r * (uint64_t)p);
}

__global__ __launch_bounds__(256) void k_sk_heads(const uint64_t *__restrict__ K, uint64_t S,
                                                  uint32_t *__restrict__ heads)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= S) return;
    heads[i] = (i == 0 || K[i] != K[i - 1]) ? 1u : 0u;
}

// run rid (exclusive scan of the heads) starts at i; nruns[0] = number of runs
__global__ __launch_bounds__(256) void k_sk_runs(const uint64_t *__restrict__ K, const uint32_t *__restrict__ hscan,
                                                 uint64_t S, uint64_t *__restrict__ run_key,
                                                 uint32_t *__restrict__ run_start, uint32_t *__restrict__ nruns)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= S) return;
    const bool head = i == 0 || K[i] != K[i - 1];
    if (head) {
        run_key[hscan[i]] = K[i];
        run_start[hscan[i]] = (uint32_t)i;
    }
    if (i == S - 1) nruns[0] = hscan[i] + (head ? 1u : 0u);
}

// Run of composite key (r << m) | b: from the direct table (m <= SK_TABLE_MAX_M: entry r 2^m + b
// holds run id + 1, 0 when the bucket is empty) or by binary search over the sorted run keys.
XYZ_DEV int64_t find_run(const uint64_t *run_key, uint32_t nr, uint64_t target, const uint32_t *table)
{
    if (table) return (int64_t)table[target] - 1;
    uint32_t lo = 0, hi = nr;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (run_key[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return (lo < nr && run_key[lo] == target) ? (int64_t)lo : -1;
}

XYZ_DEV uint32_t run_len(const uint32_t *run_start, uint32_t nr, uint64_t S, uint32_t rid)
{
    return (rid + 1 < nr ? run_start[rid + 1] : (uint32_t)S) - run_start[rid];
}

// The bucket products of run rid for response y, in the order of k_tiles: partner c,
// then (two-sided) ~c; a product is taken from its smaller key.  f(b2, rid2, a2, kind, T).
template <class F>
XYZ_DEV unsigned long long run_products(const uint64_t *run_key, const uint32_t *run_start, uint32_t nr, uint64_t S,
                                        int m, uint32_t rid, uint32_t c, int two_sided, int mfma,
                                        const uint32_t *table, F f)
{
    const uint32_t mask = (uint32_t)((1ull << m) - 1);
    const uint64_t rk = run_key[rid];
    const uint64_t rhi = rk >> m;
    const uint32_t b = (uint32_t)(rk & mask), a = run_len(run_start, nr, S, rid);
    const uint32_t cn = (~c) & mask;
    unsigned long long cand = 0;
    for (int side = 0; side < ((two_sided && cn != c) ? 2 : 1); ++side) {
        const uint32_t b2 = b ^ (side ? cn : c);
        if (b2 < b) continue;
        int64_t rid2 = rid;
        if (b2 != b) rid2 = find_run(run_key, nr, (rhi << m) | b2, table);
        if (rid2 < 0) continue;
        const uint32_t a2 = b2 == b ? a : run_len(run_start, nr, S, (uint32_t)rid2);
        unsigned long long T;
        int kind;
        const unsigned long long c = product_tiles(b, b2, a, a2, mfma, kind, T);
        cand += c;
        if (kind) f((uint32_t)rid2, a2, kind, T, c);
    }
    return cand;
}

// Per (response y, run): tile counts of the four lists into cnt[list][y][rid], and the
// repetition's statistics.  A block takes SK_ITEMS * 256 consecutive items; each thread sums its
// items per (repetition, response), flushing with atomics only when that changes, and the
// waves whose lanes end on one (repetition, response) add their sums once.
constexpr int SK_ITEMS = 16;

XYZ_DEV void sk_flush(RepInfo *info, int64_t key, const unsigned long long v[6], uint32_t mx)
{
    RepInfo *inf = info + key;
    if (v[5]) atomicAdd(&inf->big_pairs, v[5]);
    if (v[0]) atomicAdd(&inf->candidates, v[0]);
    if (v[1]) atomicAdd(&inf->tiles, v[1]);
    if (v[2]) atomicAdd(&inf->small_tiles, (unsigned)v[2]);
    if (v[3]) atomicAdd(&inf->mfma_tiles, v[3]);
    if (v[4]) atomicAdd(&inf->big_tiles, v[4]);
    atomicMax(&inf->max_bucket, mx);
}

__global__ __launch_bounds__(256) void k_sk_products(const uint64_t *__restrict__ run_key,
                                                     const uint32_t *__restrict__ run_start,
                                                     const uint32_t *__restrict__ nruns, uint64_t S, int m, int nys,
                                                     RepInfo *__restrict__ info, int two_sided, int mfma,
                                                     const uint32_t *__restrict__ table,
                                                     uint32_t *__restrict__ cnt, uint64_t cnt_stride)
{
    const uint32_t nr = nruns[0];
    const uint64_t total = (uint64_t)nr * nys;
    const uint64_t base = (uint64_t)blockIdx.x * SK_ITEMS * 256;
    int64_t key = -1;
    unsigned long long v[6] = {0, 0, 0, 0, 0, 0};
    uint32_t mx = 0;
    for (int it = 0; it < SK_ITEMS; ++it) {
        const uint64_t tid = base + (uint64_t)it * 256 + threadIdx.x;
        if (tid >= total) break;
        const uint32_t y = (uint32_t)(tid / nr), rid = (uint32_t)(tid % nr);
        const uint64_t r = run_key[rid] >> m;
        const int64_t k = (int64_t)(r * nys + y);
        if (k != key) {
            if (key >= 0) sk_flush(info, key, v, mx);
            key = k;
            v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = 0;
            mx = 0;
        }
        const uint32_t c = (uint32_t)info[k].cmask & (uint32_t)((1ull << m) - 1);
        unsigned long long tl[5] = {0, 0, 0, 0, 0}, bp = 0;
        const uint32_t a = run_len(run_start, nr, S, rid);
        v[0] += run_products(run_key, run_start, nr, S, m, rid, c, two_sided, mfma, table,
                             [&](uint32_t rid2, uint32_t a2, int kind, unsigned long long T, unsigned long long pc) {
                                 tl[kind] += T;
                                 if (kind == 4) {
                                     if (rid2 != rid) {
                                         tl[3] += thin_tiles(a, a2);
                                         bp += big_block_pairs(a, a2);
                                     } else {
                                         bp += pc;
                                     }
                                 }
                             });
        cnt[0 * cnt_stride + (uint64_t)y * nr + rid] = (uint32_t)tl[2];
        cnt[1 * cnt_stride + (uint64_t)y * nr + rid] = (uint32_t)tl[1];
        cnt[2 * cnt_stride + (uint64_t)y * nr + rid] = (uint32_t)tl[3];
        cnt[3 * cnt_stride + (uint64_t)y * nr + rid] = (uint32_t)tl[4];
        v[1] += tl[2];
        v[2] += tl[1];
        v[3] += tl[3];
        v[4] += tl[4];
        v[5] += bp;
        mx = max(mx, run_len(run_start, nr, S, rid));
    }
    // lanes that end on lane 0's (repetition, response) add their sums once per wave
    const int64_t k0 = __shfl(key, 0, 64);
    const unsigned long long same = __ballot(key == k0 || key < 0);
    if (same == ~0ull && k0 >= 0) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] += __shfl_xor(v[q], d, 64);
            mx = max(mx, (uint32_t)__shfl_xor(mx, d, 64));
        }
        if (lane_id() == 0) sk_flush(info, k0, v, mx);
    } else if (key >= 0) {
        sk_flush(info, key, v, mx);
    }
}

// Tiles of every (response, run) at pos[list][y][rid] (exclusive scan over the four lists
// laid end to end, so the popcount, small, matrix-core and big lists follow each other).
__global__ __launch_bounds__(256) void k_sk_tiles(const uint64_t *__restrict__ run_key,
                                                  const uint32_t *__restrict__ run_start,
                                                  const uint32_t *__restrict__ nruns, uint64_t S, int64_t p, int m,
                                                  int nys, const RepInfo *__restrict__ info, int two_sided, int mfma,
                                                  const uint32_t *__restrict__ table,
                                                  const uint32_t *__restrict__ pos, uint64_t cnt_stride,
                                                  Tile *__restrict__ tiles)
{
    const uint32_t nr = nruns[0];
    const uint64_t tid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (tid >= (uint64_t)nr * nys) return;
    const uint32_t y = (uint32_t)(tid / nr), rid = (uint32_t)(tid % nr);
    const uint64_t r = run_key[rid] >> m;
    const uint32_t c = (uint32_t)info[r * nys + y].cmask & (uint32_t)((1ull << m) - 1);
    const uint32_t pbase = (uint32_t)(r * (uint64_t)p);
    const uint32_t o1 = run_start[rid] - pbase, a = run_len(run_start, nr, S, rid);
    uint64_t at[5];
    at[2] = pos[0 * cnt_stride + (uint64_t)y * nr + rid];
    at[1] = pos[1 * cnt_stride + (uint64_t)y * nr + rid];
    at[3] = pos[2 * cnt_stride + (uint64_t)y * nr + rid];
    at[4] = pos[3 * cnt_stride + (uint64_t)y * nr + rid];
    run_products(run_key, run_start, nr, S, m, rid, c, two_sided, mfma, table,
                 [&](uint32_t rid2, uint32_t a2, int kind, unsigned long long T, unsigned long long) {
                     const uint32_t ts = kind_tile(kind);
                     const uint32_t o2 = run_start[rid2] - pbase;
                     const bool own = rid2 == rid;
                     for (unsigned long long t = 0; t < T; ++t)
                         tiles[at[kind] + t] = product_tile(ts, t, (uint32_t)r, y, pbase, own, o1, a, own ? o1 : o2,
                                                            own ? a : a2, mfma);
                     at[kind] += T;
                     if (kind == 4 && !own) {
                         const unsigned long long Tt = thin_tiles(a, a2);
                         for (unsigned long long t = 0; t < Tt; ++t)
                             tiles[at[3] + t] = thin_tile(t, (uint32_t)r, y, pbase, o1, a, o2, a2);
                         at[3] += Tt;
                     }
                 });
}

__global__ __launch_bounds__(256) void k_sk_table(const uint64_t *__restrict__ run_key,
                                                  const uint32_t *__restrict__ nruns, uint32_t *__restrict__ table)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nruns[0]) return;
    table[run_key[i]] = (uint32_t)i + 1;
}

__global__ __launch_bounds__(256) void k_sk_clear_info(RepInfo *__restrict__ info, int count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    info[i].candidates = 0;
    info[i].tiles = 0;
    info[i].passed = 0;
    info[i].fresh = 0;
    info[i].max_bucket = 0;
    info[i].small_tiles = 0;
    info[i].mfma_tiles = 0;
    info[i].big_tiles = 0;
    info[i].big_pairs = 0;
}

// ----------------------------------------------------------- FP4 operands --
//
// The 0/1 dot products of the exact search and of large verification tiles run
// on v_mfma_scale_f32_32x32x64_f8f6f4 with e2m1 operands: lanes 0-31 feed 32
// rows of their column, lanes 32-63 the next 32 rows, 16 bytes (32 nibbles)
// each; FP32 accumulation of the integer counts is exact below 2^24.

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

XYZ_DEV uint32_t swap02(uint32_t w)
{
    return (w & 0xAAAAAAAAu) | ((w & 0x11111111u) << 2) | ((w >> 2) & 0x11111111u);
}

// 32 bits of one column word -> 32 e2m1 nibbles (the low half of an FP4
// operand), nonzero for a set bit.  Row r = 4q + e of the word (nibble q, e in
// 0..3) goes to nibble q of dword e.  On the A side a set bit keeps its place
// in the nibble, so dwords 0, 1, 2 hold the values 0.5, 1, 2 (e2m1 0b0001,
// 0b0010, 0b0100) with one AND each, and dword 3 moves bit 3 to bit 1 (1.0).
// The exact search stages its B side with bits 0 and 2 of each nibble swapped,
// so the same masks give it the values 2, 1, 0.5, 1 (expand_b); an unstaged B
// word takes two more shifts (expand_b_plain).  Every product of two set bits
// is exactly 1.  Which rows share a nibble does not matter, because A and B
// assign rows to (dword, nibble) the same way and the product sums over all.
XYZ_DEV v8i expand_a(uint32_t w)
{
    return v8i{(int)(w & 0x11111111u), (int)(w & 0x22222222u), (int)(w & 0x44444444u),
               (int)((w >> 2) & 0x22222222u), 0, 0, 0, 0};
}

XYZ_DEV v8i expand_b(uint32_t w)
{
    return v8i{(int)(w & 0x44444444u), (int)(w & 0x22222222u), (int)(w & 0x11111111u),
               (int)((w >> 2) & 0x22222222u), 0, 0, 0, 0};
}

XYZ_DEV v8i expand_b_plain(uint32_t w)
{
    return v8i{(int)((w << 2) & 0x44444444u), (int)(w & 0x22222222u), (int)((w >> 2) & 0x11111111u),
               (int)((w >> 2) & 0x22222222u), 0, 0, 0, 0};
}

XYZ_DEV v16f mfma_fp4(v8i a, v8i b, v16f c)
{
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

// Bit plane pl of four words as one FP4 operand (word d in dword d): planes 0, 1, 2
// keep bit pl of every nibble (e2m1 values 0.5, 1, 2), plane 3 moves bit 3 to bit 1
// (value 1).  With the same plane on both sides, a product of two set bits is
// 0.25, 1, 4 or 1, and the per-block scales 2^1, 2^0, 2^-1, 2^0 on each side
// (mfma_fp4_plane) make it exactly 1: no bit swap on either side.
XYZ_DEV v8i plane_fp4(uint4 w, int pl)
{
    if (pl == 3)
        return v8i{(int)((w.x >> 2) & 0x22222222u), (int)((w.y >> 2) & 0x22222222u),
                   (int)((w.z >> 2) & 0x22222222u), (int)((w.w >> 2) & 0x22222222u), 0, 0, 0, 0};
    const uint32_t m = 0x11111111u << pl;
    return v8i{(int)(w.x & m), (int)(w.y & m), (int)(w.z & m), (int)(w.w & m), 0, 0, 0, 0};
}

XYZ_DEV v16f mfma_fp4_plane(v8i a, v8i b, v16f c, int pl)
{
    // E8M0 block scales: 128 = 2^1, 127 = 2^0, 126 = 2^-1
    switch (pl) {
    case 0: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 128, 0, 128);
    case 2: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 126, 0, 126);
    default: return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
    }
}

// ------------------------------------------------------------ verification --
//
// One wave per tile (<= 32 x 32 column pairs).  Lane (ia, ib) = (lane & 7,
// lane >> 3) owns the RA x RB block of pairs (ia + 8u, ib + 8v).  Columns are
// staged through LDS in chunks of 32 words (1024 rows): A holds z_a = y ^ x_a,
// B holds x_b, so the inner loop is one XOR and one popcount-accumulate per
// pair and 32-bit word.  RA = ceil(na/8), RB = ceil(nb/8) are wave-uniform.

// The list sizes of a verification launch whose sizes live on the device (VerifyArgs::dcnt): all
// four zero when the lists exceed the tile array, whose overflow the host resolves by rerunning.
XYZ_DEV void load_counts(VerifyArgs &a)
{
    if (!a.dcnt) return;
    const unsigned long long n0 = a.dcnt[0], n1 = a.dcnt[1], n2 = a.dcnt[2], n3 = a.dcnt[3];
    const bool fits = n0 + n1 + n2 + n3 <= a.tile_cap;
    a.ntiles = fits ? n0 : 0;
    a.nsmall = fits ? n1 : 0;
    a.nmfma = fits ? n2 : 0;
    a.nbig = fits ? n3 : 0;
}

// Candidate pairs of a tile (positions a < b only on a diagonal tile).
XYZ_DEV uint32_t tile_pairs(const Tile &t)
{
    return t.diag ? (uint32_t)t.na * (uint32_t)(t.na - 1) / 2 : (uint32_t)t.na * (uint32_t)t.nb;
}

XYZ_DEV Tile tile_from(uint4 v)
{
    Tile t;
    t.rep = v.x;
    t.a0 = v.y;
    t.b0 = v.z;
    t.na = (uint8_t)(v.w & 255u);
    t.nb = (uint8_t)((v.w >> 8) & 255u);
    t.diag = (uint8_t)((v.w >> 16) & 255u);
    t.ysel = (uint8_t)(v.w >> 24);
    return t;
}

constexpr int CW4 = 8;       // uint4 per column per chunk (32 words)
constexpr int LDS4 = CW4 + 1;  // padded row length (uint4) against bank conflicts


// Reserve room for the survivors of one tile: one atomic per wave (also
// counting them as passed for the tile's repetition).  Returns the index of
// this lane's first survivor, or ~0 when the wave has none.
XYZ_DEV unsigned long long reserve_survivors(const VerifyArgs &a, const Tile &t, int mine)
{
    const unsigned lane = lane_id();
    int incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if ((int)lane >= d) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    if (total == 0) return ~0ull;
    unsigned long long base = 0;
    if (lane == 0) {
        base = atomicAdd(a.surv_count, (unsigned long long)total);
        atomicAdd(&a.info[(int64_t)t.rep * a.nys + t.ysel].passed, (unsigned long long)total);
    }
    base = __shfl(base, 0, 64);
    return base + (unsigned long long)(incl - mine);
}

template <int RA, int RB>
XYZ_DEV void verify_bin_tile(const Tile &t, const uint32_t *colA, const uint32_t *colB, uint4 (*As)[LDS4],
                             uint4 (*Bs)[LDS4], const VerifyArgs &a)
{
    const unsigned lane = lane_id();
    const int ia = lane & 7, ib = lane >> 3;
    const int q = lane & 7, rc = lane >> 3;
    const int W4 = a.W32p >> 2;
    const uint4 *XC4 = reinterpret_cast<const uint4 *>(a.XC);
    const uint4 *y4 = reinterpret_cast<const uint4 *>(a.yb + (int64_t)t.ysel * a.W32p);
    uint32_t acc[RA][RB];
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) acc[u][v] = 0;
    const int nchunk = (W4 + CW4 - 1) / CW4;
    for (int c = 0; c < nchunk; ++c) {
        const int gq = c * CW4 + q;
        const bool inw = gq < W4;
        const uint4 yv = inw ? y4[gq] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < RA; ++u) {
            const int ci = rc + 8 * u;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ci < t.na && inw) {
                v = XC4[(int64_t)colA[ci] * W4 + gq];
                v.x ^= yv.x; v.y ^= yv.y; v.z ^= yv.z; v.w ^= yv.w;
            }
            As[ci][q] = v;
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int ci = rc + 8 * u;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (ci < t.nb && inw) v = XC4[(int64_t)colB[ci] * W4 + gq];
            Bs[ci][q] = v;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < CW4; ++w) {
            uint4 av[RA], bv[RB];
#pragma unroll
            for (int u = 0; u < RA; ++u) av[u] = As[ia + 8 * u][w];
#pragma unroll
            for (int v = 0; v < RB; ++v) bv[v] = Bs[ib + 8 * v][w];
#pragma unroll
            for (int u = 0; u < RA; ++u)
#pragma unroll
                for (int v = 0; v < RB; ++v) {
                    uint32_t x = acc[u][v];
                    x = bcnt_acc(av[u].x ^ bv[v].x, x);
                    x = bcnt_acc(av[u].y ^ bv[v].y, x);
                    x = bcnt_acc(av[u].z ^ bv[v].z, x);
                    x = bcnt_acc(av[u].w ^ bv[v].w, x);
                    acc[u][v] = x;
                }
        }
        __syncthreads();
    }
    const int64_t smin = a.smin[t.ysel];
    uint32_t passmask = 0;
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) {
            const int pa = ia + 8 * u, pb = ib + 8 * v;
            const int64_t s = a.n - 2 * (int64_t)acc[u][v];
            const bool pass = a.two_sided ? ((s < 0 ? -s : s) >= smin) : (s >= smin);
            if (pa < t.na && pb < t.nb && (!t.diag || pa < pb) && pass) passmask |= 1u << (u * RB + v);
        }
    unsigned long long idx = reserve_survivors(a, t, __popc(passmask));
    if (idx == ~0ull) return;
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v)
            if ((passmask >> (u * RB + v)) & 1u) {
                const uint32_t j = colA[ia + 8 * u], k = colB[ib + 8 * v];
                const int64_t s = a.n - 2 * (int64_t)acc[u][v];
                if (idx < a.surv_cap) {
                    Survivor sv;
                    sv.j = min(j, k);
                    sv.k = max(j, k);
                    sv.rep = (uint32_t)(a.rep_abs0 + t.rep);
                    sv.s = (int32_t)s;
                    sv.value = (double)s;
                    sv.ysel = t.ysel;
                    sv.pad = 0;
                    a.surv[idx] = sv;
                }
                ++idx;
            }
}

__global__ __launch_bounds__(64) void k_verify_bin(VerifyArgs a0)
{
    VerifyArgs a = a0;
    load_counts(a);
    __shared__ uint4 As[TILE][LDS4];
    __shared__ uint4 Bs[TILE][LDS4];
    __shared__ uint32_t colA[TILE], colB[TILE];
    const unsigned lane = lane_id();
    for (uint64_t ti = blockIdx.x; ti < a.ntiles; ti += gridDim.x) {
        const Tile t = a.tiles[ti];
        if (lane < t.na) colA[lane] = a.perm[t.a0 + lane];
        if (lane >= 32 && lane - 32 < t.nb) colB[lane - 32] = a.perm[t.b0 + lane - 32];
        __syncthreads();
        const int ra = (t.na + 7) >> 3, rb = (t.nb + 7) >> 3;
        switch (ra * 4 + rb) {
        case 5: verify_bin_tile<1, 1>(t, colA, colB, As, Bs, a); break;
        case 6: verify_bin_tile<1, 2>(t, colA, colB, As, Bs, a); break;
        case 7: verify_bin_tile<1, 3>(t, colA, colB, As, Bs, a); break;
        case 8: verify_bin_tile<1, 4>(t, colA, colB, As, Bs, a); break;
        case 9: verify_bin_tile<2, 1>(t, colA, colB, As, Bs, a); break;
        case 10: verify_bin_tile<2, 2>(t, colA, colB, As, Bs, a); break;
        case 11: verify_bin_tile<2, 3>(t, colA, colB, As, Bs, a); break;
        case 12: verify_bin_tile<2, 4>(t, colA, colB, As, Bs, a); break;
        case 13: verify_bin_tile<3, 1>(t, colA, colB, As, Bs, a); break;
        case 14: verify_bin_tile<3, 2>(t, colA, colB, As, Bs, a); break;
        case 15: verify_bin_tile<3, 3>(t, colA, colB, As, Bs, a); break;
        case 16: verify_bin_tile<3, 4>(t, colA, colB, As, Bs, a); break;
        case 17: verify_bin_tile<4, 1>(t, colA, colB, As, Bs, a); break;
        case 18: verify_bin_tile<4, 2>(t, colA, colB, As, Bs, a); break;
        case 19: verify_bin_tile<4, 3>(t, colA, colB, As, Bs, a); break;
        case 20: verify_bin_tile<4, 4>(t, colA, colB, As, Bs, a); break;
        default: break;
        }
        __syncthreads();
    }
}

// Matrix-core tiles (products of two buckets with at least MTILE_MIN columns
// each; +-1 data, n < 2^24).  One wave per MTILE x MTILE tile, as 2 x 2
// fragments of 32 x 32: the counts C = #{i : z_ia = x_ib = 1}, z = y ^ x,
// accumulate on v_mfma_scale_f32_32x32x64_f8f6f4 over 64-row steps.  A column is
// read in stages of four quads (64 bytes): one load instruction covers a stage
// of 16 columns, lane l taking quad l/16 of column l%16 (random column gathers
// run at full HBM speed only with 64 contiguous bytes or more per column and
// instruction), and v_permlane16_swap between the loads of columns 0-15 and
// 16-31 of a fragment brings them into the matrix layout: lane half h then
// holds quads 2h and 2h + 1 of column lane%32 and feeds the products' 32-row
// halves from them (any pairing of the words with the K dimension gives the
// same C, as long as both sides use it).  Lanes past the end of a bucket
// (na, nb < 64) repeat its last column, so their products duplicate real
// ones; the popcounts |z_a|, |x_b| are taken on the way.  Two stages are in
// flight per lane.  A tile side of w columns takes ceil(w / 32) fragments: a
// product with one side of at most 64 columns and the other of at most 96 is
// one tile of up to 3 x 2 fragments (neither side is read twice), and the
// remainder of a larger bucket cut into 64-column blocks takes only the
// fragments it fills.  Accumulator register r of lane l holds A
// row u*32 + (r/4)*8 + (l/32)*4 + r%4 and B column v*32 + l%32.
// v_permlane16_swap on each word: lanes 16-31 and 48-63 of lo trade places with
// lanes 0-15 and 32-47 of hi.
XYZ_DEV void swap16(uint4 &lo, uint4 &hi)
{
    auto x = __builtin_amdgcn_permlane16_swap(lo.x, hi.x, false, false);
    auto y = __builtin_amdgcn_permlane16_swap(lo.y, hi.y, false, false);
    auto z = __builtin_amdgcn_permlane16_swap(lo.z, hi.z, false, false);
    auto w = __builtin_amdgcn_permlane16_swap(lo.w, hi.w, false, false);
    lo = make_uint4(x[0], y[0], z[0], w[0]);
    hi = make_uint4(x[1], y[1], z[1], w[1]);
}

__global__ __launch_bounds__(256, 2) void k_verify_mfma(VerifyArgs a0)
{
    VerifyArgs a = a0;
    load_counts(a);
    __shared__ __align__(16) float zpop2[4][MTILE_WIDE];  // per wave: 2|z_a| of the tile's A columns
    const unsigned lane = lane_id();
    const int h = (int)(lane >> 5), c = (int)(lane & 31);
    const int lc = (int)(lane & 15), lq = (int)(lane >> 4);
    const int wv = (int)(threadIdx.x >> 6);
    const int W4 = a.W32p >> 2;
    const int NS = (W4 + 3) >> 2;                   // stages of four quads
    const uint4 *XC4 = reinterpret_cast<const uint4 *>(a.XC);
    const uint4 *T4 = reinterpret_cast<const uint4 *>(a.tiles + a.ntiles + a.nsmall);
    const uint64_t wid = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6), nwave = (uint64_t)gridDim.x * 4;
    const int32_t n32 = (int32_t)a.n;
    using T_ = std::true_type;
    using F_ = std::false_type;
    // One tile as NU x NV fragments of 32 x 32, NU = ceil(na / 32) (at most 3 x 2 or 2 x 3),
    // so that no products or loads are spent on empty fragments.
    auto tile_body = [&](const Tile &t, auto nu_c, auto nv_c) {
        constexpr int NU = decltype(nu_c)::value, NV = decltype(nv_c)::value;
        const uint4 *y4 = reinterpret_cast<const uint4 *>(a.yb + (int64_t)t.ysel * a.W32p);
        const uint4 *pa[2 * NU], *pb[2 * NV];
#pragma unroll
        for (int g = 0; g < 2 * NU; ++g)
            pa[g] = XC4 + (int64_t)a.perm[t.a0 + min(g * 16 + lc, (int)t.na - 1)] * W4;
#pragma unroll
        for (int g = 0; g < 2 * NV; ++g)
            pb[g] = XC4 + (int64_t)a.perm[t.b0 + min(g * 16 + lc, (int)t.nb - 1)] * W4;
        v16f acc[NU][NV];
        uint32_t popa[NU], popb[NV];
#pragma unroll
        for (int u = 0; u < NU; ++u) popa[u] = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) popb[v] = 0;
        struct Stage {
            uint4 a[2 * NU], b[2 * NV];  // quad 4s + l/16 of A (B) column 16g + l%16 of the tile
            uint4 y[2];                  // quads 4s + 2h and 4s + 2h + 1 of y
        };
        auto load = [&](Stage &st, int stg) {
            const int q0 = 4 * min(stg, NS - 1);
            const int q = min(q0 + lq, W4 - 1);     // clamped: quads past the column are masked
#pragma unroll
            for (int g = 0; g < 2 * NU; ++g) st.a[g] = pa[g][q];
#pragma unroll
            for (int g = 0; g < 2 * NV; ++g) st.b[g] = pb[g][q];
#pragma unroll
            for (int j = 0; j < 2; ++j) st.y[j] = y4[min(q0 + 2 * h + j, W4 - 1)];
        };
        // the stage's 8 products per fragment (quads past W4 count as zero); FIRST: the first
        // product starts the accumulators
        auto step = [&](Stage &st, int stg, auto first) {
            // matrix layout: A[u][j] = quad 4s + 2h + j of A column u*32 + c (B likewise)
            uint4 A[NU][2], B[NV][2];
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                A[u][0] = st.a[2 * u];
                A[u][1] = st.a[2 * u + 1];
                swap16(A[u][0], A[u][1]);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                B[v][0] = st.b[2 * v];
                B[v][1] = st.b[2 * v + 1];
                swap16(B[v][0], B[v][1]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint32_t keep = 4 * stg + 2 * h + j < W4 ? ~0u : 0u;
                uint4 za[NU], xb[NV];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    za[u] = make_uint4((A[u][j].x ^ st.y[j].x) & keep, (A[u][j].y ^ st.y[j].y) & keep,
                                       (A[u][j].z ^ st.y[j].z) & keep, (A[u][j].w ^ st.y[j].w) & keep);
                    popa[u] = bcnt_acc(za[u].w, bcnt_acc(za[u].z, bcnt_acc(za[u].y, bcnt_acc(za[u].x, popa[u]))));
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    xb[v] = make_uint4(B[v][j].x & keep, B[v][j].y & keep, B[v][j].z & keep, B[v][j].w & keep);
                    popb[v] = bcnt_acc(xb[v].w, bcnt_acc(xb[v].z, bcnt_acc(xb[v].y, bcnt_acc(xb[v].x, popb[v]))));
                }
                // one product per bit plane of the quad's four words
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) {
                    v8i fa[NU], fb[NV];
#pragma unroll
                    for (int u = 0; u < NU; ++u) fa[u] = plane_fp4(za[u], pl);
#pragma unroll
                    for (int v = 0; v < NV; ++v) fb[v] = plane_fp4(xb[v], pl);
#pragma unroll
                    for (int u = 0; u < NU; ++u)
#pragma unroll
                        for (int v = 0; v < NV; ++v)
                            acc[u][v] = mfma_fp4_plane(fa[u], fb[v],
                                                       (decltype(first)::value && j == 0 && pl == 0) ? v16f{}
                                                                                                    : acc[u][v],
                                                       pl);
                }
            }
            load(st, stg + 2);
            __builtin_amdgcn_sched_barrier(0);
        };
        // stage s sits in s0 (even) or s1 (odd)
        Stage s0, s1;
        load(s0, 0);
        load(s1, 1);
        step(s0, 0, T_{});
        int stg = 1;
        for (; stg + 1 < NS; stg += 2) {     // no branches inside: each wait is for the oldest loads only
            step(s1, stg, F_{});
            step(s0, stg + 1, F_{});
        }
        if (stg < NS) step(s1, stg, F_{});
        // whole-column popcounts: the two lane halves of a column hold disjoint words
#pragma unroll
        for (int u = 0; u < NU; ++u) popa[u] += __shfl_xor(popa[u], 32, 64);
#pragma unroll
        for (int v = 0; v < NV; ++v) popb[v] += __shfl_xor(popb[v], 32, 64);
        // cheap test per fragment: x = 4C - 2|z_a| over the lane's 16 rows against
        // smin - n + 2|x_b| (and -smin - n + 2|x_b| two-sided), exact in FP32
        if (h == 0) {
#pragma unroll
            for (int u = 0; u < NU; ++u) zpop2[wv][u * 32 + c] = (float)(2 * popa[u]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int32_t smin = (int32_t)a.smin[t.ysel];
        uint32_t hitmask = 0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            float tA[16];
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const float4 v4 = *reinterpret_cast<const float4 *>(&zpop2[wv][u * 32 + q4 * 8 + h * 4]);
                tA[4 * q4 + 0] = v4.x;
                tA[4 * q4 + 1] = v4.y;
                tA[4 * q4 + 2] = v4.z;
                tA[4 * q4 + 3] = v4.w;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int32_t pb2 = 2 * (int32_t)popb[v];
                float mx = -1e30f, mn = 1e30f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float x = __builtin_fmaf(4.0f, acc[u][v][r], -tA[r]);
                    mx = fmaxf(mx, x);
                    mn = fminf(mn, x);
                }
                const bool hit = mx >= (float)(smin - n32 + pb2) || (a.two_sided && mn <= (float)(-smin - n32 + pb2));
                hitmask |= (hit ? 1u : 0u) << (u * 3 + v);
            }
        }
        if (__ballot(hitmask != 0) != 0) {
            // rare: exact values and validity (padding rows and columns, a < b on a diagonal tile)
            uint32_t pm[NU][NV];
            int mine = 0;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int cb = v * 32 + c;
                    uint32_t m = 0;
                    if ((hitmask >> (u * 3 + v)) & 1u) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int ra = u * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
                            const int32_t sv = n32 - (int32_t)zpop2[wv][ra] - 2 * (int32_t)popb[v] +
                                               4 * (int32_t)acc[u][v][r];
                            const bool pass = a.two_sided ? ((sv < 0 ? -sv : sv) >= smin) : (sv >= smin);
                            const bool ok = ra < t.na && cb < t.nb && (!t.diag || ra < cb);
                            m |= (pass && ok ? 1u : 0u) << r;
                        }
                    }
                    pm[u][v] = m;
                    mine += __popc(m);
                }
            }
            unsigned long long idx = reserve_survivors(a, t, mine);
            if (idx != ~0ull) {
#pragma unroll
                for (int u = 0; u < NU; ++u)
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const int cb = v * 32 + c;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            if (!((pm[u][v] >> r) & 1u)) continue;
                            const int ra = u * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
                            const uint32_t j = a.perm[t.a0 + ra], k = a.perm[t.b0 + cb];
                            const int32_t sv = n32 - (int32_t)zpop2[wv][ra] - 2 * (int32_t)popb[v] +
                                               4 * (int32_t)acc[u][v][r];
                            if (idx < a.surv_cap) {
                                Survivor sr;
                                sr.j = min(j, k);
                                sr.k = max(j, k);
                                sr.rep = (uint32_t)(a.rep_abs0 + t.rep);
                                sr.s = sv;
                                sr.value = (double)sv;
                                sr.ysel = t.ysel;
                                sr.pad = 0;
                                a.surv[idx] = sr;
                            }
                            ++idx;
                        }
                    }
            }
        }
        // the slot is rewritten by this wave's next tile only after every lane has read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    for (uint64_t ti = wid; ti < a.nmfma; ti += nwave) {
        const Tile t = tile_from(T4[ti]);
        // fragments per side (wave-uniform); tiles are at most MTILE x MTILE_WIDE, so 3 x 3
        // does not occur
        const int fu = (t.na + 31) >> 5, fv = (t.nb + 31) >> 5;
        switch (fu * 4 + fv) {
        case 5: tile_body(t, I1{}, I1{}); break;
        case 6: tile_body(t, I1{}, I2{}); break;
        case 7: tile_body(t, I1{}, I3{}); break;
        case 9: tile_body(t, I2{}, I1{}); break;
        case 10: tile_body(t, I2{}, I2{}); break;
        case 11: tile_body(t, I2{}, I3{}); break;
        case 13: tile_body(t, I3{}, I1{}); break;
        case 14: tile_body(t, I3{}, I2{}); break;
        default: break;
        }
    }
}

// Big tiles (products of large buckets, kind 4): one workgroup of 8 waves per
// block pair of at most BIG_TILE x BIG_TILE columns, on the FP4 matrix cores as
// in the exact search.  Both blocks are gathered from the packed columns once,
// in chunks of BKQ quads (128 rows each), into LDS: the A side as z = y ^ x,
// the B side as x.  Lane half h of a fragment needs words h and h + 2 of a
// quad; they sit side by side in half row h of the quad's LDS row, so a
// fragment load is two runs of 256 contiguous bytes.  Eight consecutive
// threads read the 128 contiguous bytes of one column's chunk.  The next
// chunk's loads are in flight while the waves multiply the current one (two
// LDS buffers, one barrier per chunk).  The B side's words are expanded into
// FP4 operands with the shifts that give every product of two set bits the
// value 1 (expand_b_plain), so the staging does no arithmetic on them; the
// column popcounts |z_j| and |x_j| come precomputed per search, read with the
// first chunk.  Wave (wa, wb) owns A columns 64 wa.. and B columns 128 wb.. as
// up to 2 x 4 fragments of 32 x 32.  All 256 positions of both blocks are
// staged, those past the end of a block as copies of its last column, so the
// loads and stores carry no conditions and the products of the extra
// positions duplicate real ones (the cheap threshold test needs no masks);
// quads past the last are clamped and never read.  A workgroup runs tiles
// in turn: under the products of a tile's last chunk it reads the next
// tile's column ids and first chunk, so a tile's start waits for no memory.
constexpr int BKQ = 8;                          // quads per staged chunk (1024 rows)
constexpr int BHROW = BIG_TILE + 1;             // uint2 per LDS half row (words h, h + 2 of every column), padded
constexpr size_t BIG_LDS = (size_t)2 * 2 * BKQ * 2 * BHROW * sizeof(uint2);   // [buffer][side][quad][half][column]

template <bool TWO>
__global__ __launch_bounds__(512) void k_verify_lds(VerifyArgs a0)
{
    VerifyArgs a = a0;
    load_counts(a);
    extern __shared__ uint2 bl[];
    __shared__ __align__(16) uint32_t bpop[2][2][BIG_TILE];   // [tile parity][side][column] popcounts
    const int tid = (int)threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wa = wave >> 1, wb = wave & 1;
    const int h = lane >> 5, l32 = lane & 31;
    const int sq = tid & 7, sc = tid >> 3;       // staging: quad sq of columns sc + 64 r, r < 4
    const int W4 = a.W32p >> 2;
    const int NC = (W4 + BKQ - 1) / BKQ;
    const uint4 *XC4 = reinterpret_cast<const uint4 *>(a.XC);
    const uint4 *T4 = reinterpret_cast<const uint4 *>(a.tiles + a.ntiles + a.nsmall + a.nmfma);
    const int32_t n32 = (int32_t)a.n;
    int par = 0;
    uint64_t ti = blockIdx.x;
    if (ti >= a.nbig) return;
    // this thread's staging slots: column ids, every slot of the 256 x 256 block pair staged
    // (positions past the end of a block as copies of its last column); loads and stores are
    // unconditional, quads past the last are clamped and never read
    uint32_t col[8];
    uint32_t pops[8];
    uint4 pre[8], ypre;
    auto stage_cols = [&](const Tile &tt) {
        const int na_ = (int)tt.na + 1, nb_ = (int)tt.nb + 1;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int side = r >> 2, c = sc + 64 * (r & 3);
            col[r] = a.perm[(side ? tt.b0 : tt.a0) + min(c, (side ? nb_ : na_) - 1)];
        }
    };
    auto load_chunk = [&](const Tile &tt, int ch) {
        const uint4 *y4 = reinterpret_cast<const uint4 *>(a.yb + (int64_t)tt.ysel * a.W32p);
        const int qi = min(ch * BKQ + sq, W4 - 1);
        ypre = y4[qi];
#pragma unroll
        for (int r = 0; r < 8; ++r) pre[r] = XC4[(uint64_t)col[r] * W4 + qi];
        if (ch == 0 && sq == 0) {      // the staged columns' popcounts, stored with the first chunk
            const uint32_t *pz = a.cpop + (uint64_t)tt.ysel * (uint64_t)a.p, *px = a.cpop + (uint64_t)a.nys * a.p;
#pragma unroll
            for (int r = 0; r < 8; ++r) pops[r] = (r < 4 ? pz : px)[col[r]];
        }
    };
    // registers -> LDS buffer `buf` (A side z = y ^ x), words h and h + 2 into half row h; with
    // the first chunk, the popcounts
    auto store_chunk = [&](int buf, bool first) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int side = r >> 2, c = sc + 64 * (r & 3);
            uint4 v = pre[r];
            if (side == 0) {
                v.x ^= ypre.x;
                v.y ^= ypre.y;
                v.z ^= ypre.z;
                v.w ^= ypre.w;
            }
            uint2 *row = bl + (size_t)((buf * 2 + side) * BKQ + sq) * (2 * BHROW) + c;
            row[0] = make_uint2(v.x, v.z);
            row[BHROW] = make_uint2(v.y, v.w);
            if (first && sq == 0) bpop[par][side][c] = pops[r];
        }
    };
    Tile t = tile_from(T4[ti]);
    stage_cols(t);
    load_chunk(t, 0);
    for (;;) {
        const int na = (int)t.na + 1, nb = (int)t.nb + 1;
        const int FA = (na + 31) >> 5, FB = (nb + 31) >> 5;
        const int nua = min(max(FA - 2 * wa, 0), 2), nvb = min(max(FB - 4 * wb, 0), 4);
        v16f acc[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = v16f{};
        // the products of one chunk; FULL: all 2 x 4 fragments of the wave are inside the block pair
        auto compute = [&](int ch, int buf, auto full) {
            constexpr bool FULL = decltype(full)::value;
            const int nq = min(BKQ, W4 - ch * BKQ);
            const uint2 *LA = bl + (size_t)((buf * 2 + 0) * BKQ) * (2 * BHROW) + h * BHROW + wa * 64 + l32;
            const uint2 *LB = bl + (size_t)((buf * 2 + 1) * BKQ) * (2 * BHROW) + h * BHROW + wb * 128 + l32;
#pragma unroll
            for (int q = 0; q < BKQ; ++q) {
                if (q >= nq) break;
                uint2 fa[2], fb[4];
#pragma unroll
                for (int u = 0; u < 2; ++u) fa[u] = LA[q * 2 * BHROW + 32 * u];
#pragma unroll
                for (int v = 0; v < 4; ++v) fb[v] = LB[q * 2 * BHROW + 32 * v];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const v8i ea0 = expand_a(k ? fa[0].y : fa[0].x), ea1 = expand_a(k ? fa[1].y : fa[1].x);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const v8i eb = expand_b_plain(k ? fb[v].y : fb[v].x);
                        if (FULL || (0 < nua && v < nvb)) acc[0][v] = mfma_fp4(ea0, eb, acc[0][v]);
                        if (FULL || (1 < nua && v < nvb)) acc[1][v] = mfma_fp4(ea1, eb, acc[1][v]);
                    }
                }
            }
        };
        store_chunk(0, true);             // chunk 0 of this tile, loaded during the previous tile
        lds_barrier();
        const bool active = nua > 0 && nvb > 0, full = nua == 2 && nvb == 4;
        const uint64_t tn_i = ti + gridDim.x;
        const bool more = tn_i < a.nbig;
        Tile tn = t;
        for (int ch = 0; ch < NC; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < NC) {
                load_chunk(t, ch + 1);
            } else if (more) {            // the next tile's columns and first chunk, under this chunk's products
                tn = tile_from(T4[tn_i]);
                stage_cols(tn);
                load_chunk(tn, 0);
            }
            if (full) compute(ch, buf, std::true_type{});
            else if (active) compute(ch, buf, std::false_type{});
            if (ch + 1 < NC) store_chunk(buf ^ 1, false);
            lds_barrier();
        }
        do {
            if (!active) break;
            // cheap test per fragment: x = 4C - 2|z_a| over the lane's 16 rows against smin - n + 2|x_b|
            // (and -smin - n + 2|x_b| two-sided), exact in FP32
            const int32_t smin = (int32_t)a.smin[t.ysel];
            const uint32_t *popA = bpop[par][0], *popB = bpop[par][1];
            uint32_t hitmask = 0;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (u >= nua) break;
                float tA[16];
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const uint4 v4 = *reinterpret_cast<const uint4 *>(&popA[wa * 64 + u * 32 + q4 * 8 + h * 4]);
                    tA[4 * q4 + 0] = (float)(2 * v4.x);
                    tA[4 * q4 + 1] = (float)(2 * v4.y);
                    tA[4 * q4 + 2] = (float)(2 * v4.z);
                    tA[4 * q4 + 3] = (float)(2 * v4.w);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (v >= nvb) break;
                    const int32_t pb2 = 2 * (int32_t)popB[wb * 128 + v * 32 + l32];
                    float mx = -1e30f, mn = 1e30f;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float x = __builtin_fmaf(4.0f, acc[u][v][r], -tA[r]);
                        mx = fmaxf(mx, x);
                        if (TWO) mn = fminf(mn, x);
                    }
                    const bool hit = mx >= (float)(smin - n32 + pb2) || (TWO && mn <= (float)(-smin - n32 + pb2));
                    hitmask |= (hit ? 1u : 0u) << (u * 4 + v);
                }
            }
            if (__ballot(hitmask != 0) == 0) break;
            // rare: the fragments that hit are checked pair by pair.  Their counts go through this
            // wave's slot in the second staging buffer (free until the next tile stores its second
            // chunk, which follows a barrier that every wave reaches after this pass), so that the
            // rows are indexed at run time; each lane reads back only what it wrote.
            float *fbuf = reinterpret_cast<float *>(bl + (size_t)2 * BKQ * 2 * BHROW) + wave * 16 * 64;
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const bool fh = (hitmask >> (u * 4 + v)) & 1u;
                    if (__ballot(fh) == 0) continue;
#pragma unroll
                    for (int r = 0; r < 16; ++r) fbuf[r * 64 + lane] = acc[u][v][r];
                    const int cb = wb * 128 + v * 32 + l32;
                    const int32_t pb2 = 2 * (int32_t)popB[cb];
                    const int row0 = wa * 64 + u * 32 + h * 4;
                    uint32_t msk = 0;
                    if (fh && cb < nb) {
#pragma unroll 1
                        for (int r = 0; r < 16; ++r) {
                            const int ra = row0 + (r >> 2) * 8 + (r & 3);
                            const int32_t sv = n32 - 2 * (int32_t)popA[ra] - pb2 + 4 * (int32_t)fbuf[r * 64 + lane];
                            const bool pass = TWO ? ((sv < 0 ? -sv : sv) >= smin) : (sv >= smin);
                            if (pass && ra < na && (!t.diag || ra < cb)) msk |= 1u << r;
                        }
                    }
                    unsigned long long idx = reserve_survivors(a, t, __popc(msk));
                    if (idx == ~0ull) continue;
                    const uint32_t k = a.perm[t.b0 + min(cb, nb - 1)];
                    while (msk) {
                        const int r = __ffs(msk) - 1;
                        msk &= msk - 1;
                        const int ra = row0 + (r >> 2) * 8 + (r & 3);
                        const uint32_t j = a.perm[t.a0 + ra];
                        const int32_t sv = n32 - 2 * (int32_t)popA[ra] - pb2 + 4 * (int32_t)fbuf[r * 64 + lane];
                        if (idx < a.surv_cap) {
                            Survivor sr;
                            sr.j = min(j, k);
                            sr.k = max(j, k);
                            sr.rep = (uint32_t)(a.rep_abs0 + t.rep);
                            sr.s = sv;
                            sr.value = (double)sv;
                            sr.ysel = t.ysel;
                            sr.pad = 0;
                            a.surv[idx] = sr;
                        }
                        ++idx;
                    }
                }
        } while (0);
        if (!more) break;
        ti = tn_i;
        t = tn;
        par ^= 1;
    }
}

// Column popcounts for the big tiles: eight threads per column, each summing
// every eighth quad (the eight read 128 contiguous bytes at a time), reduced
// across the eight.  cpop[y][j] = |y_y ^ x_j| for y < nys, cpop[nys][j] = |x_j|.
__global__ __launch_bounds__(256) void k_col_pops(const uint4 *__restrict__ XC4, int W4, const uint4 *__restrict__ Y4,
                                                  int nys, int64_t p, uint32_t *__restrict__ cpop)
{
    const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3;
    const int e = (int)(threadIdx.x & 7);
    const bool ok = j < p;
    const uint4 *col = XC4 + (ok ? j : 0) * W4;
    uint32_t px = 0;
    for (int q = e; q < W4; q += 8) {
        const uint4 v = ok ? col[q] : make_uint4(0, 0, 0, 0);
        px += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    }
    px += __shfl_xor(px, 1, 64);
    px += __shfl_xor(px, 2, 64);
    px += __shfl_xor(px, 4, 64);
    if (ok && e == 0) cpop[(int64_t)nys * p + j] = px;
    for (int y = 0; y < nys; ++y) {
        uint32_t pz = 0;
        for (int q = e; q < W4; q += 8) {
            const uint4 v = ok ? col[q] : make_uint4(0, 0, 0, 0), w = Y4[(int64_t)y * W4 + q];
            pz += __popc(v.x ^ w.x) + __popc(v.y ^ w.y) + __popc(v.z ^ w.z) + __popc(v.w ^ w.w);
        }
        pz += __shfl_xor(pz, 1, 64);
        pz += __shfl_xor(pz, 2, 64);
        pz += __shfl_xor(pz, 4, 64);
        if (ok && e == 0) cpop[(int64_t)y * p + j] = pz;
    }
}

// Small tiles (high m: products of buckets holding a few columns each).  A
// wave reads 64 consecutive small tiles and packs them, in order, into groups
// of at most SG_COLS staged columns and 64 * SG_KP pairs.  The group's columns
// go through LDS in chunks of 16 words (A-side columns already XORed with y),
// and every lane verifies up to SG_KP of the group's pairs: two LDS reads, one
// XOR and one popcount-accumulate per pair and word, with all lanes busy
// whatever the tile shapes.
constexpr int SG_COLS = 64;
constexpr int SG_KP = 4;
constexpr int SCW4 = 4;              // uint4 per column per chunk
constexpr int SLDS4 = SCW4 + 1;      // padded row length

// Pair number `local` of a small tile: (pa, pb) = (local / nb, local % nb), or
// on a diagonal tile the pairs pa < pb < na in row order (row pa starts at
// pa na - pa (pa + 1) / 2).
XYZ_DEV void small_pair(uint32_t w, uint32_t local, uint32_t &pa, uint32_t &pb)
{
    const uint32_t na = w & 255u, nb = (w >> 8) & 255u, diag = (w >> 16) & 255u;
    if (diag) {
        pa = 0;
        while (pa + 1 < na && (pa + 1) * na - (pa + 1) * (pa + 2) / 2 <= local) ++pa;
        pb = pa + 1 + (local - (pa * na - pa * (pa + 1) / 2));
    } else {
        pa = nb ? local / nb : 0;
        pb = nb ? local % nb : 0;
    }
}

// Smallest lane l whose inclusive prefix v(l) exceeds x (64 if none).
XYZ_DEV int first_above(uint32_t v, uint32_t x)
{
    int L = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t u = __shfl(v, L + step - 1, 64);
        if (u <= x) L += step;
    }
    return L;
}

__global__ __launch_bounds__(64) void k_verify_small(VerifyArgs a0)
{
    VerifyArgs a = a0;
    load_counts(a);
    __shared__ uint4 Cs[SG_COLS][SLDS4];
    const unsigned lane = lane_id();
    const int W4 = a.W32p >> 2;
    const int nchunk = (W4 + SCW4 - 1) / SCW4;
    const uint4 *XC4 = reinterpret_cast<const uint4 *>(a.XC);
    const uint4 *Y4 = reinterpret_cast<const uint4 *>(a.yb);
    const uint4 *T4 = reinterpret_cast<const uint4 *>(a.tiles + a.ntiles);
    const uint64_t NS = a.nsmall;
    for (uint64_t g0 = (uint64_t)blockIdx.x * 64; g0 < NS; g0 += (uint64_t)gridDim.x * 64) {
        const int cnt = (int)min<uint64_t>(64, NS - g0);
        const bool have = (int)lane < cnt;
        const uint4 td = have ? T4[g0 + lane] : make_uint4(0, 0, 0, 0);
        const Tile mt = tile_from(td);
        const uint32_t cols = have ? (uint32_t)mt.na + mt.nb : 0u;
        const uint32_t np = have ? tile_pairs(mt) : 0u;
        uint32_t incC = cols, incP = np;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t uc = __shfl_up(incC, d, 64), up = __shfl_up(incP, d, 64);
            if ((int)lane >= d) {
                incC += uc;
                incP += up;
            }
        }
        int s0 = 0;
        uint32_t baseC = 0, baseP = 0;
        while (s0 < cnt) {
            // tiles [s0, e): every single tile fits (at most 64 columns, SMALL_TILE_PAIRS pairs)
            const bool fit = (int)lane >= s0 && have && incC - baseC <= (uint32_t)SG_COLS &&
                             incP - baseP <= 64u * SG_KP;
            const int e = s0 + (int)__popcll(__ballot(fit));
            const uint32_t C = __shfl(incC, e - 1, 64) - baseC;
            const uint32_t P = __shfl(incP, e - 1, 64) - baseP;
            // the column staged in slot `lane`
            uint32_t mycol = 0, myA = 0, myys = 0;
            {
                const int t = min(first_above(incC, baseC + lane), 63);
                const uint32_t tw = __shfl(td.w, t, 64), ta0 = __shfl(td.y, t, 64), tb0 = __shfl(td.z, t, 64);
                const uint32_t start = __shfl(incC, t, 64) - __shfl(cols, t, 64) - baseC;
                const uint32_t na = tw & 255u, local = lane - start;
                if (lane < C) {
                    if (local < na) {
                        mycol = a.perm[ta0 + local];
                        myA = 1;
                    } else {
                        mycol = a.perm[tb0 + local - na];
                    }
                    myys = tw >> 24;
                }
            }
            // the pairs of this lane: slots in LDS and the owning tile's lane
            uint32_t slot[SG_KP];
#pragma unroll
            for (int i = 0; i < SG_KP; ++i) {
                const uint32_t q = lane + 64u * i;
                const int t = min(first_above(incP, baseP + q), 63);
                const uint32_t tw = __shfl(td.w, t, 64);
                const uint32_t start = __shfl(incC, t, 64) - __shfl(cols, t, 64) - baseC;
                const uint32_t pstart = __shfl(incP, t, 64) - __shfl(np, t, 64) - baseP;
                uint32_t pa = 0, pb = 0;
                if (q < P) small_pair(tw, q - pstart, pa, pb);
                const uint32_t sa = q < P ? start + pa : 0u, sb = q < P ? start + (tw & 255u) + pb : 0u;
                slot[i] = sa | (sb << 8) | ((uint32_t)t << 16);
            }
            // staging assignment: slot (lane >> 2) + 16 u, uint4 lane & 3 of the chunk
            uint32_t scol[SG_COLS / 16], sflag[SG_COLS / 16];
#pragma unroll
            for (int u = 0; u < SG_COLS / 16; ++u) {
                const int cs = (int)(lane >> 2) + 16 * u;
                scol[u] = __shfl(mycol, cs, 64);
                sflag[u] = (__shfl(myA, cs, 64) ? 1u : 0u) | (__shfl(myys, cs, 64) << 8) | ((uint32_t)(cs < (int)C) << 1);
            }
            const int kp = (int)((P + 63) / 64);
            uint32_t acc[SG_KP];
#pragma unroll
            for (int i = 0; i < SG_KP; ++i) acc[i] = 0;
            for (int c = 0; c < nchunk; ++c) {
                const int gq = c * SCW4 + (int)(lane & 3);
#pragma unroll
                for (int u = 0; u < SG_COLS / 16; ++u) {
                    if (sflag[u] & 2u) {
                        uint4 v = make_uint4(0, 0, 0, 0);
                        if (gq < W4) {
                            v = XC4[(int64_t)scol[u] * W4 + gq];
                            if (sflag[u] & 1u) {
                                const uint4 yv = Y4[(int64_t)(sflag[u] >> 8) * W4 + gq];
                                v.x ^= yv.x; v.y ^= yv.y; v.z ^= yv.z; v.w ^= yv.w;
                            }
                        }
                        Cs[(lane >> 2) + 16 * u][lane & 3] = v;
                    }
                }
                lds_barrier();
#pragma unroll
                for (int w = 0; w < SCW4; ++w) {
#pragma unroll
                    for (int i = 0; i < SG_KP; ++i) {
                        if (i < kp) {
                            const uint4 x = Cs[slot[i] & 255u][w], z = Cs[(slot[i] >> 8) & 255u][w];
                            uint32_t r = acc[i];
                            r = bcnt_acc(x.x ^ z.x, r);
                            r = bcnt_acc(x.y ^ z.y, r);
                            r = bcnt_acc(x.z ^ z.z, r);
                            r = bcnt_acc(x.w ^ z.w, r);
                            acc[i] = r;
                        }
                    }
                }
                lds_barrier();
            }
            // threshold and survivors
#pragma unroll
            for (int i = 0; i < SG_KP; ++i) {
                const uint32_t q = lane + 64u * i;
                const int t = (int)(slot[i] >> 16);
                const uint32_t ys = __shfl(td.w, t, 64) >> 24, rep = __shfl(td.x, t, 64);
                const uint32_t j = __shfl(mycol, (int)(slot[i] & 255u), 64);
                const uint32_t k = __shfl(mycol, (int)((slot[i] >> 8) & 255u), 64);
                const int64_t sv = a.n - 2 * (int64_t)acc[i];
                const int64_t smin = a.smin[ys];
                const bool pass = q < P && (a.two_sided ? ((sv < 0 ? -sv : sv) >= smin) : (sv >= smin));
                const unsigned long long bal = __ballot(pass);
                if (bal == 0) continue;
                unsigned long long basei = 0;
                if (lane == 0) basei = atomicAdd(a.surv_count, (unsigned long long)__popcll(bal));
                basei = __shfl(basei, 0, 64);
                if (pass) {
                    const unsigned long long idx = basei + (unsigned long long)__popcll(bal & lanemask_lt());
                    if (idx < a.surv_cap) {
                        Survivor sr;
                        sr.j = min(j, k);
                        sr.k = max(j, k);
                        sr.rep = (uint32_t)(a.rep_abs0 + rep);
                        sr.s = (int32_t)sv;
                        sr.value = (double)sv;
                        sr.ysel = ys;
                        sr.pad = 0;
                        a.surv[idx] = sr;
                    }
                    atomicAdd(&a.info[(int64_t)rep * a.nys + ys].passed, 1ull);
                }
            }
            s0 = e;
            baseC = __shfl(incC, e - 1, 64);
            baseP = __shfl(incP, e - 1, 64);
        }
    }
}

// Real-valued verification: v = sum_i (Y_i X_ij) X_ik in binary64.  Rows are
// staged in chunks of 32: A holds Y_i X_ia (exact in binary64 for float
// inputs), B holds X_ib; each lane accumulates its RA x RB block with FMAs.
// Staging: load q covers 8 columns, lane l taking rows 4(l%8) .. 4(l%8) + 3 of
// column 8q + l/8 (16 contiguous bytes of float X, or one word of bits), and
// the next chunk's loads are issued before the current chunk's products.
// Rows past n are zero in Y (and in float X), so no row needs a mask.
constexpr int CR = 32;

template <int RA, int RB>
XYZ_DEV void verify_real_tile(const Tile &t, const uint32_t *colA, const uint32_t *colB, double (*As)[CR + 1],
                              double (*Bs)[CR + 1], const VerifyArgs &a, int x_real)
{
    const unsigned lane = lane_id();
    const int ia = lane & 7, ib = lane >> 3;
    const int sr = (int)(lane & 7) * 4, sc = (int)(lane >> 3);
    const double *yd = a.yd + (int64_t)t.ysel * a.nF;
    double acc[RA][RB];
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) acc[u][v] = 0.0;
    // the lane's staged columns (past the end of a bucket: its last column, never reported)
    int64_t ca[RA], cb[RB];
#pragma unroll
    for (int q = 0; q < RA; ++q) ca[q] = colA[min(8 * q + sc, (int)t.na - 1)];
#pragma unroll
    for (int q = 0; q < RB; ++q) cb[q] = colB[min(8 * q + sc, (int)t.nb - 1)];
    float4 xa[RA], xb[RB];
    uint32_t wa[RA], wb[RB];
    double2 y01, y23;
    auto load = [&](int64_t c) {
        const int64_t i0 = c * CR + sr;
        if (x_real) {
#pragma unroll
            for (int q = 0; q < RA; ++q) xa[q] = *reinterpret_cast<const float4 *>(a.XF + ca[q] * a.nF + i0);
#pragma unroll
            for (int q = 0; q < RB; ++q) xb[q] = *reinterpret_cast<const float4 *>(a.XF + cb[q] * a.nF + i0);
        } else {
#pragma unroll
            for (int q = 0; q < RA; ++q) wa[q] = a.XC[ca[q] * a.W32p + c];
#pragma unroll
            for (int q = 0; q < RB; ++q) wb[q] = a.XC[cb[q] * a.W32p + c];
        }
        y01 = *reinterpret_cast<const double2 *>(yd + i0);
        y23 = *reinterpret_cast<const double2 *>(yd + i0 + 2);
    };
    auto xval = [&](const float4 &f, uint32_t w, int e) -> double {
        if (x_real) return (double)(e == 0 ? f.x : e == 1 ? f.y : e == 2 ? f.z : f.w);
        return ((w >> (sr + e)) & 1u) ? -1.0 : 1.0;
    };
    const int64_t nchunk = a.nF / CR;
    load(0);
    for (int64_t c = 0; c < nchunk; ++c) {
        const double yv[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
        for (int q = 0; q < RA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) As[8 * q + sc][sr + e] = yv[e] * xval(xa[q], wa[q], e);
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[8 * q + sc][sr + e] = xval(xb[q], wb[q], e);
        __syncthreads();
        if (c + 1 < nchunk) load(c + 1);
#pragma unroll 4
        for (int rr = 0; rr < CR; ++rr) {
            double av[RA], bv[RB];
#pragma unroll
            for (int u = 0; u < RA; ++u) av[u] = As[ia + 8 * u][rr];
#pragma unroll
            for (int v = 0; v < RB; ++v) bv[v] = Bs[ib + 8 * v][rr];
#pragma unroll
            for (int u = 0; u < RA; ++u)
#pragma unroll
                for (int v = 0; v < RB; ++v) acc[u][v] = __fma_rn(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    const double kappa = a.kappa[t.ysel];
    const double dn = (double)a.n;
    uint32_t passmask = 0;
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v) {
            const int pa = ia + 8 * u, pb = ib + 8 * v;
            const double st = __ddiv_rn(acc[u][v], dn);
            const bool pass = a.two_sided ? (fabs(st) > kappa) : (st > kappa);
            if (pa < t.na && pb < t.nb && (!t.diag || pa < pb) && pass) passmask |= 1u << (u * RB + v);
        }
    unsigned long long idx = reserve_survivors(a, t, __popc(passmask));
    if (idx == ~0ull) return;
#pragma unroll
    for (int u = 0; u < RA; ++u)
#pragma unroll
        for (int v = 0; v < RB; ++v)
            if ((passmask >> (u * RB + v)) & 1u) {
                const uint32_t j = colA[ia + 8 * u], k = colB[ib + 8 * v];
                if (idx < a.surv_cap) {
                    Survivor sv;
                    sv.j = min(j, k);
                    sv.k = max(j, k);
                    sv.rep = (uint32_t)(a.rep_abs0 + t.rep);
                    sv.s = 0;
                    sv.value = acc[u][v];
                    sv.ysel = t.ysel;
                    sv.pad = 0;
                    a.surv[idx] = sv;
                }
                ++idx;
            }
}

// The same products on the FP64 matrix cores (v_mfma_f64_16x16x4_f64) for the
// 64 x 64 tiles of large bucket products (each column of a product staged
// once, against twice or more in 32 x 32 tiles): FA x FB fragments of 16 x 16,
// one product per 4 staged rows.  Lane l feeds A column u*16 + l%16 and B column
// v*16 + l%16 at row l/16 of the 4; accumulator element e of lane l is the pair
// (u*16 + l/16 + 4e, v*16 + l%16).  Staging as in verify_real_tile.
typedef double v4d __attribute__((ext_vector_type(4)));

template <int FA, int FB>
XYZ_DEV void verify_real_mfma_tile(const Tile &t, const uint32_t *colA, const uint32_t *colB,
                                   double (*As)[CR + 1], double (*Bs)[CR + 1], const VerifyArgs &a, int x_real)
{
    constexpr int RA = 2 * FA, RB = 2 * FB;
    const unsigned lane = lane_id();
    const int sr = (int)(lane & 7) * 4, sc = (int)(lane >> 3);
    const int li = (int)(lane & 15), lk = (int)(lane >> 4);
    const double *yd = a.yd + (int64_t)t.ysel * a.nF;
    v4d acc[FA][FB];
#pragma unroll
    for (int u = 0; u < FA; ++u)
#pragma unroll
        for (int v = 0; v < FB; ++v) acc[u][v] = v4d{0.0, 0.0, 0.0, 0.0};
    int64_t ca[RA], cb[RB];
#pragma unroll
    for (int q = 0; q < RA; ++q) ca[q] = colA[min(8 * q + sc, (int)t.na - 1)];
#pragma unroll
    for (int q = 0; q < RB; ++q) cb[q] = colB[min(8 * q + sc, (int)t.nb - 1)];
    float4 xa[RA], xb[RB];
    uint32_t wa[RA], wb[RB];
    double2 y01, y23;
    auto load = [&](int64_t c) {
        const int64_t i0 = c * CR + sr;
        if (x_real) {
#pragma unroll
            for (int q = 0; q < RA; ++q) xa[q] = *reinterpret_cast<const float4 *>(a.XF + ca[q] * a.nF + i0);
#pragma unroll
            for (int q = 0; q < RB; ++q) xb[q] = *reinterpret_cast<const float4 *>(a.XF + cb[q] * a.nF + i0);
        } else {
#pragma unroll
            for (int q = 0; q < RA; ++q) wa[q] = a.XC[ca[q] * a.W32p + c];
#pragma unroll
            for (int q = 0; q < RB; ++q) wb[q] = a.XC[cb[q] * a.W32p + c];
        }
        y01 = *reinterpret_cast<const double2 *>(yd + i0);
        y23 = *reinterpret_cast<const double2 *>(yd + i0 + 2);
    };
    auto xval = [&](const float4 &f, uint32_t w, int e) -> double {
        if (x_real) return (double)(e == 0 ? f.x : e == 1 ? f.y : e == 2 ? f.z : f.w);
        return ((w >> (sr + e)) & 1u) ? -1.0 : 1.0;
    };
    const int64_t nchunk = a.nF / CR;
    load(0);
    for (int64_t c = 0; c < nchunk; ++c) {
        const double yv[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
        for (int q = 0; q < RA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) As[8 * q + sc][sr + e] = yv[e] * xval(xa[q], wa[q], e);
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) Bs[8 * q + sc][sr + e] = xval(xb[q], wb[q], e);
        __syncthreads();
        if (c + 1 < nchunk) load(c + 1);
#pragma unroll
        for (int ks = 0; ks < CR / 4; ++ks) {
            const int k = ks * 4 + lk;
            double av[FA], bv[FB];
#pragma unroll
            for (int u = 0; u < FA; ++u) av[u] = As[u * 16 + li][k];
#pragma unroll
            for (int v = 0; v < FB; ++v) bv[v] = Bs[v * 16 + li][k];
#pragma unroll
            for (int u = 0; u < FA; ++u)
#pragma unroll
                for (int v = 0; v < FB; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
        }
        __syncthreads();
    }
    const double kappa = a.kappa[t.ysel];
    const double dn = (double)a.n;
    uint64_t passmask = 0;   // bit (u*FB + v)*4 + e: up to 64 pairs per lane
#pragma unroll
    for (int u = 0; u < FA; ++u)
#pragma unroll
        for (int v = 0; v < FB; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int pa = u * 16 + lk + 4 * e, pb = v * 16 + li;
                const double st = __ddiv_rn(acc[u][v][e], dn);
                const bool pass = a.two_sided ? (fabs(st) > kappa) : (st > kappa);
                if (pa < t.na && pb < t.nb && (!t.diag || pa < pb) && pass) passmask |= 1ull << ((u * FB + v) * 4 + e);
            }
    unsigned long long idx = reserve_survivors(a, t, __popcll(passmask));
    if (idx == ~0ull) return;
#pragma unroll
    for (int u = 0; u < FA; ++u)
#pragma unroll
        for (int v = 0; v < FB; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((passmask >> ((u * FB + v) * 4 + e)) & 1ull) {
                    const uint32_t j = colA[u * 16 + lk + 4 * e], k = colB[v * 16 + li];
                    if (idx < a.surv_cap) {
                        Survivor sv;
                        sv.j = min(j, k);
                        sv.k = max(j, k);
                        sv.rep = (uint32_t)(a.rep_abs0 + t.rep);
                        sv.s = 0;
                        sv.value = acc[u][v][e];
                        sv.ysel = t.ysel;
                        sv.pad = 0;
                        a.surv[idx] = sv;
                    }
                    ++idx;
                }
}

// 64 x 64 tiles of large products of real data, on the FP64 matrix cores (a kernel
// of its own: its accumulators and 64-row LDS tiles would cut the occupancy of
// the 32 x 32 kernel).
__global__ __launch_bounds__(64) void k_verify_real_mfma(VerifyArgs a0, int x_real)
{
    VerifyArgs a = a0;
    load_counts(a);
    __shared__ double As[MTILE][CR + 1];
    __shared__ double Bs[MTILE][CR + 1];
    __shared__ uint32_t colA[MTILE], colB[MTILE];
    const unsigned lane = lane_id();
    const Tile *T = a.tiles + a.ntiles + a.nsmall;
    for (uint64_t ti = blockIdx.x; ti < a.nmfma; ti += gridDim.x) {
        const Tile t = T[ti];
        {
            if (lane < t.na) colA[lane] = a.perm[t.a0 + lane];
            if (lane < t.nb) colB[lane] = a.perm[t.b0 + lane];
            __syncthreads();
            const int fa = (t.na + 15) >> 4, fb = (t.nb + 15) >> 4;
            switch (fa * 5 + fb) {
            case 6: verify_real_mfma_tile<1, 1>(t, colA, colB, As, Bs, a, x_real); break;
            case 7: verify_real_mfma_tile<1, 2>(t, colA, colB, As, Bs, a, x_real); break;
            case 8: verify_real_mfma_tile<1, 3>(t, colA, colB, As, Bs, a, x_real); break;
            case 9: verify_real_mfma_tile<1, 4>(t, colA, colB, As, Bs, a, x_real); break;
            case 11: verify_real_mfma_tile<2, 1>(t, colA, colB, As, Bs, a, x_real); break;
            case 12: verify_real_mfma_tile<2, 2>(t, colA, colB, As, Bs, a, x_real); break;
            case 13: verify_real_mfma_tile<2, 3>(t, colA, colB, As, Bs, a, x_real); break;
            case 14: verify_real_mfma_tile<2, 4>(t, colA, colB, As, Bs, a, x_real); break;
            case 16: verify_real_mfma_tile<3, 1>(t, colA, colB, As, Bs, a, x_real); break;
            case 17: verify_real_mfma_tile<3, 2>(t, colA, colB, As, Bs, a, x_real); break;
            case 18: verify_real_mfma_tile<3, 3>(t, colA, colB, As, Bs, a, x_real); break;
            case 19: verify_real_mfma_tile<3, 4>(t, colA, colB, As, Bs, a, x_real); break;
            case 21: verify_real_mfma_tile<4, 1>(t, colA, colB, As, Bs, a, x_real); break;
            case 22: verify_real_mfma_tile<4, 2>(t, colA, colB, As, Bs, a, x_real); break;
            case 23: verify_real_mfma_tile<4, 3>(t, colA, colB, As, Bs, a, x_real); break;
            case 24: verify_real_mfma_tile<4, 4>(t, colA, colB, As, Bs, a, x_real); break;
            default: break;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(64) void k_verify_real(VerifyArgs a0, int x_real)
{
    VerifyArgs a = a0;
    load_counts(a);
    __shared__ double As[TILE][CR + 1];
    __shared__ double Bs[TILE][CR + 1];
    __shared__ uint32_t colA[TILE], colB[TILE];
    const unsigned lane = lane_id();
    for (uint64_t ti = blockIdx.x; ti < a.ntiles + a.nsmall; ti += gridDim.x) {
        const Tile t = a.tiles[ti];
        if (lane < t.na) colA[lane] = a.perm[t.a0 + lane];
        if (lane >= 32 && lane - 32 < t.nb) colB[lane - 32] = a.perm[t.b0 + lane - 32];
        __syncthreads();
        const int ra = (t.na + 7) >> 3, rb = (t.nb + 7) >> 3;
        switch (ra * 4 + rb) {
        case 5: verify_real_tile<1, 1>(t, colA, colB, As, Bs, a, x_real); break;
        case 6: verify_real_tile<1, 2>(t, colA, colB, As, Bs, a, x_real); break;
        case 7: verify_real_tile<1, 3>(t, colA, colB, As, Bs, a, x_real); break;
        case 8: verify_real_tile<1, 4>(t, colA, colB, As, Bs, a, x_real); break;
        case 9: verify_real_tile<2, 1>(t, colA, colB, As, Bs, a, x_real); break;
        case 10: verify_real_tile<2, 2>(t, colA, colB, As, Bs, a, x_real); break;
        case 11: verify_real_tile<2, 3>(t, colA, colB, As, Bs, a, x_real); break;
        case 12: verify_real_tile<2, 4>(t, colA, colB, As, Bs, a, x_real); break;
        case 13: verify_real_tile<3, 1>(t, colA, colB, As, Bs, a, x_real); break;
        case 14: verify_real_tile<3, 2>(t, colA, colB, As, Bs, a, x_real); break;
        case 15: verify_real_tile<3, 3>(t, colA, colB, As, Bs, a, x_real); break;
        case 16: verify_real_tile<3, 4>(t, colA, colB, As, Bs, a, x_real); break;
        case 17: verify_real_tile<4, 1>(t, colA, colB, As, Bs, a, x_real); break;
        case 18: verify_real_tile<4, 2>(t, colA, colB, As, Bs, a, x_real); break;
        case 19: verify_real_tile<4, 3>(t, colA, colB, As, Bs, a, x_real); break;
        case 20: verify_real_tile<4, 4>(t, colA, colB, As, Bs, a, x_real); break;
        default: break;
        }
        __syncthreads();
    }
}


// ------------------------------------------------------- exact brute force --
//
// G = Z_A^T X_B for +-1 data on FP4 matrix cores.  With bits z = [Y_i X_ia = -1]
// and x = [X_ib = -1], Y_i X_ia X_ib = (1 - 2z)(1 - 2x), so
//   s = n - 2|z| - 2|x| + 4 C,   C = #{i : z_i = x_i = 1},
// and C is the dot product of two 0/1 vectors: exact in FP4 (e2m1 holds 0 and
// 1) with FP32 accumulation while C < 2^24.
//
// Staging (per call): each side's columns are copied into a blocked layout
// XB[block of 256 columns][quad of 4 words][column in block] (16 bytes: words
// 0, 2, 1, 3 of the quad), z = y ^ x on the A side, zero words past the data
// and zero padding columns, with the popcount of every staged column.  In a
// 32 x 32 x 64 matrix instruction, lanes 0-31 feed 32 rows of one column and
// lanes 32-63 the next 32 rows, so lane half h of a fragment reads words h and
// h + 2 of the quad: 8 contiguous bytes, and a wave's fragment load is 512
// contiguous bytes.

// One thread per (block, quad, column): XB[(blk * nq + qi) * 256 + c].  The A side
// (y given) holds z = y ^ x; the B side holds x with bits 0 and 2 of every nibble swapped.
__global__ __launch_bounds__(256) void k_brute_stage(const uint4 *__restrict__ XC4, int nq, int nw,
                                                     const int32_t *__restrict__ cols, int64_t ncols,
                                                     const uint4 *__restrict__ y4, int64_t nblk,
                                                     uint4 *__restrict__ XB)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (uint64_t)nblk * nq * BF_TILE) return;
    const int c = (int)(i % BF_TILE);
    const uint64_t bq = i / BF_TILE;
    const int qi = (int)(bq % (uint64_t)nq);
    const int64_t ci = (int64_t)(bq / (uint64_t)nq) * BF_TILE + c;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (ci < ncols) {
        const int64_t col = cols ? cols[ci] : ci;
        v = XC4[col * nq + qi];
        if (y4) {
            const uint4 yq = y4[qi];
            v.x ^= yq.x;
            v.y ^= yq.y;
            v.z ^= yq.z;
            v.w ^= yq.w;
        }
        const int w = qi * 4;
        if (w >= nw) v.x = 0;
        if (w + 1 >= nw) v.y = 0;
        if (w + 2 >= nw) v.z = 0;
        if (w + 3 >= nw) v.w = 0;
    }
    if (!y4) {
        // B side: swap bits 0 and 2 of every nibble (see expand_a / expand_b)
        v.x = swap02(v.x);
        v.y = swap02(v.y);
        v.z = swap02(v.z);
        v.w = swap02(v.w);
    }
    XB[i] = make_uint4(v.x, v.z, v.y, v.w);
}

// Popcount of every staged column (one thread per column, coalesced over c).
__global__ __launch_bounds__(256) void k_brute_pop(const uint4 *__restrict__ XB, int nq, int64_t nblk,
                                                   uint32_t *__restrict__ pop)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (uint64_t)nblk * BF_TILE) return;
    const uint64_t blk = i / BF_TILE, c = i % BF_TILE;
    const uint4 *src = XB + blk * (uint64_t)nq * BF_TILE + c;
    uint32_t pc = 0;
    for (int qi = 0; qi < nq; ++qi) {
        const uint4 v = src[(uint64_t)qi * BF_TILE];
        pc += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    }
    pop[i] = pc;
}

// A workgroup of 8 waves owns a 256 x 256 block of column pairs; wave (wa, wb)
// computes the 64 x 128 sub-block of A columns wa*64.. and B columns wb*128..
// as 2 x 4 fragments of 32 x 32.  Each lane loads its fragments' words straight
// from the staged layout (the waves of a workgroup share them through the L1
// cache), expands them in registers and feeds the matrix cores, with no barrier
// in the product loop.  Quads are loaded three steps ahead through a ring of
// three register sets, across tiles: the last three steps of a tile load the
// first three quads of the workgroup's next tile, so a tile starts with its data
// in flight.  XA and XB are kernel arguments of their own so that the compiler
// sees global, read-only pointers.
struct BruteFrag {
    uint2 a[2], b[4];        // words (h, h + 2) of quad qi for the lane's 2 A and 4 B columns
};

// Work slots: block pairs grouped in super-blocks of 8 x 8 (slot t: super-block t / 64,
// then row-major inside it), so that the 32 workgroups an XCD runs at a time share 12
// blocks in its L2.  Workgroups g = x mod 8 run on XCD x; the slot count and the grid
// are multiples of 8, so t(g) is a bijection and each XCD gets a contiguous range.
// Advances g (step gridDim.x) to the first slot at or after g that holds a block pair.
XYZ_DEV bool brute_next_tile(const BruteArgs &a, uint64_t &g, uint64_t &bi, uint64_t &bj)
{
    const uint64_t G = a.nslots, per = G / 8;
    for (; g < G; g += gridDim.x) {
        const uint64_t t = (g % 8) * per + g / 8;
        const uint64_t sb = t / 64, w = t % 64;
        uint64_t I, J;
        if (a.tri) {
            uint32_t i0, j0;
            tri_index(sb, (uint64_t)a.nsbA, i0, j0);
            I = i0;
            J = j0;
        } else {
            I = sb / (uint64_t)a.nsbB;
            J = sb % (uint64_t)a.nsbB;
        }
        bi = I * 8 + w / 8;
        bj = J * 8 + w % 8;
        if (bi < (uint64_t)a.nbA && bj < (uint64_t)a.nbB && !(a.tri && bi > bj)) return true;
    }
    return false;
}

template <bool TWO>
__global__ __launch_bounds__(512) void k_brute(BruteArgs a, const uint2 *__restrict__ XA,
                                               const uint2 *__restrict__ XB)
{
    __shared__ float fragbuf[8][16][64];             // per wave: one fragment of the rare pass
    __shared__ __align__(16) uint32_t popbuf[2][2 * BF_TILE];   // the tile's A, B popcounts (by tile parity)
    __shared__ unsigned int wg_n;                    // survivors of this workgroup so far
    const int tid = threadIdx.x;
    if (tid == 0) wg_n = 0;
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int wa = wave >> 1, wb = wave & 1;
    const int h = lane >> 5, l32 = lane & 31;
    const int nq = a.nq;
    const uint64_t qstride = 2 * BF_TILE;            // uint2 per quad of a block
    const int32_t n32 = (int32_t)a.n, smin32 = (int32_t)a.smin;
    const int la = 2 * (wa * 64 + l32) + h, lb = 2 * (wb * 128 + l32) + h;   // lane offsets in a quad
    // quad q of block b on either side (wave-uniform base; q clamped to the block)
    auto quad = [&](const uint2 *X, uint64_t blk, int q) {
        return X + (blk * (uint64_t)nq + (uint64_t)min(q, nq - 1)) * qstride;
    };
    auto load = [&](BruteFrag &f, const uint2 *qa, const uint2 *qb) {
#pragma unroll
        for (int u = 0; u < 2; ++u) f.a[u] = qa[la + 2 * 32 * u];
#pragma unroll
        for (int v = 0; v < 4; ++v) f.b[v] = qb[lb + 2 * 32 * v];
    };
    uint64_t g = blockIdx.x, bi = 0, bj = 0;
    bool have = brute_next_tile(a, g, bi, bj);
    BruteFrag f0, f1, f2;
    if (have) {
        load(f0, quad(XA, bi, 0), quad(XB, bj, 0));
        load(f1, quad(XA, bi, 1), quad(XB, bj, 1));
        load(f2, quad(XA, bi, 2), quad(XB, bj, 2));
    }
    int par = 0;
    while (have) {
        // the next tile (or this one again when there is none: its loads are then unused)
        uint64_t g2 = g + gridDim.x, bi2 = bi, bj2 = bj;
        const bool have2 = brute_next_tile(a, g2, bi2, bj2);
        if (!have2) {
            bi2 = bi;
            bj2 = bj;
        }
        // this tile's popcounts, for the epilogue: one value per thread, stored to LDS after the products
        const uint32_t popv = tid < BF_TILE ? a.popA[bi * BF_TILE + tid] : a.popB[bj * BF_TILE + tid - BF_TILE];

        v16f acc[2][4];
        // one quad: the products of its two words, then the load of quad qi + 3 into the freed
        // registers (slot s of the ring: the next tile's quad s once qi + 3 is past the end);
        // the first quad's first product starts the accumulators (a zero operand)
        auto step = [&](BruteFrag &f, int qi, int slot, auto first) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                v8i fa[2], fb[4];
#pragma unroll
                for (int u = 0; u < 2; ++u) fa[u] = expand_a(k ? f.a[u].y : f.a[u].x);
#pragma unroll
                for (int v = 0; v < 4; ++v) fb[v] = expand_b(k ? f.b[v].y : f.b[v].x);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[u][v] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            fa[u], fb[v], (decltype(first)::value && k == 0) ? v16f{} : acc[u][v], 4, 4, 0, 127, 0,
                            127);
            }
            const bool cur = qi + 3 < nq;
            load(f, cur ? quad(XA, bi, qi + 3) : quad(XA, bi2, slot), cur ? quad(XB, bj, qi + 3) : quad(XB, bj2, slot));
            // keep the loads where they are: each set is consumed three steps later
            __builtin_amdgcn_sched_barrier(0);
        };
        step(f0, 0, 0, std::true_type{});
        int qi = 1;
        for (; qi + 2 < nq; qi += 3) {      // no branches inside: each wait is for the oldest loads only
            step(f1, qi, 1, std::false_type{});
            step(f2, qi + 1, 2, std::false_type{});
            step(f0, qi + 2, 0, std::false_type{});
        }
        if (qi < nq) step(f1, qi, 1, std::false_type{});
        if (qi + 1 < nq) step(f2, qi + 1, 2, std::false_type{});
        // each stepped slot now holds the next tile's quad of the same number (all three when
        // nq >= 3; with fewer quads, the slots that were not stepped are not used either)

        popbuf[par][tid] = popv;
        __syncthreads();
        const uint32_t *popAt = popbuf[par], *popBt = popbuf[par] + BF_TILE;

        // epilogue: accumulator register r of lane l holds row (r/4)*8 + (l/32)*4 + r%4, column l%32.
        // s = n - 2|z_a| - 2|x_b| + 4C >= smin  <=>  4C - 2|z_a| >= smin - n + 2|x_b|, exact in FP32
        // (|values| < 2^26).  A cheap test of the row maximum (and minimum, two-sided) runs on every
        // fragment; the rare fragments that hit are checked pair by pair.
        const bool diag = a.tri && bi == bj;
        // 2|z_a| of the lane's 16 rows of A fragment u
        auto rows_pop2 = [&](int u, float *tA) {
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const uint4 v4 = *reinterpret_cast<const uint4 *>(&popAt[wa * 64 + u * 32 + q4 * 8 + h * 4]);
                tA[4 * q4 + 0] = (float)(2 * (int32_t)v4.x);
                tA[4 * q4 + 1] = (float)(2 * (int32_t)v4.y);
                tA[4 * q4 + 2] = (float)(2 * (int32_t)v4.z);
                tA[4 * q4 + 3] = (float)(2 * (int32_t)v4.w);
            }
        };
        uint32_t hitmask = 0;     // bit u*4+v: this lane has a candidate in fragment (u, v)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            float tA[16];
            rows_pop2(u, tA);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t pb2 = 2 * (int32_t)popBt[wb * 128 + v * 32 + l32];
                float mx = -1e30f, mn = 1e30f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float x = __builtin_fmaf(4.0f, acc[u][v][r], -tA[r]);
                    mx = fmaxf(mx, x);
                    if (TWO) mn = fminf(mn, x);
                }
                const bool hit = mx >= (float)(smin32 - n32 + pb2) || (TWO && mn <= (float)(-smin32 - n32 + pb2));
                hitmask |= (hit ? 1u : 0u) << (u * 4 + v);
            }
        }
        if (__ballot(hitmask != 0) != 0) {
            // pair-by-pair pass on the fragments that hit (rare): x = 4C - 2|z_a| of the fragment goes
            // to the wave's LDS slot, so that the pass can index its rows at run time, then validity
            // (padding columns, j != k, a < b on a diagonal block) and the survivors' slots, with one
            // atomic per fragment and wave.  s = n - 2|x_b| + x.
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                float tA[16];
                rows_pop2(u, tA);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (__ballot((hitmask >> (u * 4 + v)) & 1u) == 0) continue;
#pragma unroll
                    for (int r = 0; r < 16; ++r) fragbuf[wave][r][lane] = __builtin_fmaf(4.0f, acc[u][v][r], -tA[r]);
                    const int cb = wb * 128 + v * 32 + l32;
                    const int64_t cjb = (int64_t)bj * BF_TILE + cb;
                    const bool okb = cjb < a.nB && ((hitmask >> (u * 4 + v)) & 1u);
                    const int32_t gb = cjb < a.nB ? (a.colsB ? a.colsB[cjb] : (int32_t)cjb) : -1;
                    const int32_t pb2 = 2 * (int32_t)popBt[cb];
                    const int32_t hi = smin32 - n32 + pb2, lo = -smin32 - n32 + pb2;
                    const int row0 = wa * 64 + u * 32 + h * 4;
                    uint32_t m = 0;
                    if (okb) {
#pragma unroll 4
                        for (int r = 0; r < 16; ++r) {
                            const int ra = row0 + (r >> 2) * 8 + (r & 3);
                            const int32_t x = (int32_t)fragbuf[wave][r][lane];
                            const bool pass = x >= hi || (TWO && x <= lo);
                            const bool ok = (int64_t)bi * BF_TILE + ra < a.nA && !(diag && ra >= cb);
                            m |= (pass && ok ? 1u : 0u) << r;
                        }
                    }
                    // with column lists a column can meet itself (the same id on both sides); with
                    // identity lists that happens only on a diagonal block, excluded by a < b
                    if (a.colsA || a.colsB) {
                        for (uint32_t mm = m; mm;) {
                            const int r = __ffs(mm) - 1;
                            mm &= mm - 1;
                            const int64_t cja = (int64_t)bi * BF_TILE + row0 + (r >> 2) * 8 + (r & 3);
                            if ((a.colsA ? a.colsA[cja] : (int32_t)cja) == gb) m &= ~(1u << r);
                        }
                    }
                    const int mine = __popc(m);
                    int incl = mine;
#pragma unroll
                    for (int d = 1; d < 64; d <<= 1) {
                        const int yv = __shfl_up(incl, d, 64);
                        if (lane >= d) incl += yv;
                    }
                    const int total = __shfl(incl, 63, 64);
                    if (total == 0) continue;
                    unsigned int base = 0;
                    if (lane == 0) base = atomicAdd(&wg_n, (unsigned int)total);
                    base = __shfl(base, 0, 64);
                    uint64_t idx = base + (uint64_t)(incl - mine);
                    Survivor *mysurv = a.surv + (uint64_t)blockIdx.x * a.cap_wg;
                    while (m) {
                        const int r = __ffs(m) - 1;
                        m &= m - 1;
                        const int64_t cja = (int64_t)bi * BF_TILE + row0 + (r >> 2) * 8 + (r & 3);
                        const int32_t ga = a.colsA ? a.colsA[cja] : (int32_t)cja;
                        if (idx < a.cap_wg) {
                            Survivor sv;
                            sv.j = (uint32_t)min(ga, gb);
                            sv.k = (uint32_t)max(ga, gb);
                            sv.rep = 0;
                            sv.s = n32 - pb2 + (int32_t)fragbuf[wave][r][lane];
                            sv.value = (double)sv.s;
                            sv.ysel = 0;
                            sv.pad = 0;
                            mysurv[idx] = sv;
                        }
                        ++idx;
                    }
                }
            }
        }
        g = g2;
        bi = bi2;
        bj = bj2;
        have = have2;
        par ^= 1;
    }
    __syncthreads();
    if (tid == 0) a.wg_count[blockIdx.x] = wg_n;
}

// Dense copy of the workgroups' survivor regions: workgroup g's count[g] survivors
// (at most cap each) go to dense[offs[g] ...].
__global__ __launch_bounds__(256) void k_brute_compact(const Survivor *__restrict__ sparse, uint64_t cap,
                                                       const unsigned int *__restrict__ count,
                                                       const unsigned long long *__restrict__ offs,
                                                       Survivor *__restrict__ dense)
{
    const int g = blockIdx.x;
    const unsigned int c = count[g];
    for (unsigned int i = threadIdx.x; i < c; i += 256) dense[offs[g] + i] = sparse[(uint64_t)g * cap + i];
}

// ---------------------------------------------------------------- planner --

// One wave per pair.  Binary Y: gamma = 1 - popcount(y ^ x_j ^ x_k) / n.
// Real Y: gamma = sum of |Y_i| over agreeing rows / ||Y||_1 (the collision
// probability of one |Y|-weighted row draw, Section 3.1).
__global__ __launch_bounds__(256) void k_pair_strengths(const uint32_t *__restrict__ XC, int W32p,
                                                        const uint32_t *__restrict__ yb,
                                                        const double *__restrict__ yd, int64_t n, int64_t p,
                                                        int real_y, uint64_t seed, int64_t npairs,
                                                        double *__restrict__ gamma)
{
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= npairs) return;
    const unsigned lane = lane_id();
    const uint64_t u = splitmix64_at(seed, 2ull * q + 1), v = splitmix64_at(seed, 2ull * q + 2);
    const int64_t j = (int64_t)__umul64hi(u, (uint64_t)p);
    int64_t k = (int64_t)__umul64hi(v, (uint64_t)(p - 1));
    k += (k >= j) ? 1 : 0;
    const uint32_t *xj = XC + j * (int64_t)W32p, *xk = XC + k * (int64_t)W32p;
    if (!real_y) {
        uint32_t c = 0;
        for (int w = lane; w < W32p; w += 64) c += __popc(yb[w] ^ xj[w] ^ xk[w]);
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
        if (lane == 0) gamma[q] = 1.0 - (double)c / (double)n;
        return;
    }
    double agree = 0.0, tot = 0.0;
    for (int64_t i = lane; i < n; i += 64) {
        const double a = fabs(yd[i]);
        const uint32_t bit = ((yb[i >> 5] ^ xj[i >> 5] ^ xk[i >> 5]) >> (i & 31)) & 1u;
        tot += a;
        if (!bit) agree += a;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        agree += __shfl_xor(agree, d, 64);
        tot += __shfl_xor(tot, d, 64);
    }
    if (lane == 0) gamma[q] = tot > 0.0 ? agree / tot : 0.0;
}

// ------------------------------------------------------- scan, radix sort --

constexpr int RS_NT = 256, RS_IPT = 8, RS_TILE = RS_NT * RS_IPT;
constexpr uint64_t RS_SMALL = 32768;   // survivor counts merged by one workgroup

__global__ __launch_bounds__(RS_NT) void k_scan_reduce(const uint32_t *__restrict__ in, uint64_t cnt,
                                                       uint32_t *__restrict__ partial)
{
    __shared__ unsigned long long shm[RS_NT / 64 + 1];
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    unsigned long long s = 0;
    for (int e = 0; e < RS_IPT; ++e) {
        const uint64_t i = base + (uint64_t)e * RS_NT + threadIdx.x;
        if (i < cnt) s += in[i];
    }
    s = block_sum<RS_NT>(s, shm);
    if (threadIdx.x == 0) partial[blockIdx.x] = (uint32_t)s;
}

__global__ __launch_bounds__(1024) void k_scan_single(uint32_t *__restrict__ v, uint64_t cnt)
{
    __shared__ unsigned long long shm[17];
    const uint64_t seg = (cnt + 1023) / 1024;
    const uint64_t i0 = min(cnt, (uint64_t)threadIdx.x * seg), i1 = min(cnt, i0 + seg);
    unsigned long long loc = 0;
    for (uint64_t i = i0; i < i1; ++i) loc += v[i];
    unsigned long long tot;
    unsigned long long pre = block_scan_excl<1024>(loc, shm, &tot);
    for (uint64_t i = i0; i < i1; ++i) {
        const uint32_t x = v[i];
        v[i] = (uint32_t)pre;
        pre += x;
    }
}

// Exclusive scan of in[0..cnt) into out (may alias in), given exclusive block offsets.
__global__ __launch_bounds__(RS_NT) void k_scan_apply(const uint32_t *in, uint64_t cnt, const uint32_t *partial,
                                                      uint32_t *out)
{
    __shared__ unsigned long long shm[RS_NT / 64 + 1];
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE + (uint64_t)threadIdx.x * RS_IPT;
    uint32_t vals[RS_IPT];
    unsigned long long s = 0;
    for (int e = 0; e < RS_IPT; ++e) {
        const uint64_t i = base + e;
        vals[e] = i < cnt ? in[i] : 0;
        s += vals[e];
    }
    unsigned long long tot;
    unsigned long long pre = block_scan_excl<RS_NT>(s, shm, &tot) + partial[blockIdx.x];
    for (int e = 0; e < RS_IPT; ++e) {
        const uint64_t i = base + e;
        if (i < cnt) out[i] = (uint32_t)pre;
        pre += vals[e];
    }
}

__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t *__restrict__ keys, uint64_t S, int shift,
                                                   uint32_t *__restrict__ hist, uint32_t nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int e = 0; e < RS_IPT; ++e) {
        const uint64_t i = base + (uint64_t)e * RS_NT + threadIdx.x;
        if (i < S) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items are taken in index order, 256 per step; within a step
// the rank of an item among equal digits is (count in earlier waves) + (rank
// among its wave's peers, found by 8 ballots on the digit bits).
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
                                                      uint32_t *__restrict__ vout, uint64_t S, int shift,
                                                      const uint32_t *__restrict__ hist, uint32_t nblocks)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[RS_NT / 64][256];
    const int tid = threadIdx.x, w = tid >> 6;
    run[tid] = hist[(uint64_t)tid * nblocks + blockIdx.x];
    const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
    for (int e = 0; e < RS_IPT; ++e) {
#pragma unroll
        for (int q = 0; q < RS_NT / 64; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        const uint64_t i = base + (uint64_t)e * RS_NT + tid;
        const bool valid = i < S;
        uint64_t k = 0;
        uint32_t v = 0, d = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
            d = (uint32_t)(k >> shift) & 255u;
        }
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < RS_NT / 64; ++q) add += wcnt[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_dedup_keys(const Survivor *__restrict__ surv, uint64_t S, int64_t p,
                                                    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const Survivor s = surv[i];
    keys[i] = ((uint64_t)s.ysel * (uint64_t)p + s.j) * (uint64_t)p + s.k;
    vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_dedup_heads(const uint64_t *__restrict__ keys, uint64_t S,
                                                     uint32_t *__restrict__ heads)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    heads[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// The unique pair whose first sorted record is at position i goes to out[u]: first repetition,
// hits, and the per-response and per-repetition counters (lanes with equal targets add once).
// Called by the lanes that hold a head only.
XYZ_DEV void dedup_emit_head(uint64_t i, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                             const Survivor *__restrict__ surv, uint64_t S, uint64_t u, int64_t n, int nys,
                             OutPair *__restrict__ out, unsigned long long *__restrict__ ycount,
                             RepInfo *__restrict__ info, int64_t rep_abs0)
{
    const Survivor s0 = surv[vals[i]];
    uint32_t first = s0.rep;
    int32_t hits = 0;
    for (uint64_t q = i; q < S && keys[q] == keys[i]; ++q) {
        first = min(first, surv[vals[q]].rep);
        ++hits;
    }
    OutPair o;
    o.j = (int32_t)s0.j;
    o.k = (int32_t)s0.k;
    o.s = s0.s;
    o.value = s0.value;
    o.stat = __ddiv_rn(s0.value, (double)n);
    o.first_rep = (int32_t)first;
    o.hits = hits;
    out[u] = o;
    // per-response and per-repetition counters: lanes with equal targets add once
    unsigned long long todo = __ballot(1);
    const unsigned long long key_y = s0.ysel;
    const unsigned long long key_f = ((unsigned long long)(first - rep_abs0) << 8) | s0.ysel;
    const unsigned lane = lane_id();
    unsigned long long left = todo;
    while (left) {
        const int leader = __ffsll((long long)left) - 1;
        const unsigned long long v = __shfl(key_y, leader, 64);
        const unsigned long long same = __ballot(key_y == v) & left;
        if ((int)lane == leader) atomicAdd(&ycount[v], (unsigned long long)__popcll(same));
        left &= ~same;
    }
    left = todo;
    while (left) {
        const int leader = __ffsll((long long)left) - 1;
        const unsigned long long v = __shfl(key_f, leader, 64);
        const unsigned long long same = __ballot(key_f == v) & left;
        if ((int)lane == leader)
            atomicAdd(&info[(int64_t)(v >> 8) * nys + (int64_t)(v & 255)].fresh, (unsigned long long)__popcll(same));
        left &= ~same;
    }
}

__global__ __launch_bounds__(256) void k_dedup_emit(const uint64_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ vals,
                                                    const Survivor *__restrict__ surv, uint64_t S,
                                                    const uint32_t *__restrict__ heads_scan, int64_t n, int nys,
                                                    OutPair *__restrict__ out, unsigned long long *__restrict__ ycount,
                                                    RepInfo *__restrict__ info, int64_t rep_abs0)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    if (i != 0 && keys[i] == keys[i - 1]) return;
    dedup_emit_head(i, keys, vals, surv, S, heads_scan[i], n, nys, out, ycount, info, rep_abs0);
}

// Merges of at most RS_SMALL survivors run in one workgroup each: the sort's passes and the
// heads' prefix sum stay inside one launch instead of a few launches per pass.
constexpr int RSS_NT = 1024;

// Stable LSD radix sort of S (key, value) pairs on the low `bits` bits, 8 bits per pass, by one
// workgroup: items are taken in index order, RSS_NT per step, each ranked among equal digits
// by (count in earlier waves of the step) + (rank among its wave's peers, 8 ballots).
// Ping-pongs between (k0, v0) and (k1, v1): the result is in (k0, v0) after an even number of
// passes, else in (k1, v1).
__global__ __launch_bounds__(RSS_NT) void k_rs_sort_small(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                                                          uint32_t S, int bits)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[RSS_NT / 64][256];
    const int tid = threadIdx.x, w = tid >> 6;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int shift = 0; shift < bits; shift += 8) {
        if (tid < 256) run[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < S; i += RSS_NT) atomicAdd(&run[(uint32_t)(ka[i] >> shift) & 255u], 1u);
        __syncthreads();
        if (tid < 64) {                              // exclusive scan of the 256 counts by one wave
            const uint32_t c0 = run[4 * tid], c1 = run[4 * tid + 1], c2 = run[4 * tid + 2], c3 = run[4 * tid + 3];
            const uint32_t sum = c0 + c1 + c2 + c3;
            uint32_t inc = sum;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t t = __shfl_up(inc, d, 64);
                if (tid >= d) inc += t;
            }
            const uint32_t ex = inc - sum;
            run[4 * tid] = ex;
            run[4 * tid + 1] = ex + c0;
            run[4 * tid + 2] = ex + c0 + c1;
            run[4 * tid + 3] = ex + c0 + c1 + c2;
        }
        __syncthreads();
        for (uint32_t base = 0; base < S; base += RSS_NT) {
#pragma unroll
            for (int q = 0; q < RSS_NT / 64 / 4; ++q) wcnt[(tid >> 8) + 4 * q][tid & 255] = 0;
            __syncthreads();
            const uint32_t i = base + tid;
            const bool valid = i < S;
            uint64_t k = 0;
            uint32_t v = 0, d = 0;
            if (valid) {
                k = ka[i];
                v = va[i];
                d = (uint32_t)(k >> shift) & 255u;
            }
            unsigned long long peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bal = __ballot(valid && bit);
                peers &= bit ? bal : ~bal;
            }
            const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
            if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t pos = run[d] + rank;
                for (int q = 0; q < w; ++q) pos += wcnt[q][d];
                kb[pos] = k;
                vb[pos] = v;
            }
            __syncthreads();
            if (tid < 256) {
                uint32_t add = 0;
#pragma unroll
                for (int q = 0; q < RSS_NT / 64; ++q) add += wcnt[q][tid];
                run[tid] += add;
            }
            __syncthreads();
        }
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
}

// Heads of the sorted keys, their prefix sum and the unique pairs, by one workgroup.
__global__ __launch_bounds__(RSS_NT) void k_dedup_small(const uint64_t *__restrict__ keys,
                                                        const uint32_t *__restrict__ vals,
                                                        const Survivor *__restrict__ surv, uint32_t S, int64_t n,
                                                        int nys, OutPair *__restrict__ out,
                                                        unsigned long long *__restrict__ nout,
                                                        unsigned long long *__restrict__ ycount,
                                                        RepInfo *__restrict__ info, int64_t rep_abs0)
{
    __shared__ uint32_t wsum[RSS_NT / 64];
    const int tid = threadIdx.x, w = tid >> 6;
    uint32_t u0 = 0;
    for (uint32_t base = 0; base < S; base += RSS_NT) {
        const uint32_t i = base + tid;
        const bool head = i < S && (i == 0 || keys[i] != keys[i - 1]);
        const unsigned long long hb = __ballot(head);
        if ((tid & 63) == 0) wsum[w] = (uint32_t)__popcll(hb);
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int q = 0; q < RSS_NT / 64; ++q) {
            const uint32_t c = wsum[q];
            before += q < w ? c : 0u;
            total += c;
        }
        if (head)
            dedup_emit_head(i, keys, vals, surv, S, u0 + before + (uint32_t)__popcll(hb & lanemask_lt()), n, nys, out,
                            ycount, info, rep_abs0);
        u0 += total;
        __syncthreads();
    }
    if (tid == 0) *nout = u0;
}

__global__ void k_dedup_count(const uint32_t *__restrict__ heads_scan, const uint64_t *__restrict__ keys, uint64_t S,
                              unsigned long long *__restrict__ nout)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (S == 0) {
        *nout = 0;
        return;
    }
    const bool last_head = (S == 1) || keys[S - 1] != keys[S - 2];
    *nout = (unsigned long long)heads_scan[S - 1] + (last_head ? 1ull : 0ull);
}

// ------------------------------------------------------------- launchers --

static inline unsigned grid1(uint64_t work, unsigned per) { return (unsigned)((work + per - 1) / per); }

__global__ __launch_bounds__(256) void k_zero(uint32_t *__restrict__ p, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st)
{
    const uint64_t count = bytes / 4;
    if (count == 0) return hipSuccess;
    k_zero<<<(unsigned)std::min<uint64_t>(grid1(count, 256), 4096), 256, 0, st>>>((uint32_t *)p, count);
    return hipGetLastError();
}

hipError_t kernels_init()
{
    hipError_t e = hipFuncSetAttribute((const void *)k_bucket, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)std::max<size_t>((size_t)4 << MAX_M_LDS, BUCKET_LDS));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_verify_lds<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)BIG_LDS);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_verify_lds<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)BIG_LDS);
    return e;
}

hipError_t launch_pack_x_i8(const int8_t *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC, int *err,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x_i8, dim3(grid1(p, 4)), dim3(256), 0, st, X, ld, n, p, W32p, XC, err);
    return hipGetLastError();
}

hipError_t launch_pack_x_i8_rows(const int8_t *X, int64_t ld, int64_t n, int64_t p, uint64_t *XR, int64_t P64,
                                 int *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x_i8_rows, dim3(grid1((uint64_t)n * (uint64_t)P64, 4)), dim3(256), 0, st, X, ld, n, p,
                       XR, P64, err);
    return hipGetLastError();
}

hipError_t launch_transpose_rc(const uint64_t *XR, int64_t n, int64_t p, int64_t P64, int W32p, uint32_t *XC,
                               hipStream_t st)
{
    const uint64_t waves = (uint64_t)P64 * (uint64_t)(W32p / 4);
    hipLaunchKernelGGL(k_transpose_rc, dim3(grid1(waves, 4)), dim3(256), 0, st, XR, n, p, P64, W32p, XC);
    return hipGetLastError();
}

hipError_t launch_pack_x_f32(const float *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC, float *XF,
                             int64_t nF, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x_f32, dim3(grid1(p, 4)), dim3(256), 0, st, X, ld, n, p, W32p, XC, XF, nF, err);
    return hipGetLastError();
}

hipError_t launch_pack_x_bits(const uint64_t *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_x_bits, dim3(grid1((uint64_t)p * (W32p / 2), 256)), dim3(256), 0, st, X, ld, n, p,
                       W32p, XC);
    return hipGetLastError();
}

hipError_t launch_transpose(const uint32_t *XC, int64_t n, int64_t p, int W32p, uint64_t *XR, int64_t P64,
                            hipStream_t st)
{
    const uint64_t waves = (uint64_t)((p + 63) / 64) * (uint64_t)(W32p / 4);
    hipLaunchKernelGGL(k_transpose, dim3(grid1(waves, 4)), dim3(256), 0, st, XC, n, p, W32p, XR, P64);
    return hipGetLastError();
}

hipError_t launch_pack_y(const void *Y, int yfmt, int64_t n, int W32p, uint32_t *yb, double *yd, int64_t nF,
                         int *err, hipStream_t st)
{
    const int64_t nb = (int64_t)W32p * 32;
    const int64_t lim = nb > nF ? nb : nF;
    hipLaunchKernelGGL(k_pack_y, dim3(grid1(lim, 256)), dim3(256), 0, st, Y, yfmt, n, W32p, yb, yd, nF, err);
    return hipGetLastError();
}

hipError_t launch_cdf(const double *yd, int64_t n, double *cdf, int64_t *last, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_cdf, dim3(1), dim3(64), 0, st, yd, n, cdf, last, err);
    return hipGetLastError();
}

hipError_t launch_sample(uint64_t seed, int64_t rep0, int nrep, int m, int64_t n, int weighted, const double *cdf,
                         const int64_t *last, int32_t *rows, hipStream_t st)
{
    if (m == 0 || nrep == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample, dim3(grid1((uint64_t)nrep * m, 256)), dim3(256), 0, st, seed, rep0, nrep, m, n,
                       weighted, cdf, last, rows);
    return hipGetLastError();
}

hipError_t launch_cmask(const int32_t *rows, int nrep, int m, int nys, const uint32_t *yb, int yb_stride,
                        RepInfo *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_cmask, dim3(grid1((uint64_t)nrep * nys, 256)), dim3(256), 0, st, rows, nrep, m, nys, yb,
                       yb_stride, info);
    return hipGetLastError();
}

hipError_t launch_row_absmax(const float *XF, int64_t nF, int64_t n, int64_t p, float cap, uint32_t *nu,
                             hipStream_t st)
{
    const hipError_t e = launch_zero(nu, sizeof(uint32_t) * (size_t)n, st);
    if (e != hipSuccess) return e;
    const int64_t slices = std::min<int64_t>(std::max<int64_t>(p / 64, 1), 4096);
    const int64_t per = (p + slices - 1) / slices;
    uint32_t capb;
    std::memcpy(&capb, &cap, sizeof capb);
    hipLaunchKernelGGL(k_row_absmax, dim3(grid1(n, 256), (unsigned)slices), dim3(256), 0, st, XF, nF, n, p, per, capb,
                       nu);
    return hipGetLastError();
}

hipError_t launch_cdf_unbiased(const double *yd, const uint32_t *nu, int64_t n, double *cdf, int64_t *last, int *err,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_cdf_unbiased, dim3(1), dim3(64), 0, st, yd, nu, n, cdf, last, err);
    return hipGetLastError();
}

hipError_t launch_hash_unbiased(const float *XF, int64_t nF, int64_t p, int m, int nrep, const int32_t *rows,
                                const uint32_t *nu, float cap, uint64_t seed, int64_t rep0, uint32_t *keys,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_hash_unbiased, dim3(grid1(p, 256), nrep), dim3(256), 0, st, XF, nF, p, m, rows, nu, cap,
                       seed, rep0, keys);
    return hipGetLastError();
}

hipError_t launch_hash(const uint64_t *XR, int64_t P64, int64_t p, int m, int nrep, const int32_t *rows,
                       uint32_t *keys, hipStream_t st)
{
    hipLaunchKernelGGL(k_hash, dim3(grid1(p, 256 * HASH_COLS), nrep), dim3(256), 0, st, XR, P64, p, m, rows, keys);
    return hipGetLastError();
}

hipError_t launch_bucket(const uint32_t *keys, int64_t p, int m, int nrep, int nys, RepInfo *info, int two_sided,
                         int mfma, uint32_t *offs, uint32_t *perm, hipStream_t st)
{
    // chunked scatter while the bucket counters, the chunk's offsets and cursors and a chunk of
    // ids and 16-bit keys fit in BUCKET_LDS with runs of at least two ids per bucket on average
    // (m <= 12); direct scatter above
    const int nb = 1 << m;
    const size_t base = (size_t)4 * (3 * (size_t)nb + 1), budget = BUCKET_LDS;
    int ch = 0;
    if (base + 8 * 4096 <= budget) ch = (int)std::min<size_t>((budget - base) / 8 / 1024 * 1024, 65536);
    if (ch < 2 * nb) ch = 0;
    const size_t lds = ch ? base + 8 * (size_t)ch : (size_t)4 << m;
    hipLaunchKernelGGL(k_bucket, dim3(nrep), dim3(1024), lds, st, keys, p, m, nys, info, two_sided, mfma, offs,
                       perm, ch);
    return hipGetLastError();
}

hipError_t launch_tile_scan(const RepInfo *info, int count, unsigned long long *base, unsigned long long *totals,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, info, count, base, totals);
    return hipGetLastError();
}

hipError_t launch_tiles(const uint32_t *offs, int64_t p, int m, int nrep, int nys, const RepInfo *info,
                        int two_sided, int mfma, const unsigned long long *base, Tile *tiles, uint64_t cap,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_tiles, dim3(nrep * nys), dim3(256), 0, st, offs, p, m, nys, info, two_sided, mfma, base,
                       tiles, cap);
    return hipGetLastError();
}

hipError_t launch_verify_bin(const VerifyArgs &a, int grid, hipStream_t st)
{
    if (a.ntiles)
        hipLaunchKernelGGL(k_verify_bin, dim3((unsigned)std::min<uint64_t>(a.ntiles, (uint64_t)grid)), dim3(64), 0, st,
                           a);
    if (a.nmfma)
        hipLaunchKernelGGL(k_verify_mfma, dim3((unsigned)std::min<uint64_t>((a.nmfma + 3) / 4, (uint64_t)grid)),
                           dim3(256), 0, st, a);
    if (a.nsmall) {
        const uint64_t groups = (a.nsmall + 63) / 64;                  // 64 small tiles per wave step
        hipLaunchKernelGGL(k_verify_small, dim3((unsigned)std::min<uint64_t>(groups, (uint64_t)grid)), dim3(64), 0, st,
                           a);
    }
    return hipGetLastError();
}

hipError_t launch_col_pops(const uint32_t *XC, int W32p, const uint32_t *yb, int nys, int64_t p, uint32_t *cpop,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_col_pops, dim3(grid1((uint64_t)p * 8, 256)), dim3(256), 0, st,
                       reinterpret_cast<const uint4 *>(XC), W32p / 4, reinterpret_cast<const uint4 *>(yb), nys, p, cpop);
    return hipGetLastError();
}

hipError_t launch_verify_big(const VerifyArgs &a, int grid, hipStream_t st)
{
    if (a.nbig) {
        const unsigned g = (unsigned)std::min<uint64_t>(a.nbig, (uint64_t)std::max(grid, 1));
        if (a.two_sided)
            hipLaunchKernelGGL(k_verify_lds<true>, dim3(g), dim3(512), BIG_LDS, st, a);
        else
            hipLaunchKernelGGL(k_verify_lds<false>, dim3(g), dim3(512), BIG_LDS, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_verify_real(const VerifyArgs &a, int x_real, int grid, hipStream_t st)
{
    if (a.ntiles + a.nsmall > 0)
        hipLaunchKernelGGL(k_verify_real, dim3(grid), dim3(64), 0, st, a, x_real);
    if (a.nmfma > 0)
        hipLaunchKernelGGL(k_verify_real_mfma, dim3((unsigned)std::min<uint64_t>(a.nmfma, (uint64_t)grid)), dim3(64), 0,
                           st, a, x_real);
    return hipGetLastError();
}

hipError_t launch_brute_stage(const uint32_t *XC, int W32p, int nw, const int32_t *cols, int64_t ncols,
                              const uint32_t *yb, uint4 *XB, uint32_t *pop, hipStream_t st)
{
    const int nq = W32p >> 2;
    const int64_t nblk = (ncols + BF_TILE - 1) / BF_TILE;
    if (nblk == 0) return hipSuccess;
    const uint64_t total = (uint64_t)nblk * nq * BF_TILE;
    hipLaunchKernelGGL(k_brute_stage, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const uint4 *>(XC), nq, nw, cols, ncols, reinterpret_cast<const uint4 *>(yb),
                       nblk, XB);
    hipLaunchKernelGGL(k_brute_pop, dim3((unsigned)((nblk * BF_TILE + 255) / 256)), dim3(256), 0, st, XB, nq, nblk,
                       pop);
    return hipGetLastError();
}

int brute_grid(const BruteArgs &a)
{
    return (int)std::min<uint64_t>(a.nslots, (uint64_t)a.grid_blocks);
}

hipError_t launch_brute_compact(const Survivor *sparse, uint64_t cap, const unsigned int *count,
                                const unsigned long long *offs, int grid, Survivor *dense, hipStream_t st)
{
    hipLaunchKernelGGL(k_brute_compact, dim3(grid), dim3(256), 0, st, sparse, cap, count, offs, dense);
    return hipGetLastError();
}

hipError_t launch_brute(const BruteArgs &a, hipStream_t st)
{
    if (a.ntiles == 0) return hipSuccess;
    const uint64_t grid = (uint64_t)brute_grid(a);
    const uint2 *XA = reinterpret_cast<const uint2 *>(a.XBA), *XB = reinterpret_cast<const uint2 *>(a.XBB);
    if (a.two_sided)
        hipLaunchKernelGGL(k_brute<true>, dim3((unsigned)grid), dim3(512), 0, st, a, XA, XB);
    else
        hipLaunchKernelGGL(k_brute<false>, dim3((unsigned)grid), dim3(512), 0, st, a, XA, XB);
    return hipGetLastError();
}

hipError_t launch_pair_strengths(const uint32_t *XC, int W32p, const uint32_t *yb, const double *yd, int64_t n,
                                 int64_t p, int real_y, uint64_t seed, int64_t npairs, double *gamma,
                                 hipStream_t st)
{
    if (npairs <= 0 || p < 2) return hipSuccess;
    hipLaunchKernelGGL(k_pair_strengths, dim3(grid1((uint64_t)npairs, 4)), dim3(256), 0, st, XC, W32p, yb, yd, n, p,
                       real_y, seed, npairs, gamma);
    return hipGetLastError();
}

size_t radix_hist_entries(uint64_t S)
{
    const uint64_t nb = (S + RS_TILE - 1) / RS_TILE;
    const uint64_t h = 256 * (nb ? nb : 1);
    return (size_t)(h + (h + RS_TILE - 1) / RS_TILE + 16);
}

// Exclusive scan in place of v[0..cnt) using partial (cdiv(cnt, RS_TILE) entries).
static hipError_t scan_u32(uint32_t *v, uint64_t cnt, uint32_t *partial, hipStream_t st)
{
    const uint64_t nb = (cnt + RS_TILE - 1) / RS_TILE;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(RS_NT), 0, st, v, cnt, partial);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, partial, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(RS_NT), 0, st, v, cnt, partial, v);
    return hipGetLastError();
}

hipError_t launch_scan_u32(uint32_t *v, uint64_t cnt, uint32_t *partial, hipStream_t st)
{
    return scan_u32(v, cnt, partial, st);
}

hipError_t launch_sk_sort(const uint32_t *keys, int64_t p, int m, int nrep, uint64_t *K, uint32_t *V, uint64_t *K2,
                          uint32_t *V2, uint32_t *hist, uint32_t *perm, uint64_t **Ksorted, hipStream_t st)
{
    const uint64_t S = (uint64_t)nrep * (uint64_t)p;
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sk_init, dim3(grid1(S, 256)), dim3(256), 0, st, keys, S, p, m, K, V);
    int rbits = 0;
    while ((1ll << rbits) < nrep) ++rbits;
    uint32_t *Vs = nullptr;
    hipError_t e = launch_radix_sort(K, V, K2, V2, S, m + rbits, hist, Ksorted, &Vs, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(perm, Vs, sizeof(uint32_t) * S, hipMemcpyDeviceToDevice, st);
}

hipError_t launch_radix_sort(uint64_t *K, uint32_t *V, uint64_t *K2, uint32_t *V2, uint64_t S, int bits,
                             uint32_t *hist, uint64_t **Kout, uint32_t **Vout, hipStream_t st)
{
    const uint32_t nb = (uint32_t)((S + RS_TILE - 1) / RS_TILE);
    const uint64_t hent = 256ull * nb;
    uint32_t *partial = hist + hent;
    uint64_t *ka = K, *kb = K2;
    uint32_t *va = V, *vb = V2;
    for (int shift = 0; S > 0 && shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_NT), 0, st, ka, S, shift, hist, nb);
        hipError_t e = scan_u32(hist, hent, partial, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_NT), 0, st, ka, va, kb, vb, S, shift, hist, nb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    *Kout = ka;
    *Vout = va;
    return hipGetLastError();
}

hipError_t launch_sk_runs(const uint64_t *K, uint64_t S, uint32_t *heads, uint32_t *partial, uint64_t *run_key,
                          uint32_t *run_start, uint32_t *nruns, hipStream_t st)
{
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sk_heads, dim3(grid1(S, 256)), dim3(256), 0, st, K, S, heads);
    hipError_t e = scan_u32(heads, S, partial, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sk_runs, dim3(grid1(S, 256)), dim3(256), 0, st, K, heads, S, run_key, run_start, nruns);
    return hipGetLastError();
}

hipError_t launch_sk_table(const uint64_t *run_key, const uint32_t *nruns, uint32_t nr, uint64_t entries,
                           uint32_t *table, hipStream_t st)
{
    hipError_t e = launch_zero(table, sizeof(uint32_t) * entries, st);
    if (e != hipSuccess || nr == 0) return e;
    hipLaunchKernelGGL(k_sk_table, dim3(grid1(nr, 256)), dim3(256), 0, st, run_key, nruns, table);
    return hipGetLastError();
}

hipError_t launch_sk_products(const uint64_t *run_key, const uint32_t *run_start, const uint32_t *nruns, uint32_t nr,
                              uint64_t S, int m, int nys, RepInfo *info, int count, int two_sided, int mfma,
                              const uint32_t *table, uint32_t *cnt, hipStream_t st)
{
    hipLaunchKernelGGL(k_sk_clear_info, dim3((count + 255) / 256), dim3(256), 0, st, info, count);
    const uint64_t work = (uint64_t)nr * nys;
    if (work == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_sk_products, dim3(grid1(work, 256 * SK_ITEMS)), dim3(256), 0, st, run_key, run_start, nruns,
                       S, m, nys, info, two_sided, mfma, table, cnt, work);
    return hipGetLastError();
}

hipError_t launch_sk_tiles(const uint64_t *run_key, const uint32_t *run_start, const uint32_t *nruns, uint32_t nr,
                           uint64_t S, int64_t p, int m, int nys, const RepInfo *info, int two_sided, int mfma,
                           const uint32_t *table, const uint32_t *pos, Tile *tiles, hipStream_t st)
{
    const uint64_t work = (uint64_t)nr * nys;
    if (work == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sk_tiles, dim3(grid1(work, 256)), dim3(256), 0, st, run_key, run_start, nruns, S, p, m, nys,
                       info, two_sided, mfma, table, pos, work, tiles);
    return hipGetLastError();
}

hipError_t launch_dedup(const Survivor *surv, uint64_t S, int64_t p, int64_t n, int nys, uint64_t *keys,
                        uint32_t *vals, uint64_t *keys2, uint32_t *vals2, uint32_t *hist, uint32_t *heads,
                        OutPair *out, unsigned long long *nout, unsigned long long *ycount, RepInfo *info,
                        int64_t rep_abs0, hipStream_t st)
{
    if (S == 0) {
        hipLaunchKernelGGL(k_dedup_count, dim3(1), dim3(64), 0, st, heads, keys, (uint64_t)0, nout);
        return hipGetLastError();
    }
    const unsigned g = grid1(S, 256);
    hipLaunchKernelGGL(k_dedup_keys, dim3(g), dim3(256), 0, st, surv, S, p, keys, vals);
    // number of key bits: ceil(log2(nys * p * p))
    const double span = (double)nys * (double)p * (double)p;
    int bits = 1;
    while (bits < 64 && (double)(1ull << bits) < span) ++bits;
    if (S <= RS_SMALL) {
        hipLaunchKernelGGL(k_rs_sort_small, dim3(1), dim3(RSS_NT), 0, st, keys, vals, keys2, vals2, (uint32_t)S, bits);
        const bool odd = ((bits + 7) / 8) & 1;
        hipLaunchKernelGGL(k_dedup_small, dim3(1), dim3(RSS_NT), 0, st, odd ? keys2 : keys, odd ? vals2 : vals, surv,
                           (uint32_t)S, n, nys, out, nout, ycount, info, rep_abs0);
        return hipGetLastError();
    }
    const uint32_t nb = (uint32_t)((S + RS_TILE - 1) / RS_TILE);
    const uint64_t hent = 256ull * nb;
    uint32_t *partial = hist + hent;
    uint64_t *ka = keys, *kb = keys2;
    uint32_t *va = vals, *vb = vals2;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_NT), 0, st, ka, S, shift, hist, nb);
        hipError_t e = scan_u32(hist, hent, partial, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_NT), 0, st, ka, va, kb, vb, S, shift, hist, nb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    hipLaunchKernelGGL(k_dedup_heads, dim3(g), dim3(256), 0, st, ka, S, heads);
    hipError_t e = scan_u32(heads, S, hist, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dedup_emit, dim3(g), dim3(256), 0, st, ka, va, surv, S, heads, n, nys, out, ycount, info,
                       rep_abs0);
    hipLaunchKernelGGL(k_dedup_count, dim3(1), dim3(64), 0, st, heads, ka, S, nout);
    return hipGetLastError();
}

}  // namespace xyz
