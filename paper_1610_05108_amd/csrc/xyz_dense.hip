// xyz_dense.hip -- Algorithm 1 with dense projections (Section 2.1, class (a);
// compared with minimal subsampling in Section 5.1 and Theorem 1).
//
// Repetition l projects every column of X and of Z = Y o X onto an integer
// vector R_l: x = X^T R_l and z = Z^T R_l = X^T (Y o R_l), exact in int32
// because the caller bounds sum_i |R_i| below 2^31.  The projections of 8
// repetitions at a time are one integer matrix product on the int8 matrix
// cores (+-1 X against the base-256 digits of the weights).  The z of a
// repetition are sorted (with the column ids), and column j walks the window of
// sorted z with |x_j - z_k| <= tau, starting from an index of the sorted z: that
// is E_l.  Each unordered pair {j, k} of E_l u E_l^T is checked once, from the
// side that owns it (j when (j, k) is in E_l and, if k < j, (k, j) is not), by
// s = n - 2 popcount(y ^ x_j ^ x_k) against the integer threshold of eq. (1).
#include "xyz_internal.h"

#include <algorithm>

namespace xyz {

namespace {

constexpr int DP_R = 8;        // repetitions per projection pass (one group)

__device__ __forceinline__ unsigned dp_lane() { return threadIdx.x & 63u; }

}  // namespace

typedef int dp_v4i __attribute__((ext_vector_type(4)));
typedef int dp_v16i __attribute__((ext_vector_type(16)));

// The projection x = X^T R is a contraction over the rows; it runs on the int8 matrix cores.
// A weight w (R_i or Y_i R_i, |w| < 2^31) is written in balanced base-256 digits,
// w = d0 + 2^8 d1 + 2^16 d2 + 2^24 d3 with every d in [-128, 127], so that
// x = sum_k 2^(8k) (X^T D_k) exactly; each X^T D_k is at most 128 n in magnitude (exact in
// int32 for n < 2^24).  Output column c of a repetition group is 2r (R of repetition r) or
// 2r + 1 (Y o R); the matrix product's 64 columns are digit k = n / 16 of output column
// c = n % 16.
__device__ __forceinline__ int dp_digit(int32_t w, int k)
{
    int32_t v = w;
    for (int q = 0; q < k; ++q) v = (v - (int32_t)(int8_t)(v & 0xff)) >> 8;
    return (int)(int8_t)(v & 0xff);
}

// Digits of repetition group g in the matrix cores' B layout: WL[((g nK + ks) 2 + h) 64 + n]
// is 16 bytes, byte s = digit n / 16 of weight column n % 16 at row 32 ks + 16 h + s
// (0 for rows past n and repetitions past nrep).
__global__ __launch_bounds__(256) void k_dense_weights(const int32_t *__restrict__ R, int64_t n, int nrep,
                                                       const uint32_t *__restrict__ yb, int nK,
                                                       uint4 *__restrict__ WL)
{
    const int g = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (ks, h, col) of the group
    if (e >= (int64_t)nK * 128) return;
    const int col = (int)(e & 63), h = (int)((e >> 6) & 1);
    const int64_t ks = e >> 7;
    const int k = col >> 4, c = col & 15, rep = g * DP_R + (c >> 1);
    uint32_t wd[4] = {0, 0, 0, 0};
    if (rep < nrep) {
        for (int sb = 0; sb < 16; ++sb) {
            const int64_t i = ks * 32 + 16 * h + sb;
            if (i >= n) break;
            int32_t w = R[(int64_t)rep * n + i];
            if ((c & 1) && ((yb[i >> 5] >> (i & 31)) & 1u)) w = -w;
            wd[sb >> 2] |= ((uint32_t)dp_digit(w, k) & 0xffu) << (8 * (sb & 3));
        }
    }
    WL[((int64_t)g * nK + ks) * 128 + h * 64 + col] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
}

// x and z of DP_R repetitions for 32 columns per wave, over all rows: the A operand is 16
// rows of one column as int8 +-1 (bit b of a nibble spread to byte b by one multiply), the B
// operand the weight digits.  Lane l takes column l % 32 and row half l / 32 of every 32-row
// step; accumulator r of lane l holds column (r/4)*8 + (l/32)*4 + r%4 of the wave's 32 and
// product column l % 32.  Writes xs, zs [rep][p] and the sort keys (rep << 32) | (z + 2^31)
// with the column id.
__global__ __launch_bounds__(256) void k_dense_project(const uint32_t *__restrict__ XC, int W32p, int64_t p,
                                                       int nK, const uint4 *__restrict__ WL, int nrep,
                                                       int32_t *__restrict__ xs, int32_t *__restrict__ zs,
                                                       uint64_t *__restrict__ K, uint32_t *__restrict__ V)
{
    const unsigned lane = dp_lane();
    const int64_t j0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    if (j0 >= p) return;                            // the whole wave lies past the last column
    const int g = blockIdx.y;
    const int h = (int)(lane >> 5), lc = (int)(lane & 31);
    const int64_t col = j0 + lc < p ? j0 + lc : p - 1;
    const uint4 *xc4 = reinterpret_cast<const uint4 *>(XC + col * (int64_t)W32p);
    const uint4 *wl = WL + (int64_t)g * nK * 128 + h * 64 + lc;
    dp_v16i acc0 = {}, acc1 = {};
    for (int q = 0; 4 * q < nK; ++q) {
        const uint4 w4 = xc4[q];                    // rows 128 q .. 128 q + 127 (W32p is a multiple of 4)
        const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ks = 4 * q + e;
            if (ks >= nK) break;
            const uint32_t bits = (ws[e] >> (16 * h)) & 0xffffu;
            dp_v4i av;
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const uint32_t m = (((bits >> (4 * q4)) & 15u) * 0x00204081u) & 0x01010101u;
                av[q4] = (int)(0x01010101u | (m * 0xfeu));   // byte b: -1 when bit b is set, else +1
            }
            const uint4 b0 = wl[(int64_t)ks * 128], b1 = wl[(int64_t)ks * 128 + 32];
            const dp_v4i bv0 = {(int)b0.x, (int)b0.y, (int)b0.z, (int)b0.w};
            const dp_v4i bv1 = {(int)b1.x, (int)b1.y, (int)b1.z, (int)b1.w};
            acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv1, acc1, 0, 0, 0);
        }
    }
    // digits 0 and 1 of output column c sit in lanes c and c + 16 of acc0, digits 2 and 3 in acc1
    const int c = lc & 15, rep = g * DP_R + (c >> 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int32_t d1 = __shfl_xor(acc0[r], 16, 64), d3 = __shfl_xor(acc1[r], 16, 64);
        const int64_t v = (int64_t)acc0[r] + ((int64_t)d1 << 8) + ((int64_t)acc1[r] << 16) + ((int64_t)d3 << 24);
        const int64_t j = j0 + (r >> 2) * 8 + h * 4 + (r & 3);
        if (lc < 16 && j < p && rep < nrep) {
            const int64_t t = (int64_t)rep * p + j;
            if (c & 1) {
                zs[t] = (int32_t)v;
                K[t] = ((uint64_t)rep << 32) | (uint64_t)((uint32_t)(int32_t)v ^ 0x80000000u);
                V[t] = (uint32_t)j;
            } else {
                xs[t] = (int32_t)v;
            }
        }
    }
}

namespace {

__device__ __forceinline__ int32_t dp_zval(uint64_t key) { return (int32_t)((uint32_t)key ^ 0x80000000u); }

// Buckets of the index: nb equal slices of [zmin, zmax], bucket(v) = floor((v - zmin) scale)
// with scale = nb / (zmax - zmin + 1) in binary64 (v - zmin < 2^33 is exact; rounding keeps the
// map non-decreasing in v, and both the index and the search use this one function).
__device__ __forceinline__ uint32_t dp_bucket(int64_t v, int64_t zmin, double scale, uint32_t nb)
{
    const uint32_t b = (uint32_t)((double)(v - zmin) * scale);
    return b < nb ? b : nb - 1;
}

}  // namespace

// Index of each repetition's sorted z: idx[rep][b] = first position t with bucket(z_t) >= b
// (b = 0 .. nb; idx[rep][nb] = p).  Thread t writes the entries of the buckets in
// (bucket(z_{t-1}), bucket(z_t)], so that every entry is written once.
__global__ __launch_bounds__(256) void k_dense_index(const uint64_t *__restrict__ Ks, int64_t p, uint32_t nb,
                                                     uint32_t *__restrict__ idx)
{
    const int rep = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= p) return;
    const uint64_t *K = Ks + (int64_t)rep * p;
    uint32_t *ix = idx + (int64_t)rep * (nb + 1);
    const int64_t zmin = dp_zval(K[0]), zmax = dp_zval(K[p - 1]);
    const double scale = (double)nb / ((double)(zmax - zmin) + 1.0);
    const uint32_t b = dp_bucket(dp_zval(K[t]), zmin, scale, nb);
    const int64_t b0 = t == 0 ? -1 : (int64_t)dp_bucket(dp_zval(K[t - 1]), zmin, scale, nb);
    for (int64_t q = b0 + 1; q <= (int64_t)b; ++q) ix[q] = (uint32_t)t;
    if (t == p - 1)
        for (int64_t q = (int64_t)b + 1; q <= (int64_t)nb; ++q) ix[q] = (uint32_t)p;
}

namespace {

// First position t in [0, p) of a repetition's sorted keys K with z >= v (p if none), via the
// index: the position lies in [ix[bucket(v)], ix[bucket(v) + 1]].
__device__ __forceinline__ uint32_t dp_first_ge(const uint64_t *K, const uint32_t *ix, uint32_t p, uint32_t nb,
                                                int64_t zmin, int64_t zmax, int64_t v)
{
    if (v <= zmin) return 0;
    if (v > zmax) return p;
    const uint32_t b = dp_bucket(v, zmin, (double)nb / ((double)(zmax - zmin) + 1.0), nb);
    uint32_t lo = ix[b], hi = ix[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((int64_t)dp_zval(K[mid]) < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace

// E_l and its check.  Grid (ceil(p / 256), nrep): thread (rep, j) walks the window of the
// repetition's sorted z with |x_j - z_k| <= tau: its start from the index and a binary
// search inside one bucket, its end by walking while z_k <= x_j + tau.
__global__ __launch_bounds__(256) void k_dense_verify(const int32_t *__restrict__ xs, const int32_t *__restrict__ zs,
                                                      const uint64_t *__restrict__ Ks,
                                                      const uint32_t *__restrict__ Vs,
                                                      const uint32_t *__restrict__ idx, uint32_t nb, int64_t p,
                                                      int64_t tau,
                                                      const uint32_t *__restrict__ XC, int W32p,
                                                      const uint32_t *__restrict__ yb, int64_t n, int64_t smin,
                                                      int64_t rep_abs0, Survivor *__restrict__ surv,
                                                      unsigned long long *__restrict__ surv_count, uint64_t surv_cap,
                                                      RepInfo *__restrict__ info)
{
    const int rep = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t base = (int64_t)rep * p;
    unsigned long long cand = 0, passed = 0;
    uint32_t window = 0;
    if (j < p) {
        const int32_t xj = xs[base + j], zj = zs[base + j];
        const uint64_t *K = Ks + base;
        const int64_t zmin = dp_zval(K[0]), zmax = dp_zval(K[p - 1]);
        const int64_t zhi = (int64_t)xj + tau;
        const uint32_t lo = dp_first_ge(K, idx + (int64_t)rep * (nb + 1), (uint32_t)p, nb, zmin, zmax,
                                        (int64_t)xj - tau);
        const uint4 *xj4 = reinterpret_cast<const uint4 *>(XC + j * (int64_t)W32p);
        const uint4 *y4 = reinterpret_cast<const uint4 *>(yb);
        const int W4 = W32p >> 2;
        uint32_t t = lo;
        for (; t < (uint32_t)p && (int64_t)dp_zval(K[t]) <= zhi; ++t) {
            const uint32_t k = Vs[base + t];
            if ((int64_t)k == j) continue;
            if ((int64_t)k < j) {                  // (k, j) in E_l as well: the pair is k's
                const int64_t d = (int64_t)xs[base + k] - zj;
                if (d <= tau && d >= -tau) continue;
            }
            ++cand;
            const uint4 *xk4 = reinterpret_cast<const uint4 *>(XC + (int64_t)k * W32p);
            uint32_t pop = 0;
            for (int w = 0; w < W4; ++w) {
                const uint4 a = xj4[w], b = xk4[w], c = y4[w];
                pop += __popc(a.x ^ b.x ^ c.x) + __popc(a.y ^ b.y ^ c.y) + __popc(a.z ^ b.z ^ c.z) +
                       __popc(a.w ^ b.w ^ c.w);
            }
            const int64_t s = n - 2 * (int64_t)pop;
            if (s >= smin) {
                ++passed;
                const unsigned long long idx = atomicAdd(surv_count, 1ull);
                if (idx < surv_cap) {
                    Survivor sv;
                    sv.j = (int64_t)k < j ? k : (uint32_t)j;
                    sv.k = (int64_t)k < j ? (uint32_t)j : k;
                    sv.rep = (uint32_t)(rep_abs0 + rep);
                    sv.s = (int32_t)s;
                    sv.value = (double)s;
                    sv.ysel = 0;
                    sv.pad = 0;
                    surv[idx] = sv;
                }
            }
        }
        window = t - lo;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        cand += __shfl_xor(cand, d, 64);
        passed += __shfl_xor(passed, d, 64);
        window = max(window, (uint32_t)__shfl_xor((int)window, d, 64));
    }
    if (dp_lane() == 0) {
        if (cand) atomicAdd(&info[rep].candidates, cand);
        if (passed) atomicAdd(&info[rep].passed, passed);
        if (window) atomicMax(&info[rep].max_bucket, window);
    }
}

// ------------------------------------------------------------ launchers --

size_t dense_weight_bytes(int64_t n, int nrep)
{
    const int64_t nK = (n + 31) / 32, ng = (nrep + DP_R - 1) / DP_R;
    return (size_t)(ng * nK * 128) * sizeof(uint4);
}

hipError_t launch_dense_project(const uint64_t *XR, int64_t P64, const uint32_t *XC, int W32p, int64_t p, int64_t n,
                                const int32_t *R, int nrep, const uint32_t *yb, void *W, int32_t *xs, int32_t *zs,
                                uint64_t *K, uint32_t *V, hipStream_t st)
{
    (void)XR;
    (void)P64;
    if (nrep <= 0 || p <= 0) return hipSuccess;
    const int ng = (nrep + DP_R - 1) / DP_R;
    const int nK = (int)((n + 31) / 32);
    uint4 *WL = static_cast<uint4 *>(W);
    hipLaunchKernelGGL(k_dense_weights, dim3((unsigned)(((int64_t)nK * 128 + 255) / 256), ng), dim3(256), 0, st, R, n,
                       nrep, yb, nK, WL);
    hipLaunchKernelGGL(k_dense_project, dim3((unsigned)((p + 127) / 128), ng), dim3(256), 0, st, XC, W32p, p, nK, WL,
                       nrep, xs, zs, K, V);
    return hipGetLastError();
}

uint32_t dense_index_buckets(int64_t p) { return (uint32_t)std::max<int64_t>(1, p / 4); }

hipError_t launch_dense_verify(const int32_t *xs, const int32_t *zs, const uint64_t *Ks, const uint32_t *Vs,
                               uint32_t *idx, int64_t p, int nrep, int64_t tau, const uint32_t *XC, int W32p,
                               const uint32_t *yb, int64_t n, int64_t smin, int64_t rep_abs0, Survivor *surv,
                               unsigned long long *surv_count, uint64_t surv_cap, RepInfo *info, hipStream_t st)
{
    if (nrep <= 0 || p <= 0) return hipSuccess;
    const uint32_t nb = dense_index_buckets(p);
    const dim3 grid((unsigned)((p + 255) / 256), (unsigned)nrep);
    hipLaunchKernelGGL(k_dense_index, grid, dim3(256), 0, st, Ks, p, nb, idx);
    hipLaunchKernelGGL(k_dense_verify, grid, dim3(256), 0, st, xs, zs, Ks, Vs, idx, nb, p, tau, XC, W32p, yb, n, smin,
                       rep_abs0, surv, surv_count, surv_cap, info);
    return hipGetLastError();
}

}  // namespace xyz
