// xyz_dense.hip -- Algorithm 1 with dense projections (Section 2.1, class (a);
// compared with minimal subsampling in Section 5.1 and Theorem 1).
//
// Repetition l projects every column of X and of Z = Y o X onto an integer
// vector R_l: x = X^T R_l and z = Z^T R_l.  For +-1 data
//     x_j = sum_i R_i - 2 sum_{i : X_ij = -1} R_i,
//     z_j = sum_i Y_i R_i - 2 sum_{i : X_ij = -1} Y_i R_i,
// exact in int32 because the caller bounds sum_i |R_i| below 2^31.  The z of a
// repetition are sorted (with the column ids), and column j walks the window of
// sorted z with |x_j - z_k| <= tau, starting from an index of the sorted z: that is E_l.
// Each unordered pair {j, k} of E_l u E_l^T is checked once, from the side that
// owns it (j when (j, k) is in E_l and, if k < j, (k, j) is not), by
// s = n - 2 popcount(y ^ x_j ^ x_k) against the integer threshold of eq. (1).
#include "xyz_internal.h"

#include <algorithm>

namespace xyz {

namespace {

constexpr int DP_R = 8;        // repetitions per projection pass (one group)
constexpr int DP_ROWS = 256;   // rows per projection workgroup slice (more when n needs > DP_SLICES)
constexpr int DP_SLICES = 32768;

__device__ __forceinline__ unsigned dp_lane() { return threadIdx.x & 63u; }

}  // namespace

// Weights of repetition group g interleaved per row for the projection:
// W[((g n + i) DP_R + r) 2 + 0] = R_{gDP_R+r, i}, [.. + 1] = Y_i R_{gDP_R+r, i}
// (zero for repetitions past nrep), and the per-repetition sums rs[rep] =
// sum_i R_i, rys[rep] = sum_i Y_i R_i (int32: bounded by sum_i |R_i| < 2^31).
__global__ __launch_bounds__(256) void k_dense_weights(const int32_t *__restrict__ R, int64_t n, int nrep,
                                                       const uint32_t *__restrict__ yb, int32_t *__restrict__ W,
                                                       int32_t *__restrict__ rs, int32_t *__restrict__ rys)
{
    const int g = blockIdx.y;
    __shared__ int32_t part[2][DP_R][4];
    int32_t sr[DP_R], sy[DP_R];
#pragma unroll
    for (int r = 0; r < DP_R; ++r) sr[r] = sy[r] = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int32_t ys = ((yb[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
        int32_t *o = W + (((int64_t)g * n + i) * DP_R) * 2;
#pragma unroll
        for (int r = 0; r < DP_R; ++r) {
            const int rep = g * DP_R + r;
            const int32_t v = rep < nrep ? R[(int64_t)rep * n + i] : 0;
            o[2 * r] = v;
            o[2 * r + 1] = ys * v;
            sr[r] += v;
            sy[r] += ys * v;
        }
    }
#pragma unroll
    for (int r = 0; r < DP_R; ++r) {
        for (int d = 32; d >= 1; d >>= 1) {
            sr[r] += __shfl_xor(sr[r], d, 64);
            sy[r] += __shfl_xor(sy[r], d, 64);
        }
    }
    const int w = threadIdx.x >> 6;
    if (dp_lane() == 0) {
#pragma unroll
        for (int r = 0; r < DP_R; ++r) {
            part[0][r][w] = sr[r];
            part[1][r][w] = sy[r];
        }
    }
    __syncthreads();
    if (threadIdx.x < DP_R) {
        const int r = threadIdx.x, rep = g * DP_R + r;
        if (rep < nrep) {
            atomicAdd(&rs[rep], part[0][r][0] + part[0][r][1] + part[0][r][2] + part[0][r][3]);
            atomicAdd(&rys[rep], part[1][r][0] + part[1][r][1] + part[1][r][2] + part[1][r][3]);
        }
    }
}

// Partial sums over one slice of `rows` rows: sx[rep][j] += sum_{i : X_ij = -1} R_i and
// sz[rep][j] += sum_{i : X_ij = -1} Y_i R_i.  One thread per column; the 64 columns of a
// wave read one word of each row of XR (bit j % 64 of word j / 64 is 1 iff X_ij = -1).
__global__ __launch_bounds__(256) void k_dense_project(const uint64_t *__restrict__ XR, int64_t P64, int64_t p,
                                                       int64_t n, int64_t rows, const int32_t *__restrict__ W,
                                                       int nrep, int32_t *__restrict__ sx, int32_t *__restrict__ sz)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int q = __builtin_amdgcn_readfirstlane((int)(j >> 6));
    if (q >= P64) return;                           // the whole wave lies past the last word
    const int g = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.z * rows, i1 = i0 + rows < n ? i0 + rows : n;
    const unsigned lane = dp_lane();
    int32_t ax[DP_R], az[DP_R];
#pragma unroll
    for (int r = 0; r < DP_R; ++r) ax[r] = az[r] = 0;
    const uint64_t *col = XR + q;
    const int4 *Wg = reinterpret_cast<const int4 *>(W + (int64_t)g * n * DP_R * 2);
#pragma unroll 2
    for (int64_t i = i0; i < i1; ++i) {
        const uint64_t w = col[i * P64];
        const int32_t m = -(int32_t)((w >> lane) & 1u);      // all ones iff X_ij = -1
        const int4 *wr = Wg + i * (DP_R / 2);
#pragma unroll
        for (int h = 0; h < DP_R / 2; ++h) {
            const int4 v = wr[h];                            // R, YR of repetitions 2h, 2h + 1
            ax[2 * h] += v.x & m;
            az[2 * h] += v.y & m;
            ax[2 * h + 1] += v.z & m;
            az[2 * h + 1] += v.w & m;
        }
    }
    if (j >= p) return;
#pragma unroll
    for (int r = 0; r < DP_R; ++r) {
        const int rep = g * DP_R + r;
        if (rep < nrep) {
            atomicAdd(&sx[(int64_t)rep * p + j], ax[r]);
            atomicAdd(&sz[(int64_t)rep * p + j], az[r]);
        }
    }
}

// x = rs - 2 sx and z = rys - 2 sz in place; sort keys (rep << 32) | (z + 2^31) with the
// column id as value (keys of one repetition are contiguous after the sort).
__global__ __launch_bounds__(256) void k_dense_keys(int32_t *__restrict__ xs, int32_t *__restrict__ zs, int64_t p,
                                                    int nrep, const int32_t *__restrict__ rs,
                                                    const int32_t *__restrict__ rys, uint64_t *__restrict__ K,
                                                    uint32_t *__restrict__ V)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nrep * p) return;
    const int rep = (int)(t / p);
    const int32_t x = (int32_t)((uint32_t)rs[rep] - 2u * (uint32_t)xs[t]);
    const int32_t z = (int32_t)((uint32_t)rys[rep] - 2u * (uint32_t)zs[t]);
    xs[t] = x;
    zs[t] = z;
    K[t] = ((uint64_t)rep << 32) | (uint64_t)((uint32_t)z ^ 0x80000000u);
    V[t] = (uint32_t)(t - (int64_t)rep * p);
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

int dense_group_reps() { return DP_R; }

hipError_t launch_dense_project(const uint64_t *XR, int64_t P64, int64_t p, int64_t n, const int32_t *R, int nrep,
                                const uint32_t *yb, int32_t *W, int32_t *rs, int32_t *rys, int32_t *xs, int32_t *zs,
                                uint64_t *K, uint32_t *V, hipStream_t st)
{
    if (nrep <= 0 || p <= 0) return hipSuccess;
    const int ng = (nrep + DP_R - 1) / DP_R;
    hipError_t e = hipMemsetAsync(rs, 0, sizeof(int32_t) * nrep, st);
    if (e == hipSuccess) e = hipMemsetAsync(rys, 0, sizeof(int32_t) * nrep, st);
    if (e == hipSuccess) e = hipMemsetAsync(xs, 0, sizeof(int32_t) * nrep * p, st);
    if (e == hipSuccess) e = hipMemsetAsync(zs, 0, sizeof(int32_t) * nrep * p, st);
    if (e != hipSuccess) return e;
    const unsigned wblocks = (unsigned)std::min<int64_t>((n + 255) / 256, 64);
    hipLaunchKernelGGL(k_dense_weights, dim3(wblocks, ng), dim3(256), 0, st, R, n, nrep, yb, W, rs, rys);
    const unsigned bx = (unsigned)((p + 255) / 256);
    const int64_t rows = std::max<int64_t>(DP_ROWS, (n + DP_SLICES - 1) / DP_SLICES);
    const unsigned bz = (unsigned)((n + rows - 1) / rows);
    hipLaunchKernelGGL(k_dense_project, dim3(bx, ng, bz), dim3(256), 0, st, XR, P64, p, n, rows, W, nrep, xs, zs);
    const int64_t tot = (int64_t)nrep * p;
    hipLaunchKernelGGL(k_dense_keys, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, xs, zs, p, nrep, rs, rys,
                       K, V);
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
