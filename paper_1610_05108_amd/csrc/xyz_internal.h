// Internal declarations shared by the libxyz sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace xyz {

// Verification tiles cover at most TILE columns per side (Algorithm 2's
// E_l is a union of Cartesian products of two buckets; each product is cut
// into TILE x TILE blocks).
constexpr int TILE = 32;
// Largest m handled by the single-pass LDS bucket sort (2^m counters in LDS).
constexpr int MAX_M_LDS = 15;
// A bucket product that fits one tile and has at most this many candidate
// pairs goes to the small-tile list (verified many tiles per wave).
constexpr uint32_t SMALL_TILE_PAIRS = 96;
// Bucket products whose sides both have at least MTILE_MIN columns (MTILE_MIN_DIAG
// for a bucket's own pairs) are verified on the matrix cores in MTILE x MTILE tiles
// (+-1 data, n < 2^24; FP4).
constexpr int MTILE = 64;
constexpr uint32_t MTILE_MIN = 16;
constexpr uint32_t MTILE_MIN_DIAG = 24;
// Real data: only products too large for one 32 x 32 tile on both sides go to the
// 64 x 64 FP64 matrix-core tiles (smaller ones pack better into the 32 x 32 tiles).
constexpr uint32_t MTILE_MIN_REAL = 33;
// +-1 data: a product with one side of at most MTILE columns and the other of at most
// MTILE_WIDE is verified as one tile (up to 3 x 2 fragments of 32 x 32), so that neither
// side is read twice; larger products are cut into MTILE x MTILE tiles.
constexpr uint32_t MTILE_WIDE = 96;
// +-1 data: products larger than that whose shorter side has at least BIG_MIN_SHORT columns
// are verified by one workgroup per block pair of at most BIG_TILE x BIG_TILE columns, with
// both blocks staged through LDS once (k_verify_lds): the fourth tile list.  A big tile stores
// its sides minus one (1..BIG_TILE columns in a byte).
constexpr int BIG_TILE = 256;
constexpr uint32_t BIG_MIN_SHORT = 33;

struct Tile {            // 16 bytes
    uint32_t rep;        // repetition index relative to the launch's first repetition
    uint32_t a0;         // first position of the A block in perm (absolute)
    uint32_t b0;         // first position of the B block in perm (absolute)
    uint8_t na, nb;      // block sizes (1..TILE, or 1..MTILE_WIDE for matrix-core tiles)
    uint8_t diag;        // 1: A and B are the same block of one bucket; keep positions a < b only
    uint8_t ysel;        // response index within a batch
};

struct Survivor {        // 32 bytes
    uint32_t j, k;       // j < k
    uint32_t rep;        // absolute repetition index
    int32_t s;           // exact Y^T(X_j o X_k) for +-1 data
    double value;        // inner product as double (binary64 sum for real data)
    uint32_t ysel;       // response index within a batch
    uint32_t pad;
};

struct OutPair {         // layout of xyz_pair
    int32_t j, k;
    int64_t s;
    double value;
    double stat;
    int32_t first_rep, hits;
};

struct RepInfo {         // per repetition and response, filled on the device
    unsigned long long candidates;
    unsigned long long tiles;
    unsigned long long passed;
    unsigned long long fresh;
    unsigned long long cmask;
    unsigned int max_bucket;
    unsigned int small_tiles; // one-tile bucket products with at most SMALL_TILE_PAIRS pairs
    unsigned long long mfma_tiles; // MTILE x MTILE tiles of products verified on the matrix cores
    unsigned long long big_tiles;  // BIG_TILE x BIG_TILE block pairs of products staged through LDS
    unsigned long long big_pairs;  // candidate pairs of those products
};

// ------------------------------------------------------------ launchers --
// All launchers enqueue on `st` and return the hipError_t of the launch.

// X (int8 +-1, column-major, ld) -> XC bits [p][W32p] u32.  err |= 1 on a bad value.
hipError_t launch_pack_x_i8(const int8_t *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC,
                            int *err, hipStream_t st);
// X (int8 +-1, row-major, ld >= p) -> XR [n][P64] directly (columns past p: bit 0).  err |= 1 on a bad value.
hipError_t launch_pack_x_i8_rows(const int8_t *X, int64_t ld, int64_t n, int64_t p, uint64_t *XR, int64_t P64,
                                 int *err, hipStream_t st);
// XR [n][P64] -> XC [p][W32p] (the inverse bit transpose; rows past n: bit 0).
hipError_t launch_transpose_rc(const uint64_t *XR, int64_t n, int64_t p, int64_t P64, int W32p, uint32_t *XC,
                               hipStream_t st);
// X (float32, column-major, ld) -> sign bits XC and the zero-padded copy XF [p][nF].  err |= 2 on NaN/Inf.
hipError_t launch_pack_x_f32(const float *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC,
                             float *XF, int64_t nF, int *err, hipStream_t st);
// X (uint64 bits, column-major, ld words) -> XC (tail bits past n cleared).
hipError_t launch_pack_x_bits(const uint64_t *X, int64_t ld, int64_t n, int64_t p, int W32p, uint32_t *XC,
                              hipStream_t st);
// XC [p][W32p] -> XR [n][P64] (row-major bits, bit j%64 of word j/64).
hipError_t launch_transpose(const uint32_t *XC, int64_t n, int64_t p, int W32p, uint64_t *XR, int64_t P64,
                            hipStream_t st);
// X (float32) -> int8 +-1 of the signs, or int8 copy, for matrix-core brute force (not used yet).

// Y -> yb bits [W32p] u32, yd binary64 [nF] (zero padded).  yfmt: 0 int8, 1 f32, 2 f64.  err |= 4 bad value.
hipError_t launch_pack_y(const void *Y, int yfmt, int64_t n, int W32p, uint32_t *yb, double *yd, int64_t nF,
                         int *err, hipStream_t st);
// Running sum of |Y| in binary64, left to right (one thread); last[0] = largest i with Y_i != 0.  err |= 8 if all zero.
hipError_t launch_cdf(const double *yd, int64_t n, double *cdf, int64_t *last, int *err, hipStream_t st);
// Unbiased transform (Section 3.2): row maxima nu_i = max_j |X_ij| of the float
// copy XF [p][nF] (nu as float bits, zeroed here), the running sum of the row
// weights |yd_i| * (nu_i * nu_i) in binary64 (ascending i, last = last row of
// positive weight), and the keys of nrep repetitions from the transformed
// entries of the sampled rows (draws keyed by seed and rep0 + r).
// nu_i = max_j min(|X_ij|, cap) as float bits (cap = +inf: no capping).
hipError_t launch_row_absmax(const float *XF, int64_t nF, int64_t n, int64_t p, float cap, uint32_t *nu,
                             hipStream_t st);
hipError_t launch_cdf_unbiased(const double *yd, const uint32_t *nu, int64_t n, double *cdf, int64_t *last, int *err,
                               hipStream_t st);
hipError_t launch_hash_unbiased(const float *XF, int64_t nF, int64_t p, int m, int nrep, const int32_t *rows,
                                const uint32_t *nu, float cap, uint64_t seed, int64_t rep0, uint32_t *keys,
                                hipStream_t st);
// Row draws for repetitions [rep0, rep0 + nrep): rows [nrep][m].  weighted: cdf/last used.
hipError_t launch_sample(uint64_t seed, int64_t rep0, int nrep, int m, int64_t n, int weighted, const double *cdf,
                         const int64_t *last, int32_t *rows, hipStream_t st);
// cmask of every (repetition, response): info[r * nys + y].cmask from rows and yb + y * yb_stride.
hipError_t launch_cmask(const int32_t *rows, int nrep, int m, int nys, const uint32_t *yb, int yb_stride,
                        RepInfo *info, hipStream_t st);
// keys[r][j] for r < nrep (projection of column j on the sampled rows).
hipError_t launch_hash(const uint64_t *XR, int64_t P64, int64_t p, int m, int nrep, const int32_t *rows,
                       uint32_t *keys, hipStream_t st);
// Bucket sort of each repetition's keys (one workgroup per repetition) plus the histogram-only
// statistics of nys responses (info[r * nys + y]): candidates, tile counts of the four lists
// (matrix-core and big tiles only when mfma != 0), max bucket.  offs [nrep][2^m + 1], perm [nrep][p].
hipError_t launch_bucket(const uint32_t *keys, int64_t p, int m, int nrep, int nys, RepInfo *info,
                         int two_sided, int mfma, uint32_t *offs, uint32_t *perm, hipStream_t st);
// Exclusive scans over count = nrep*nys entries into base [NLISTS (count + 1)] (u64): list K
// (0: popcount tiles, 1: small tiles, 2: matrix-core tiles, 3: big tiles) at base + K (count + 1),
// its total at base[K (count + 1) + count] and, if totals is not NULL, at totals[K].
constexpr int NLISTS = 4;
hipError_t launch_tile_scan(const RepInfo *info, int count, unsigned long long *base, unsigned long long *totals,
                            hipStream_t st);
// Emit the tiles of every (repetition, response): popcount tiles first, then small tiles,
// then matrix-core tiles (MTILE x MTILE), then big tiles, each list ordered by (repetition,
// response).
// Tiles past cap are not written.
hipError_t launch_tiles(const uint32_t *offs, int64_t p, int m, int nrep, int nys, const RepInfo *info,
                        int two_sided, int mfma, const unsigned long long *base, Tile *tiles, uint64_t cap,
                        hipStream_t st);

// Bucketing for m > MAX_M_LDS (keys sorted instead of counted in LDS):
// sort the nrep * p keys by (repetition, key) with the radix sort (K, V, K2, V2: scratch of
// nrep * p entries; hist: radix_hist_entries(nrep * p) u32), write the sorted column ids to perm
// [nrep][p] and return the sorted composite keys in *Ksorted (K or K2).
hipError_t launch_sk_sort(const uint32_t *keys, int64_t p, int m, int nrep, uint64_t *K, uint32_t *V, uint64_t *K2,
                          uint32_t *V2, uint32_t *hist, uint32_t *perm, uint64_t **Ksorted, hipStream_t st);
// Runs of equal keys (the non-empty buckets): run_key, run_start (position in perm); nruns[0] on
// the device.  heads: S u32 scratch; partial: scan scratch (radix_hist_entries(S) is enough).
hipError_t launch_sk_runs(const uint64_t *K, uint64_t S, uint32_t *heads, uint32_t *partial, uint64_t *run_key,
                          uint32_t *run_start, uint32_t *nruns, hipStream_t st);
// Largest m with a direct bucket -> run table (nrep 2^m u32) instead of binary search.
constexpr int SK_TABLE_MAX_M = 22;
// table[(r << m) | b] = run id + 1 for every run, 0 for empty buckets (entries = nrep 2^m).
hipError_t launch_sk_table(const uint64_t *run_key, const uint32_t *nruns, uint32_t nr, uint64_t entries,
                           uint32_t *table, hipStream_t st);
// Clears the statistics of info[0..count) (keeping cmask), then per (response, run) counts the
// tiles of its bucket products in cnt[list][y][rid] (lists: popcount, small, matrix-core, big;
// NLISTS * nys * nr entries) and adds the statistics to info.  table: as above, or null (binary search).
hipError_t launch_sk_products(const uint64_t *run_key, const uint32_t *run_start, const uint32_t *nruns, uint32_t nr,
                              uint64_t S, int m, int nys, RepInfo *info, int count, int two_sided, int mfma,
                              const uint32_t *table, uint32_t *cnt, hipStream_t st);
// Emits the tiles at pos[list][y][rid] (the exclusive scan of cnt laid end to end).
hipError_t launch_sk_tiles(const uint64_t *run_key, const uint32_t *run_start, const uint32_t *nruns, uint32_t nr,
                           uint64_t S, int64_t p, int m, int nys, const RepInfo *info, int two_sided, int mfma,
                           const uint32_t *table, const uint32_t *pos, Tile *tiles, hipStream_t st);
// Exclusive scan in place of v[0..cnt) (partial: cdiv(cnt, 2048) + 16 u32 of scratch).
hipError_t launch_scan_u32(uint32_t *v, uint64_t cnt, uint32_t *partial, hipStream_t st);

// Shared arguments of the verification kernels.
struct VerifyArgs {
    const Tile *tiles;
    uint64_t ntiles;         // large tiles: tiles[0, ntiles)
    uint64_t nsmall;         // small tiles: tiles[ntiles, ntiles + nsmall)
    uint64_t nmfma;          // matrix-core tiles: tiles[ntiles + nsmall, ... + nmfma)
    uint64_t nbig;           // big tiles: tiles[ntiles + nsmall + nmfma, ... + nbig)
    // With dcnt set, the four list sizes are read on the device (dcnt[0..3]: popcount, small,
    // matrix-core, big; the tile scan's totals) instead of the fields above, which then only
    // bound the launch grids; a kernel does nothing when the sizes sum past tile_cap (the host
    // then grows the list and reruns the chunk).
    const unsigned long long *dcnt;
    uint64_t tile_cap;
    const uint32_t *perm;
    const uint32_t *XC;      // [p][W32p] bits
    int W32p;
    const float *XF;         // [p][nF] values (continuous X) or null
    int64_t nF;
    const uint32_t *yb;      // [nys][W32p] bits of Y
    const uint32_t *cpop;    // big tiles: [nys + 1][p] popcounts |y_y ^ x_j| (rows y < nys) and |x_j| (row nys)
    int64_t p;
    const double *yd;        // [nys][nF] values of Y
    int64_t n;
    const int64_t *smin;     // [nys] integer thresholds (binary data)
    const double *kappa;     // [nys] thresholds (real data)
    int two_sided;
    int nys;
    int64_t rep_abs0;        // absolute index of relative repetition 0
    Survivor *surv;
    unsigned long long *surv_count;
    uint64_t surv_cap;
    RepInfo *info;           // [nrep][nys]
};
// Column popcounts for the big tiles: cpop[y][j] = |y_y ^ x_j| for y < nys, cpop[nys][j] = |x_j|.
hipError_t launch_col_pops(const uint32_t *XC, int W32p, const uint32_t *yb, int nys, int64_t p, uint32_t *cpop,
                           hipStream_t st);
// Popcount-XOR verification of +-1 candidates: s = n - 2 popcount(y ^ x_j ^ x_k) (popcount, small
// and matrix-core tiles).
hipError_t launch_verify_bin(const VerifyArgs &a, int grid, hipStream_t st);
// The big tiles of +-1 candidates (LDS-staged block pairs on the FP4 matrix cores), on at most
// grid workgroups.
hipError_t launch_verify_big(const VerifyArgs &a, int grid, hipStream_t st);
// Binary64 verification of real-valued candidates (x_real: values from XF, else +-1 from XC).
hipError_t launch_verify_real(const VerifyArgs &a, int x_real, int grid, hipStream_t st);

// Merge S survivors into unique pairs sorted by (ysel, j, k).  Scratch: keys/keys2 (u64) and
// vals/vals2 (u32) of S entries, hist of radix_hist_entries(S) u32, heads of S + 1 u32.
// out: unique pairs (ysel in the pad word of first_rep's neighbour is not kept: pairs of one
// response are contiguous and their count per response goes to ycount[y]).  nout: device count.
// Fresh counts go to info[(first_rep - rep_abs0) * nys + ysel].fresh.
hipError_t launch_dedup(const Survivor *surv, uint64_t S, int64_t p, int64_t n, int nys, uint64_t *keys,
                        uint32_t *vals, uint64_t *keys2, uint32_t *vals2, uint32_t *hist, uint32_t *heads,
                        OutPair *out, unsigned long long *nout, unsigned long long *ycount, RepInfo *info,
                        int64_t rep_abs0, hipStream_t st);

// Exact search of eq. (1) over column blocks on FP4 matrix cores.
struct BruteArgs {
    const uint4 *XBA;        // A side staged: [nbA][nq][BF_TILE] quads of z = y ^ x (zero padded, words 0,2,1,3)
    const uint4 *XBB;        // B side staged: [nbB][nq][BF_TILE] quads of x (nibble bits 0, 2 swapped)
    const uint32_t *popA;    // [nbA * BF_TILE] popcounts of the staged A columns
    const uint32_t *popB;    // [nbB * BF_TILE]
    int nq;                  // quads (4 words, 128 rows) per column
    const int32_t *colsA;    // column ids of the A side (null: identity)
    int64_t nA;
    const int32_t *colsB;    // column ids of the B side (null: identity)
    int64_t nB;
    int tri;                 // A and B are the same list: only block pairs bi <= bj, and a < b on the diagonal
    int64_t nbA, nbB;        // number of 256-column blocks per side
    uint64_t ntiles;         // block pairs
    int64_t nsbA, nsbB;      // super-blocks of 8 x 8 block pairs per side (ceil(nb / 8))
    uint64_t nslots;         // work slots: 64 per super-block (upper triangle of super-blocks when tri)
    int64_t n;
    int64_t smin;
    int two_sided;
    Survivor *surv;          // [grid][cap_wg]: workgroup g writes its survivors at g * cap_wg
    uint64_t cap_wg;
    unsigned int *wg_count;  // [grid]: survivors found by each workgroup (may exceed cap_wg)
    int grid_blocks;         // persistent grid bound (a multiple of 8)
};
constexpr int BF_TILE = 256;
// Stage ncols columns (cols: device ids, or null for 0..ncols-1) into XB [nblk][W32p/4][BF_TILE]
// quads (words in the order 0, 2, 1, 3): with yb, the A side z = y ^ x; without, the B side x
// with bits 0 and 2 of every nibble swapped; words >= nw and padding columns zero; and their
// popcounts into pop [nblk * BF_TILE].
hipError_t launch_brute_stage(const uint32_t *XC, int W32p, int nw, const int32_t *cols, int64_t ncols,
                              const uint32_t *yb, uint4 *XB, uint32_t *pop, hipStream_t st);
// Workgroups of the persistent brute-force launch (a multiple of 8, at most grid_blocks).
int brute_grid(const BruteArgs &a);
hipError_t launch_brute(const BruteArgs &a, hipStream_t st);
// dense[offs[g] + i] = sparse[g * cap + i] for i < count[g], g < grid.
hipError_t launch_brute_compact(const Survivor *sparse, uint64_t cap, const unsigned int *count,
                                const unsigned long long *offs, int grid, Survivor *dense, hipStream_t st);

// Collision strengths of uniformly drawn column pairs (for the planner).
// Pair q: draws u = SplitMix64(seed, 2q+1), v = SplitMix64(seed, 2q+2);
// j = floor(u p / 2^64), k = floor(v (p-1) / 2^64), k += (k >= j).  gamma[q] is
// the probability that one sampled row agrees: the fraction of rows with
// sgn(Y_i) = X~_ij X~_ik, weighted by |Y_i| / ||Y||_1 for real Y.
hipError_t launch_pair_strengths(const uint32_t *XC, int W32p, const uint32_t *yb, const double *yd, int64_t n,
                                 int64_t p, int real_y, uint64_t seed, int64_t npairs, double *gamma,
                                 hipStream_t st);

// Radix histogram scratch size (u32 entries) for S items.
size_t radix_hist_entries(uint64_t S);
// Stable LSD radix sort of S (key, value) pairs on the low `bits` bits of the keys, ping-ponging
// between (K, V) and (K2, V2); hist holds radix_hist_entries(S) u32.  *Kout / *Vout name the
// buffers that hold the sorted sequence.
hipError_t launch_radix_sort(uint64_t *K, uint32_t *V, uint64_t *K2, uint32_t *V2, uint64_t S, int bits,
                             uint32_t *hist, uint64_t **Kout, uint32_t **Vout, hipStream_t st);

// ------------------------------------------- dense projections (Algorithm 1) --
// Repetitions are projected in groups of 8 on the int8 matrix cores; dense_weight_bytes is the
// size of the weight-digit buffer W of launch_dense_project for n rows and nrep repetitions.
size_t dense_weight_bytes(int64_t n, int nrep);
// x = X^T R_r and z = (Y o X)^T R_r (int32, exact when sum_i |R_r,i| < 2^31) for the nrep rows of
// R [nrep][n] (device), from the column bits XC [p][W32p], into xs / zs [nrep][p]; sort keys
// K [nrep][p] = (r << 32) | (z + 2^31) with the column id in V.
hipError_t launch_dense_project(const uint64_t *XR, int64_t P64, const uint32_t *XC, int W32p, int64_t p, int64_t n,
                                const int32_t *R, int nrep, const uint32_t *yb, void *W, int32_t *xs, int32_t *zs,
                                uint64_t *K, uint32_t *V, hipStream_t st);
// Buckets of the per-repetition index of the sorted z (idx holds nrep * (buckets + 1) u32).
uint32_t dense_index_buckets(int64_t p);
// E_r = {(j, k) : |x_j - z_k| <= tau} from the sorted keys Ks / column ids Vs of each repetition,
// and the check s >= smin of every unordered pair of E_r u E_r^T (j != k) once.  Survivors as
// in launch_verify_bin; info[r].candidates / passed / max_bucket (largest window) accumulate.
hipError_t launch_dense_verify(const int32_t *xs, const int32_t *zs, const uint64_t *Ks, const uint32_t *Vs,
                               uint32_t *idx, int64_t p, int nrep, int64_t tau, const uint32_t *XC, int W32p,
                               const uint32_t *yb, int64_t n, int64_t smin, int64_t rep_abs0, Survivor *surv,
                               unsigned long long *surv_count, uint64_t surv_cap, RepInfo *info, hipStream_t st);
// Zero `bytes` bytes at p (a multiple of 4, p 4-byte aligned) with a fill kernel: used instead of
// hipMemsetAsync for every counter and flag of the search path.
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
// Set kernel attributes (large dynamic LDS); called once per device.
hipError_t kernels_init();

}  // namespace xyz
