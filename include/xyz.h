/*
 * xyz.h -- C ABI of libxyz, a GPU (AMD Instinct MI355X, gfx950) implementation
 * of the xyz interaction search of Thanei, Meinshausen & Shah, "The xyz
 * algorithm for fast interaction search in high-dimensional data".
 *
 * The problem (eq. (1), Section 1): given X (n x p) and Y (n), keep every pair
 * of columns (j, k), j < k, with  Y^T (X_j o X_k) / n > kappa.
 * The method (Algorithm 2, Section 2.2): in each of L repetitions, sample m
 * rows, project every column of X and of Z = Y o X onto them, collect the
 * pairs whose projections collide (x_j = z_k), and verify each candidate
 * exactly.  Continuous Y (Section 3.1) is handled by |Y|-weighted row
 * sampling with Z = sgn(Y) o X; continuous X (Section 3.2) is hashed on its
 * signs (the "sign transform") and verified on its values.
 *
 * Conventions
 *  - Every function returns xyz_status (0 = XYZ_OK, < 0 error) unless stated.
 *    On error, xyz_last_error() returns a message (thread-local, valid until the
 *    next xyz_* call on the same thread).  No C++ exception crosses the ABI.
 *  - Indices are 0-based.  Reported pairs are unordered with j < k; the
 *    diagonal j == k is never reported.
 *  - Input pointers are borrowed for the duration of the call and copied.
 *    `mem` says whether a pointer is host memory (XYZ_MEM_HOST) or device
 *    memory on the context's GPU (XYZ_MEM_DEVICE).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls that return a
 *    result synchronise that stream before returning.
 *  - Handles have a single owner and are released with their _destroy/_free.
 *  - A context is not thread-safe: use one per thread, or serialise calls.
 *    The serving API (xyz_serve_*) is thread-safe.
 */
#ifndef XYZ_H
#define XYZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xyz_status;
#define XYZ_OK            0
#define XYZ_EINVAL       (-1)  /* bad shape, value or range (m out of range, L < 1, kappa not finite,
                                  a +-1 input holding another value, NaN or Inf in real data) */
#define XYZ_ENOMEM       (-2)  /* device allocation failed or the context's memory budget is exceeded */
#define XYZ_EDEVICE      (-3)  /* a HIP call failed; the context should be destroyed */
#define XYZ_EAGAIN       (-4)  /* serving: the request is not finished yet */
#define XYZ_ECANCELED    (-5)  /* serving: the request was cancelled or the server stopped */
#define XYZ_EUNSUPPORTED (-6)  /* valid request outside what this build implements */

#define XYZ_MEM_HOST   0
#define XYZ_MEM_DEVICE 1

/* X formats.  All are column-major: column j starts at element j * ld. */
#define XYZ_X_I8_PM1 0   /* int8 in {-1, +1}; ld >= n elements */
#define XYZ_X_BITS   1   /* uint64 words; bit (i % 64) of word i / 64 is 1 iff X_ij = -1; ld >= ceil(n/64) words;
                            bits of rows >= n are ignored */
#define XYZ_X_F32    2   /* float32, finite; ld >= n elements.  Hashing uses the sign transform
                            (x < 0 -> -1, else +1; Section 3.2), verification uses the values */

/* Y formats */
#define XYZ_Y_I8_PM1 0   /* int8 in {-1, +1}: rows are sampled uniformly (eq. (6)) */
#define XYZ_Y_F32    1   /* float32, finite, not all zero: rows sampled with probability |Y_i|/||Y||_1 */
#define XYZ_Y_F64    2   /* float64, same as XYZ_Y_F32 */

/* flags */
#define XYZ_TWO_SIDED 1u  /* also search -Y (Section 4 runs +r and -r in turn): keep |Y^T(X_j o X_k)|/n > kappa */
#define XYZ_PROFILE   2u  /* time the GPU stages with HIP events and report them in xyz_timing */

#define XYZ_MAX_M 30      /* largest supported number of sampled rows per repetition */

typedef struct xyz_ctx xyz_ctx;
typedef struct xyz_x xyz_x;
typedef struct xyz_result xyz_result;
typedef struct xyz_server xyz_server;

/* Parameters of Algorithm 2 (Section 2.2): subsample size M (here m), number of
 * projections L and the threshold on the inner-product scale (kappa of eq. (1);
 * the paper's strength threshold gamma equals (1 + kappa) / 2 by eq. (4)). */
typedef struct {
    int32_t m;            /* rows sampled per repetition, 0 <= m <= XYZ_MAX_M (0: every pair collides) */
    int32_t L;            /* repetitions, >= 1 */
    double kappa;         /* keep Y^T(X_j o X_k)/n > kappa (strict), finite */
    uint64_t seed;        /* row sampler seed */
    uint32_t flags;       /* XYZ_TWO_SIDED | XYZ_PROFILE */
    int32_t rep_offset;   /* index of the first repetition (split or resumed runs); >= 0 */
    const int32_t *rows;  /* optional host table of L*m row indices in [0, n) replacing the sampler;
                             repetition l uses rows[l*m .. l*m+m-1] */
} xyz_params;

/* One reported pair.  For +-1 data s is exact and stat = s/n (binary64
 * division); for real data s = 0 and value is the binary64 inner product. */
typedef struct {
    int32_t j, k;         /* j < k */
    int64_t s;            /* Y^T(X_j o X_k) for +-1 data */
    double value;         /* Y^T(X_j o X_k) (as double) */
    double stat;          /* value / n */
    int32_t first_rep;    /* first repetition that found the pair (-1 for brute force) */
    int32_t hits;         /* repetitions that found the pair (0 for brute force) */
} xyz_pair;

/* Per-repetition statistics (repetition rep_offset + index). */
typedef struct {
    int64_t candidates;   /* |E_l|: unordered colliding pairs j < k */
    int64_t passed;       /* candidates that passed the strength check */
    int64_t fresh;        /* reported pairs first found in this repetition */
    uint64_t cmask;       /* bit t = [Y_{r_t} < 0] for the sampled rows r_0..r_{m-1} */
    int32_t max_bucket;   /* largest number of columns sharing one projected value */
    int32_t reserved;
} xyz_rep_stats;

/* GPU time per stage (milliseconds, summed over launches), filled when the
 * call had XYZ_PROFILE. */
typedef struct {
    double total_ms;      /* whole call, host wall clock */
    double pack_ms;       /* packing Y (and X for brute force) */
    double sample_ms;     /* row sampling */
    double hash_ms;       /* key packing (projection) */
    double bucket_ms;     /* bucket sort and per-repetition statistics */
    double tiles_ms;      /* work-list construction */
    double verify_ms;     /* candidate verification (the dominant stage) */
    double dedup_ms;      /* merging repetitions into the reported set */
    double brute_ms;      /* brute-force kernel */
    int64_t verify_launches;
    int64_t candidates;   /* sum of candidates over repetitions */
    int64_t tiles;        /* verification tiles processed */
} xyz_timing;

/* Library version string (static storage). */
const char *xyz_version(void);
const char *xyz_last_error(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold (0 = no bound). */
xyz_status xyz_init(int device, uint64_t hbm_budget_bytes, xyz_ctx **out);
void xyz_fini(xyz_ctx *ctx);
/* Device bytes currently held by the context (resident X and workspaces). */
uint64_t xyz_ctx_bytes(const xyz_ctx *ctx);

/* Make X resident on the device in the packed layouts the search reads
 * (term (i) of eq. (8)).  X: n x p column-major in format `fmt` (XYZ_X_*),
 * leading dimension ld (elements, or words for XYZ_X_BITS), host or device
 * memory per `mem`.  n >= 1, 1 <= p < 2^31, n < 2^31.  The caller keeps
 * ownership of X. */
xyz_status xyz_x_create(xyz_ctx *ctx, const void *X, int fmt, int mem, int64_t n, int64_t p,
                        int64_t ld, void *stream, xyz_x **out);
void xyz_x_destroy(xyz_x *x);
int64_t xyz_x_n(const xyz_x *x);
int64_t xyz_x_p(const xyz_x *x);

/* Algorithm 2 on resident X and response Y (n entries, format yfmt, memory
 * per mem).  Returns when the result is ready.  Results depend only on
 * (X, Y, params); they are the same when run alone, split over rep_offset
 * ranges, or batched. */
xyz_status xyz_search(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem,
                      const xyz_params *params, void *stream, xyz_result **out);

/* nY searches on the same X in one pass.  Y[q] / params[q] / outs[q] per
 * search.  Searches with uniform sampling (+-1 Y), the same seed, m and
 * repetition range share their projections and bucket sort. */
xyz_status xyz_search_batch(xyz_ctx *ctx, const xyz_x *x, int32_t nY, const void *const *Y, int yfmt,
                            int mem, const xyz_params *params, void *stream, xyz_result **outs);

/* Exact search of eq. (1) over the pairs (a, b), a in colsA, b in colsB,
 * a != b, reported once as (min, max) (brute force, int8 matrix cores for
 * +-1 data).  colsA / colsB: host arrays of column indices, or NULL for all
 * columns.  flags: XYZ_TWO_SIDED | XYZ_PROFILE. */
xyz_status xyz_bruteforce(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                          uint32_t flags, const int32_t *colsA, int64_t nA, const int32_t *colsB,
                          int64_t nB, void *stream, xyz_result **out);

int64_t xyz_result_npairs(const xyz_result *r);
const xyz_pair *xyz_result_pairs(const xyz_result *r);      /* sorted by (j, k), unique */
int32_t xyz_result_nreps(const xyz_result *r);
const xyz_rep_stats *xyz_result_reps(const xyz_result *r);
const xyz_timing *xyz_result_timing(const xyz_result *r);
void xyz_result_free(xyz_result *r);

/* Integer threshold used by the binary path: the smallest s in [-n, n] with
 * (double)s / (double)n > kappa, or n + 1 when there is none (eq. (1)).
 * With two_sided, the smallest s in [0, n] with that property, applied to |s|. */
int64_t xyz_smin(int64_t n, double kappa, int two_sided);

#ifdef __cplusplus
}
#endif
#endif /* XYZ_H */
