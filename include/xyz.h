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
#define XYZ_EUNSUPPORTED (-6)  /* valid request outside what the library implements */
#define XYZ_EINTERNAL    (-7)  /* an internal consistency check failed (a bug in the library) */

#define XYZ_MEM_HOST   0
#define XYZ_MEM_DEVICE 1

/* X formats.  XYZ_X_I8_PM1, XYZ_X_BITS and XYZ_X_F32 are column-major: column j starts at element
 * j * ld.  XYZ_X_I8_PM1_ROWMAJOR is row-major: row i starts at element i * ld. */
#define XYZ_X_I8_PM1 0   /* int8 in {-1, +1}; ld >= n elements */
#define XYZ_X_BITS   1   /* uint64 words; bit (i % 64) of word i / 64 is 1 iff X_ij = -1; ld >= ceil(n/64) words;
                            bits of rows >= n are ignored */
#define XYZ_X_F32    2   /* float32, finite; ld >= n elements.  Hashing uses the sign transform
                            (x < 0 -> -1, else +1; Section 3.2), verification uses the values */
#define XYZ_X_I8_PM1_ROWMAJOR 3  /* int8 in {-1, +1}, row-major (n rows of p entries); ld >= p elements */

/* Y formats */
#define XYZ_Y_I8_PM1 0   /* int8 in {-1, +1}: rows are sampled uniformly (eq. (6)) */
#define XYZ_Y_F32    1   /* float32, finite, not all zero: rows sampled with probability |Y_i|/||Y||_1 */
#define XYZ_Y_F64    2   /* float64, same as XYZ_Y_F32 */

/* flags */
#define XYZ_TWO_SIDED 1u  /* also search -Y (Section 4 runs +r and -r in turn): keep |Y^T(X_j o X_k)|/n > kappa */
#define XYZ_PROFILE   2u  /* time the GPU stages with HIP events and report them in xyz_timing */
#define XYZ_EXACT     4u  /* xyz_serve_submit only: answer with the exact search of eq. (1), as xyz_bruteforce
                             over all columns; m, L, seed, rep_offset and rows are ignored */
#define XYZ_ROUTE    16u  /* xyz_serve_submit only: the server chooses between the exact search and xyz with the
                             request's L (see xyz_serve_submit); m, seed and rows are ignored */
#define XYZ_UNBIASED  8u  /* float32 X only: hash with the unbiased transform of Section 3.2 (Proposition 4)
                             instead of the sign transform.  Each row is divided by its largest absolute
                             entry nu_i and Y_i multiplied by nu_i^2, so rows are drawn with probability
                             proportional to |Y_i| nu_i^2 (+-1 Y: nu_i^2), and every sampled entry becomes +1
                             with probability (1 + X_ij / nu_i) / 2, drawn afresh for each repetition, draw
                             and column from a counter-based SplitMix64 stream (draw t of repetition l: stream
                             seed = output 1 + l*2^16 + t of SplitMix64 seeded with seed ^ 0x2545F4914F6CDD1D;
                             column j: top 24 bits u of that stream's output 1 + j; +1 exactly when, in
                             binary64, (u * 2) * nu_i < (nu_i + X_ij) * 2^24; on an all-zero row, when
                             u < 2^23).  With xyz_params.cap > 0 the entries are first capped at
                             +-cap (Section 3.2's remark on capping; cap rounded to float32): nu_i, the
                             row weights and the transform then use min(max(X_ij, -cap), cap).  The
                             strength check stays eq. (1) on the original X and Y.
                             XYZ_EUNSUPPORTED for int8 or bit-packed X. */

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
    uint32_t flags;       /* XYZ_TWO_SIDED | XYZ_PROFILE | XYZ_UNBIASED */
    int32_t rep_offset;   /* index of the first repetition (split or resumed runs); >= 0 */
    const int32_t *rows;  /* optional host table of L*m row indices in [0, n) replacing the sampler;
                             repetition l uses rows[l*m .. l*m+m-1] */
    double cap;           /* XYZ_UNBIASED only: 0 for no capping, else cap |X_ij| at cap (> 0, finite or
                             +inf, at least the smallest positive float32) before the transform;
                             XYZ_EINVAL otherwise */
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
    double big_ms;        /* the part of verify_ms spent on products of large buckets (LDS-staged block pairs on
                             the matrix cores) */
    int64_t big_launches;
    int64_t big_candidates;   /* candidates verified in those products */
    int64_t chunks;           /* chunks of repetitions the search ran (each stage launches once per chunk) */
    int64_t host_syncs;       /* host waits on the stream during the search: one per chunk (three for m > 15),
                                 one after the inputs are checked, two for the merged result, and one more
                                 per chunk redone when a tile list or the survivor buffer grew */
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
 * (term (i) of eq. (8)).  X: n x p in format `fmt` (XYZ_X_*: column-major, or
 * row-major for XYZ_X_I8_PM1_ROWMAJOR), leading dimension ld (elements, or
 * words for XYZ_X_BITS), host or device
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

/* xyz_search for callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same search, with the same result, but no device memory is
 * allocated or freed, and no host memory either.  Every workspace is carved from one static device
 * array of XYZ_NOALLOC_SCRATCH_BYTES per device, held from the library's first xyz_init on that
 * device until the process ends; calls that overlap on one device race on it (serialise them).
 * Y: n entries per yfmt / mem; params: as xyz_search, without XYZ_PROFILE (XYZ_EUNSUPPORTED).
 * pairs: caller-owned host array of pairs_cap entries (NULL when pairs_cap = 0); *npairs receives the
 * number of pairs found, sorted by (j, k); when it exceeds pairs_cap nothing is written to pairs and
 * XYZ_ENOMEM is returned (call again with room for *npairs).  reps: caller-owned host array of L
 * entries.  A search whose workspace exceeds the scratch fails with XYZ_ENOMEM: before any launch
 * when the statistics of L repetitions, packed Y and one repetition's keys, permutation and bucket
 * offsets need more than half of it; during the search when tiles, survivors and merge scratch
 * need more than the rest. */
#define XYZ_NOALLOC_SCRATCH_BYTES (256ull << 20)
xyz_status xyz_search_noalloc(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem,
                              const xyz_params *params, void *stream, xyz_pair *pairs, int64_t pairs_cap,
                              int64_t *npairs, xyz_rep_stats *reps);

/* Launch shapes of Algorithm 2 that do not change a search's result: how many repetitions one
 * chunk holds (its workspace budget: keys, permutations and bucket offsets; more repetitions per
 * chunk give the hash and bucket launches more workgroups) and the workgroups per compute unit of
 * the tile-verification and big-tile launches. */
typedef struct {
    double chunk_gib;          /* workspace budget of one chunk, GiB (default 8) */
    int32_t verify_wg_per_cu;  /* tile-verification launches (default 24) */
    int32_t big_wg_per_cu;     /* big-tile launch (default 8) */
    int32_t from_cache;        /* 1: read from the cache file, nothing was timed */
    int32_t variants;          /* searches timed (0 when read from the cache) */
    double ms;                 /* wall time of the search under the chosen shapes, ms (as recorded) */
} xyz_tuning;

/* Times the search (x, Y, params) under a few launch shapes, one choice at a time from the
 * defaults, and keeps the fastest for every later search of the same shape in the context: the
 * same device architecture and compute units, n, p, m, X and Y formats, XYZ_TWO_SIDED and
 * XYZ_UNBIASED.  cache_path (or NULL): a text file of tuned shapes; when it holds this shape the
 * record is used and nothing is timed, else the choice is added to it (written to cache_path.tmp,
 * then renamed).  The search runs several times (params as xyz_search, without XYZ_PROFILE);
 * every run must give the same pairs (XYZ_EINTERNAL otherwise).  Chunk budgets above the default
 * are tried only with room in free device memory.  out: the choice. */
xyz_status xyz_autotune(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, const xyz_params *params,
                        void *stream, const char *cache_path, xyz_tuning *out);

/* Exact search of eq. (1) over the pairs (a, b), a in colsA, b in colsB,
 * a != b, reported once as (min, max) (brute force, FP4 e2m1 matrix cores for
 * +-1 data).  colsA / colsB: host arrays of column indices, or NULL for all
 * columns.  flags: XYZ_TWO_SIDED | XYZ_PROFILE. */
xyz_status xyz_bruteforce(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                          uint32_t flags, const int32_t *colsA, int64_t nA, const int32_t *colsB,
                          int64_t nB, void *stream, xyz_result **out);

/* --------------------------------------------------- dense projections --
 * Algorithm 1 (Section 2.1) with a dense projection vector per repetition
 * (class (a) of Section 2.1), the scheme that Section 5.1 and Theorem 1
 * compare with minimal subsampling.  Repetition l projects the columns of X
 * and of Z = Y o X onto R_l, x = X^T R_l and z = Z^T R_l; E_l holds the ordered
 * pairs (j, k), j != k, with |x_j - z_k| <= tau; every unordered pair {j, k}
 * with (j, k) or (k, j) in E_l is checked once against eq. (1) (strict
 * Y^T(X_j o X_k)/n > kappa) and kept pairs are reported as (min, max).
 *
 * X: resident, +-1 (XYZ_X_I8_PM1 or XYZ_X_BITS; float X is XYZ_EUNSUPPORTED).
 * Y: n entries, XYZ_Y_I8_PM1 only, host or device memory per mem.
 * R: host array of L * n int32 weights, repetition l uses R[l*n .. l*n+n-1]:
 *    the projection vector on a fixed-point grid chosen by the caller (for a
 *    Gaussian F, round(2^b N(0, 1))).  sum_i |R[l*n+i]| must not exceed
 *    2^31 - 1 and no |R[l*n+i]| may exceed 2^31 - 2^24 (XYZ_EINVAL otherwise):
 *    projections are then exact int32 sums, so E_l does not depend on
 *    summation order.  Copied before the call returns.
 * tau: close-pairs threshold on the same grid, >= 0.  L >= 1; rep_offset >= 0
 *    numbers the repetitions (first_rep) as in xyz_search.
 * flags: XYZ_PROFILE only (others: XYZ_EUNSUPPORTED).
 * Result: pairs as from xyz_search (s exact); per repetition, candidates =
 * unordered pairs checked, passed, fresh, cmask = 0 and max_bucket = the
 * largest window max_j |{k : |x_j - z_k| <= tau}| (k = j included).  The
 * caller frees it with xyz_result_free. */
xyz_status xyz_dense_search(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, const int32_t *R,
                            int32_t L, int64_t tau, double kappa, int32_t rep_offset, uint32_t flags, void *stream,
                            xyz_result **out);

/* ---------------------------------------------------- parameter choice --
 * Section 2.3: a pair of strength gamma (eq. (3); gamma = (1 + s/n)/2 by
 * eq. (4)) lands in E_l with probability gamma^m, so it is found within L
 * repetitions with probability eta = 1 - (1 - gamma^m)^L (eq. (9)). */

/* eq. (9). */
double xyz_eta(double gamma, int32_t m, int64_t L);
/* eq. (15): the smallest L with 1 - (1 - beta)^L >= eta, beta = gamma^m in (0, 1]; -1 if beta <= 0 or eta
 * not in (0, 1). */
int64_t xyz_L_for(double eta, double beta);
/* The largest m in [0, m_max] with eta(gamma, m, L) >= eta, or -1 (the rule for a request with fixed L). */
int32_t xyz_m_for_L(double gamma, int64_t L, double eta, int32_t m_max);
/* eq. (11): M* = argmin over M in [1, m_max] of -(M p + p log p + n S(M)) / log(1 - gamma^M), with
 * S(M) = total_pairs * mean(gammas^M) estimated from ns sampled strengths (Section 2.3: "estimated by
 * sampling"); returns -1 on invalid input. */
int32_t xyz_mstar(double gamma, int64_t n, int64_t p, const double *gammas, int64_t ns, double total_pairs,
                  int32_t m_max);

/* Section 5.1, dense Gaussian projections at the budget of minimal subsampling (the mean
 * size of E_1 is p when every pair has strength 1/2), for +-1 data and R ~ N(0, sd^2 I): the
 * projected distance x_j - z_k of a pair of strength gamma is exactly N(0, 4 n (1 - gamma) sd^2).
 * xyz_tau_dense: the threshold tau with P(|x_j - z_k| <= tau) = 1/p at gamma = 1/2 (the
 * (1/p)-quantile of |W|); NAN unless p >= 2, n >= 1, sd > 0.
 * xyz_eta_dense: the probability that the ordered pair (j, k) of strength gamma lands in E_1
 * at that tau, erf(erfinv(1/p) sqrt(1/2 / (1 - gamma))), free of n; NAN unless p >= 2 and
 * 0 <= gamma <= 1. */
double xyz_tau_dense(int64_t p, int64_t n, double sd);
double xyz_eta_dense(double gamma, int64_t p);

/* Strengths of npairs column pairs drawn uniformly (j != k) with SplitMix64(seed): gamma = fraction of rows
 * with sgn(Y_i) = X~_ij X~_ik, weighted by |Y_i|/||Y||_1 for real Y (the collision probability of one row
 * draw, Section 3.1).  out: host array of npairs doubles. */
xyz_status xyz_sample_strengths(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, int64_t npairs,
                                uint64_t seed, void *stream, double *out);

#define XYZ_PLAN_XYZ   0
#define XYZ_PLAN_BRUTE 1
typedef struct {
    int32_t method;             /* XYZ_PLAN_XYZ or XYZ_PLAN_BRUTE */
    int32_t m, L;               /* the xyz parameters (m = 0, L = 1 for brute force) */
    int32_t mstar;              /* eq. (11) under the paper's cost model, for reference */
    double predicted_ms;        /* predicted GPU time of the chosen plan */
    double predicted_recall;    /* eq. (9) at gamma_target (1 for brute force) */
    double expected_candidates; /* sum over repetitions of E|E_l| (unordered pairs) */
    double brute_ms;            /* predicted time of the exact search */
} xyz_plan_info;

/* Autotuner: choose brute force or xyz (m, L) for a search at threshold kappa that must find pairs of
 * strength >= gamma_target (gamma scale) with probability >= eta_target.  Samples pair strengths to predict
 * E|E_l| per m, takes L from eq. (15), times short runs of the candidate plans on this X and Y, and picks
 * the fastest.  flags: XYZ_TWO_SIDED. */
xyz_status xyz_plan(xyz_ctx *ctx, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                    double gamma_target, double eta_target, uint32_t flags, void *stream, xyz_plan_info *out);

/* -------------------------------------------------------------- serving --
 * A server owns `workers` threads, each with its own context (workspaces) and
 * HIP stream on the device of ctx.  Requests on resident X (any context of the
 * same device; X must outlive its requests) wait in one FIFO queue; a free
 * worker takes the oldest request whose estimated device bytes fit within
 * hbm_budget_bytes (0: no bound) beside what the other workers hold or run
 * (their workspaces are counted while idle, and a worker keeps at most
 * budget / workers bytes between groups), together with up to
 * max_batch - 1 queued requests it can share a pass with (same X, m, L, seed,
 * rep_offset and flags, +-1 Y, no row table: one row draw, projection and
 * bucket sort serve them all).  Groups on different workers overlap on the
 * device.  Each result equals the request's stand-alone xyz_search.  A request
 * larger than the budget runs fewer repetitions per chunk; if one repetition
 * does not fit, submission fails with XYZ_ENOMEM.  All xyz_serve_* calls are
 * thread-safe. */
typedef struct {
    uint64_t submitted, completed, canceled, failed;
    uint64_t batches;           /* groups run */
    int32_t max_batch;          /* largest group */
    int32_t queued, inflight;   /* requests waiting / running now */
    uint64_t bytes_inflight;    /* estimated device bytes of running groups */
    double p50_ms, p99_ms, max_ms;  /* submit-to-completion latency of completed requests */
    uint64_t bytes_held;        /* device bytes the workers' contexts may hold now: the larger of what each
                                   holds and the estimate of the group it runs */
} xyz_serve_stats;

xyz_status xyz_serve_start(xyz_ctx *ctx, uint64_t hbm_budget_bytes, int32_t workers, int32_t max_batch,
                           xyz_server **out);
/* Queue a search; Y (host memory, format yfmt) and params (including its row table) are copied.
 * With XYZ_EXACT in params->flags the request is answered by the exact search (result as from
 * xyz_bruteforce); such requests are never grouped with others.
 * With XYZ_ROUTE (+-1 X and Y) the server picks the method, as Section 2.3 compares xyz with the
 * O(n p^2) search: xyz with the request's L and the largest m <= 15 whose recall eq. (9) at the
 * threshold's own strength gamma = (1 + kappa)/2 is at least 0.95 (xyz_m_for_L), or the exact
 * search, whichever its cost model predicts faster.  The cost model prices the exact search at
 * p(p-1)/2 pairs of n rows and xyz at L repetitions of p columns plus E|E_l| candidates of n rows,
 * E|E_l| = p(p-1)/2 times the mean of gamma_jk^m over 4096 sampled pairs (xyz_sample_strengths;
 * Section 2.3 estimates the strengths by sampling); its rates start from values measured on this
 * part and follow the server's completed requests.  A routed xyz request samples its rows with
 * the shared seed XYZ_SERVE_SEED, so that routed requests on the same X with the same L, m and
 * flags share a pass.  xyz_result_route tells what was run. */
#define XYZ_SERVE_SEED 0x9E3779B97F4A7C15ull
xyz_status xyz_serve_submit(xyz_server *s, const xyz_x *x, const void *Y, int yfmt, const xyz_params *params,
                            uint64_t *ticket);
/* XYZ_EAGAIN while the request is queued or running; otherwise the request's result (or its error, or
 * XYZ_ECANCELED) is returned once and the ticket is forgotten. */
xyz_status xyz_serve_poll(xyz_server *s, uint64_t ticket, xyz_result **out);
/* Like xyz_serve_poll but blocks until the request is finished. */
xyz_status xyz_serve_wait(xyz_server *s, uint64_t ticket, xyz_result **out);
/* Cancel a queued request (XYZ_EAGAIN if it is already running). */
xyz_status xyz_serve_cancel(xyz_server *s, uint64_t ticket);
xyz_status xyz_serve_stats_get(xyz_server *s, xyz_serve_stats *out);
/* Cancel queued requests, wait for running ones, free the server and every unclaimed result. */
xyz_status xyz_serve_stop(xyz_server *s);

/* What produced a result: the method (XYZ_PLAN_XYZ or XYZ_PLAN_BRUTE), xyz's m, L and seed (0, 1, 0
 * for the exact search) and, for a request routed by a server (XYZ_ROUTE), the cost model's
 * predictions for the chosen and the other method (0 otherwise). */
typedef struct {
    int32_t method;
    int32_t m, L;
    int32_t routed;             /* 1 when the server chose the method */
    uint64_t seed;
    double predicted_ms;
    double alternative_ms;
} xyz_route;
xyz_status xyz_result_route(const xyz_result *r, xyz_route *out);
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
