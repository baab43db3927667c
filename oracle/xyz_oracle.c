/*
 * xyz_oracle.c -- plain CPU oracle for the xyz interaction search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path loads, links or calls
 * this file: it exists so that tests, the smoke check and the benchmark's CPU
 * baseline can compare the GPU library against an independent, slow and
 * obviously correct implementation written directly from the paper
 * (Thanei, Meinshausen & Shah, "The xyz algorithm for fast interaction search
 * in high-dimensional data").  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes
 *  - Problem (eq. (1), Section 1): keep the pairs (j,k) with
 *    Y^T (X_j o X_k) / n > kappa.  Pairs are unordered, j < k.
 *  - Algorithm 2 (Section 2.2, "final version of xyz"): form Z = Y o X, then
 *    for each of L repetitions draw M row indices i.i.d. with replacement
 *    (eq. (6) with tau = 0, "minimal subsampling"), find all (j,k) whose X_j
 *    and Z_k agree on every sampled row (the event x_j = z_k of the random
 *    projection, Section 2.1), and keep the candidates that pass the strength
 *    check.  The equal-pairs search sorts the 2p projected values and walks
 *    the distinct values, recording X-side x Z-side index sets (Section 2.2,
 *    Figure 2).
 *  - Continuous Y (Section 3.1): Z = sgn(Y) o X, rows drawn with probability
 *    |Y_i| / ||Y||_1.  Continuous X (Section 3.2): X is first mapped to its
 *    signs (the "sign transform"), or, on request, by the unbiased transform
 *    of Section 3.2 (Proposition 4): each row is divided by its largest
 *    absolute entry nu_i and Y_i is multiplied by nu_i^2 (the paper's remark
 *    after Proposition 4), so rows are drawn with probability proportional to
 *    |Y_i| nu_i^2, and every sampled entry becomes +1 with probability
 *    (1 + X_ij / nu_i) / 2, drawn afresh for each repetition, draw and column;
 *    the Z side uses the same draw, Z~_ij = sgn(Y_i) X~_ij.  Optionally the
 *    entries are first capped at +-c (Section 3.2's remark on capping): the
 *    transform, the row maxima and the row weights then all see the capped
 *    entries min(max(X_ij, -c), c).
 *
 * Readings where the paper leaves a choice (each is also listed in the
 * design notes of the repository):
 *  - the strength check uses eq. (1)'s strict ">" on s/n, evaluated as an
 *    IEEE binary64 division of the exact integer s by n (binary data) or of
 *    the binary64 sum v = sum_i (Y_i X_ij) X_ik taken in ascending i
 *    (continuous data);
 *  - the projection x_j is represented exactly by the tuple of column j's
 *    entries on the sampled rows: with tau = 0 and a continuous weight
 *    distribution, x_j = z_k holds exactly when the tuples agree (Section
 *    2.1), and comparing tuples avoids any chance collision by rounding;
 *  - a sign-transformed entry is -1 when x < 0 and +1 otherwise (so +-0 map
 *    to +1) instead of the paper's coin toss for zeros;
 *  - row draws come from SplitMix64 (Steele, Lea & Flood 2014, the
 *    generator of Vigna's public-domain splitmix64.c): draw t of repetition l
 *    is output number 1 + l*2^16 + t of the generator seeded with `seed`;
 *    a uniform row is floor(u * n / 2^64); a |Y|-weighted row is the first i
 *    whose running sum |Y_0| + ... + |Y_i| exceeds (u >> 11) * 2^-53 * ||Y||_1;
 *  - two-sided search (Section 4 runs xyz on +r and -r in turn) adds the
 *    equal pairs of X against -Z and keeps |s|/n > kappa;
 *  - the unbiased transform's draws are counter based: draw t of repetition
 *    l seeds a stream, output number 1 + l*2^16 + t of SplitMix64 seeded with
 *    seed ^ 0x2545F4914F6CDD1D, and column j takes the top 24 bits u of that
 *    stream's output number 1 + j; X~_ij = +1 exactly when, in binary64,
 *    (u * 2) * nu_i < (nu_i + X_ij) * 2^24 (u / 2^24 < (1 + X_ij / nu_i) / 2
 *    without a division), and with probability 1/2 (u < 2^23) on a row whose
 *    entries are all zero (nu_i = 0; such a row is drawn only from a row table);
 *    the row weights are |Y_i| * (nu_i * nu_i), summed left to right;
 *  - the cap c of the unbiased transform is taken in float32, as X is: c is
 *    the caller's value rounded to the nearest float32, so that every capped
 *    entry is a float32 value; the strength check stays eq. (1) on the
 *    original, uncapped X.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define XO_OK 0
#define XO_EINVAL (-1)
#define XO_ENOMEM (-2)

typedef struct {
    int32_t j, k;        /* j < k */
    int64_t s;           /* exact Y^T(X_j o X_k) for binary data, else 0 */
    double value;        /* the inner product (exact integer as double, or the binary64 sum) */
    double stat;         /* value / n */
    int32_t first_rep;   /* smallest repetition index in which the pair was found (-1 for brute force) */
    int32_t hits;        /* number of repetitions in which the pair was found */
} xo_pair;

typedef struct {
    int64_t candidates;  /* |E_l|, unordered pairs j < k */
    int64_t passed;      /* candidates of E_l that pass the strength check */
    int64_t fresh;       /* pairs whose first_rep is this repetition */
    uint64_t cmask;      /* bit t = [Y_{r_t} < 0] */
    int32_t max_bucket;  /* largest number of X-side columns sharing one projected value */
    int32_t pad;
} xo_rep;

/* ------------------------------------------------------------------ RNG -- */

/* Output number k (k >= 1) of SplitMix64 seeded with `seed`. */
uint64_t xo_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t draw_u64(uint64_t seed, int64_t l, int t)
{
    return xo_splitmix64(seed, 1ull + (uint64_t)l * 65536ull + (uint64_t)t);
}

/* Uniform row (Section 2.1, eq. (6): i.i.d. indices, with replacement). */
static int64_t uniform_row(uint64_t u, int64_t n)
{
    return (int64_t)(((unsigned __int128)u * (unsigned __int128)(uint64_t)n) >> 64);
}

/* |Y|-weighted row (Section 3.1): P(i) = |Y_i| / ||Y||_1, by inverting the
 * running sum cdf[i] = |Y_0| + ... + |Y_i| (binary64, left to right). */
static int64_t weighted_row(uint64_t u, const double *cdf, const double *Y, int64_t n)
{
    double v = ((double)(u >> 11) * 0x1p-53) * cdf[n - 1];
    for (int64_t i = 0; i < n; i++)
        if (cdf[i] > v) return i;
    for (int64_t i = n - 1; i >= 0; i--)
        if (Y[i] != 0.0) return i;
    return -1;
}

/* Row draws of repetition l with probability proportional to w_i >= 0 (a
 * row of weight 0 is never drawn; the last row of positive weight catches a
 * draw at the very top of the running sum). */
static int draw_rows_w(const double *w, int64_t n, uint64_t seed, int64_t l, int m, int32_t *out)
{
    double *cdf = (double *)malloc(sizeof(double) * (size_t)n);
    if (!cdf) return XO_ENOMEM;
    double acc = 0.0;
    for (int64_t i = 0; i < n; i++) { acc = acc + w[i]; cdf[i] = acc; }
    if (!(acc > 0.0)) { free(cdf); return XO_EINVAL; }
    for (int t = 0; t < m; t++) {
        uint64_t u = draw_u64(seed, l, t);
        out[t] = (int32_t)weighted_row(u, cdf, w, n);
    }
    free(cdf);
    return XO_OK;
}

/* Unbiased transform (Section 3.2, Proposition 4) of entry x of a row with
 * largest absolute entry nu, for draw t of repetition l and column j:
 * +1 with probability (1 + x / nu) / 2. */
#define XO_UNBIASED_STREAM 0x2545F4914F6CDD1Dull
static int8_t unbiased_sign(uint64_t seed, int64_t l, int t, int64_t j, double x, double nu)
{
    uint64_t stream = xo_splitmix64(seed ^ XO_UNBIASED_STREAM, 1ull + (uint64_t)l * 65536ull + (uint64_t)t);
    uint64_t u = xo_splitmix64(stream, 1ull + (uint64_t)j) >> 40;
    int plus;
    if (nu > 0.0) plus = ((double)u * 2.0) * nu < (nu + x) * 16777216.0;
    else plus = u < 8388608ull;
    return plus ? 1 : -1;
}

/* Row draws of repetition l.  Y == NULL selects the uniform sampler. */
int xo_draw_rows(const double *Y, int64_t n, uint64_t seed, int64_t l, int m, int32_t *out)
{
    if (n <= 0 || m < 0) return XO_EINVAL;
    double *cdf = NULL;
    if (Y) {
        cdf = (double *)malloc(sizeof(double) * (size_t)n);
        if (!cdf) return XO_ENOMEM;
        double acc = 0.0;
        for (int64_t i = 0; i < n; i++) { acc = acc + fabs(Y[i]); cdf[i] = acc; }
        if (!(acc > 0.0)) { free(cdf); return XO_EINVAL; }
    }
    for (int t = 0; t < m; t++) {
        uint64_t u = draw_u64(seed, l, t);
        out[t] = (int32_t)(Y ? weighted_row(u, cdf, Y, n) : uniform_row(u, n));
    }
    free(cdf);
    return XO_OK;
}

/* ------------------------------------------------------- inner products -- */

/* eq. (1): s = Y^T (X_j o X_k) for +-1 data, exactly. X column-major (n x p). */
int64_t xo_pair_s(const int8_t *X, const int8_t *Y, int64_t n, int64_t j, int64_t k)
{
    const int8_t *a = X + j * n, *b = X + k * n;
    int64_t s = 0;
    for (int64_t i = 0; i < n; i++) s += (int64_t)Y[i] * a[i] * b[i];
    return s;
}

/* eq. (1) for real data: v = sum_i (Y_i X_ij) X_ik in binary64, ascending i. */
double xo_pair_v(const double *X, const double *Y, int64_t n, int64_t j, int64_t k)
{
    const double *a = X + j * n, *b = X + k * n;
    double v = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double t = Y[i] * a[i];
        t = t * b[i];
        v = v + t;
    }
    return v;
}

/* --------------------------------------------------------- equal pairs -- */

typedef struct { int32_t idx; int32_t side; } entry;   /* side 0: x (X), side 1: z (Z) */

typedef struct { const int8_t *tx, *tz; int m; } tuple_ctx;

static const int8_t *tuple_of(const tuple_ctx *c, const entry *e)
{
    return (e->side ? c->tz : c->tx) + (size_t)e->idx * (size_t)c->m;
}

static int cmp_entry(const void *pa, const void *pb, void *ctx)
{
    const tuple_ctx *c = (const tuple_ctx *)ctx;
    const entry *a = (const entry *)pa, *b = (const entry *)pb;
    int r = c->m ? memcmp(tuple_of(c, a), tuple_of(c, b), (size_t)c->m) : 0;
    if (r) return r;
    if (a->side != b->side) return a->side - b->side;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct { int64_t *v; size_t n, cap; } vec64;

static int vpush(vec64 *a, int64_t x)
{
    if (a->n == a->cap) {
        size_t nc = a->cap ? a->cap * 2 : 1024;
        int64_t *nv = (int64_t *)realloc(a->v, nc * sizeof(int64_t));
        if (!nv) return XO_ENOMEM;
        a->v = nv; a->cap = nc;
    }
    a->v[a->n++] = x;
    return XO_OK;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Equal-pairs search of Section 2.2: sort the 2p projected values (here:
 * the tuples of X_j and of Z_k on the sampled rows), walk the distinct
 * values, and for every value held by both sides record the X-side x Z-side
 * index sets.  Every ordered (j,k), j != k, is pushed as the unordered key
 * min*p + max.  Returns the largest X-side group size in *maxb. */
static int equal_pairs(const int8_t *tx, const int8_t *tz, int64_t p, int m,
                       vec64 *out, int32_t *maxb)
{
    entry *e = (entry *)malloc(sizeof(entry) * (size_t)(2 * p));
    int32_t *A = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    int32_t *B = (int32_t *)malloc(sizeof(int32_t) * (size_t)p);
    if (!e || !A || !B) { free(e); free(A); free(B); return XO_ENOMEM; }
    for (int64_t j = 0; j < p; j++) { e[j].idx = (int32_t)j; e[j].side = 0; }
    for (int64_t k = 0; k < p; k++) { e[p + k].idx = (int32_t)k; e[p + k].side = 1; }
    tuple_ctx c = { tx, tz, m };
    qsort_r(e, (size_t)(2 * p), sizeof(entry), cmp_entry, &c);
    int rc = XO_OK;
    int64_t g0 = 0;
    while (g0 < 2 * p && rc == XO_OK) {
        int64_t g1 = g0 + 1;
        while (g1 < 2 * p &&
               (m == 0 || memcmp(tuple_of(&c, &e[g0]), tuple_of(&c, &e[g1]), (size_t)m) == 0))
            g1++;
        int64_t na = 0, nb = 0;
        for (int64_t q = g0; q < g1; q++) {
            if (e[q].side == 0) A[na++] = e[q].idx; else B[nb++] = e[q].idx;
        }
        if (na > *maxb) *maxb = (int32_t)na;
        for (int64_t a = 0; a < na && rc == XO_OK; a++)
            for (int64_t b = 0; b < nb && rc == XO_OK; b++) {
                int64_t j = A[a], k = B[b];
                if (j == k) continue;
                int64_t lo = j < k ? j : k, hi = j < k ? k : j;
                rc = vpush(out, lo * p + hi);
            }
        g0 = g1;
    }
    free(e); free(A); free(B);
    return rc;
}

/* -------------------------------------------------------------- search -- */

typedef struct { int64_t key; int32_t rep; double value; int64_t s; } record;

static int cmp_record(const void *pa, const void *pb)
{
    const record *a = (const record *)pa, *b = (const record *)pb;
    if (a->key != b->key) return (a->key > b->key) - (a->key < b->key);
    return (a->rep > b->rep) - (a->rep < b->rep);
}

/*
 * Algorithm 2.  X: n x p column-major, int8 +-1 (xkind 0) or binary64
 * (xkind 1).  Y: int8 +-1 (ykind 0, uniform row sampling) or binary64
 * (ykind 1, |Y|-weighted sampling).  rows: optional L x m table overriding
 * the sampler.  Outputs malloc'ed arrays (free with xo_free); reps must hold
 * L entries.
 */
/* Entry x capped at +-c (c = +inf: unchanged). */
static double capped(double x, double c)
{
    return x > c ? c : (x < -c ? -c : x);
}

/* transform: 0 = sign transform of real X (or +-1 X as is), 1 = unbiased
 * transform of real X (Section 3.2).  cap (transform 1 only): 0 for none,
 * else the entries are capped at +-cap (rounded to float32) before the
 * transform. */
int xo_search_ex(const void *Xv, int xkind, const void *Yv, int ykind, int64_t n, int64_t p,
                 int m, int L, double kappa, uint64_t seed, int two_sided, int rep_offset,
                 const int32_t *rows_in, int transform, double cap, xo_pair **out_pairs, int64_t *out_npairs,
                 xo_rep *reps)
{
    if (n <= 0 || p <= 0 || m < 0 || m > 64 || L < 0 || !(kappa == kappa) || isinf(kappa))
        return XO_EINVAL;
    if (transform != 0 && (transform != 1 || xkind != 1)) return XO_EINVAL;
    if (!(cap >= 0.0) || (cap != 0.0 && transform != 1)) return XO_EINVAL;
    const double c = cap == 0.0 ? INFINITY : (double)(float)cap;
    if (!(c > 0.0)) return XO_EINVAL;
    const int8_t *Xb = (const int8_t *)Xv; const double *Xd = (const double *)Xv;
    const int8_t *Yb = (const int8_t *)Yv; const double *Yd = (const double *)Yv;
    int binary = (xkind == 0 && ykind == 0);

    /* X~ (sign transform for real X), sgn(Y), and Z = sgn(Y) o X~ (Algorithm 2, first step). */
    int8_t *Xs = (int8_t *)malloc((size_t)(n * p));
    int8_t *Z = (int8_t *)malloc((size_t)(n * p));
    int8_t *Ys = (int8_t *)malloc((size_t)n);
    double *Ydw = NULL;
    if (!Xs || !Z || !Ys) { free(Xs); free(Z); free(Ys); return XO_ENOMEM; }
    for (int64_t i = 0; i < n; i++) {
        if (ykind == 0) {
            if (Yb[i] != 1 && Yb[i] != -1) { free(Xs); free(Z); free(Ys); return XO_EINVAL; }
            Ys[i] = Yb[i];
        } else {
            if (!(Yd[i] == Yd[i]) || isinf(Yd[i])) { free(Xs); free(Z); free(Ys); return XO_EINVAL; }
            Ys[i] = Yd[i] < 0.0 ? -1 : 1;
        }
    }
    for (int64_t j = 0; j < p; j++)
        for (int64_t i = 0; i < n; i++) {
            int8_t x;
            if (xkind == 0) {
                x = Xb[j * n + i];
                if (x != 1 && x != -1) { free(Xs); free(Z); free(Ys); return XO_EINVAL; }
            } else {
                double d = Xd[j * n + i];
                if (!(d == d) || isinf(d)) { free(Xs); free(Z); free(Ys); return XO_EINVAL; }
                x = d < 0.0 ? -1 : 1;
            }
            Xs[j * n + i] = x;
            Z[j * n + i] = (int8_t)(Ys[i] * x);
        }
    /* real-valued copies for the continuous inner product */
    double *Xdw = NULL;
    if (!binary) {
        Ydw = (double *)malloc(sizeof(double) * (size_t)n);
        if (xkind == 0) Xdw = (double *)malloc(sizeof(double) * (size_t)(n * p));
        if (!Ydw || (xkind == 0 && !Xdw)) { free(Xs); free(Z); free(Ys); free(Ydw); free(Xdw); return XO_ENOMEM; }
        for (int64_t i = 0; i < n; i++) Ydw[i] = ykind == 0 ? (double)Yb[i] : Yd[i];
        if (xkind == 0) for (int64_t q = 0; q < n * p; q++) Xdw[q] = (double)Xb[q];
    }
    const double *Xreal = xkind == 1 ? Xd : Xdw;
    if (ykind == 1) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; i++) acc = acc + fabs(Yd[i]);
        if (!(acc > 0.0)) { free(Xs); free(Z); free(Ys); free(Ydw); free(Xdw); return XO_EINVAL; }
    }

    /* unbiased transform: row maxima nu_i and row weights |Y_i| nu_i^2 */
    double *nu = NULL, *wrow = NULL;
    if (transform == 1) {
        nu = (double *)malloc(sizeof(double) * (size_t)n);
        wrow = (double *)malloc(sizeof(double) * (size_t)n);
        if (!nu || !wrow) { free(Xs); free(Z); free(Ys); free(Ydw); free(Xdw); free(nu); free(wrow); return XO_ENOMEM; }
        for (int64_t i = 0; i < n; i++) {
            double v = 0.0;
            for (int64_t j = 0; j < p; j++) {
                double a = fabs(capped(Xd[j * n + i], c));
                if (a > v) v = a;
            }
            nu[i] = v;
            wrow[i] = fabs(ykind == 0 ? (double)Yb[i] : Yd[i]) * (v * v);
        }
    }

    int mm = m > 0 ? m : 1;
    int8_t *tx = (int8_t *)malloc((size_t)(p * mm));
    int8_t *tz = (int8_t *)malloc((size_t)(p * mm));
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)mm);
    vec64 cand = { 0 };
    record *rec = NULL; size_t nrec = 0, caprec = 0;
    int rc = (tx && tz && rows) ? XO_OK : XO_ENOMEM;

    for (int li = 0; li < L && rc == XO_OK; li++) {
        int64_t l = (int64_t)rep_offset + li;
        /* draw R: M row indices (eq. (6)) */
        if (rows_in) {
            for (int t = 0; t < m; t++) {
                rows[t] = rows_in[(size_t)li * (size_t)m + t];
                if (rows[t] < 0 || rows[t] >= n) { rc = XO_EINVAL; break; }
            }
            if (rc != XO_OK) break;
        } else if (transform == 1) {
            rc = draw_rows_w(wrow, n, seed, l, m, rows);
            if (rc != XO_OK) break;
        } else {
            rc = xo_draw_rows(ykind == 1 ? Yd : NULL, n, seed, l, m, rows);
            if (rc != XO_OK) break;
        }
        uint64_t cm = 0;
        for (int t = 0; t < m; t++) if (Ys[rows[t]] < 0) cm |= 1ull << t;
        reps[li].cmask = cm;
        /* projections x = X^T R, z = Z^T R, represented by the sampled tuples */
        for (int64_t j = 0; j < p; j++)
            for (int t = 0; t < m; t++) {
                if (transform == 1) {
                    int64_t i = rows[t];
                    int8_t xt = unbiased_sign(seed, l, t, j, capped(Xd[j * n + i], c), nu[i]);
                    tx[j * m + t] = xt;
                    tz[j * m + t] = (int8_t)(Ys[i] * xt);
                } else {
                    tx[j * m + t] = Xs[j * n + rows[t]];
                    tz[j * m + t] = Z[j * n + rows[t]];
                }
            }
        cand.n = 0;
        int32_t maxb = 0;
        rc = equal_pairs(tx, tz, p, m, &cand, &maxb);
        if (rc == XO_OK && two_sided) {
            /* -Y: the Z side changes sign */
            for (int64_t q = 0; q < p * m; q++) tz[q] = (int8_t)(-tz[q]);
            rc = equal_pairs(tx, tz, p, m, &cand, &maxb);
        }
        if (rc != XO_OK) break;
        /* E_l as a set of unordered pairs */
        qsort(cand.v, cand.n, sizeof(int64_t), cmp_i64);
        size_t u = 0;
        for (size_t q = 0; q < cand.n; q++)
            if (q == 0 || cand.v[q] != cand.v[q - 1]) cand.v[u++] = cand.v[q];
        cand.n = u;
        reps[li].candidates = (int64_t)u;
        reps[li].max_bucket = maxb;
        reps[li].fresh = 0;
        reps[li].pad = 0;
        /* strength check, eq. (1) */
        int64_t passed = 0;
        for (size_t q = 0; q < u; q++) {
            int64_t j = cand.v[q] / p, k = cand.v[q] % p;
            int64_t s = 0; double v;
            if (binary) { s = xo_pair_s(Xb, Yb, n, j, k); v = (double)s; }
            else v = xo_pair_v(Xreal, Ydw, n, j, k);
            double st = v / (double)n;
            int pass = two_sided ? (fabs(st) > kappa) : (st > kappa);
            if (!pass) continue;
            passed++;
            if (nrec == caprec) {
                size_t nc = caprec ? caprec * 2 : 1024;
                record *nr = (record *)realloc(rec, nc * sizeof(record));
                if (!nr) { rc = XO_ENOMEM; break; }
                rec = nr; caprec = nc;
            }
            rec[nrec].key = cand.v[q]; rec[nrec].rep = (int32_t)l; rec[nrec].value = v; rec[nrec].s = s;
            nrec++;
        }
        reps[li].passed = passed;
    }

    xo_pair *pairs = NULL; int64_t np_ = 0;
    if (rc == XO_OK) {
        /* I: union over repetitions */
        qsort(rec, nrec, sizeof(record), cmp_record);
        pairs = (xo_pair *)malloc(sizeof(xo_pair) * (nrec ? nrec : 1));
        if (!pairs) rc = XO_ENOMEM;
        for (size_t q = 0; rc == XO_OK && q < nrec; ) {
            size_t q1 = q;
            while (q1 < nrec && rec[q1].key == rec[q].key) q1++;
            xo_pair *o = &pairs[np_++];
            o->j = (int32_t)(rec[q].key / p); o->k = (int32_t)(rec[q].key % p);
            o->s = rec[q].s; o->value = rec[q].value; o->stat = rec[q].value / (double)n;
            o->first_rep = rec[q].rep; o->hits = (int32_t)(q1 - q);
            reps[rec[q].rep - rep_offset].fresh++;
            q = q1;
        }
    }
    free(Xs); free(Z); free(Ys); free(Ydw); free(Xdw); free(tx); free(tz); free(rows);
    free(cand.v); free(rec); free(nu); free(wrow);
    if (rc != XO_OK) { free(pairs); return rc; }
    *out_pairs = pairs; *out_npairs = np_;
    return XO_OK;
}

int xo_search(const void *Xv, int xkind, const void *Yv, int ykind, int64_t n, int64_t p,
              int m, int L, double kappa, uint64_t seed, int two_sided, int rep_offset,
              const int32_t *rows_in, xo_pair **out_pairs, int64_t *out_npairs, xo_rep *reps)
{
    return xo_search_ex(Xv, xkind, Yv, ykind, n, p, m, L, kappa, seed, two_sided, rep_offset, rows_in, 0, 0.0,
                        out_pairs, out_npairs, reps);
}

/* The plain definition T(kappa) = {j < k : Y^T(X_j o X_k)/n > kappa} (eq. (1)),
 * by enumerating every pair.  Same input conventions as xo_search. */
int xo_brute(const void *Xv, int xkind, const void *Yv, int ykind, int64_t n, int64_t p,
             double kappa, int two_sided, xo_pair **out_pairs, int64_t *out_npairs)
{
    if (n <= 0 || p <= 0 || !(kappa == kappa) || isinf(kappa)) return XO_EINVAL;
    int binary = (xkind == 0 && ykind == 0);
    const int8_t *Xb = (const int8_t *)Xv; const int8_t *Yb = (const int8_t *)Yv;
    double *Xr = NULL, *Yr = NULL;
    if (!binary) {
        Yr = (double *)malloc(sizeof(double) * (size_t)n);
        Xr = (double *)malloc(sizeof(double) * (size_t)(n * p));
        if (!Yr || !Xr) { free(Yr); free(Xr); return XO_ENOMEM; }
        for (int64_t i = 0; i < n; i++) Yr[i] = ykind == 0 ? (double)Yb[i] : ((const double *)Yv)[i];
        for (int64_t q = 0; q < n * p; q++) Xr[q] = xkind == 0 ? (double)Xb[q] : ((const double *)Xv)[q];
    }
    size_t cap = 1024, cnt = 0;
    xo_pair *out = (xo_pair *)malloc(sizeof(xo_pair) * cap);
    if (!out) { free(Yr); free(Xr); return XO_ENOMEM; }
    for (int64_t j = 0; j < p; j++)
        for (int64_t k = j + 1; k < p; k++) {
            int64_t s = 0; double v;
            if (binary) { s = xo_pair_s(Xb, Yb, n, j, k); v = (double)s; }
            else v = xo_pair_v(Xr, Yr, n, j, k);
            double st = v / (double)n;
            int pass = two_sided ? (fabs(st) > kappa) : (st > kappa);
            if (!pass) continue;
            if (cnt == cap) {
                xo_pair *no = (xo_pair *)realloc(out, sizeof(xo_pair) * cap * 2);
                if (!no) { free(out); free(Yr); free(Xr); return XO_ENOMEM; }
                out = no; cap *= 2;
            }
            xo_pair *o = &out[cnt++];
            o->j = (int32_t)j; o->k = (int32_t)k; o->s = s; o->value = v; o->stat = st;
            o->first_rep = -1; o->hits = 0;
        }
    free(Yr); free(Xr);
    *out_pairs = out; *out_npairs = (int64_t)cnt;
    return XO_OK;
}

void xo_free(void *p) { free(p); }
