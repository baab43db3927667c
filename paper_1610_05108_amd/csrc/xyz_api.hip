// xyz_api.hip -- host runtime and C ABI of libxyz (see include/xyz.h).
//
// The host side validates arguments, converts the threshold kappa of eq. (1)
// into the integer threshold used for +-1 data, owns device memory, splits
// the repetitions of Algorithm 2 into chunks that fit the workspace, and
// enqueues the kernels of xyz_kernels.hip.  Every step of the search itself
// (packing, row sampling, projection, bucket sort, candidate expansion,
// verification, merging) runs on the GPU.
#include "xyz_runtime.h"

#include <algorithm>
#include <limits>
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace xyz;
using namespace xyz_rt;

namespace {
thread_local std::string g_last_error;
}  // namespace

xyz_status xyz_rt::fail(xyz_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

namespace {

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// HIP events around the stages of one call, summed after the final sync.
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    hipStream_t st = nullptr;
    int open_stage = -1;
    hipEvent_t open_ev = nullptr;
    hipEvent_t get()
    {
        hipEvent_t e;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return nullptr;
        }
        return e;
    }
    void begin(int stage)
    {
        if (!on) return;
        open_stage = stage;
        open_ev = get();
        if (open_ev) (void)hipEventRecord(open_ev, st);
    }
    void end()
    {
        if (!on || !open_ev) return;
        hipEvent_t e = get();
        if (!e) return;
        (void)hipEventRecord(e, st);
        marks.push_back({open_stage, {open_ev, e}});
        open_ev = nullptr;
    }
    // stage ids: 0 pack, 1 sample, 2 hash, 3 bucket, 4 tiles, 5 verify, 6 dedup, 7 brute, 8 big tiles
    // (counted in verify as well)
    void collect(xyz_timing &t)
    {
        for (auto &m : marks) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, m.second.first, m.second.second);
            double *dst[9] = {&t.pack_ms, &t.sample_ms, &t.hash_ms, &t.bucket_ms,
                              &t.tiles_ms, &t.verify_ms, &t.dedup_ms, &t.brute_ms, &t.big_ms};
            if (m.first >= 0 && m.first < 9) *dst[m.first] += ms;
            if (m.first == 8) t.verify_ms += ms;
            pool.push_back(m.second.first);
            pool.push_back(m.second.second);
        }
        marks.clear();
    }
    ~Timer()
    {
        for (auto &m : marks) {
            (void)hipEventDestroy(m.second.first);
            (void)hipEventDestroy(m.second.second);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace

namespace {

xyz_status dev_alloc(xyz_ctx *c, size_t bytes, void **out)
{
    bytes = (size_t)round_up((int64_t)std::max<size_t>(bytes, 256), 256);
    if (c->budget && c->used + bytes > c->budget)
        return fail(XYZ_ENOMEM, "device memory budget exceeded: %llu in use + %zu requested > %llu",
                    (unsigned long long)c->used, bytes, (unsigned long long)c->budget);
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) return fail(XYZ_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    c->used += bytes;
    return XYZ_OK;
}

void dev_free(xyz_ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    bytes = (size_t)round_up((int64_t)std::max<size_t>(bytes, 256), 256);
    c->used -= std::min<uint64_t>(c->used, bytes);
}

// Arena mode: carve the slot from the context's arena (bump pointer, 256-byte aligned); a slot
// that is the last carved region grows in place.  Nothing is allocated or freed.
xyz_status arena_get(xyz_ctx *c, DevBuf &b, size_t bytes, void **out)
{
    const size_t want = (size_t)round_up((int64_t)std::max<size_t>(bytes, 256), 256);
    const bool top = b.p && (char *)b.p + b.bytes == c->arena + c->arena_used;
    const size_t start = top ? (size_t)((char *)b.p - c->arena) : c->arena_used;
    if (start + want > c->arena_size)
        return fail(XYZ_ENOMEM, "the search needs more than the %zu bytes of static scratch (%zu in use, %zu more "
                    "requested)", c->arena_size, c->arena_used, want);
    b.p = c->arena + start;
    b.bytes = want;
    c->arena_used = start + want;
    *out = b.p;
    return XYZ_OK;
}

// Grow-only workspace slot.
xyz_status ws_get(xyz_ctx *c, int slot, size_t bytes, void **out)
{
    DevBuf &b = c->ws[slot];
    if (b.p && b.bytes >= bytes) {
        *out = b.p;
        return XYZ_OK;
    }
    if (c->arena) return arena_get(c, b, bytes, out);
    size_t want = std::max(bytes, b.bytes + b.bytes / 4);
    want = (size_t)round_up((int64_t)std::max<size_t>(want, 256), 256);
    dev_free(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
    void *p = nullptr;
    xyz_status s = dev_alloc(c, want, &p);
    if (s != XYZ_OK && want > bytes) s = dev_alloc(c, bytes, &p), want = bytes;
    if (s != XYZ_OK) return s;
    b.p = p;
    b.bytes = (size_t)round_up((int64_t)std::max<size_t>(want, 256), 256);
    *out = p;
    return XYZ_OK;
}

template <class T>
xyz_status ws(xyz_ctx *c, int slot, size_t count, T **out)
{
    void *p = nullptr;
    XYZ_TRY(ws_get(c, slot, std::max<size_t>(count, 1) * sizeof(T), &p));
    *out = static_cast<T *>(p);
    return XYZ_OK;
}

xyz_status err_flag_status(int h)
{
    if (h & 1) return fail(XYZ_EINVAL, "X holds a value other than -1 or +1");
    if (h & 2) return fail(XYZ_EINVAL, "X holds NaN or Inf");
    if (h & 4) return fail(XYZ_EINVAL, "Y holds an invalid value (not +-1 for the +-1 format, or NaN/Inf)");
    if (h & 8) return fail(XYZ_EINVAL, "Y is zero everywhere: the |Y|-weighted sampler has no row to draw");
    return XYZ_OK;
}

xyz_status check_err_flag(int *d_err, hipStream_t st, xyz_ctx *c = nullptr)
{
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (c) ++c->syncs;
    return err_flag_status(h);
}

// A host wait on the stream within a search (counted in xyz_timing.host_syncs).
xyz_status host_wait(xyz_ctx *c, hipStream_t st)
{
    ++c->syncs;
    HIP_TRY(hipStreamSynchronize(st));
    return XYZ_OK;
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ------------------------------------------------------------------ ABI --

extern "C" const char *xyz_version(void) { return "libxyz 0.1 (gfx950)"; }

extern "C" const char *xyz_last_error(void) { return g_last_error.c_str(); }

extern "C" int64_t xyz_smin(int64_t n, double kappa, int two_sided)
{
    if (n <= 0) return 1;
    const double dn = (double)n;
    int64_t lo = two_sided ? 0 : -n, hi = n;
    if (!((double)hi / dn > kappa)) return n + 1;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((double)mid / dn > kappa) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

extern "C" xyz_status xyz_init(int device, uint64_t hbm_budget_bytes, xyz_ctx **out)
{
    if (!out) return fail(XYZ_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(XYZ_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(XYZ_EUNSUPPORTED, "libxyz is built for gfx950; device %d is %s", device, prop.gcnArchName);
    HIP_TRY(kernels_init());
    XYZ_TRY(scratch_setup(device));
    xyz_ctx *c = new xyz_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->cu_count = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    *out = c;
    return XYZ_OK;
}

extern "C" void xyz_fini(xyz_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    for (auto &b : c->ws) dev_free(c, b.p, b.bytes);
    delete c;
}

extern "C" uint64_t xyz_ctx_bytes(const xyz_ctx *c) { return c ? c->used : 0; }

extern "C" xyz_status xyz_x_create(xyz_ctx *c, const void *X, int fmt, int mem, int64_t n, int64_t p, int64_t ld,
                                   void *stream, xyz_x **out)
{
    if (!c || !out || !X) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (n < 1 || n >= (1ll << 31) || p < 1 || p >= (1ll << 31))
        return fail(XYZ_EINVAL, "shape n=%lld p=%lld out of range", (long long)n, (long long)p);
    if (fmt != XYZ_X_I8_PM1 && fmt != XYZ_X_BITS && fmt != XYZ_X_F32 && fmt != XYZ_X_I8_PM1_ROWMAJOR)
        return fail(XYZ_EINVAL, "unknown X format %d", fmt);
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    const bool rowmajor = fmt == XYZ_X_I8_PM1_ROWMAJOR;
    const int64_t minld = fmt == XYZ_X_BITS ? (n + 63) / 64 : (rowmajor ? p : n);
    if (ld < minld) return fail(XYZ_EINVAL, "ld=%lld < %lld", (long long)ld, (long long)minld);
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    xyz_x *x = new xyz_x();
    x->ctx = c;
    x->n = n;
    x->p = p;
    x->fmt = fmt;
    x->W32p = (int)round_up((n + 31) / 32, 4);
    x->P64 = (p + 63) / 64;
    x->nF = round_up(n, 32);
    auto cleanup = [&](xyz_status s) {
        xyz_x_destroy(x);
        return s;
    };
    const size_t xc_bytes = (size_t)p * x->W32p * 4, xr_bytes = (size_t)n * x->P64 * 8;
    void *pc = nullptr, *pr = nullptr, *pf = nullptr;
    xyz_status s = dev_alloc(c, xc_bytes, &pc);
    if (s != XYZ_OK) return cleanup(s);
    x->XC = (uint32_t *)pc;
    x->bytes += xc_bytes;
    s = dev_alloc(c, xr_bytes, &pr);
    if (s != XYZ_OK) return cleanup(s);
    x->XR = (uint64_t *)pr;
    x->bytes += xr_bytes;
    if (fmt == XYZ_X_F32) {
        const size_t xf_bytes = (size_t)p * x->nF * 4;
        s = dev_alloc(c, xf_bytes, &pf);
        if (s != XYZ_OK) return cleanup(s);
        x->XF = (float *)pf;
        x->bytes += xf_bytes;
    }
    // source on the device
    const size_t esz = fmt == XYZ_X_BITS ? 8 : (fmt == XYZ_X_F32 ? 4 : 1);
    const size_t src_bytes = ((size_t)((rowmajor ? n : p) - 1) * ld + minld) * esz;
    const void *src = X;
    if (mem == XYZ_MEM_HOST) {
        void *tmp = nullptr;
        s = ws_get(c, WS_XIN, src_bytes, &tmp);
        if (s != XYZ_OK) return cleanup(s);
        if (hipMemcpyAsync(tmp, X, src_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return cleanup(fail(XYZ_EDEVICE, "copying X to the device failed"));
        src = tmp;
    }
    int *err = nullptr;
    s = ws(c, WS_ERR, 4, &err);
    if (s != XYZ_OK) return cleanup(s);
    if (launch_zero(err, sizeof(int), st) != hipSuccess) return cleanup(fail(XYZ_EDEVICE, "zeroing the error flag failed"));
    hipError_t e;
    if (rowmajor) {
        // row-major input packs straight into the row layout; the column layout is its transpose
        e = launch_pack_x_i8_rows((const int8_t *)src, ld, n, p, x->XR, x->P64, err, st);
        if (e == hipSuccess) e = launch_transpose_rc(x->XR, n, p, x->P64, x->W32p, x->XC, st);
    } else {
        if (fmt == XYZ_X_I8_PM1) e = launch_pack_x_i8((const int8_t *)src, ld, n, p, x->W32p, x->XC, err, st);
        else if (fmt == XYZ_X_F32) e = launch_pack_x_f32((const float *)src, ld, n, p, x->W32p, x->XC, x->XF, x->nF, err, st);
        else e = launch_pack_x_bits((const uint64_t *)src, ld, n, p, x->W32p, x->XC, st);
        if (e == hipSuccess) e = launch_transpose(x->XC, n, p, x->W32p, x->XR, x->P64, st);
    }
    if (e != hipSuccess) return cleanup(fail(XYZ_EDEVICE, "packing X failed: %s", hipGetErrorString(e)));
    s = check_err_flag(err, st);
    if (s != XYZ_OK) return cleanup(s);
    *out = x;
    return XYZ_OK;
}

extern "C" void xyz_x_destroy(xyz_x *x)
{
    if (!x) return;
    xyz_ctx *c = x->ctx;
    (void)hipSetDevice(c->device);
    dev_free(c, x->XC, (size_t)x->p * x->W32p * 4);
    dev_free(c, x->XR, (size_t)x->n * x->P64 * 8);
    if (x->XF) dev_free(c, x->XF, (size_t)x->p * x->nF * 4);
    delete x;
}

extern "C" int64_t xyz_x_n(const xyz_x *x) { return x ? x->n : 0; }
extern "C" int64_t xyz_x_p(const xyz_x *x) { return x ? x->p : 0; }

int64_t xyz_rt::chunk_reps(const xyz_ctx *c, int64_t L, int64_t p, int m, int64_t chunk_bytes)
{
    int64_t chunk = std::min<int64_t>(L, 4096);
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, ((1ll << 32) - 1) / p));   // u32 positions in perm
    // bytes per repetition: keys and permutation, plus the LDS path's bucket offsets or the sort
    // path's scratch (two key/value buffers, heads, runs and per-run tile counts)
    const int64_t per_rep = m <= MAX_M_LDS ? 8 * p + 4 * ((1ll << m) + 1)
                                           : 64 * p + (m <= SK_TABLE_MAX_M ? 4 * (1ll << m) : 0);
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, chunk_bytes / per_rep));   // default 8 GiB of 288
    chunk = std::min<int64_t>(chunk, 65535);                                           // grid y of k_hash
    if (c->max_chunk > 0) chunk = std::min<int64_t>(chunk, c->max_chunk);
    return std::max<int64_t>(chunk, 1);
}

void xyz_rt::ws_release(xyz_ctx *c)
{
    for (auto &b : c->ws) {
        dev_free(c, b.p, b.bytes);
        b.p = nullptr;
        b.bytes = 0;
    }
}

xyz_status xyz_rt::validate_params(const xyz_x *x, const xyz_params *P, int yfmt)
{
    if (!P) return fail(XYZ_EINVAL, "params is NULL");
    if (P->m < 0 || P->m > XYZ_MAX_M) return fail(XYZ_EINVAL, "m=%d out of range [0, %d]", P->m, XYZ_MAX_M);
    if (P->L < 1) return fail(XYZ_EINVAL, "L=%d < 1", P->L);
    if (!std::isfinite(P->kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
    if (P->rep_offset < 0) return fail(XYZ_EINVAL, "rep_offset < 0");
    if ((int64_t)P->rep_offset + P->L > (1ll << 31)) return fail(XYZ_EINVAL, "repetition index overflow");
    if (P->flags & ~(uint32_t)(XYZ_TWO_SIDED | XYZ_PROFILE | XYZ_UNBIASED))
        return fail(XYZ_EINVAL, "unknown flags 0x%x", P->flags);
    if ((P->flags & XYZ_UNBIASED) && x->fmt != XYZ_X_F32)
        return fail(XYZ_EUNSUPPORTED, "the unbiased transform needs float32 X");
    if (P->cap != 0.0) {
        if (!(P->flags & XYZ_UNBIASED)) return fail(XYZ_EINVAL, "cap applies to the unbiased transform only");
        if (!(P->cap > 0.0) || !((float)P->cap > 0.0f))
            return fail(XYZ_EINVAL, "cap=%g: must be positive and at least the smallest positive float32", P->cap);
    }
    if (yfmt != XYZ_Y_I8_PM1 && yfmt != XYZ_Y_F32 && yfmt != XYZ_Y_F64) return fail(XYZ_EINVAL, "unknown Y format %d", yfmt);
    if (P->rows) {
        const int64_t cnt = (int64_t)P->L * P->m;
        for (int64_t q = 0; q < cnt; ++q)
            if (P->rows[q] < 0 || P->rows[q] >= x->n)
                return fail(XYZ_EINVAL, "rows[%lld]=%d out of range [0, %lld)", (long long)q, P->rows[q], (long long)x->n);
    }
    return XYZ_OK;
}

namespace {

size_t y_bytes(int yfmt, int64_t n) { return (size_t)n * (yfmt == XYZ_Y_I8_PM1 ? 1 : (yfmt == XYZ_Y_F32 ? 4 : 8)); }

// Pack nys responses into yb [nys][W32p] bits and yd [nys][nF] values; err is
// the device error flag (zeroed here, checked by the caller).
xyz_status pack_ys(xyz_ctx *c, const xyz_x *x, int nys, const void *const *Ys, int yfmt, int mem, hipStream_t st,
                   uint32_t **yb_out, double **yd_out, int **err_out)
{
    uint32_t *yb = nullptr;
    double *yd = nullptr;
    int *err = nullptr;
    XYZ_TRY(ws(c, WS_YB, (size_t)nys * x->W32p, &yb));
    XYZ_TRY(ws(c, WS_YD, (size_t)nys * x->nF, &yd));
    XYZ_TRY(ws(c, WS_ERR, 1, &err));
    HIP_TRY(launch_zero(err, sizeof(int), st));
    for (int y = 0; y < nys; ++y) {
        const void *src = Ys[y];
        if (mem == XYZ_MEM_HOST) {
            void *tmp = nullptr;
            XYZ_TRY(ws_get(c, WS_YIN, y_bytes(yfmt, x->n), &tmp));
            HIP_TRY(hipMemcpyAsync(tmp, Ys[y], y_bytes(yfmt, x->n), hipMemcpyHostToDevice, st));
            src = tmp;
        }
        HIP_TRY(launch_pack_y(src, yfmt, x->n, x->W32p, yb + (size_t)y * x->W32p, yd + (size_t)y * x->nF, x->nF,
                              err, st));
    }
    *yb_out = yb;
    *yd_out = yd;
    *err_out = err;
    return XYZ_OK;
}

xyz_status merge_results(xyz_ctx *c, const xyz_x *x, int nys, int L, int rep_offset, const Survivor *surv,
                         uint64_t S, RepInfo *info, Timer &tm, xyz_timing &timing, double t0, hipStream_t st,
                         xyz_result **outs, const DirectOut *direct = nullptr);

// The survivor buffer overflowed (cnt records for capacity *cap): grow it, keep the first
// `done` records (earlier chunks), and reset the device count to `done` so that the chunk
// can be run again.
xyz_status grow_survivors(xyz_ctx *c, unsigned long long cnt, uint64_t done, unsigned long long *scnt,
                          Survivor **surv, uint64_t *cap, hipStream_t st)
{
    const uint64_t ncap = std::max<uint64_t>(cnt + cnt / 2, *cap * 2);
    Survivor *tmp = nullptr;
    XYZ_TRY(ws(c, WS_SURV2, done, &tmp));
    if (done) HIP_TRY(hipMemcpyAsync(tmp, *surv, done * sizeof(Survivor), hipMemcpyDeviceToDevice, st));
    XYZ_TRY(host_wait(c, st));
    XYZ_TRY(ws(c, WS_SURV, ncap, surv));
    if (done) HIP_TRY(hipMemcpyAsync(*surv, tmp, done * sizeof(Survivor), hipMemcpyDeviceToDevice, st));
    *cap = ncap;
    const unsigned long long keep = done;
    HIP_TRY(hipMemcpyAsync(scnt, &keep, sizeof keep, hipMemcpyHostToDevice, st));
    XYZ_TRY(host_wait(c, st));
    return XYZ_OK;
}

// One group of searches sharing X, m, L, seed, rep_offset and flags.  With
// nys > 1 every Y must be +-1 and no row table may be given, so the row draws,
// projections and bucket sort are shared (Z = Y o X changes only the partner mask).
}  // namespace

xyz_status xyz_rt::run_group(xyz_ctx *c, const xyz_x *x, int nys, const void *const *Ys, int yfmt, int mem,
                             const xyz_params *const *Ps, hipStream_t st, xyz_result **outs, const DirectOut *direct)
{
    if (nys < 1 || nys > 255 || (direct && nys != 1)) return fail(XYZ_EINVAL, "group of %d searches", nys);
    const double t0 = now_ms();
    c->syncs = 0;
    const xyz_params &P = *Ps[0];
    const int64_t n = x->n, p = x->p;
    const int m = P.m, L = P.L;
    const int two = (P.flags & XYZ_TWO_SIDED) ? 1 : 0;
    const bool real_y = yfmt != XYZ_Y_I8_PM1;
    const bool real_x = x->fmt == XYZ_X_F32;
    const bool real = real_x || real_y;
    const bool unbiased = (P.flags & XYZ_UNBIASED) != 0 && real_x;
    // Section 3.2's capping of the unbiased transform, in float32 like X (+inf: none)
    const float cap_f = P.cap > 0.0 ? (float)P.cap : std::numeric_limits<float>::infinity();
    // large bucket products go to the matrix cores in 64 x 64 tiles: FP4 with exact FP32
    // counts for +-1 data (n < 2^24, mfma = 1), FP64 for real data (mfma = 2)
    const int mfma = real ? 2 : (n < (1 << 24) ? 1 : 0);
    Timer tm;
    tm.on = (P.flags & XYZ_PROFILE) != 0;
    tm.st = st;
    xyz_timing timing{};

    // ---- Y
    uint32_t *yb = nullptr;
    double *yd = nullptr;
    int *err = nullptr;
    tm.begin(0);
    XYZ_TRY(pack_ys(c, x, nys, Ys, yfmt, mem, st, &yb, &yd, &err));
    double *cdf = nullptr;
    int64_t *last = nullptr;
    uint32_t *nu = nullptr;
    if (unbiased && m > 0) {
        // Section 3.2: rows scaled by their largest absolute entry, weights |Y_i| nu_i^2
        XYZ_TRY(ws(c, WS_NU, (size_t)n, &nu));
        XYZ_TRY(ws(c, WS_CDF, (size_t)n, &cdf));
        XYZ_TRY(ws(c, WS_LAST, 1, &last));
        HIP_TRY(launch_row_absmax(x->XF, x->nF, n, p, cap_f, nu, st));
        HIP_TRY(launch_cdf_unbiased(yd, nu, n, cdf, last, err, st));
    } else if (real_y && m > 0) {
        XYZ_TRY(ws(c, WS_CDF, (size_t)n, &cdf));
        XYZ_TRY(ws(c, WS_LAST, 1, &last));
        HIP_TRY(launch_cdf(yd, n, cdf, last, err, st));
    }
    tm.end();
    // thresholds (fixed arrays: this path allocates no host memory either)
    int64_t hsmin[255];
    double hkap[255];
    for (int y = 0; y < nys; ++y) {
        hkap[y] = Ps[y]->kappa;
        hsmin[y] = xyz_smin(n, Ps[y]->kappa, two);
    }
    int64_t *dsmin = nullptr;
    double *dkap = nullptr;
    XYZ_TRY(ws(c, WS_SMIN, nys, &dsmin));
    XYZ_TRY(ws(c, WS_KAPPA, nys, &dkap));
    HIP_TRY(hipMemcpyAsync(dsmin, hsmin, sizeof(int64_t) * nys, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dkap, hkap, sizeof(double) * nys, hipMemcpyHostToDevice, st));
    XYZ_TRY(check_err_flag(err, st, c));

    // column popcounts for the big tiles (+-1 data on the matrix cores)
    uint32_t *cpop = nullptr;
    if (mfma == 1) {
        XYZ_TRY(ws(c, WS_CPOP, (size_t)(nys + 1) * p, &cpop));
        HIP_TRY(launch_col_pops(x->XC, x->W32p, yb, nys, p, cpop, st));
    }

    // ---- repetitions, in chunks
    const int nb = 1 << m;
    const Knobs kn = knobs_for(c, x, m, yfmt, P.flags);
    const int64_t chunk = chunk_reps(c, L, p, m, kn.chunk_bytes);
    RepInfo *info = nullptr;
    XYZ_TRY(ws(c, WS_INFO, (size_t)L * nys, &info));
    int32_t *rows = nullptr;
    uint32_t *keys = nullptr, *offs = nullptr, *perm = nullptr;
    unsigned long long *base = nullptr, *scnt = nullptr;
    XYZ_TRY(ws(c, WS_ROWS, (size_t)chunk * std::max(m, 1), &rows));
    XYZ_TRY(ws(c, WS_KEYS, (size_t)chunk * p, &keys));
    if (m <= MAX_M_LDS) XYZ_TRY(ws(c, WS_OFFS, (size_t)chunk * (nb + 1), &offs));
    XYZ_TRY(ws(c, WS_PERM, (size_t)chunk * p, &perm));
    XYZ_TRY(ws(c, WS_BASE, NLISTS * ((size_t)chunk * nys + 1), &base));
    // scnt[0]: survivors so far; scnt[1..4]: the chunk's four tile-list sizes (m <= MAX_M_LDS),
    // read back with the survivor count in one transfer per chunk
    XYZ_TRY(ws(c, WS_SCNT, 1 + NLISTS, &scnt));
    HIP_TRY(launch_zero(scnt, sizeof(unsigned long long), st));
    uint64_t surv_cap = std::max<uint64_t>(c->ws[WS_SURV].bytes / sizeof(Survivor), 1 << 16);
    Survivor *surv = nullptr;
    XYZ_TRY(ws(c, WS_SURV, surv_cap, &surv));
    uint64_t surv_done = 0;
    const int grid = std::max(1, c->cu_count * kn.verify_per_cu);
    const int big_grid = std::max(1, c->cu_count * kn.big_per_cu);

    for (int64_t r0 = 0; r0 < L; r0 += chunk) {
        const int R = (int)std::min<int64_t>(chunk, L - r0);
        timing.chunks += 1;
        const int64_t rep_abs0 = (int64_t)P.rep_offset + r0;
        RepInfo *cinfo = info + (size_t)r0 * nys;
        tm.begin(1);
        if (m > 0) {
            if (P.rows) {
                HIP_TRY(hipMemcpyAsync(rows, P.rows + (size_t)r0 * m, sizeof(int32_t) * R * m, hipMemcpyHostToDevice, st));
            } else {
                HIP_TRY(launch_sample(P.seed, rep_abs0, R, m, n, (real_y || unbiased) ? 1 : 0, cdf, last, rows, st));
            }
        }
        HIP_TRY(launch_cmask(rows, R, m, nys, yb, x->W32p, cinfo, st));
        tm.end();
        tm.begin(2);
        if (unbiased && m > 0)
            HIP_TRY(launch_hash_unbiased(x->XF, x->nF, p, m, R, rows, nu, cap_f, P.seed, rep_abs0, keys, st));
        else
            HIP_TRY(launch_hash(x->XR, x->P64, p, m, R, rows, keys, st));
        tm.end();
        bool redo = true;
        while (redo) {
            redo = false;
            unsigned long long ntiles = 0, nsmall = 0, nmfma = 0, nbig = 0;
            Tile *tiles = nullptr;
            // m <= MAX_M_LDS: the list sizes stay on the device; the tile list has the capacity
            // it has (grown when a chunk overflows it) and the verification kernels read the sizes
            const bool device_counts = m <= MAX_M_LDS;
            uint64_t tile_cap = 0;
            if (device_counts) {
                tm.begin(3);
                HIP_TRY(launch_bucket(keys, p, m, R, nys, cinfo, two, mfma, offs, perm, st));
                tm.end();
                tm.begin(4);
                HIP_TRY(launch_tile_scan(cinfo, R * nys, base, scnt + 1, st));
                tile_cap = std::max<uint64_t>(c->ws[WS_TILES].bytes / sizeof(Tile), 1 << 16);
                XYZ_TRY(ws(c, WS_TILES, (size_t)tile_cap, &tiles));
                HIP_TRY(launch_tiles(offs, p, m, R, nys, cinfo, two, mfma, base, tiles, tile_cap, st));
                tm.end();
                // launch bounds only (matrix-core tiles need mfma, big tiles +-1 data)
                ntiles = nsmall = tile_cap;
                nmfma = mfma ? tile_cap : 0;
                nbig = mfma == 1 ? tile_cap : 0;
            } else {
                // m > MAX_M_LDS: sort the keys, take runs of equal keys as buckets
                const uint64_t S = (uint64_t)R * (uint64_t)p;
                uint64_t *K = nullptr, *K2 = nullptr, *Ks = nullptr, *rkey = nullptr;
                uint32_t *V = nullptr, *V2 = nullptr, *hist = nullptr, *heads = nullptr, *rstart = nullptr;
                uint32_t *dnr = nullptr, *cnt = nullptr;
                XYZ_TRY(ws(c, WS_SKK, S, &K));
                XYZ_TRY(ws(c, WS_SKK2, S, &K2));
                XYZ_TRY(ws(c, WS_SKV, S, &V));
                XYZ_TRY(ws(c, WS_SKV2, S, &V2));
                XYZ_TRY(ws(c, WS_SKHIST, radix_hist_entries(S), &hist));
                XYZ_TRY(ws(c, WS_SKHEADS, S, &heads));
                XYZ_TRY(ws(c, WS_SKRK, S, &rkey));
                XYZ_TRY(ws(c, WS_SKRS, S, &rstart));
                XYZ_TRY(ws(c, WS_SKN, 1, &dnr));
                tm.begin(3);
                HIP_TRY(launch_sk_sort(keys, p, m, R, K, V, K2, V2, hist, perm, &Ks, st));
                HIP_TRY(launch_sk_runs(Ks, S, heads, hist, rkey, rstart, dnr, st));
                uint32_t nr = 0;
                HIP_TRY(hipMemcpyAsync(&nr, dnr, sizeof nr, hipMemcpyDeviceToHost, st));
                XYZ_TRY(host_wait(c, st));
                uint32_t *table = nullptr;
                if (m <= SK_TABLE_MAX_M) {
                    XYZ_TRY(ws(c, WS_SKTAB, (size_t)R << m, &table));
                    HIP_TRY(launch_sk_table(rkey, dnr, nr, (uint64_t)R << m, table, st));
                }
                const uint64_t ncnt = (uint64_t)NLISTS * nys * nr;
                XYZ_TRY(ws(c, WS_SKCNT, ncnt + 1, &cnt));
                HIP_TRY(launch_zero(cnt + ncnt, sizeof(uint32_t), st));
                HIP_TRY(launch_sk_products(rkey, rstart, dnr, nr, S, m, nys, cinfo, R * nys, two, mfma, table, cnt,
                                           st));
                tm.end();
                tm.begin(4);
                // positions of every (list, response, run) in the tile array; list starts and total
                XYZ_TRY(ws(c, WS_SKHIST, std::max<size_t>(radix_hist_entries(S), (size_t)((ncnt + 1) / 2048 + 16)), &hist));
                HIP_TRY(launch_scan_u32(cnt, ncnt + 1, hist, st));
                uint32_t bnd[4] = {0, 0, 0, 0};
                const uint64_t stride = (uint64_t)nys * nr;
                HIP_TRY(hipMemcpyAsync(&bnd[0], cnt + stride, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&bnd[1], cnt + 2 * stride, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&bnd[2], cnt + 3 * stride, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(&bnd[3], cnt + ncnt, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
                XYZ_TRY(host_wait(c, st));
                ntiles = bnd[0];
                nsmall = bnd[1] - bnd[0];
                nmfma = bnd[2] - bnd[1];
                nbig = bnd[3] - bnd[2];
                XYZ_TRY(ws(c, WS_TILES, (size_t)(ntiles + nsmall + nmfma + nbig), &tiles));
                HIP_TRY(launch_sk_tiles(rkey, rstart, dnr, nr, S, p, m, nys, cinfo, two, mfma, table, cnt, tiles, st));
                tm.end();
            }
            VerifyArgs va{};
            va.tiles = tiles;
            va.ntiles = ntiles;
            va.nsmall = nsmall;
            va.nmfma = nmfma;
            va.nbig = nbig;
            va.perm = perm;
            va.XC = x->XC;
            va.W32p = x->W32p;
            va.XF = x->XF;
            va.nF = x->nF;
            va.yb = yb;
            va.cpop = cpop;
            va.p = p;
            va.yd = yd;
            va.n = n;
            va.smin = dsmin;
            va.kappa = dkap;
            va.two_sided = two;
            va.nys = nys;
            va.rep_abs0 = rep_abs0;
            va.surv = surv;
            va.surv_count = scnt;
            va.surv_cap = surv_cap;
            va.info = cinfo;
            if (device_counts) {
                va.dcnt = scnt + 1;
                va.tile_cap = tile_cap;
            }
            const int g = (int)std::min<unsigned long long>(std::max(ntiles + nsmall + nmfma + nbig, 1ull),
                                                            (unsigned long long)grid);
            tm.begin(5);
            if (real) HIP_TRY(launch_verify_real(va, real_x ? 1 : 0, g, st));
            else HIP_TRY(launch_verify_bin(va, g, st));
            tm.end();
            if (nbig) {
                tm.begin(8);
                HIP_TRY(launch_verify_big(va, big_grid, st));
                tm.end();
            }
            // the one transfer of the chunk: the survivor count and (device_counts) the list sizes
            unsigned long long hc[1 + NLISTS] = {0, ntiles, nsmall, nmfma, nbig};
            HIP_TRY(hipMemcpyAsync(hc, scnt, sizeof(unsigned long long) * (device_counts ? 1 + NLISTS : 1),
                                   hipMemcpyDeviceToHost, st));
            XYZ_TRY(host_wait(c, st));
            const unsigned long long cnt = hc[0];
            ntiles = hc[1], nsmall = hc[2], nmfma = hc[3], nbig = hc[4];
            const uint64_t need = ntiles + nsmall + nmfma + nbig;
            if (device_counts && need > tile_cap) {
                // nothing was verified: grow the list and redo the chunk
                XYZ_TRY(ws(c, WS_TILES, (size_t)need, &tiles));
                redo = true;
                continue;
            }
            if (nbig) timing.big_launches += 1;
            timing.verify_launches += (ntiles ? 1 : 0) + (nsmall && !real ? 1 : 0) + (nmfma ? 1 : 0) + (nbig ? 1 : 0);
            timing.tiles += (int64_t)need;
            if (cnt > surv_cap) {
                XYZ_TRY(grow_survivors(c, cnt, surv_done, scnt, &surv, &surv_cap, st));
                redo = true;
            } else {
                surv_done = cnt;
            }
        }
    }

    // ---- merge repetitions
    const xyz_status ms = merge_results(c, x, nys, L, P.rep_offset, surv, surv_done, info, tm, timing, t0, st, outs,
                                        direct);
    if (ms == XYZ_OK && !direct)
        for (int y = 0; y < nys; ++y) {
            outs[y]->route.method = XYZ_PLAN_XYZ;
            outs[y]->route.m = m;
            outs[y]->route.L = L;
            outs[y]->route.seed = Ps[y]->seed;
        }
    return ms;
}

namespace {

// One search's result into caller-owned host buffers (xyz_search_noalloc): the pairs, if they
// fit, and the statistics of every repetition, converted through a small stack buffer.
xyz_status copy_direct(xyz_ctx *c, const unsigned long long *nout, const OutPair *dout, const RepInfo *info,
                       int L, hipStream_t st, const DirectOut &d)
{
    unsigned long long U = 0;
    HIP_TRY(hipMemcpyAsync(&U, nout, sizeof U, hipMemcpyDeviceToHost, st));
    XYZ_TRY(host_wait(c, st));
    *d.npairs = (int64_t)U;
    if ((int64_t)U > d.cap)
        return fail(XYZ_ENOMEM, "the search found %llu pairs; the pair buffer holds %lld", U, (long long)d.cap);
    static_assert(sizeof(OutPair) == sizeof(xyz_pair), "OutPair is the layout of xyz_pair");
    if (U) HIP_TRY(hipMemcpyAsync(d.pairs, dout, sizeof(xyz_pair) * U, hipMemcpyDeviceToHost, st));
    RepInfo buf[64];
    for (int l0 = 0; l0 < L; l0 += 64) {
        const int cnt = std::min(64, L - l0);
        HIP_TRY(hipMemcpyAsync(buf, info + l0, sizeof(RepInfo) * cnt, hipMemcpyDeviceToHost, st));
        XYZ_TRY(host_wait(c, st));
        for (int i = 0; i < cnt; ++i) {
            xyz_rep_stats &o = d.reps[l0 + i];
            o.candidates = (int64_t)buf[i].candidates;
            o.passed = (int64_t)buf[i].passed;
            o.fresh = (int64_t)buf[i].fresh;
            o.cmask = buf[i].cmask;
            o.max_bucket = (int32_t)buf[i].max_bucket;
            o.reserved = 0;
        }
    }
    XYZ_TRY(host_wait(c, st));
    return XYZ_OK;
}

// Merge the S survivors of a finished search into one result per response: unique pairs
// sorted by (j, k) with their first repetition and hits (Algorithm 2, "add to I"), and the
// per-repetition statistics of info [L][nys].
xyz_status merge_results(xyz_ctx *c, const xyz_x *x, int nys, int L, int rep_offset, const Survivor *surv,
                         uint64_t S, RepInfo *info, Timer &tm, xyz_timing &timing, double t0, hipStream_t st,
                         xyz_result **outs, const DirectOut *direct)
{
    const int64_t n = x->n, p = x->p;
    uint64_t *dk = nullptr, *dk2 = nullptr;
    uint32_t *dv = nullptr, *dv2 = nullptr, *hist = nullptr, *heads = nullptr;
    OutPair *dout = nullptr;
    unsigned long long *nout = nullptr, *ycnt = nullptr;
    XYZ_TRY(ws(c, WS_DKEYS, S, &dk));
    XYZ_TRY(ws(c, WS_DKEYS2, S, &dk2));
    XYZ_TRY(ws(c, WS_DVALS, S, &dv));
    XYZ_TRY(ws(c, WS_DVALS2, S, &dv2));
    XYZ_TRY(ws(c, WS_HIST, radix_hist_entries(S), &hist));
    XYZ_TRY(ws(c, WS_HEADS, S + 1, &heads));
    XYZ_TRY(ws(c, WS_OUT, S, &dout));
    XYZ_TRY(ws(c, WS_NOUT, 1, &nout));
    XYZ_TRY(ws(c, WS_YCNT, nys, &ycnt));
    HIP_TRY(launch_zero(ycnt, sizeof(unsigned long long) * nys, st));
    tm.begin(6);
    HIP_TRY(launch_dedup(surv, S, p, n, nys, dk, dv, dk2, dv2, hist, heads, dout, nout, ycnt, info,
                         (int64_t)rep_offset, st));
    tm.end();
    if (direct) return copy_direct(c, nout, dout, info, L, st, *direct);
    unsigned long long U = 0;
    std::vector<unsigned long long> hy(nys);
    HIP_TRY(hipMemcpyAsync(&U, nout, sizeof U, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hy.data(), ycnt, sizeof(unsigned long long) * nys, hipMemcpyDeviceToHost, st));
    std::vector<RepInfo> hinfo((size_t)L * nys);
    HIP_TRY(hipMemcpyAsync(hinfo.data(), info, sizeof(RepInfo) * hinfo.size(), hipMemcpyDeviceToHost, st));
    XYZ_TRY(host_wait(c, st));
    std::vector<xyz_pair> all(U);
    if (U) HIP_TRY(hipMemcpyAsync(all.data(), dout, sizeof(xyz_pair) * U, hipMemcpyDeviceToHost, st));
    XYZ_TRY(host_wait(c, st));
    tm.collect(timing);
    int64_t cand_total = 0, big_total = 0;
    for (auto &ri : hinfo) {
        cand_total += (int64_t)ri.candidates;
        big_total += (int64_t)ri.big_pairs;
    }
    timing.candidates = cand_total;
    timing.big_candidates = big_total;
    timing.total_ms = now_ms() - t0;
    timing.host_syncs = c->syncs;

    size_t off = 0;
    for (int y = 0; y < nys; ++y) {
        xyz_result *r = new xyz_result();
        r->pairs.assign(all.begin() + off, all.begin() + off + hy[y]);
        off += hy[y];
        r->reps.resize(L);
        for (int l = 0; l < L; ++l) {
            const RepInfo &ri = hinfo[(size_t)l * nys + y];
            xyz_rep_stats &o = r->reps[l];
            o.candidates = (int64_t)ri.candidates;
            o.passed = (int64_t)ri.passed;
            o.fresh = (int64_t)ri.fresh;
            o.cmask = ri.cmask;
            o.max_bucket = (int32_t)ri.max_bucket;
            o.reserved = 0;
        }
        r->timing = timing;
        outs[y] = r;
    }
    return XYZ_OK;
}

}  // namespace

extern "C" xyz_status xyz_search(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem,
                                 const xyz_params *params, void *stream, xyz_result **out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    XYZ_TRY(validate_params(x, params, yfmt));
    HIP_TRY(hipSetDevice(c->device));
    const void *ys[1] = {Y};
    const xyz_params *ps[1] = {params};
    return run_group(c, x, 1, ys, yfmt, mem, ps, (hipStream_t)stream, out);
}

extern "C" xyz_status xyz_search_batch(xyz_ctx *c, const xyz_x *x, int32_t nY, const void *const *Y, int yfmt,
                                       int mem, const xyz_params *params, void *stream, xyz_result **outs)
{
    if (!c || !x || !Y || !outs || !params) return fail(XYZ_EINVAL, "NULL argument");
    if (nY < 0) return fail(XYZ_EINVAL, "nY < 0");
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    for (int q = 0; q < nY; ++q) {
        outs[q] = nullptr;
        if (!Y[q]) return fail(XYZ_EINVAL, "Y[%d] is NULL", q);
        XYZ_TRY(validate_params(x, &params[q], yfmt));
    }
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    std::vector<char> done(nY, 0);
    for (int q = 0; q < nY; ++q) {
        if (done[q]) continue;
        std::vector<int> grp{q};
        const xyz_params &a = params[q];
        const bool shareable = yfmt == XYZ_Y_I8_PM1 && !a.rows;
        if (shareable)
            for (int r = q + 1; r < nY && grp.size() < 255; ++r) {
                const xyz_params &b = params[r];
                if (!done[r] && !b.rows && b.m == a.m && b.L == a.L && b.seed == a.seed &&
                    b.rep_offset == a.rep_offset && b.flags == a.flags && b.cap == a.cap)
                    grp.push_back(r);
            }
        std::vector<const void *> ys;
        std::vector<const xyz_params *> ps;
        for (int g : grp) {
            ys.push_back(Y[g]);
            ps.push_back(&params[g]);
            done[g] = 1;
        }
        std::vector<xyz_result *> res(grp.size(), nullptr);
        xyz_status s = run_group(c, x, (int)grp.size(), ys.data(), yfmt, mem, ps.data(), st, res.data());
        if (s != XYZ_OK) {
            for (int r = 0; r < nY; ++r) {
                if (outs[r]) xyz_result_free(outs[r]);
                outs[r] = nullptr;
            }
            return s;
        }
        for (size_t g = 0; g < grp.size(); ++g) outs[grp[g]] = res[g];
    }
    return XYZ_OK;
}

extern "C" int64_t xyz_result_npairs(const xyz_result *r) { return r ? (int64_t)r->pairs.size() : 0; }
extern "C" const xyz_pair *xyz_result_pairs(const xyz_result *r) { return r && !r->pairs.empty() ? r->pairs.data() : nullptr; }
extern "C" int32_t xyz_result_nreps(const xyz_result *r) { return r ? (int32_t)r->reps.size() : 0; }
extern "C" const xyz_rep_stats *xyz_result_reps(const xyz_result *r) { return r && !r->reps.empty() ? r->reps.data() : nullptr; }
extern "C" const xyz_timing *xyz_result_timing(const xyz_result *r) { return r ? &r->timing : nullptr; }
extern "C" void xyz_result_free(xyz_result *r) { delete r; }
extern "C" xyz_status xyz_result_route(const xyz_result *r, xyz_route *out)
{
    if (!r || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = r->route;
    return XYZ_OK;
}

extern "C" xyz_status xyz_bruteforce(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                                     uint32_t flags, const int32_t *colsA, int64_t nA, const int32_t *colsB,
                                     int64_t nB, void *stream, xyz_result **out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    return brute_run(c, x, Y, yfmt, mem, kappa, flags, colsA, nA, colsB, nB, (hipStream_t)stream, out);
}

xyz_status xyz_rt::brute_run(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                             uint32_t flags, const int32_t *colsA, int64_t nA, const int32_t *colsB, int64_t nB,
                             hipStream_t st, xyz_result **out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (x->ctx->device != c->device) return fail(XYZ_EINVAL, "X lives on another device");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    if (yfmt != XYZ_Y_I8_PM1 && yfmt != XYZ_Y_F32 && yfmt != XYZ_Y_F64) return fail(XYZ_EINVAL, "unknown Y format %d", yfmt);
    if (!std::isfinite(kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
    if (flags & ~(uint32_t)(XYZ_TWO_SIDED | XYZ_PROFILE)) return fail(XYZ_EINVAL, "unknown flags 0x%x", flags);
    const int64_t p = x->p, n = x->n;
    if (!colsA) nA = p;
    if (!colsB) nB = p;
    if (nA < 0 || nB < 0) return fail(XYZ_EINVAL, "negative column count");
    for (int64_t q = 0; colsA && q < nA; ++q)
        if (colsA[q] < 0 || colsA[q] >= p) return fail(XYZ_EINVAL, "colsA[%lld] out of range", (long long)q);
    for (int64_t q = 0; colsB && q < nB; ++q)
        if (colsB[q] < 0 || colsB[q] >= p) return fail(XYZ_EINVAL, "colsB[%lld] out of range", (long long)q);
    HIP_TRY(hipSetDevice(c->device));
    const bool real = x->fmt == XYZ_X_F32 || yfmt != XYZ_Y_I8_PM1;
    if (!real && n >= (1ll << 24))
        return fail(XYZ_EUNSUPPORTED, "brute force needs n < 2^24 (exact FP32 accumulation of the matrix cores)");
    if (real) {
        // real-valued data: the exhaustive search (m = 0, every pair collides) verified in binary64
        if (colsA || colsB) return fail(XYZ_EUNSUPPORTED, "column lists are supported for +-1 data only");
        xyz_params P{};
        P.m = 0;
        P.L = 1;
        P.kappa = kappa;
        P.flags = flags;
        const void *ys[1] = {Y};
        const xyz_params *ps[1] = {&P};
        xyz_result *r = nullptr;
        XYZ_TRY(run_group(c, x, 1, ys, yfmt, mem, ps, st, &r));
        for (auto &pr : r->pairs) {
            pr.first_rep = -1;
            pr.hits = 0;
        }
        r->reps.clear();
        r->timing.brute_ms = r->timing.verify_ms;
        r->route = xyz_route{};
        r->route.method = XYZ_PLAN_BRUTE;
        r->route.L = 1;
        *out = r;
        return XYZ_OK;
    }
    const double t0 = now_ms();
    Timer tm;
    tm.on = (flags & XYZ_PROFILE) != 0;
    tm.st = st;
    xyz_timing timing{};
    const int two = (flags & XYZ_TWO_SIDED) ? 1 : 0;
    uint32_t *yb = nullptr;
    double *yd = nullptr;
    int *err = nullptr;
    const void *ys[1] = {Y};
    tm.begin(0);
    XYZ_TRY(pack_ys(c, x, 1, ys, yfmt, mem, st, &yb, &yd, &err));
    tm.end();
    // the packing's error flag is read back with the survivor counts below (no wait here)
    int herr = 0;
    int32_t *dA = nullptr, *dB = nullptr;
    if (colsA) {
        XYZ_TRY(ws(c, WS_ROWS, (size_t)nA + (colsB ? nB : 0), &dA));
        HIP_TRY(hipMemcpyAsync(dA, colsA, sizeof(int32_t) * nA, hipMemcpyHostToDevice, st));
    }
    if (colsB) {
        if (!dA) {
            XYZ_TRY(ws(c, WS_ROWS, (size_t)nB, &dA));
            dB = dA;
        } else {
            dB = dA + nA;
        }
        HIP_TRY(hipMemcpyAsync(dB, colsB, sizeof(int32_t) * nB, hipMemcpyHostToDevice, st));
    }
    RepInfo *info = nullptr;
    XYZ_TRY(ws(c, WS_INFO, 1, &info));
    HIP_TRY(launch_zero(info, sizeof(RepInfo), st));
    BruteArgs ba{};
    const int nw = (int)((n + 31) / 32);
    ba.nq = x->W32p >> 2;
    ba.colsA = colsA ? dA : nullptr;
    ba.nA = nA;
    ba.colsB = colsB ? dB : nullptr;
    ba.nB = nB;
    ba.tri = (!colsA && !colsB) ? 1 : 0;
    ba.nbA = (nA + BF_TILE - 1) / BF_TILE;
    ba.nbB = (nB + BF_TILE - 1) / BF_TILE;
    ba.ntiles = ba.tri ? (uint64_t)ba.nbA * (ba.nbA + 1) / 2 : (uint64_t)ba.nbA * ba.nbB;
    ba.nsbA = (ba.nbA + 7) / 8;
    ba.nsbB = (ba.nbB + 7) / 8;
    ba.nslots = 64 * (ba.tri ? (uint64_t)ba.nsbA * (ba.nsbA + 1) / 2 : (uint64_t)ba.nsbA * ba.nsbB);
    {
        // blocked copies of both sides (z = y ^ x on the A side) and their popcounts
        uint4 *xa = nullptr, *xb = nullptr;
        uint32_t *pops = nullptr;
        XYZ_TRY(ws(c, WS_BXA, (size_t)ba.nbA * ba.nq * BF_TILE, &xa));
        XYZ_TRY(ws(c, WS_BXB, (size_t)ba.nbB * ba.nq * BF_TILE, &xb));
        XYZ_TRY(ws(c, WS_BPOP, (size_t)(ba.nbA + ba.nbB) * BF_TILE, &pops));
        tm.begin(0);
        HIP_TRY(launch_brute_stage(x->XC, x->W32p, nw, ba.colsA, nA, yb, xa, pops, st));
        HIP_TRY(launch_brute_stage(x->XC, x->W32p, nw, ba.colsB, nB, nullptr, xb, pops + ba.nbA * BF_TILE, st));
        tm.end();
        ba.XBA = xa;
        ba.XBB = xb;
        ba.popA = pops;
        ba.popB = pops + ba.nbA * BF_TILE;
    }
    ba.n = n;
    ba.smin = xyz_smin(n, kappa, two);
    ba.two_sided = two;
    ba.grid_blocks = std::max(8, c->cu_count / 8 * 8);
    if (ba.nslots > 0x7fffffffull) return fail(XYZ_EUNSUPPORTED, "too many column blocks for one launch");
    // each workgroup of the persistent launch owns cap_wg survivor slots; a workgroup that
    // finds more reports its count, and the launch is redone with room for the largest
    const int grid = ba.ntiles ? brute_grid(ba) : 1;
    uint64_t cap_wg = std::max<uint64_t>(c->ws[WS_SURV].bytes / sizeof(Survivor) / grid, 1024);
    unsigned int *wcnt = nullptr;
    XYZ_TRY(ws(c, WS_BCNT, grid, &wcnt));
    std::vector<unsigned int> hcnt(grid);
    Survivor *surv = nullptr;
    uint64_t S = 0;
    for (;;) {
        XYZ_TRY(ws(c, WS_SURV, cap_wg * grid, &surv));
        HIP_TRY(launch_zero(wcnt, sizeof(unsigned int) * grid, st));
        ba.surv = surv;
        ba.cap_wg = cap_wg;
        ba.wg_count = wcnt;
        tm.begin(7);
        HIP_TRY(launch_brute(ba, st));
        tm.end();
        timing.verify_launches += 1;
        HIP_TRY(hipMemcpyAsync(hcnt.data(), wcnt, sizeof(unsigned int) * grid, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        XYZ_TRY(err_flag_status(herr));
        uint64_t mx = 0;
        S = 0;
        for (unsigned int v : hcnt) {
            mx = std::max<uint64_t>(mx, v);
            S += v;
        }
        if (mx <= cap_wg) break;
        cap_wg = mx + mx / 4 + 64;
    }
    // dense survivor list
    Survivor *dense = nullptr;
    unsigned long long *doff = nullptr;
    XYZ_TRY(ws(c, WS_SURV2, std::max<uint64_t>(S, 1), &dense));
    XYZ_TRY(ws(c, WS_BOFF, grid, &doff));
    std::vector<unsigned long long> hoff(grid);
    {
        unsigned long long acc = 0;
        for (int g = 0; g < grid; ++g) {
            hoff[g] = acc;
            acc += hcnt[g];
        }
    }
    HIP_TRY(hipMemcpyAsync(doff, hoff.data(), sizeof(unsigned long long) * grid, hipMemcpyHostToDevice, st));
    tm.begin(6);
    if (S) HIP_TRY(launch_brute_compact(surv, cap_wg, wcnt, doff, grid, dense, st));
    tm.end();
    uint64_t *dk = nullptr, *dk2 = nullptr;
    uint32_t *dv = nullptr, *dv2 = nullptr, *hist = nullptr, *heads = nullptr;
    OutPair *dout = nullptr;
    unsigned long long *nout = nullptr, *ycnt = nullptr;
    XYZ_TRY(ws(c, WS_DKEYS, S, &dk));
    XYZ_TRY(ws(c, WS_DKEYS2, S, &dk2));
    XYZ_TRY(ws(c, WS_DVALS, S, &dv));
    XYZ_TRY(ws(c, WS_DVALS2, S, &dv2));
    XYZ_TRY(ws(c, WS_HIST, radix_hist_entries(S), &hist));
    XYZ_TRY(ws(c, WS_HEADS, S + 1, &heads));
    XYZ_TRY(ws(c, WS_OUT, S, &dout));
    XYZ_TRY(ws(c, WS_NOUT, 1, &nout));
    XYZ_TRY(ws(c, WS_YCNT, 1, &ycnt));
    HIP_TRY(launch_zero(ycnt, sizeof(unsigned long long), st));
    tm.begin(6);
    HIP_TRY(launch_dedup(dense, S, p, n, 1, dk, dv, dk2, dv2, hist, heads, dout, nout, ycnt, info, 0, st));
    tm.end();
    unsigned long long U = 0;
    HIP_TRY(hipMemcpyAsync(&U, nout, sizeof U, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    xyz_result *r = new xyz_result();
    r->pairs.resize(U);
    if (U) HIP_TRY(hipMemcpyAsync(r->pairs.data(), dout, sizeof(xyz_pair) * U, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (auto &pr : r->pairs) {
        pr.first_rep = -1;
        pr.hits = 0;
    }
    tm.collect(timing);
    timing.candidates = ba.tri ? (int64_t)(nA * (nA - 1) / 2) : (int64_t)nA * nB;
    timing.tiles = (int64_t)ba.ntiles;
    timing.total_ms = now_ms() - t0;
    r->timing = timing;
    r->route.method = XYZ_PLAN_BRUTE;
    r->route.L = 1;
    *out = r;
    return XYZ_OK;
}

// ------------------------------------------------------- parameter choice --

extern "C" double xyz_eta(double gamma, int32_t m, int64_t L)
{
    if (!(gamma >= 0.0 && gamma <= 1.0) || m < 0 || L < 0) return NAN;
    return 1.0 - std::pow(1.0 - std::pow(gamma, (double)m), (double)L);
}

namespace {

// erf^{-1}(y) for y in (0, 1/2]: Newton's method on erf(x) - y (derivative 2/sqrt(pi) exp(-x^2))
// from the first term of the series, x = y sqrt(pi) / 2; erf is concave on x > 0, so the
// iterates increase monotonically to the root.
double erf_inv_small(double y)
{
    double x = y * 0.88622692545275801365;
    for (int it = 0; it < 60; ++it) {
        const double d = (std::erf(x) - y) / (1.12837916709551257390 * std::exp(-x * x));
        x -= d;
        if (std::fabs(d) <= 1e-17 * x) break;
    }
    return x;
}

}  // namespace

extern "C" double xyz_tau_dense(int64_t p, int64_t n, double sd)
{
    if (p < 2 || n < 1 || !(sd > 0.0) || !std::isfinite(sd)) return NAN;
    // W ~ N(0, 4 n (1 - 1/2) sd^2): P(|W| <= tau) = erf(tau / (sd sqrt(2n) sqrt 2)) = 1/p
    return 2.0 * std::sqrt((double)n) * sd * erf_inv_small(1.0 / (double)p);
}

extern "C" double xyz_eta_dense(double gamma, int64_t p)
{
    if (p < 2 || !(gamma >= 0.0 && gamma <= 1.0)) return NAN;
    if (gamma >= 1.0) return 1.0;
    return std::erf(erf_inv_small(1.0 / (double)p) * std::sqrt(0.5 / (1.0 - gamma)));
}

extern "C" int64_t xyz_L_for(double eta, double beta)
{
    if (!(eta > 0.0 && eta < 1.0) || !(beta > 0.0) || beta > 1.0) return -1;
    if (beta >= 1.0) return 1;
    const double L = std::ceil(std::log(1.0 - eta) / std::log1p(-beta));
    int64_t Li = (int64_t)std::max(1.0, L);
    // guard against rounding on either side of the exact boundary: 1 - (1 - beta)^L >= eta
    auto found = [beta](int64_t l) { return 1.0 - std::pow(1.0 - beta, (double)l); };
    while (Li > 1 && found(Li - 1) >= eta) --Li;
    while (found(Li) < eta) ++Li;
    return Li;
}

extern "C" int32_t xyz_m_for_L(double gamma, int64_t L, double eta, int32_t m_max)
{
    if (!(gamma > 0.0 && gamma <= 1.0) || L < 1 || !(eta > 0.0 && eta < 1.0) || m_max < 0) return -1;
    int32_t best = -1;
    for (int32_t m = 0; m <= m_max; ++m)
        if (xyz_eta(gamma, m, L) >= eta) best = m;
    return best;
}

extern "C" int32_t xyz_mstar(double gamma, int64_t n, int64_t p, const double *gammas, int64_t ns,
                             double total_pairs, int32_t m_max)
{
    if (!(gamma > 0.0 && gamma < 1.0) || n < 1 || p < 2 || !gammas || ns < 1 || m_max < 1) return -1;
    int32_t best = -1;
    double best_v = INFINITY;
    const double lp = std::log((double)p);
    for (int32_t M = 1; M <= m_max; ++M) {
        double acc = 0.0;
        for (int64_t q = 0; q < ns; ++q) acc += std::pow(gammas[q], (double)M);
        const double S = total_pairs * acc / (double)ns;
        const double b = std::pow(gamma, (double)M);
        const double cost = (double)M * p + p * lp + (double)n * S;
        const double v = b >= 1.0 ? cost : -cost / std::log1p(-b);
        if (v < best_v) {
            best_v = v;
            best = M;
        }
    }
    return best;
}

extern "C" xyz_status xyz_sample_strengths(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem,
                                           int64_t npairs, uint64_t seed, void *stream, double *out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    return sample_strengths(c, x, Y, yfmt, mem, npairs, seed, (hipStream_t)stream, out);
}

xyz_status xyz_rt::sample_strengths(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, int64_t npairs,
                                    uint64_t seed, hipStream_t stream, double *out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    if (x->ctx->device != c->device) return fail(XYZ_EINVAL, "X lives on another device");
    if (npairs < 0) return fail(XYZ_EINVAL, "npairs < 0");
    if (x->p < 2) return fail(XYZ_EINVAL, "X has fewer than two columns");
    if (yfmt != XYZ_Y_I8_PM1 && yfmt != XYZ_Y_F32 && yfmt != XYZ_Y_F64) return fail(XYZ_EINVAL, "unknown Y format %d", yfmt);
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    if (npairs == 0) return XYZ_OK;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    uint32_t *yb = nullptr;
    double *yd = nullptr;
    int *err = nullptr;
    const void *ys[1] = {Y};
    XYZ_TRY(pack_ys(c, x, 1, ys, yfmt, mem, st, &yb, &yd, &err));
    XYZ_TRY(check_err_flag(err, st));
    double *g = nullptr;
    XYZ_TRY(ws(c, WS_CDF, (size_t)npairs, &g));
    HIP_TRY(launch_pair_strengths(x->XC, x->W32p, yb, yd, x->n, x->p, yfmt != XYZ_Y_I8_PM1 ? 1 : 0, seed, npairs, g, st));
    HIP_TRY(hipMemcpyAsync(out, g, sizeof(double) * npairs, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return XYZ_OK;
}

// Largest m the planner considers (the sort path serves m > 15).
constexpr int PLAN_MAX_M = 24;

extern "C" xyz_status xyz_plan(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa,
                               double gamma_target, double eta_target, uint32_t flags, void *stream,
                               xyz_plan_info *out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    if (!(gamma_target > 0.0 && gamma_target <= 1.0)) return fail(XYZ_EINVAL, "gamma_target must be in (0, 1]");
    if (!(eta_target > 0.0 && eta_target < 1.0)) return fail(XYZ_EINVAL, "eta_target must be in (0, 1)");
    if (!std::isfinite(kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
    if (flags & ~(uint32_t)XYZ_TWO_SIDED) return fail(XYZ_EINVAL, "unknown flags 0x%x", flags);
    const int64_t n = x->n, p = x->p;
    if (p < 2) return fail(XYZ_EINVAL, "X has fewer than two columns");
    const double P = (double)p * (double)(p - 1) / 2.0;
    const bool two = (flags & XYZ_TWO_SIDED) != 0;
    // 1. sampled strengths -> expected candidates per repetition for each m
    const int64_t ns = std::min<int64_t>(1 << 16, (int64_t)std::max(2.0, P));
    std::vector<double> g(ns);
    XYZ_TRY(xyz_sample_strengths(c, x, Y, yfmt, mem, ns, 0x5eed5eedull, stream, g.data()));
    std::vector<double> cand(PLAN_MAX_M + 1, 0.0);
    for (int m = 0; m <= PLAN_MAX_M; ++m) {
        double acc = 0.0;
        for (double gq : g) acc += std::pow(gq, (double)m) + (two && m > 0 ? std::pow(1.0 - gq, (double)m) : 0.0);
        cand[m] = m == 0 ? P : P * acc / (double)ns;
    }
    xyz_plan_info best{};
    best.mstar = xyz_mstar(std::min(gamma_target, 1.0 - 1e-12), n, p, g.data(), ns, (double)p * (double)p, 64);
    // 2. brute force: time a square block of up to 4096 x 4096 columns
    const int64_t nb = std::min<int64_t>(p, 4096);
    std::vector<int32_t> cols(nb);
    for (int64_t q = 0; q < nb; ++q) cols[q] = (int32_t)q;
    double brute_ms = INFINITY;
    {
        xyz_result *r = nullptr;
        const bool real = x->fmt == XYZ_X_F32 || yfmt != XYZ_Y_I8_PM1;
        if (!real) {
            for (int rep = 0; rep < 2; ++rep) {
                XYZ_TRY(xyz_bruteforce(c, x, Y, yfmt, mem, 1.0, XYZ_PROFILE, cols.data(), nb, cols.data(), nb, stream, &r));
                const double ms = r->timing.brute_ms;
                xyz_result_free(r);
                brute_ms = ms * P / ((double)nb * (double)nb);
            }
        } else {
            xyz_params P0{};
            P0.m = 0;
            P0.L = 1;
            P0.kappa = 1e300;
            P0.flags = XYZ_PROFILE;
            // real data: exhaustive search on the first nb columns is not available through
            // column lists; time the exhaustive search on the whole X only when it is small
            if (p <= 8192) {
                XYZ_TRY(xyz_search(c, x, Y, yfmt, mem, &P0, stream, &r));
                brute_ms = r->timing.total_ms;
                xyz_result_free(r);
            }
        }
    }
    best.method = XYZ_PLAN_BRUTE;
    best.m = 0;
    best.L = 1;
    best.predicted_ms = brute_ms;
    best.predicted_recall = 1.0;
    best.expected_candidates = P;
    best.brute_ms = brute_ms;
    // 3. xyz: L from eq. (15); rank m by the analytic work, time the most promising ones
    struct Cand {
        int m;
        int64_t L;
        double work;
    };
    std::vector<Cand> cs;
    for (int m = 1; m <= PLAN_MAX_M; ++m) {
        const int64_t L = xyz_L_for(eta_target, std::pow(gamma_target, (double)m));
        if (L < 1 || L > 2000000) continue;
        const double work = (double)L * (cand[m] * std::ceil(n / 32.0) * 2.0 / 1.5e13 + (double)p * 2e-10);
        cs.push_back({m, L, work});
    }
    std::sort(cs.begin(), cs.end(), [](const Cand &a, const Cand &b) { return a.work < b.work; });
    if (cs.size() > 4) cs.resize(4);
    for (const Cand &cd : cs) {
        xyz_params Pc{};
        Pc.m = cd.m;
        Pc.L = (int32_t)std::min<int64_t>(cd.L, 32);
        Pc.kappa = kappa;
        Pc.seed = 0x9a1ull;
        Pc.flags = XYZ_PROFILE | (two ? XYZ_TWO_SIDED : 0);
        xyz_result *r = nullptr;
        XYZ_TRY(xyz_search(c, x, Y, yfmt, mem, &Pc, stream, &r));
        const xyz_timing &t = r->timing;
        const double per_rep = (t.sample_ms + t.hash_ms + t.bucket_ms + t.tiles_ms + t.verify_ms) / Pc.L;
        const double fixed = t.pack_ms + t.dedup_ms;
        xyz_result_free(r);
        const double pred = fixed + per_rep * (double)cd.L;
        if (pred < best.predicted_ms) {
            best.method = XYZ_PLAN_XYZ;
            best.m = cd.m;
            best.L = (int32_t)std::min<int64_t>(cd.L, 0x7fffffff);
            best.predicted_ms = pred;
            best.predicted_recall = xyz_eta(gamma_target, cd.m, cd.L);
            best.expected_candidates = cand[cd.m] * (double)cd.L;
        }
    }
    *out = best;
    return XYZ_OK;
}

extern "C" xyz_status xyz_dense_search(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem,
                                       const int32_t *R, int32_t L, int64_t tau, double kappa, int32_t rep_offset,
                                       uint32_t flags, void *stream, xyz_result **out)
{
    if (!c || !x || !Y || !R || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    if (L < 1) return fail(XYZ_EINVAL, "L=%d < 1", (int)L);
    if (tau < 0) return fail(XYZ_EINVAL, "tau=%lld < 0", (long long)tau);
    if (!std::isfinite(kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
    if (rep_offset < 0) return fail(XYZ_EINVAL, "rep_offset=%d < 0", (int)rep_offset);
    if ((int64_t)rep_offset + L > (1ll << 31)) return fail(XYZ_EINVAL, "repetition index overflow");
    if (flags & ~XYZ_PROFILE) return fail(XYZ_EUNSUPPORTED, "the dense search takes XYZ_PROFILE only");
    if (x->fmt == XYZ_X_F32) return fail(XYZ_EUNSUPPORTED, "the dense search takes +-1 X");
    if (yfmt != XYZ_Y_I8_PM1) return fail(XYZ_EUNSUPPORTED, "the dense search takes +-1 Y");
    const int64_t n = x->n, p = x->p;
    // the projections are int32 sums; each weight is four balanced base-256 digits on the
    // matrix cores, which hold |w| <= 127 (1 + 2^8 + 2^16 + 2^24) > 2^31 - 2^24
    for (int64_t l = 0; l < L; ++l) {
        int64_t a = 0, mx = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t v = R[l * n + i] < 0 ? -(int64_t)R[l * n + i] : (int64_t)R[l * n + i];
            a += v;
            mx = std::max(mx, v);
        }
        if (a > INT32_MAX)
            return fail(XYZ_EINVAL, "sum of |R| of repetition %lld is %lld > 2^31 - 1", (long long)l, (long long)a);
        if (mx > (1ll << 31) - (1ll << 24))
            return fail(XYZ_EINVAL, "|R| of repetition %lld reaches %lld > 2^31 - 2^24", (long long)l, (long long)mx);
    }
    const int64_t taub = std::min<int64_t>(tau, 1ll << 33);   // |x_j - z_k| < 2^32 always
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const double t0 = now_ms();
    Timer tm;
    tm.on = (flags & XYZ_PROFILE) != 0;
    tm.st = st;
    xyz_timing timing{};

    uint32_t *yb = nullptr;
    double *yd = nullptr;
    int *err = nullptr;
    tm.begin(0);
    const void *ys[1] = {Y};
    XYZ_TRY(pack_ys(c, x, 1, ys, yfmt, mem, st, &yb, &yd, &err));
    tm.end();
    XYZ_TRY(check_err_flag(err, st));
    const int64_t smin = xyz_smin(n, kappa, 0);

    // repetitions in chunks of whole projection groups of 8: 32 bytes per (repetition, column)
    const int64_t G = 8;
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(256, (1ll << 30) / (32 * p)));
    if (c->max_chunk > 0) chunk = std::min<int64_t>(chunk, c->max_chunk);
    if (chunk >= G) chunk -= chunk % G;
    chunk = std::min<int64_t>(chunk, L);
    RepInfo *info = nullptr;
    int32_t *dR = nullptr, *xs = nullptr, *zs = nullptr;
    void *dW = nullptr;
    uint64_t *K = nullptr, *K2 = nullptr;
    uint32_t *V = nullptr, *V2 = nullptr, *hist = nullptr;
    unsigned long long *scnt = nullptr;
    XYZ_TRY(ws(c, WS_INFO, (size_t)L, &info));
    XYZ_TRY(ws(c, WS_DPR, (size_t)(chunk * n), &dR));
    XYZ_TRY(ws_get(c, WS_DPW, dense_weight_bytes(n, (int)chunk), &dW));
    XYZ_TRY(ws(c, WS_DPX, (size_t)(chunk * p), &xs));
    XYZ_TRY(ws(c, WS_DPZ, (size_t)(chunk * p), &zs));
    XYZ_TRY(ws(c, WS_SKK, (size_t)(chunk * p), &K));
    XYZ_TRY(ws(c, WS_SKK2, (size_t)(chunk * p), &K2));
    XYZ_TRY(ws(c, WS_SKV, (size_t)(chunk * p), &V));
    XYZ_TRY(ws(c, WS_SKV2, (size_t)(chunk * p), &V2));
    XYZ_TRY(ws(c, WS_SKHIST, radix_hist_entries((uint64_t)(chunk * p)), &hist));
    uint32_t *didx = nullptr;
    XYZ_TRY(ws(c, WS_DPI, (size_t)chunk * (dense_index_buckets(p) + 1), &didx));
    XYZ_TRY(ws(c, WS_SCNT, 1, &scnt));
    HIP_TRY(launch_zero(info, sizeof(RepInfo) * L, st));
    HIP_TRY(launch_zero(scnt, sizeof(unsigned long long), st));
    uint64_t surv_cap = std::max<uint64_t>(c->ws[WS_SURV].bytes / sizeof(Survivor), 1 << 16);
    Survivor *surv = nullptr;
    XYZ_TRY(ws(c, WS_SURV, surv_cap, &surv));
    uint64_t surv_done = 0;

    for (int64_t r0 = 0; r0 < L; r0 += chunk) {
        const int nr = (int)std::min<int64_t>(chunk, L - r0);
        RepInfo *cinfo = info + r0;
        tm.begin(1);
        HIP_TRY(hipMemcpyAsync(dR, R + r0 * n, sizeof(int32_t) * nr * n, hipMemcpyHostToDevice, st));
        tm.end();
        tm.begin(2);
        HIP_TRY(launch_dense_project(x->XR, x->P64, x->XC, x->W32p, p, n, dR, nr, yb, dW, xs, zs, K, V, st));
        tm.end();
        int rbits = 0;
        while ((1 << rbits) < nr) ++rbits;
        uint64_t *Ks = nullptr;
        uint32_t *Vs = nullptr;
        tm.begin(3);
        HIP_TRY(launch_radix_sort(K, V, K2, V2, (uint64_t)nr * p, 32 + rbits, hist, &Ks, &Vs, st));
        tm.end();
        for (bool redo = true; redo;) {
            redo = false;
            HIP_TRY(launch_zero(cinfo, sizeof(RepInfo) * nr, st));
            tm.begin(5);
            HIP_TRY(launch_dense_verify(xs, zs, Ks, Vs, didx, p, nr, taub, x->XC, x->W32p, yb, n, smin,
                                        (int64_t)rep_offset + r0, surv, scnt, surv_cap, cinfo, st));
            tm.end();
            timing.verify_launches += 1;
            unsigned long long cnt = 0;
            HIP_TRY(hipMemcpyAsync(&cnt, scnt, sizeof cnt, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (cnt > surv_cap) {
                XYZ_TRY(grow_survivors(c, cnt, surv_done, scnt, &surv, &surv_cap, st));
                redo = true;
            } else {
                surv_done = cnt;
            }
        }
    }
    return merge_results(c, x, 1, L, rep_offset, surv, surv_done, info, tm, timing, t0, st, out);
}
