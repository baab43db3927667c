// xyz_serve.hip -- serving loop of libxyz (xyz_serve_* in include/xyz.h).
//
// Requests arrive from any thread and wait in one FIFO queue.  Each worker
// thread owns a context (its own workspaces) and a HIP stream on the server's
// device.  A free worker takes the oldest request that fits the memory budget
// together with every queued request it can share a pass with (same resident
// X, m, L, seed, first repetition and flags, +-1 responses, no row table:
// these share the row draws, projections and bucket sort, Section 2.2), runs
// them as one group, and publishes each result.  Workers run concurrently, so
// groups overlap on the device.  A request's result never depends on what it
// was grouped with: every per-response quantity is computed from its own Y.
#include "xyz_runtime.h"

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace xyz_rt;

namespace {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    const xyz_x *x = nullptr;
    std::vector<uint8_t> y;      // host copy of Y
    int yfmt = 0;
    xyz_params params{};
    std::vector<int32_t> rows;   // host copy of the row table, if any
    double t_submit = 0.0;
    uint64_t bytes = 0;          // estimated device bytes while running
    int64_t chunk = 0;           // repetitions per chunk that keep it within budget
    bool running = false, done = false, canceled = false;
    xyz_status status = XYZ_OK;
    xyz_result *result = nullptr;
    xyz_route route{};           // what the router chose (routed requests)
    double base_ms = 0.0;        // the cost model's unscaled prediction of the chosen method
};

size_t y_size(int yfmt, int64_t n) { return (size_t)n * (yfmt == XYZ_Y_I8_PM1 ? 1 : (yfmt == XYZ_Y_F32 ? 4 : 8)); }

// Device bytes of one request with `chunk` repetitions per chunk, from the buffers its path
// allocates.  Algorithm 2: keys and permutation (8p per repetition), bucket offsets (or the
// sort path's scratch), the tile list (about one 16-byte tile per 24 x 24 candidates, at least
// p/24 per repetition), the initial survivor buffer and merge scratch, and packed Y.  The exact
// search of +-1 data (brute_run): both sides staged in 256-column blocks of the packed columns
// (2 p n / 8 bytes) with their popcounts, one survivor region of at least 1024 records per
// workgroup of the persistent launch, and the merge.  The exact search of real data runs the
// m = 0 search: one bucket of p columns cut into 64 x 64 matrix-core tiles.
uint64_t estimate_bytes(const xyz_x *x, const xyz_params &P, int64_t chunk, int yfmt)
{
    const double p = (double)x->p;
    const double ybytes = (double)x->W32p * 4 + (double)x->nF * 8 + (double)x->n * 8 + 4096;
    const double merge = (double)(1 << 16) * (32 + 72);      // initial survivors + dedup scratch per record
    if (P.flags & XYZ_EXACT) {
        const bool real = x->fmt == XYZ_X_F32 || yfmt != XYZ_Y_I8_PM1;
        if (!real) {
            const double blocks = std::ceil(p / 256.0);
            const double staged = 2 * blocks * 256.0 * (double)x->W32p * 4 + 2 * blocks * 256.0 * 4;
            const double grid = 256;                         // workgroups of the persistent launch (cu_count / 8 * 8)
            const double surv = grid * 1024 * 32 + grid * 12;
            return (uint64_t)(staged + surv + merge + ybytes);
        }
        const double t = std::ceil(p / 64.0);
        const double tiles = t * (t + 1) / 2;
        return (uint64_t)(8 * p + 64 + 16 * tiles + 80 + merge + ybytes);
    }
    const double nb = std::ldexp(1.0, P.m);
    const double cand = p * (p - 1) / 2 / nb;
    const double tiles = std::max(p / 24.0, cand / 576.0);
    // the sort path (m > 15) replaces the 2^m bucket offsets by about 56 bytes of scratch per column
    const double per_rep = 8 * p + (P.m <= 15 ? 4 * (nb + 1) : 56 * p) + 16 * tiles + 80;
    // column popcounts of the big tiles: |x_j| once and |y ^ x_j| per response
    const double fixed = merge + ybytes + (double)P.L * 64 + (yfmt != XYZ_Y_I8_PM1 ? (double)x->n * 12 : 8.0 * p);
    return (uint64_t)(per_rep * (double)chunk + fixed);
}

// Unscaled cost model of the router (Section 2.3 compares the two methods the same way).  Rates of
// this part: the exact search runs about 2.7e15 pair-rows per second on the FP4 matrix cores, xyz
// verifies about 4.5e13 candidate words per second and spends about 8e-11 s per column and
// repetition on sampling, projection, bucket sort and candidate expansion.
constexpr double RATE_EXACT_PAIR_ROWS = 2.7e15;
constexpr double RATE_VERIFY_WORDS = 4.5e13;
constexpr double SEC_PER_REP_COLUMN = 8e-11;

double exact_ms(const xyz_x *x)
{
    const double p = (double)x->p;
    return p * (p - 1) / 2 * (double)x->n / RATE_EXACT_PAIR_ROWS * 1e3 + 0.05;
}

double xyz_ms(const xyz_x *x, int L, double cand_per_rep)
{
    const double words = std::ceil((double)x->n / 32.0);
    return (double)L * (cand_per_rep * words / RATE_VERIFY_WORDS + (double)x->p * SEC_PER_REP_COLUMN) * 1e3 + 0.05;
}

bool same_group(const Request &a, const Request &b)
{
    if ((a.params.flags | b.params.flags) & XYZ_EXACT) return false;
    return a.x == b.x && a.yfmt == XYZ_Y_I8_PM1 && b.yfmt == XYZ_Y_I8_PM1 && a.rows.empty() && b.rows.empty() &&
           a.params.m == b.params.m && a.params.L == b.params.L && a.params.seed == b.params.seed &&
           a.params.rep_offset == b.params.rep_offset && a.params.flags == b.params.flags && a.chunk == b.chunk;
}

}  // namespace

struct xyz_server {
    int device = 0;
    uint64_t budget = 0;
    int max_batch = 64;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<std::thread> threads;
    std::vector<xyz_ctx *> wctx;
    uint64_t next_ticket = 1;
    bool stopping = false;
    uint64_t bytes_inflight = 0;
    int inflight = 0;
    std::vector<uint64_t> held;   // device bytes each worker's context held after its last group
    std::vector<uint64_t> est;    // estimated bytes of the group each worker runs (0: idle)
    xyz_serve_stats st{};
    std::vector<double> lat;
    // router (XYZ_ROUTE): a context of its own for sampling strengths, and the cost model's
    // scale factors (measured time / unscaled prediction, exponential average of completed groups)
    std::mutex rmu;
    xyz_ctx *rctx = nullptr;
    // measured over predicted time per method, by resident X: requests on one X calibrate each
    // other, and a small data set whose fixed costs dominate does not skew the scale of a large one
    struct Scales {
        double exact = 1.0, xyz = 1.0;
    };
    std::unordered_map<const xyz_x *, Scales> scales;
};

namespace {

// Device bytes the workers' contexts may hold if worker w runs a group of `bytes` now: each
// running worker its estimate (or more, if its context already holds more), each idle worker
// what its context holds.  Lock held.
uint64_t footprint(const xyz_server *s, int w, uint64_t bytes)
{
    uint64_t t = 0;
    for (size_t v = 0; v < s->held.size(); ++v)
        t += std::max(s->held[v], (int)v == w ? bytes : s->est[v]);
    return t;
}

void worker_loop(xyz_server *s, int w)
{
    (void)hipSetDevice(s->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    xyz_ctx *ctx = s->wctx[w];
    for (;;) {
        std::vector<Request *> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [s, w] {
                if (s->stopping) return true;
                if (s->queue.empty()) return false;
                const Request *h = s->queue.front();
                return s->inflight == 0 || s->budget == 0 || footprint(s, w, h->bytes) <= s->budget;
            });
            if (s->stopping) break;
            if (s->budget && footprint(s, w, s->queue.front()->bytes) > s->budget) {
                // nothing runs (inflight == 0), yet the idle contexts' workspaces leave no room:
                // free them all (their threads touch their contexts only after taking a group,
                // which needs this lock)
                for (size_t v = 0; v < s->wctx.size(); ++v) {
                    ws_release(s->wctx[v]);
                    s->held[v] = s->wctx[v]->used;
                }
            }
            Request *h = s->queue.front();
            s->queue.pop_front();
            batch.push_back(h);
            uint64_t bytes = h->bytes;
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)batch.size() < s->max_batch;) {
                Request *r = *it;
                // a group shares its workspace: extra members add only their response buffers
                if (same_group(*h, *r)) {
                    batch.push_back(r);
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            for (Request *r : batch) r->running = true;
            s->est[w] = bytes;
            s->bytes_inflight += bytes;
            s->inflight += (int)batch.size();
            s->st.batches += 1;
            s->st.max_batch = std::max<int32_t>(s->st.max_batch, (int32_t)batch.size());
        }
        std::vector<const void *> ys;
        std::vector<const xyz_params *> ps;
        for (Request *r : batch) {
            ys.push_back(r->y.data());
            r->params.rows = r->rows.empty() ? nullptr : r->rows.data();
            ps.push_back(&r->params);
        }
        std::vector<xyz_result *> outs(batch.size(), nullptr);
        ctx->max_chunk = batch[0]->chunk;
        const xyz_params &P0 = batch[0]->params;
        const double tg0 = now_ms();
        const xyz_status rc =
            (P0.flags & XYZ_EXACT)
                ? brute_run(ctx, batch[0]->x, ys[0], batch[0]->yfmt, XYZ_MEM_HOST, P0.kappa,
                            P0.flags & ~XYZ_EXACT, nullptr, 0, nullptr, 0, stream, outs.data())
                : run_group(ctx, batch[0]->x, (int)batch.size(), ys.data(), batch[0]->yfmt, XYZ_MEM_HOST,
                            ps.data(), stream, outs.data());
        // keep at most this worker's share of the budget between groups, so that idle workers
        // together never hold more than the budget
        if (s->budget && ctx->used > s->budget / s->wctx.size()) ws_release(ctx);
        const double tg = now_ms() - tg0;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->held[w] = ctx->used;
            s->est[w] = 0;
            // the router's scale factors of this X follow the measured group times (a group of
            // routed xyz requests shares its row draws and bucket sort but verifies every member:
            // its prediction is the sum of the members', an upper bound)
            double base = 0.0;
            for (Request *r : batch) base += r->base_ms;
            if (rc == XYZ_OK && base > 0.0 && batch[0]->route.routed) {
                auto &sc = s->scales[batch[0]->x];
                double &f = (P0.flags & XYZ_EXACT) ? sc.exact : sc.xyz;
                f = 0.7 * f + 0.3 * std::min(100.0, std::max(0.01, tg / base));
            }
            const double t = now_ms();
            for (size_t q = 0; q < batch.size(); ++q) {
                Request *r = batch[q];
                r->running = false;
                r->done = true;
                r->status = rc;
                r->result = rc == XYZ_OK ? outs[q] : nullptr;
                if (r->result && r->route.routed) {
                    r->result->route.routed = 1;
                    r->result->route.predicted_ms = r->route.predicted_ms;
                    r->result->route.alternative_ms = r->route.alternative_ms;
                }
                if (rc == XYZ_OK) {
                    s->st.completed += 1;
                    s->lat.push_back(t - r->t_submit);
                } else {
                    s->st.failed += 1;
                    if (outs[q]) xyz_result_free(outs[q]);
                }
            }
            s->bytes_inflight -= batch[0]->bytes;
            s->inflight -= (int)batch.size();
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" xyz_status xyz_serve_start(xyz_ctx *ctx, uint64_t hbm_budget_bytes, int32_t workers, int32_t max_batch,
                                      xyz_server **out)
{
    if (!ctx || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (workers < 1 || workers > 16) return fail(XYZ_EINVAL, "workers=%d out of range [1, 16]", workers);
    if (max_batch < 1 || max_batch > 255) return fail(XYZ_EINVAL, "max_batch=%d out of range [1, 255]", max_batch);
    xyz_server *s = new xyz_server();
    s->device = ctx->device;
    s->budget = hbm_budget_bytes;
    s->max_batch = max_batch;
    for (int w = 0; w < workers; ++w) {
        xyz_ctx *c = nullptr;
        const xyz_status rc = xyz_init(ctx->device, 0, &c);
        if (rc != XYZ_OK) {
            for (auto *q : s->wctx) xyz_fini(q);
            delete s;
            return rc;
        }
        s->wctx.push_back(c);
    }
    {
        const xyz_status rc = xyz_init(ctx->device, 0, &s->rctx);
        if (rc != XYZ_OK) {
            for (auto *q : s->wctx) xyz_fini(q);
            delete s;
            return rc;
        }
    }
    s->held.assign(workers, 0);
    s->est.assign(workers, 0);
    for (int w = 0; w < workers; ++w) s->threads.emplace_back(worker_loop, s, w);
    *out = s;
    return XYZ_OK;
}

extern "C" xyz_status xyz_serve_submit(xyz_server *s, const xyz_x *x, const void *Y, int yfmt,
                                       const xyz_params *params, uint64_t *ticket)
{
    if (!s || !x || !Y || !params || !ticket) return fail(XYZ_EINVAL, "NULL argument");
    if (x->ctx->device != s->device) return fail(XYZ_EINVAL, "X lives on another device");
    xyz_params rp = *params;
    xyz_route route{};
    double base_ms = 0.0;
    if (params->flags & XYZ_ROUTE) {
        // the router: xyz at the request's L with m from eq. (9) at gamma = (1 + kappa)/2, or the exact
        // search, whichever the cost model predicts faster
        if (params->flags & (XYZ_EXACT | XYZ_UNBIASED | XYZ_PROFILE))
            return fail(XYZ_EINVAL, "XYZ_ROUTE combines with XYZ_TWO_SIDED only");
        if (x->fmt == XYZ_X_F32 || yfmt != XYZ_Y_I8_PM1) return fail(XYZ_EUNSUPPORTED, "XYZ_ROUTE needs +-1 X and Y");
        if (params->L < 1) return fail(XYZ_EINVAL, "L=%d < 1", params->L);
        if (!std::isfinite(params->kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
        const bool two = (params->flags & XYZ_TWO_SIDED) != 0;
        const double g = std::min(1.0, std::max(1e-9, 0.5 * (1.0 + std::fabs(params->kappa))));
        const int32_t m = g >= 1.0 ? -1 : xyz_m_for_L(g, params->L, 0.95, xyz::MAX_M_LDS);
        const double t_exact = exact_ms(x);
        double t_xyz = INFINITY;
        if (m >= 1 && x->p >= 2) {
            constexpr int NS = 4096;
            double gs[NS];
            xyz_status rc;
            {
                std::lock_guard<std::mutex> lk(s->rmu);
                rc = sample_strengths(s->rctx, x, Y, yfmt, XYZ_MEM_HOST, NS, 0x5eedull, nullptr, gs);
            }
            if (rc != XYZ_OK) return rc;
            double acc = 0.0;
            for (int q = 0; q < NS; ++q) acc += std::pow(gs[q], m) + (two ? std::pow(1.0 - gs[q], m) : 0.0);
            const double P = (double)x->p * (double)(x->p - 1) / 2;
            t_xyz = xyz_ms(x, params->L, P * acc / NS);
        }
        double se, sx;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const auto it = s->scales.find(x);
            se = it == s->scales.end() ? 1.0 : it->second.exact;
            sx = it == s->scales.end() ? 1.0 : it->second.xyz;
        }
        route.routed = 1;
        rp.rows = nullptr;
        rp.rep_offset = 0;
        rp.flags &= ~XYZ_ROUTE;
        if (t_xyz * sx < t_exact * se) {
            rp.m = m;
            rp.seed = XYZ_SERVE_SEED;
            route.method = XYZ_PLAN_XYZ;
            route.m = m;
            route.L = params->L;
            route.seed = XYZ_SERVE_SEED;
            route.predicted_ms = t_xyz * sx;
            route.alternative_ms = t_exact * se;
            base_ms = t_xyz;
        } else {
            rp.flags |= XYZ_EXACT;
            route.method = XYZ_PLAN_BRUTE;
            route.L = 1;
            route.predicted_ms = t_exact * se;
            route.alternative_ms = t_xyz * sx;
            base_ms = t_exact;
        }
        params = &rp;
    }
    if (params->flags & XYZ_EXACT) {
        if (!std::isfinite(params->kappa)) return fail(XYZ_EINVAL, "kappa is not finite");
        if (params->flags & ~(uint32_t)(XYZ_TWO_SIDED | XYZ_PROFILE | XYZ_EXACT))
            return fail(XYZ_EINVAL, "unknown flags 0x%x", params->flags);
        if (yfmt != XYZ_Y_I8_PM1 && yfmt != XYZ_Y_F32 && yfmt != XYZ_Y_F64)
            return fail(XYZ_EINVAL, "unknown Y format %d", yfmt);
    } else {
        const xyz_status v = validate_params(x, params, yfmt);
        if (v != XYZ_OK) return v;
    }
    Request *r = new Request();
    r->x = x;
    r->yfmt = yfmt;
    r->y.resize(y_size(yfmt, x->n));
    std::memcpy(r->y.data(), Y, r->y.size());
    r->params = *params;
    r->route = route;
    r->base_ms = base_ms;
    if (params->rows && !(params->flags & XYZ_EXACT))
        r->rows.assign(params->rows, params->rows + (size_t)params->L * params->m);
    r->params.rows = nullptr;
    // repetitions per chunk: as many as the budget allows (at least one)
    xyz_ctx probe{};
    int64_t chunk = (params->flags & XYZ_EXACT) ? 1 : chunk_reps(&probe, params->L, x->p, params->m);
    if (s->budget) {
        while (chunk > 1 && estimate_bytes(x, r->params, chunk, yfmt) > s->budget) chunk = (chunk + 1) / 2;
        if (estimate_bytes(x, r->params, chunk, yfmt) > s->budget) {
            delete r;
            return fail(XYZ_ENOMEM, "request needs about %llu bytes even one repetition at a time, budget %llu",
                        (unsigned long long)estimate_bytes(x, *params, 1, yfmt), (unsigned long long)s->budget);
        }
    }
    r->chunk = chunk;
    r->bytes = estimate_bytes(x, r->params, chunk, yfmt);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete r;
            return fail(XYZ_ECANCELED, "server is stopping");
        }
        r->ticket = s->next_ticket++;
        r->t_submit = now_ms();
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
        s->st.submitted += 1;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return XYZ_OK;
}

namespace {

// Hands out a finished request's outcome and forgets the ticket (lock held).
xyz_status claim(xyz_server *s, Request *r, xyz_result **out)
{
    xyz_status rc = r->canceled ? fail(XYZ_ECANCELED, "request %llu was cancelled", (unsigned long long)r->ticket)
                                : r->status;
    if (rc == XYZ_OK) *out = r->result;
    else if (r->status != XYZ_OK && !r->canceled) fail(r->status, "request %llu failed", (unsigned long long)r->ticket);
    s->reqs.erase(r->ticket);
    delete r;
    return rc;
}

}  // namespace

extern "C" xyz_status xyz_serve_poll(xyz_server *s, uint64_t ticket, xyz_result **out)
{
    if (!s || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(XYZ_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second->done) return XYZ_EAGAIN;
    return claim(s, it->second, out);
}

extern "C" xyz_status xyz_serve_wait(xyz_server *s, uint64_t ticket, xyz_result **out)
{
    if (!s || !out) return fail(XYZ_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(XYZ_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    s->cv_done.wait(lk, [r] { return r->done; });
    return claim(s, r, out);
}

extern "C" xyz_status xyz_serve_cancel(xyz_server *s, uint64_t ticket)
{
    if (!s) return fail(XYZ_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(XYZ_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->done) return XYZ_OK;
    if (r->running) return XYZ_EAGAIN;
    s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), r), s->queue.end());
    r->canceled = true;
    r->done = true;
    s->st.canceled += 1;
    s->cv_done.notify_all();
    return XYZ_OK;
}

extern "C" xyz_status xyz_serve_stats_get(xyz_server *s, xyz_serve_stats *out)
{
    if (!s || !out) return fail(XYZ_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int32_t)s->queue.size();
    out->inflight = s->inflight;
    out->bytes_inflight = s->bytes_inflight;
    out->bytes_held = 0;
    for (size_t v = 0; v < s->held.size(); ++v) out->bytes_held += std::max(s->held[v], s->est[v]);
    if (!s->lat.empty()) {
        std::vector<double> v = s->lat;
        std::sort(v.begin(), v.end());
        auto q = [&v](double f) { return v[std::min(v.size() - 1, (size_t)std::floor(f * (double)(v.size() - 1) + 0.5))]; };
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        out->max_ms = v.back();
    }
    return XYZ_OK;
}

extern "C" xyz_status xyz_serve_stop(xyz_server *s)
{
    if (!s) return fail(XYZ_EINVAL, "NULL argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (Request *r : s->queue) {
            r->canceled = true;
            r->done = true;
            s->st.canceled += 1;
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto &t : s->threads) t.join();
    for (auto &kv : s->reqs) {
        if (kv.second->result) xyz_result_free(kv.second->result);
        delete kv.second;
    }
    for (auto *c : s->wctx) xyz_fini(c);
    xyz_fini(s->rctx);
    delete s;
    return XYZ_OK;
}
