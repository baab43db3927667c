// xyz_tune.hip -- xyz_autotune: launch shapes of Algorithm 2 timed once per search shape and
// kept in a cache file.
//
// The choices are those that leave a search's result unchanged: how many repetitions one
// chunk holds (the workspace budget of keys, permutations and bucket offsets, which sets the
// workgroups of the hash and bucket launches) and how many workgroups per compute unit the
// tile-verification and big-tile launches use.  The tuner times the caller's search under a
// few candidates, one choice at a time, keeps the fastest, and records it under a key of the
// device architecture, compute units, n, p, m, the X and Y formats and the flags that change
// the path.  A later xyz_autotune of the same shape reads the record instead of timing, and
// every search of that shape in the context uses it.
#include "xyz_runtime.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

using namespace xyz;
using namespace xyz_rt;

namespace {

double wall_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

Tuned *find_tuned(xyz_ctx *c, const std::string &key)
{
    for (auto &t : c->tuned)
        if (t.key == key) return &t;
    return nullptr;
}

void install(xyz_ctx *c, const Tuned &t)
{
    if (Tuned *e = find_tuned(c, t.key)) *e = t;
    else c->tuned.push_back(t);
}

// Cache file: one record per line, "key chunk_bytes verify_per_cu big_per_cu ms"; lines
// starting with '#' and malformed lines are skipped.
std::vector<Tuned> read_cache(const char *path)
{
    std::vector<Tuned> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream ss(line);
        Tuned t;
        long long cb = 0;
        if (!(ss >> t.key >> cb >> t.k.verify_per_cu >> t.k.big_per_cu >> t.ms)) continue;
        if (cb < (1ll << 20) || t.k.verify_per_cu < 1 || t.k.verify_per_cu > 1024 || t.k.big_per_cu < 1 ||
            t.k.big_per_cu > 1024)
            continue;
        t.k.chunk_bytes = cb;
        out.push_back(t);
    }
    return out;
}

// Rewrites the cache with t replacing any record of its key (temporary file, then rename).
xyz_status write_cache(const char *path, const Tuned &t)
{
    std::vector<Tuned> all = read_cache(path);
    bool found = false;
    for (auto &e : all)
        if (e.key == t.key) e = t, found = true;
    if (!found) all.push_back(t);
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return fail(XYZ_EINVAL, "cannot write the tuning cache %s", tmp.c_str());
        f << "# xyz_autotune: key chunk_bytes verify_wg_per_cu big_wg_per_cu ms\n";
        for (const auto &e : all)
            f << e.key << ' ' << (long long)e.k.chunk_bytes << ' ' << e.k.verify_per_cu << ' ' << e.k.big_per_cu << ' '
              << e.ms << '\n';
        if (!f) return fail(XYZ_EINVAL, "cannot write the tuning cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(XYZ_EINVAL, "cannot replace the tuning cache %s", path);
    return XYZ_OK;
}

void to_public(const Tuned &t, int from_cache, int variants, xyz_tuning *out)
{
    out->chunk_gib = (double)t.k.chunk_bytes / (double)(1ll << 30);
    out->verify_wg_per_cu = t.k.verify_per_cu;
    out->big_wg_per_cu = t.k.big_per_cu;
    out->from_cache = from_cache;
    out->variants = variants;
    out->ms = t.ms;
}

}  // namespace

std::string xyz_rt::tune_key(const xyz_ctx *c, const xyz_x *x, int m, int yfmt, uint32_t flags)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s:cu%d:n%lld:p%lld:m%d:x%d:y%d:f%u", c->arch.empty() ? "gfx" : c->arch.c_str(),
                  c->cu_count, (long long)x->n, (long long)x->p, m, x->fmt, yfmt,
                  (unsigned)(flags & (XYZ_TWO_SIDED | XYZ_UNBIASED)));
    std::string k = buf;
    for (char &ch : k)
        if (ch == ' ') ch = '_';
    return k;
}

Knobs xyz_rt::knobs_for(const xyz_ctx *c, const xyz_x *x, int m, int yfmt, uint32_t flags)
{
    if (c->force_knobs) return *c->force_knobs;
    if (c->tuned.empty()) return Knobs{};
    const std::string key = tune_key(c, x, m, yfmt, flags);
    for (const auto &t : c->tuned)
        if (t.key == key) return t.k;
    return Knobs{};
}

extern "C" xyz_status xyz_autotune(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem,
                                   const xyz_params *params, void *stream, const char *cache_path,
                                   xyz_tuning *out)
{
    if (!c || !x || !Y || !out) return fail(XYZ_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof *out);
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    const xyz_status vs = validate_params(x, params, yfmt);
    if (vs != XYZ_OK) return vs;
    if (params->flags & XYZ_PROFILE) return fail(XYZ_EUNSUPPORTED, "xyz_autotune does not take XYZ_PROFILE");
    const std::string key = tune_key(c, x, params->m, yfmt, params->flags);
    if (cache_path)
        for (const Tuned &t : read_cache(cache_path))
            if (t.key == key) {
                install(c, t);
                to_public(t, 1, 0, out);
                return XYZ_OK;
            }
    HIP_TRY(hipSetDevice(c->device));
    const hipStream_t st = (hipStream_t)stream;
    const void *ys[1] = {Y};
    const xyz_params *ps[1] = {params};
    int variants = 0;
    int64_t ref_pairs = -1, ref_hits = -1;
    bool had_big = false;
    // one search under knobs k: its wall time, checked to give the same pairs as the first
    auto timed = [&](const Knobs &k, double *ms) -> xyz_status {
        c->force_knobs = &k;
        xyz_result *r = nullptr;
        const double t0 = wall_ms();
        const xyz_status s = run_group(c, x, 1, ys, yfmt, mem, ps, st, &r);
        *ms = wall_ms() - t0;
        c->force_knobs = nullptr;
        if (s != XYZ_OK) return s;
        int64_t hits = 0;
        for (const auto &q : r->pairs) hits += q.hits;
        const int64_t np = (int64_t)r->pairs.size();
        had_big = had_big || r->timing.big_launches > 0;
        xyz_result_free(r);
        ++variants;
        if (ref_pairs < 0) ref_pairs = np, ref_hits = hits;
        else if (np != ref_pairs || hits != ref_hits)
            return fail(XYZ_EINTERNAL, "launch shapes changed the search result (%lld pairs, %lld hits; first %lld, %lld)",
                        (long long)np, (long long)hits, (long long)ref_pairs, (long long)ref_hits);
        return XYZ_OK;
    };
    Knobs best{};
    double best_ms = 0.0, ms = 0.0;
    XYZ_TRY(timed(best, &ms));                       // warm-up: workspaces, code objects
    XYZ_TRY(timed(best, &best_ms));
    // chunk budget: candidates that change the repetitions per chunk, within free memory
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    std::vector<int64_t> seen{chunk_reps(c, params->L, x->p, params->m, best.chunk_bytes)};
    for (int64_t gib : {2ll, 4ll, 16ll, 32ll}) {
        Knobs k = best;
        k.chunk_bytes = gib << 30;
        const int64_t reps = chunk_reps(c, params->L, x->p, params->m, k.chunk_bytes);
        if (std::find(seen.begin(), seen.end(), reps) != seen.end()) continue;
        if (k.chunk_bytes > (int64_t)Knobs{}.chunk_bytes && (uint64_t)k.chunk_bytes * 5 / 4 > free_b) continue;
        seen.push_back(reps);
        XYZ_TRY(timed(k, &ms));
        if (ms < best_ms) best_ms = ms, best = k;
    }
    for (int v : {8, 48}) {
        Knobs k = best;
        k.verify_per_cu = v;
        XYZ_TRY(timed(k, &ms));
        if (ms < best_ms) best_ms = ms, best = k;
    }
    if (had_big)
        for (int b : {2, 4, 16}) {
            Knobs k = best;
            k.big_per_cu = b;
            XYZ_TRY(timed(k, &ms));
            if (ms < best_ms) best_ms = ms, best = k;
        }
    Tuned t;
    t.key = key;
    t.k = best;
    t.ms = best_ms;
    install(c, t);
    if (cache_path) XYZ_TRY(write_cache(cache_path, t));
    to_public(t, 0, variants, out);
    return XYZ_OK;
}
