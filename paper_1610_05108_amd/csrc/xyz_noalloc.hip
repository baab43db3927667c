// xyz_noalloc.hip -- xyz_search_noalloc: Algorithm 2 with no allocation.
//
// The search's workspaces (keys, permutation, bucket offsets, tile lists,
// survivors, merge scratch) are carved from one static device array,
// `scratch`, instead of being allocated: the entry point serves callers that
// cannot allocate device memory.  Each device that loads the library holds its
// own copy of the array until the process ends.  Every call on a device uses
// that device's copy and leaves its contents behind; the search zeroes every
// counter it reads with a fill kernel, so stale contents never matter.  Calls
// that overlap on one device race on the array.
#include "xyz_runtime.h"

#include <algorithm>
#include <cmath>
#include <mutex>

using namespace xyz;
using namespace xyz_rt;

static __device__ __align__(256) unsigned char scratch[XYZ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};   // device address of `scratch`, per device

void *scratch_ptr(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < MAX_DEVICES ? g_scratch_ptr[device] : nullptr;
}

inline uint64_t round256(uint64_t b) { return (std::max<uint64_t>(b, 1) + 255) / 256 * 256; }

// Workspace bytes of run_group that do not depend on the number of repetitions per chunk
// (packed Y, thresholds, statistics of every repetition, the initial survivor buffer).
uint64_t fixed_bytes(const xyz_x *x, const xyz_params &P, int yfmt)
{
    const uint64_t n = (uint64_t)x->n;
    uint64_t b = round256((uint64_t)x->W32p * 4) + round256((uint64_t)x->nF * 8) + 3 * 256;
    b += round256(n * (yfmt == XYZ_Y_I8_PM1 ? 1 : (yfmt == XYZ_Y_F32 ? 4 : 8)));   // host Y staged on the device
    if (yfmt != XYZ_Y_I8_PM1 || (P.flags & XYZ_UNBIASED)) b += round256(n * 8) + round256(n * 4) + 256;
    b += round256((uint64_t)P.L * sizeof(RepInfo));
    b += round256((uint64_t)(1 << 16) * sizeof(Survivor));
    b += round256(2 * (uint64_t)x->p * 4);                      // column popcounts of the big tiles
    return b;
}

// Workspace bytes per repetition of a chunk: row draws, keys, permutation, bucket offsets
// (m <= 15) or the radix-sort scratch of the sort path (m > 15), tile-list bases.
uint64_t per_rep_bytes(const xyz_x *x, int m)
{
    const uint64_t p = (uint64_t)x->p;
    uint64_t b = 4 * (uint64_t)std::max(m, 1) + 8 * p + 8 * NLISTS;
    if (m <= MAX_M_LDS) b += 4 * ((1ull << m) + 1);
    else b += (48 + 4 * NLISTS) * p + (m <= SK_TABLE_MAX_M ? 4ull << m : 0);
    return b;
}

}  // namespace

xyz_status xyz_rt::scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return fail(XYZ_EUNSUPPORTED, "device %d: the static scratch supports devices 0..%d", device, MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return XYZ_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(XYZ_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return XYZ_OK;
}

extern "C" xyz_status xyz_search_noalloc(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem,
                                         const xyz_params *params, void *stream, xyz_pair *pairs, int64_t pairs_cap,
                                         int64_t *npairs, xyz_rep_stats *reps)
{
    if (!c || !x || !Y || !npairs || !reps) return fail(XYZ_EINVAL, "NULL argument");
    *npairs = 0;
    if (pairs_cap < 0 || (pairs_cap > 0 && !pairs)) return fail(XYZ_EINVAL, "pair buffer: cap %lld at %p",
                                                                (long long)pairs_cap, (void *)pairs);
    if (x->ctx != c) return fail(XYZ_EINVAL, "X belongs to another context");
    if (mem != XYZ_MEM_HOST && mem != XYZ_MEM_DEVICE) return fail(XYZ_EINVAL, "unknown memory kind %d", mem);
    const xyz_status vs = validate_params(x, params, yfmt);
    if (vs != XYZ_OK) return vs;
    if (params->flags & XYZ_PROFILE) return fail(XYZ_EUNSUPPORTED, "xyz_search_noalloc does not take XYZ_PROFILE");
    void *base = scratch_ptr(c->device);
    if (!base) return fail(XYZ_EDEVICE, "the static scratch of device %d is not set up", c->device);
    // sizes known before the search: reject what cannot fit even one repetition per chunk
    const uint64_t cap = (uint64_t)XYZ_NOALLOC_SCRATCH_BYTES;
    const uint64_t fixed = fixed_bytes(x, *params, yfmt), per_rep = per_rep_bytes(x, params->m);
    if (fixed + per_rep > cap / 2)
        return fail(XYZ_ENOMEM, "p=%lld, m=%d, L=%d needs %llu bytes of workspace before any candidate; "
                    "xyz_search_noalloc has %llu bytes of static scratch (at most half for these)",
                    (long long)x->p, params->m, params->L, (unsigned long long)(fixed + per_rep),
                    (unsigned long long)cap);
    const int64_t chunk = (int64_t)std::min<uint64_t>((uint64_t)params->L, (cap / 2 - fixed) / per_rep);
    if (hipSetDevice(c->device) != hipSuccess) return fail(XYZ_EDEVICE, "hipSetDevice(%d) failed", c->device);
    // a context of the same device whose workspaces live in the scratch array
    xyz_ctx a;
    a.device = c->device;
    a.cu_count = c->cu_count;
    a.max_chunk = chunk;
    a.arena = static_cast<char *>(base);
    a.arena_size = (size_t)cap;
    a.arena_used = 0;
    const void *ys[1] = {Y};
    const xyz_params *ps[1] = {params};
    const DirectOut d{pairs, pairs_cap, npairs, reps};
    return run_group(&a, x, 1, ys, yfmt, mem, ps, (hipStream_t)stream, nullptr, &d);
}
