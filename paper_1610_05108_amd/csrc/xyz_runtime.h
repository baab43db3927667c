// xyz_runtime.h -- host-runtime internals shared by the libxyz sources (not part of the ABI).
#pragma once
#include "xyz.h"
#include "xyz_internal.h"

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

// Return from the enclosing xyz_status function on a failed HIP call (XYZ_EDEVICE, with the
// call and its error as the last-error message) or on a failed library call.
#define HIP_TRY(expr)                                                                                       \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) return fail(XYZ_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                              \
    } while (0)

#define XYZ_TRY(expr)                  \
    do {                               \
        xyz_status s_ = (expr);        \
        if (s_ != XYZ_OK) return s_;   \
    } while (0)

namespace xyz_rt {

enum Slot {
    WS_XIN, WS_YIN, WS_YB, WS_YD, WS_CDF, WS_LAST, WS_ERR, WS_ROWS, WS_INFO, WS_KEYS, WS_OFFS, WS_PERM, WS_BASE,
    WS_TILES, WS_SURV, WS_SURV2, WS_SCNT, WS_SMIN, WS_KAPPA, WS_DKEYS, WS_DVALS, WS_DKEYS2, WS_DVALS2, WS_HIST,
    WS_HEADS, WS_OUT, WS_NOUT, WS_YCNT, WS_BXA, WS_BXB, WS_BPOP, WS_BCNT, WS_BOFF, WS_SKK, WS_SKK2, WS_SKV, WS_SKV2, WS_SKHIST, WS_SKHEADS,
    WS_SKRK, WS_SKRS, WS_SKN, WS_SKCNT, WS_SKTAB, WS_NU, WS_DPR, WS_DPW, WS_DPX, WS_DPZ, WS_DPI, WS_CPOP, NWS
};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Launch-shape choices of a search that do not change its result: the workspace budget of
// one chunk of repetitions and the workgroups per compute unit of the verification launches.
struct Knobs {
    int64_t chunk_bytes = 8ll << 30;
    int verify_per_cu = 24;
    int big_per_cu = 8;
};

// A tuned choice for one shape of search (xyz_autotune).
struct Tuned {
    std::string key;
    Knobs k;
    double ms = 0.0;
};

}  // namespace xyz_rt

struct xyz_ctx {
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;
    int cu_count = 256;
    int64_t max_chunk = 0;   // repetitions per chunk (0: the default bound); the server lowers it to fit its budget
    xyz_rt::DevBuf ws[xyz_rt::NWS];
    // Arena mode (xyz_search_noalloc): workspaces are carved from [arena, arena + arena_size)
    // by a bump pointer instead of being allocated, and are never freed.
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    // Tuned launch shapes by search shape (xyz_autotune), and the shape the tuner is timing.
    std::string arch;
    std::vector<xyz_rt::Tuned> tuned;
    const xyz_rt::Knobs *force_knobs = nullptr;
    int64_t syncs = 0;   // host waits on the stream since the current search started
};

struct xyz_x {
    xyz_ctx *ctx = nullptr;
    int64_t n = 0, p = 0;
    int fmt = 0;
    int W32p = 0;
    int64_t P64 = 0;
    int64_t nF = 0;
    uint32_t *XC = nullptr;
    uint64_t *XR = nullptr;
    float *XF = nullptr;
    size_t bytes = 0;
};

struct xyz_result {
    std::vector<xyz_pair> pairs;
    std::vector<xyz_rep_stats> reps;
    xyz_timing timing{};
    xyz_route route{};
};

namespace xyz_rt {

// Sets the thread's last error and returns code.
xyz_status fail(xyz_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
xyz_status validate_params(const xyz_x *x, const xyz_params *P, int yfmt);
// Exact search of eq. (1) (xyz_bruteforce after its argument checks); x may belong to another
// context on the same device.
xyz_status brute_run(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, double kappa, uint32_t flags,
                     const int32_t *colsA, int64_t nA, const int32_t *colsB, int64_t nB, hipStream_t st,
                     xyz_result **out);
// Caller-owned host buffers that receive one search's result instead of an xyz_result.
struct DirectOut {
    xyz_pair *pairs;       // room for cap pairs
    int64_t cap;
    int64_t *npairs;       // number of pairs found (also when it exceeds cap)
    xyz_rep_stats *reps;   // L entries
};
// Searches sharing X, m, L, seed, rep_offset and flags (nys > 1 requires +-1 Y and no row table;
// nys <= 255).  X may belong to another context on the same device.  With direct (nys = 1), the
// result goes to the caller's buffers and outs is not used.
xyz_status run_group(xyz_ctx *c, const xyz_x *x, int nys, const void *const *Ys, int yfmt, int mem,
                     const xyz_params *const *Ps, hipStream_t st, xyz_result **outs,
                     const DirectOut *direct = nullptr);
// xyz_sample_strengths without the check that X belongs to c (X may belong to another context on
// the same device).
xyz_status sample_strengths(xyz_ctx *c, const xyz_x *x, const void *Y, int yfmt, int mem, int64_t npairs,
                            uint64_t seed, hipStream_t stream, double *out);
// Repetitions per chunk for p columns and 2^m buckets under the context's limits and a chunk
// budget of chunk_bytes.
int64_t chunk_reps(const xyz_ctx *c, int64_t L, int64_t p, int m, int64_t chunk_bytes = 8ll << 30);
// Key of a search shape in the tuning table and cache file.
std::string tune_key(const xyz_ctx *c, const xyz_x *x, int m, int yfmt, uint32_t flags);
// The launch shapes of a search: the tuner's forced choice, a tuned entry, or the defaults.
Knobs knobs_for(const xyz_ctx *c, const xyz_x *x, int m, int yfmt, uint32_t flags);
// Frees every workspace of the context.
void ws_release(xyz_ctx *c);
// Device address of the static scratch array of xyz_search_noalloc on `device` (looked up once
// per device, with that device current; called by xyz_init).
xyz_status scratch_setup(int device);

}  // namespace xyz_rt
