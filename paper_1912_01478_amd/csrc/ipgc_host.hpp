// Host-side pieces shared by the translation units of the IPGC library:
// error reporting, checked HIP calls, growable device buffers and the
// validated form of ipgc_options.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ipgc.h"
#include "ipgc_device.hpp"

namespace ipgc {

constexpr int kDefaultLightMax = 32;
constexpr int kDefaultHubMin = 1024;
constexpr int kDefaultTailGroups = 32;  // workgroups kept for small data-driven rounds (0: all)

// Message of the last failing call on this thread (ipgc_last_error).
extern thread_local char g_err[512];

// Formats the message into g_err and returns code.
int fail(int code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(IPGC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define TRY(expr)             \
    do {                      \
        int rc_ = (expr);     \
        if (rc_) return rc_;  \
    } while (0)

template <typename T>
inline int grow(T **p, int64_t *cap, int64_t want) {
    if (want <= *cap) return IPGC_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    const int64_t alloc = std::max<int64_t>(want, 1024);
    if (hipMalloc(p, sizeof(T) * alloc) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(IPGC_ENOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * alloc));
    }
    *cap = alloc;
    return IPGC_OK;
}

// A device buffer that only grows (its contents are not kept when it does).
template <typename T>
struct DBuf {
    T *p = nullptr;
    int64_t cap = 0;
    int reserve(int64_t n) { return grow(&p, &cap, n); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Options after validation.
struct Params {
    int light_max = kDefaultLightMax;
    int hub_min = kDefaultHubMin;
    bool check_ids = true;
    bool stepped = false;
    int64_t threshold = 0;  // 0: floor(6n/10) for HYBRID
    int workgroups = 0;     // 0: automatic
    int tail_groups = 0;    // workgroups kept for small data-driven rounds (0: all)
    int light = -1;         // -1: automatic, 0: push into every byte map, 1: class L pulls
    bool racy = false;      // in-place (timing-dependent) mode
    int mode = IPGC_MODE_HYBRID;
    ipgc_profile *prof = nullptr;
};

// Validates options (NULL: defaults) and mode into p; clears the out fields of a profile.
int parse_options(const ipgc_options *opt, int mode, Params *p);

// Frees the cached buffers of the BFS entry point on every device.
void release_bfs_workspaces();

}  // namespace ipgc
