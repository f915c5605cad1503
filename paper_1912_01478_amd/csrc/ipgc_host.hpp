// Host-side pieces shared by the translation units of the IPGC library:
// error reporting, checked HIP calls, growable device buffers and the
// validated form of ipgc_options.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <new>

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

// Body of an extern "C" entry point: no C++ exception crosses the C ABI (host
// containers can throw std::bad_alloc).
#define IPGC_GUARD(expr)                                                             \
    do {                                                                             \
        try {                                                                        \
            return (expr);                                                           \
        } catch (const std::bad_alloc &) {                                           \
            return ::ipgc::fail(IPGC_ENOMEM, "host memory allocation failed");       \
        } catch (...) {                                                              \
            return ::ipgc::fail(IPGC_EHIP, "unexpected exception in the library");   \
        }                                                                            \
    } while (0)

#define TRY(expr)             \
    do {                      \
        int rc_ = (expr);     \
        if (rc_) return rc_;  \
    } while (0)

// Where a device buffer came from: the allocation hook in force when it was
// taken (null functions: hipMalloc / hipFree), so that it goes back to the same
// pair even if the hook has been replaced since.
struct AllocOwner {
    ipgc_alloc_fn alloc = nullptr;
    ipgc_free_fn free = nullptr;
    void *user = nullptr;
    int device = 0;
};

// Takes `bytes` of device memory on the current device through the installed
// hook (or hipMalloc) and records the owner; IPGC_ENOMEM on failure.
int dev_alloc(void **p, size_t bytes, AllocOwner *owner);
// Returns memory taken by dev_alloc to its owner (p may be null).
void dev_free(void *p, size_t bytes, const AllocOwner &owner);

template <typename T>
inline int grow(T **p, int64_t *cap, AllocOwner *owner, int64_t want) {
    if (want <= *cap) return IPGC_OK;
    if (*p) dev_free(*p, sizeof(T) * (size_t)*cap, *owner);
    *p = nullptr;
    *cap = 0;
    // at least 4 KiB, so that small buffers are not re-taken for every call
    const int64_t alloc = std::max<int64_t>(want, (int64_t)((4096 + sizeof(T) - 1) / sizeof(T)));
    void *q = nullptr;
    const int rc = dev_alloc(&q, sizeof(T) * (size_t)alloc, owner);
    if (rc) return rc;
    *p = static_cast<T *>(q);
    *cap = alloc;
    return IPGC_OK;
}

// A device buffer that only grows (its contents are not kept when it does), or
// a borrowed piece of memory the library does not own (never grown or freed).
template <typename T>
struct DBuf {
    T *p = nullptr;
    int64_t cap = 0;
    AllocOwner owner;
    bool borrowed = false;
    int reserve(int64_t n) {
        if (borrowed) {
            if (n <= cap) return IPGC_OK;
            return fail(IPGC_ETOOBIG, "a borrowed buffer of %lld entries cannot hold %lld", (long long)cap, (long long)n);
        }
        return grow(&p, &cap, &owner, n);
    }
    void lend(T *q, int64_t n) {
        release();
        p = q;
        cap = n;
        borrowed = true;
    }
    void release() {
        if (p && !borrowed) dev_free(p, sizeof(T) * (size_t)cap, owner);
        p = nullptr;
        cap = 0;
        borrowed = false;
    }
};

// Options after validation.
struct Params {
    int light_max = kDefaultLightMax;
    int hub_min = kDefaultHubMin;
    bool check_ids = true;
    bool full = false;      // IPGC_VALIDATE_FULL: also a simple symmetric graph
    bool stepped = false;
    int barrier_ms = 60000; // grid-barrier wait limit (-1: give up at once)
    int64_t threshold = 0;  // 0: floor(6n/10) for HYBRID
    int workgroups = 0;     // 0: automatic
    int tail_groups = 0;    // workgroups kept for small data-driven rounds (0: all)
    int light = -1;         // -1: automatic, 0: push into every byte map, 1: class L pulls
    bool racy = false;      // in-place (timing-dependent) mode
    bool per_graph = false; // batches: a schedule decision per graph (H_g) instead of one per round
    int mode = IPGC_MODE_HYBRID;
    ipgc_profile *prof = nullptr;
};

// Validates options (NULL: defaults) and mode into p; clears the out fields of a profile.
int parse_options(const ipgc_options *opt, int mode, Params *p);

// Frees the cached buffers of the BFS entry point on every device.
void release_bfs_workspaces();

// Wall-clock ticks a grid-barrier wait may last (Params::barrier_ms at the
// device's wall-clock rate; 0 for a limit of -1).
int barrier_limit_ticks(int dev, int barrier_ms, uint64_t *ticks);

// IPGC_OK, or IPGC_EBADCSR with a message for the kFull* bits of a full check.
int full_check_verdict(int bits);

// Zeroes `bytes` device bytes at p on stream s with a fill kernel (no memset node).
inline int clear(void *p, size_t bytes, hipStream_t s) {
    if (!bytes) return IPGC_OK;
    const int blocks = (int)std::min<uint64_t>(4096, (bytes / 16 + 255) / 256 + 1);
    k_zero<<<blocks, 256, 0, s>>>(static_cast<unsigned char *>(p), (uint64_t)bytes);
    HIP_TRY(hipGetLastError());
    return IPGC_OK;
}

}  // namespace ipgc
