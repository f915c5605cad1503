// Worklist push micro-benchmark of Section III (Listings 1 and 2 of Rai, M P,
// Pai, arXiv 1912.01478): Push_WL iterates over the worklist, Push_NoWL over
// every node; both keep a worklist and, in iteration i, deactivate nodes
// [COUNT*i, COUNT*(i+1)) (the text's description; the listing's test
// `node > COUNT * iter_count` is off by the first block).  One kernel launch
// per iteration, as a Pipe of the paper runs it; the first workgroup of each
// launch stamps the device wall clock, so the time of iteration i is the gap
// between the stamps of launches i and i + 1 (its kernel plus the launch).
//
// Two ways to push are measured: the segmented append of the coloring kernels
// (each workgroup appends to its own segment with shared-memory counters, no
// global atomic) and a single global worklist filled through one atomicAdd per
// wavefront (the usual GPU worklist).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ipgc.h"
#include "ipgc_device.hpp"
#include "ipgc_host.hpp"

namespace ipgc {
namespace micro {

constexpr int kBlock = 1024;

struct MicroDev {
    int32_t *list[2];     // worklists (segmented: grid segments of cap entries; atomic: one array)
    int32_t *seg[2];      // segmented: entries per segment of each list
    int32_t *cnt;         // atomic: three rotating sizes (iteration i reads i % 3, fills (i + 1) % 3)
    int32_t cap;          // segmented: entries per segment
    int64_t n;
    int32_t count;        // nodes deactivated per iteration
    int32_t nowl;         // 1: iterate over every node (Push_NoWL), 0: over the worklist (Push_WL)
    int32_t atomic;       // 1: one global worklist filled with wavefront-aggregated atomics
    uint64_t *ticks;      // wall clock at the start of every launch
    int32_t *sizes;       // worklist size at the start of every iteration
};

// One iteration.  Every loop below is bounded by the worklist or node count.
__global__ __launch_bounds__(kBlock) void k_push_micro(MicroDev m, int64_t it) {
    __shared__ int32_t pre[kMaxRoundBlocks + 1];
    __shared__ int s_cnt;
    const int src = (int)(it & 1), dst = src ^ 1;
    const int nb = gridDim.x, lane = lane_id();
    int32_t size;
    if (m.atomic) {
        size = m.cnt[it % 3];
    } else {
        const int x = threadIdx.x < (unsigned)nb ? m.seg[src][threadIdx.x] : 0;
        int tot;
        const int ex = block_scan(x, &tot);
        if (threadIdx.x < (unsigned)nb) pre[threadIdx.x] = ex;
        if (threadIdx.x == 0) pre[nb] = tot;
        size = tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        m.ticks[it] = wall_clock64();
        m.sizes[it] = size;
        if (m.atomic) m.cnt[(it + 2) % 3] = 0;  // the size the next launch fills
    }
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t keep_from = (it + 1) * (int64_t)m.count;  // nodes below are deactivated now
    const int64_t items = size == 0 ? 0 : (m.nowl ? m.n : size);
    const int64_t nt = (int64_t)nb * blockDim.x;
    // the loop runs the same number of times in every lane of a wavefront (ballots below)
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < items; i0 += nt) {
        const int64_t i = i0 + threadIdx.x;
        int32_t v = -1;
        if (i < items) {
            if (m.nowl) {
                v = (int32_t)i;
            } else if (m.atomic) {
                v = m.list[src][i];
            } else {
                int lo = 0, hi = nb;  // the segment holding item i
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (pre[mid] <= i) lo = mid;
                    else hi = mid;
                }
                v = m.list[src][(int64_t)lo * m.cap + (i - pre[lo])];
            }
        }
        const bool push = v >= 0 && v >= keep_from;
        const uint64_t pm = __ballot(push);
        const int below = __popcll(pm & lanes_below());
        int base = 0;
        if (lane == 0 && pm) base = m.atomic ? atomicAdd(&m.cnt[(it + 1) % 3], __popcll(pm)) : atomicAdd(&s_cnt, __popcll(pm));
        base = __shfl(base, 0);
        if (push) {
            if (m.atomic) m.list[dst][base + below] = v;
            else m.list[dst][(int64_t)blockIdx.x * m.cap + base + below] = v;
        }
    }
    __syncthreads();
    if (!m.atomic && threadIdx.x == 0) m.seg[dst][blockIdx.x] = s_cnt;
}

}  // namespace micro
}  // namespace ipgc

extern "C" int ipgc_push_microbench(int64_t n, int32_t count, int32_t nowl, int32_t atomic, uint64_t *ticks,
                                    int32_t *sizes, int64_t capacity, int64_t *iterations, int64_t *tick_khz) {
    using namespace ipgc;
    using namespace ipgc::micro;
    if (n <= 0 || n >= INT32_MAX || count <= 0 || !ticks || !sizes || !iterations || !tick_khz)
        return fail(IPGC_EINVAL, "bad micro-benchmark arguments");
    const int64_t iters = (n + count - 1) / count + 1;  // the last launch finds the worklist empty
    if (capacity < iters + 1) return fail(IPGC_EINVAL, "ticks and sizes need %lld entries", (long long)(iters + 1));
    int dev = 0, cus = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const int grid = std::max(1, std::min(kMaxRoundBlocks, 2 * cus));
    MicroDev m{};
    m.cap = (int32_t)((n + grid - 1) / grid) + kBlock;
    const int64_t list_len = atomic ? n : (int64_t)grid * m.cap;
    DBuf<int32_t> l0, l1, s0, s1, cnt, sz;
    DBuf<uint64_t> tk;
    int rc = IPGC_OK;
    do {
        if ((rc = l0.reserve(list_len)) || (rc = l1.reserve(list_len)) || (rc = s0.reserve(kMaxRoundBlocks)) ||
            (rc = s1.reserve(kMaxRoundBlocks)) || (rc = cnt.reserve(3)) || (rc = sz.reserve(iters + 1)) ||
            (rc = tk.reserve(iters + 1)))
            break;
        // initial worklist: every node (segmented: workgroup b holds nodes [b*span, (b+1)*span))
        std::vector<int32_t> h_list(list_len), h_seg(kMaxRoundBlocks, 0);
        const int32_t h_cnt[3] = {(int32_t)n, 0, 0};
        if (atomic) {
            for (int64_t v = 0; v < n; ++v) h_list[v] = (int32_t)v;
        } else {
            const int64_t span = (n + grid - 1) / grid;
            for (int b = 0; b < grid; ++b) {
                const int64_t lo = b * span, hi = std::min<int64_t>(n, lo + span);
                for (int64_t v = lo; v < hi; ++v) h_list[(int64_t)b * m.cap + (v - lo)] = (int32_t)v;
                h_seg[b] = (int32_t)std::max<int64_t>(0, hi - lo);
            }
        }
        if (hipMemcpy(l0.p, h_list.data(), sizeof(int32_t) * list_len, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s0.p, h_seg.data(), sizeof(int32_t) * kMaxRoundBlocks, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(s1.p, 0, sizeof(int32_t) * kMaxRoundBlocks) != hipSuccess ||
            hipMemcpy(cnt.p, h_cnt, sizeof h_cnt, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(sz.p, 0, sizeof(int32_t) * (iters + 1)) != hipSuccess ||
            hipMemset(tk.p, 0, sizeof(uint64_t) * (iters + 1)) != hipSuccess) {
            rc = fail(IPGC_EHIP, "micro-benchmark set-up failed");
            break;
        }
        m.list[0] = l0.p;
        m.list[1] = l1.p;
        m.seg[0] = s0.p;
        m.seg[1] = s1.p;
        m.cnt = cnt.p;
        m.n = n;
        m.count = count;
        m.nowl = nowl ? 1 : 0;
        m.atomic = atomic ? 1 : 0;
        m.ticks = tk.p;
        m.sizes = sz.p;
        for (int64_t it = 0; it <= iters; ++it) k_push_micro<<<grid, kBlock>>>(m, it);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            rc = fail(IPGC_EHIP, "micro-benchmark launch failed");
            break;
        }
        if (hipMemcpy(ticks, tk.p, sizeof(uint64_t) * (iters + 1), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(sizes, sz.p, sizeof(int32_t) * (iters + 1), hipMemcpyDeviceToHost) != hipSuccess) {
            rc = fail(IPGC_EHIP, "micro-benchmark read-back failed");
            break;
        }
        int64_t k = 0;
        while (k < iters && sizes[k] > 0) ++k;
        *iterations = k;
        *tick_khz = khz;
    } while (false);
    l0.release(); l1.release(); s0.release(); s1.release(); cnt.release(); sz.release(); tk.release();
    if (rc == IPGC_OK) g_err[0] = 0;
    return rc;
}
