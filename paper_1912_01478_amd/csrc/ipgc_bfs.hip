// Level-synchronous breadth-first search under the keep-the-worklist hybrid
// schedule (Section IV of Rai, M P, Pai, arXiv 1912.01478, applied to another
// worklist algorithm, as its conclusion proposes).  Level L expands the
// frontier (the nodes at distance L): a topology-driven level sweeps every node
// and expands those with dist == L; a data-driven level walks the worklist.
// Both kinds push every newly reached node onto the worklist of level L + 1, so
// the worklist is kept in every level, and a level is topology-driven iff the
// frontier holds more than H nodes.
//
// A neighbour u is claimed with one compare-and-swap on dist[u] (-1 -> L + 1),
// so each node enters exactly one frontier, once.  Nodes of degree up to 32
// expand with one thread; wider ones are handed to a wavefront of the same
// workgroup.  Pushes go to the workgroup's own segment (shared-memory counter,
// no global atomic); a segment that fills up spills into an overflow list
// through one atomicAdd per spilled node.  All levels run in one cooperative
// launch with the grid barrier of the coloring kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "ipgc.h"
#include "ipgc_device.hpp"
#include "ipgc_host.hpp"

namespace ipgc {
namespace bfs {

constexpr int kBlock = 1024;
constexpr int kLightDeg = 32;     // wider frontier nodes are expanded by a wavefront
constexpr int kHeavyPerBlock = 1024;

struct BfsDev {
    const int32_t *rowptr;
    const int32_t *colidx;
    int32_t *dist;
    int32_t *seg[2];      // frontier lists: grid segments of cap entries
    int32_t *seg_cnt[2];  // entries per segment (at most cap)
    int32_t *ovf[2];      // overflow lists
    int32_t *ovf_cnt;     // three rotating overflow sizes: level L reads L % 3, fills (L + 1) % 3
    int32_t *trace;       // frontier size per level
    int64_t trace_cap;
    int64_t n;
    int64_t threshold;    // topology-driven level iff |frontier| > threshold
    int32_t cap;
    int32_t *levels;      // out: non-empty levels (stays -1 if a grid-barrier wait gave up)
    Barrier *bar;
    uint64_t bar_limit;   // wall-clock ticks a grid-barrier wait may last
};

// Prefix sums over the grid segments plus the overflow list (grid + 1 parts) in shared memory.
__device__ int32_t frontier_view(const BfsDev &d, int p, int lvl, int32_t *pre) {
    const int nb = gridDim.x;
    int x = 0;
    if (threadIdx.x < (unsigned)nb) x = d.seg_cnt[p][threadIdx.x];
    else if (threadIdx.x == (unsigned)nb) x = d.ovf_cnt[lvl % 3];
    int tot;
    const int ex = block_scan(x, &tot);
    if (threadIdx.x <= (unsigned)nb) pre[threadIdx.x] = ex;
    if (threadIdx.x == 0) pre[nb + 1] = tot;
    __syncthreads();
    return tot;
}

__device__ __forceinline__ int32_t frontier_at(const BfsDev &d, int p, const int32_t *pre, int32_t i) {
    int lo = 0, hi = gridDim.x + 1;  // part lo with pre[lo] <= i < pre[lo + 1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    if (lo == (int)gridDim.x) return d.ovf[p][i - pre[lo]];
    return d.seg[p][(int64_t)lo * d.cap + (i - pre[lo])];
}

// Claims u for level `next`; the winner appends it to this workgroup's segment (or the overflow list).
__device__ __forceinline__ void visit(const BfsDev &d, int32_t u, int32_t next, int dst, int *s_cnt) {
    if (__hip_atomic_load(&d.dist[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1) return;
    if (atomicCAS(&d.dist[u], -1, next) != -1) return;
    const int p = atomicAdd(s_cnt, 1);
    if (p < d.cap) d.seg[dst][(int64_t)blockIdx.x * d.cap + p] = u;
    else d.ovf[dst][atomicAdd(&d.ovf_cnt[next % 3], 1)] = u;
}

__global__ __launch_bounds__(kBlock) void k_bfs(BfsDev d) {
    __shared__ int32_t pre[kMaxRoundBlocks + 2];
    __shared__ int32_t heavy[kHeavyPerBlock];
    __shared__ int s_cnt, s_heavy;
    GridBarrier gb;
    if (!gb.setup(d.bar, d.bar_limit)) return;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int lane = lane_id(), w = threadIdx.x / kWave, nwv = blockDim.x / kWave;
    int32_t lvl = 0;
    for (;; ++lvl) {
        const int src = lvl & 1, dst = src ^ 1;
        const int32_t size = frontier_view(d, src, lvl, pre);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (lvl < d.trace_cap) d.trace[lvl] = size;
            if (size == 0) *d.levels = lvl;
            d.ovf_cnt[(lvl + 2) % 3] = 0;  // the overflow size level lvl + 1 fills (read last at level lvl - 1)
        }
        if (size == 0) break;
        const bool topo = (int64_t)size > d.threshold;
        const int64_t items = topo ? d.n : size;
        const int32_t next = lvl + 1;
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_heavy = 0;
        }
        __syncthreads();
        if (!gb.sync()) return;  // every part of the frontier is read before any segment of the next one is written
        for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < items; i0 += nt) {
            const int64_t i = i0 + threadIdx.x;
            int32_t v = -1;
            if (i < items) {
                if (topo) v = d.dist[i] == lvl ? (int32_t)i : -1;
                else v = frontier_at(d, src, pre, (int32_t)i);
            }
            if (v >= 0) {
                const int32_t b = d.rowptr[v], e = d.rowptr[v + 1];
                if (e - b > kLightDeg) {
                    const int h = atomicAdd(&s_heavy, 1);
                    if (h < kHeavyPerBlock) heavy[h] = v;
                    else v = -2;  // the list is full: expand it here
                }
                if (e - b <= kLightDeg || v == -2) {
                    for (int32_t k = b; k < e; ++k) visit(d, d.colidx[k], next, dst, &s_cnt);
                }
            }
            // the heavy list fills up at most blockDim entries per pass: drain it before the next
            __syncthreads();
            const int nh = min(s_heavy, kHeavyPerBlock);
            for (int h = w; h < nh; h += nwv) {
                const int32_t u = heavy[h];
                const int32_t b = d.rowptr[u], e = d.rowptr[u + 1];
                for (int32_t k = b + lane; k < e; k += kWave) visit(d, d.colidx[k], next, dst, &s_cnt);
            }
            __syncthreads();
            if (threadIdx.x == 0) s_heavy = 0;
            __syncthreads();
        }
        if (threadIdx.x == 0) d.seg_cnt[dst][blockIdx.x] = min(s_cnt, d.cap);
        if (!gb.sync()) return;
    }
}

// Buffers of one device, kept between calls (they only grow).
struct BfsWorkspace {
    DBuf<int32_t> seg0, seg1, cnt0, cnt1, ovf0, ovf1, ovfc, tr, lv, bad;
    DBuf<Barrier> bar;
};
std::mutex g_bfs_mutex;
std::vector<BfsWorkspace> g_bfs_ws;

// Row pointers non-decreasing inside [0, m] and every column id inside [0, n).
__global__ __launch_bounds__(256) void k_bfs_check(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m,
                                                   int32_t *bad) {
    int b = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = rowptr[v], e = rowptr[v + 1];
        if (a < 0 || e < a || e > m) {
            b = 1;
            continue;
        }
        for (int64_t k = a; k < e; ++k) b |= colidx[k] < 0 || colidx[k] >= n;
    }
    if (__ballot(b) && lane_id() == 0) *bad = 1;
}

}  // namespace bfs

void release_bfs_workspaces() {
    std::lock_guard<std::mutex> lock(bfs::g_bfs_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t dv = 0; dv < bfs::g_bfs_ws.size(); ++dv) {
        if (hipSetDevice((int)dv) != hipSuccess) continue;
        bfs::BfsWorkspace &w = bfs::g_bfs_ws[dv];
        w.seg0.release(); w.seg1.release(); w.cnt0.release(); w.cnt1.release(); w.ovf0.release(); w.ovf1.release();
        w.ovfc.release(); w.tr.release(); w.lv.release(); w.bad.release(); w.bar.release();
    }
    (void)hipSetDevice(cur);
    bfs::g_bfs_ws.clear();
}

}  // namespace ipgc

extern "C" int ipgc_bfs(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m, int64_t source, int mode,
                        const ipgc_options *options, void *stream, int32_t *out_dist, int32_t *out_levels,
                        ipgc_trace *trace) {
    using namespace ipgc;
    using namespace ipgc::bfs;
    if (!out_levels) return fail(IPGC_EINVAL, "null out_levels");
    *out_levels = -1;
    if (n < 0 || m < 0) return fail(IPGC_EINVAL, "negative n or m");
    if (n >= INT32_MAX || m >= INT32_MAX) return fail(IPGC_ETOOBIG, "n or m does not fit the int32 CSR");
    if (mode == IPGC_MODE_REBUILD) return fail(IPGC_EINVAL, "BFS runs TOPOLOGY, DATA or HYBRID");
    Params P;
    TRY(parse_options(options, mode, &P));
    if (P.stepped || P.racy || P.prof) return fail(IPGC_EINVAL, "BFS takes no flags and no profile");
    if (trace) trace->recorded = 0;
    if (n == 0) {
        *out_levels = 0;
        g_err[0] = 0;
        return IPGC_OK;
    }
    if (source < 0 || source >= n) return fail(IPGC_EINVAL, "source %lld outside [0, n)", (long long)source);
    if (!rowptr || !out_dist || (m > 0 && !colidx)) return fail(IPGC_EINVAL, "null device pointer");
    hipStream_t s = (hipStream_t)stream;
    int32_t ends[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&ends[0], rowptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ends[1], rowptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != m) return fail(IPGC_EBADCSR, "rowptr[0] != 0 or rowptr[n] != m");

    int dev = 0, cus = 0, per_cu = 0, coop = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(IPGC_EHIP, "the device cannot launch cooperatively");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_bfs), kBlock, 0));
    // the frontier view keeps one prefix entry per workgroup plus the overflow list in a block of kBlock threads
    const int cap_grid = std::max(1, std::min(std::min(kMaxRoundBlocks, kBlock) - 1, cus * std::max(1, per_cu)));
    const int64_t want = P.workgroups > 0 ? P.workgroups : (n + 4 * kBlock - 1) / (4 * kBlock);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, cap_grid));

    int64_t H;
    if (P.mode == IPGC_MODE_TOPOLOGY) H = -1;
    else if (P.mode == IPGC_MODE_DATA) H = INT64_MAX;
    else H = P.threshold > 0 ? P.threshold : (6 * n) / 10;

    std::lock_guard<std::mutex> lock(g_bfs_mutex);
    if ((int)g_bfs_ws.size() <= dev) g_bfs_ws.resize(dev + 1);
    BfsWorkspace &w = g_bfs_ws[dev];
    DBuf<int32_t> &seg0 = w.seg0, &seg1 = w.seg1, &cnt0 = w.cnt0, &cnt1 = w.cnt1, &ovf0 = w.ovf0, &ovf1 = w.ovf1,
                  &ovfc = w.ovfc, &tr = w.tr, &lv = w.lv, &bad = w.bad;
    DBuf<Barrier> &bar = w.bar;
    BfsDev d{};
    d.cap = (int32_t)((n + grid - 1) / grid) + kBlock;
    const int64_t seg_len = (int64_t)grid * d.cap;
    int rc = IPGC_OK;
    do {
        if ((rc = seg0.reserve(seg_len)) || (rc = seg1.reserve(seg_len)) || (rc = cnt0.reserve(kMaxRoundBlocks)) ||
            (rc = cnt1.reserve(kMaxRoundBlocks)) || (rc = ovf0.reserve(n)) || (rc = ovf1.reserve(n)) ||
            (rc = ovfc.reserve(3)) || (rc = tr.reserve(n + 1)) || (rc = lv.reserve(1)) || (rc = bad.reserve(1)) ||
            (rc = bar.reserve(1)))
            break;
        // ids in range and rows non-decreasing (the kernel reads rows through them)
        if (P.check_ids) {
            int32_t h_bad = 0;
            if (hipMemsetAsync(bad.p, 0, sizeof(int32_t), s) != hipSuccess) {
                rc = fail(IPGC_EHIP, "BFS set-up failed");
                break;
            }
            k_bfs_check<<<(int)std::min<int64_t>(4096, (n + 255) / 256), 256, 0, s>>>(rowptr, colidx, n, m, bad.p);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(&h_bad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = fail(IPGC_EHIP, "BFS checks failed to run");
                break;
            }
            if (h_bad) {
                rc = fail(IPGC_EBADCSR, "decreasing rowptr or a column id outside [0, n)");
                break;
            }
        }
        const int32_t zero3[3] = {0, 0, 0}, src32 = (int32_t)source, dist0 = 0, unset = -1;
        std::vector<int32_t> cnt(kMaxRoundBlocks, 0);
        cnt[0] = 1;
        if (hipMemsetAsync(out_dist, 0xff, sizeof(int32_t) * n, s) != hipSuccess ||
            hipMemcpyAsync(out_dist + source, &dist0, sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(seg0.p, &src32, sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(cnt0.p, cnt.data(), sizeof(int32_t) * kMaxRoundBlocks, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemsetAsync(cnt1.p, 0, sizeof(int32_t) * kMaxRoundBlocks, s) != hipSuccess ||
            hipMemcpyAsync(ovfc.p, zero3, sizeof zero3, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(lv.p, &unset, sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemsetAsync(bar.p, 0, sizeof(Barrier), s) != hipSuccess) {
            rc = fail(IPGC_EHIP, "BFS set-up failed");
            break;
        }
        d.rowptr = rowptr;
        d.colidx = colidx;
        d.dist = out_dist;
        d.seg[0] = seg0.p;
        d.seg[1] = seg1.p;
        d.seg_cnt[0] = cnt0.p;
        d.seg_cnt[1] = cnt1.p;
        d.ovf[0] = ovf0.p;
        d.ovf[1] = ovf1.p;
        d.ovf_cnt = ovfc.p;
        d.trace = tr.p;
        d.trace_cap = n + 1;
        d.n = n;
        d.threshold = H;
        d.levels = lv.p;
        d.bar = bar.p;
        if ((rc = barrier_limit_ticks(dev, P.barrier_ms, &d.bar_limit))) break;
        void *args[] = {&d};
        if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_bfs), dim3(grid), dim3(kBlock), args, 0, s) !=
            hipSuccess) {
            rc = fail(IPGC_EHIP, "BFS launch failed");
            break;
        }
        int32_t levels = -1;
        if (hipMemcpyAsync(&levels, lv.p, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(IPGC_EHIP, "BFS read-back failed");
            break;
        }
        if (levels < 0) {
            rc = fail(IPGC_EHIP, "a grid-barrier wait exceeded %d ms: not every workgroup of the cooperative launch ran "
                      "(%d workgroups)", P.barrier_ms, grid);
            break;
        }
        if (trace) {
            const int64_t k = std::min<int64_t>(trace->capacity, levels);
            if (k > 0 && trace->wl_size &&
                hipMemcpy(trace->wl_size, tr.p, sizeof(int32_t) * k, hipMemcpyDeviceToHost) != hipSuccess) {
                rc = fail(IPGC_EHIP, "BFS trace read-back failed");
                break;
            }
            if (k > 0 && trace->topology && trace->wl_size)
                for (int64_t i = 0; i < k; ++i) trace->topology[i] = (int8_t)((int64_t)trace->wl_size[i] > H);
            trace->recorded = k;
        }
        *out_levels = levels;
    } while (false);
    if (rc == IPGC_OK) g_err[0] = 0;
    return rc;
}
