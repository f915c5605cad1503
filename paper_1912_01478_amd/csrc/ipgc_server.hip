// Device-resident job server with continuous batching (ipgc_server_* in ipgc.h).
//
// Jobs live in one arena: each resident job owns a range of node slots (its
// n nodes plus one sentinel whose row start ends the job's last row), a range
// of CSR entry slots (its column ids, local to the job, and the rings of its
// W/M nodes) and a range of byte-map bytes.  The three ranges come from three
// first-fit allocators, so a job's byte maps sit at a per-job shift from the
// position rowptr[v] + v that the round kernels compute; the kernels add that
// shift (DevT::fshift).  Node slots outside every resident job carry class
// kNoNode and never enter a list.
//
// The round kernels see the resident jobs as one graph, the disjoint union,
// exactly as for a packed batch (each job's local ids are shifted by its first
// node slot).  A step:
//   1. admit queued jobs in FIFO order while the arena has room: copy the CSR
//      in, then k_srv_admit (row starts, classes, state) and k_srv_prep (id
//      checks, rings); jobs that fail the checks are retired at once;
//   2. k_srv_scan: the worklist of the next round (every uncolored node of a
//      resident job) in the segmented layout, and, if the resident set
//      changed, the static class lists (k_srv_static_offsets/fill);
//   3. k_rounds for up to rounds_per_step rounds (one cooperative launch);
//   4. read the per-job counts of uncommitted nodes and retire the jobs whose
//      count reached zero (colors copied to the caller's host array).
// Between steps every byte of state stays on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "ipgc.h"
#include "ipgc_device.hpp"
#include "ipgc_host.hpp"

namespace ipgc {
namespace srv {

constexpr int8_t kNoNode = -1;   // class of node slots that belong to no resident job
constexpr int kSrvBlock = 1024;  // workgroup of the scan kernels
constexpr int kFPad = 64;        // byte-map guard bytes before and after the arena (word reads)
constexpr int kDefaultQuantum = 8;

using SDev = DevT<int64_t>;

// ------------------------------------------------------------------ kernels

// Admission of one job: its local row pointers rp (n + 1) become union row
// starts at node slot v0 (entries from e0), plus the sentinel slot v0 + n;
// classes by degree; every node uncolored.  Bad row pointers set gerr[slot].
struct AdmitJob {
    const int32_t *rp;  // the job's local row pointers (n + 1), on the device
    int64_t n, m;
    int64_t e0;         // first entry slot
    int64_t fshift;     // byte-map shift
    int32_t v0;         // first node slot
    int32_t slot;
    int32_t r_adm;      // the last round before the job's first
};

__global__ __launch_bounds__(256) void k_srv_admit(AdmitJob j, int32_t light_max, int32_t hub_min, int64_t *growptr,
                                                   int32_t *gbase, int32_t *gidx, int8_t *cls, int32_t *c, uint64_t *mask,
                                                   uint32_t *pend,
                                                   int32_t *lstart, int32_t *llen, int64_t *gend, int64_t *gfshift,
                                                   int32_t *gleft, int32_t *grounds, int32_t *gerr) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
    const int32_t *rp = j.rp;
    const int64_t n = j.n, m = j.m, e0 = j.e0;
    const int32_t v0 = j.v0, slot = j.slot;
    if (gt == 0) {
        gend[slot] = v0 + n;
        gfshift[slot] = j.fshift;
        gleft[slot] = (int32_t)n;
        grounds[slot] = j.r_adm;
    }
    int bad = 0;
    for (int64_t lv = gt; lv <= n; lv += nt) {
        const int32_t v = v0 + (int32_t)lv;
        const int64_t a = rp[lv];
        if (lv == 0) bad |= a != 0;
        gbase[v] = v0;
        gidx[v] = slot;
        lstart[v] = 0;
        llen[v] = 0;
        mask[v] = 0;
        pend[v] = 0;
        if (lv == n) {  // sentinel: ends the last row
            bad |= a != m;
            growptr[v] = e0 + m;
            cls[v] = kNoNode;
            c[v] = 1;
            continue;
        }
        const int64_t e = rp[lv + 1];
        const bool ok = a >= 0 && e >= a && e <= m;
        bad |= !ok;
        growptr[v] = e0 + a;
        const int64_t dv = ok ? e - a : 0;
        cls[v] = (int8_t)node_class(dv, light_max, hub_min);
        if (cls[v] == kL) pend[v] = dv >= 32 ? ~0u : (1u << dv) - 1u;
        c[v] = 0;
    }
    if (__ballot(bad) && lane_id() == 0) gerr[slot] = 1;
}

// Column checks of one admitted job (ids local to the job, in [0, n)) and the
// rings of its W/M nodes; a wavefront per node.  Skipped if its rows failed.
__global__ __launch_bounds__(256) void k_srv_prep(SDev d, int32_t v0, int64_t n, int32_t slot, int32_t *gerr) {
    if (gerr[slot]) return;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const int lane = lane_id();
    int bad = 0, unsorted = 0;
    for (int64_t i = gw; i < n; i += nw) {
        const int32_t v = v0 + (int32_t)i;
        if (d.cls[v] != kL) {
            ring_build_wave(d, v, v0, v0 + n, bad, unsorted);
            continue;
        }
        const int64_t b = d.rowptr[v], e = d.rowptr[v + 1];
        for (int64_t k = b + lane; k < e; k += kWave) {
            const int32_t u = d.colidx[k];
            bad |= u < 0 || u >= n;
        }
    }
    if (__ballot(bad) && lane == 0) gerr[slot] = 1;
}

// A job whose checks failed leaves the union before any round sees it.
__global__ __launch_bounds__(256) void k_srv_reject(int8_t *cls, int32_t v0, int64_t cnt, int32_t slot,
                                                    const int32_t *gerr) {
    if (!gerr[slot]) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        cls[v0 + i] = kNoNode;
}

// Marks node slots [v0, v0 + cnt) as belonging to no job.
__global__ __launch_bounds__(256) void k_srv_retire(int8_t *cls, int32_t v0, int64_t cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        cls[v0 + i] = kNoNode;
}

// Workgroup b of the round grid takes node slots [b*span, (b+1)*span): its
// uncolored nodes of each class go, in ascending order, to its own segment of
// list `par` (the list the next round reads), with their degree sums; its
// resident nodes per class are counted into block_cnt for the static lists.
__global__ __launch_bounds__(kSrvBlock) void k_srv_scan(SDev d, int64_t nhigh, int32_t span, int par,
                                                       int32_t *block_cnt) {
    __shared__ int s_cnt[kNumClasses], s_static[kNumClasses];
    __shared__ unsigned long long s_deg[kNumClasses];
    if (threadIdx.x < kNumClasses) {
        s_cnt[threadIdx.x] = 0;
        s_static[threadIdx.x] = 0;
        s_deg[threadIdx.x] = 0;
    }
    __syncthreads();
    const int b = blockIdx.x, nb = gridDim.x;
    const int64_t lo = (int64_t)b * span, hi = min<int64_t>(lo + span, nhigh);
    for (int64_t c0 = lo; c0 < hi; c0 += blockDim.x) {
        const int64_t v = c0 + threadIdx.x;
        const int k = v < hi ? d.cls[v] : kNoNode;
        const bool act = k >= 0 && d.c[v] <= 0;
        const int64_t deg = act ? d.rowptr[v + 1] - d.rowptr[v] : 0;
        for (int q = 0; q < kNumClasses; ++q) {
            const uint64_t live = __ballot(k == q);
            if (lane_id() == 0 && live) atomicAdd(&s_static[q], __popcll(live));
            const int64_t ds = wave_sum(act && k == q ? deg : 0);
            if (lane_id() == 0 && ds) atomicAdd(&s_deg[q], (unsigned long long)ds);
            const int p = block_append(act && k == q, &s_cnt[q]);
            if (act && k == q) d.seg_list[par][d.ct->seg_off[q] + (int64_t)b * d.ct->seg_cap[q] + p] = (int32_t)v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
        d.seg_cnt[par][threadIdx.x * nb + b] = s_cnt[threadIdx.x];
        d.seg_deg[par][threadIdx.x * nb + b] = (int64_t)s_deg[threadIdx.x];
        block_cnt[threadIdx.x * nb + b] = s_static[threadIdx.x];
    }
}

// Static list layout from the per-workgroup class counts (one workgroup):
// block_cnt becomes each workgroup's first position per class.
__global__ __launch_bounds__(kSrvBlock) void k_srv_static_offsets(SDev d, int32_t *block_cnt, int32_t nhigh) {
    const int nb = d.grid;
    int base = 0;
    for (int q = 0; q < kNumClasses; ++q) {
        const int x = threadIdx.x < (unsigned)nb ? block_cnt[q * nb + threadIdx.x] : 0;
        int tot;
        const int ex = block_scan(x, &tot);
        if (threadIdx.x < (unsigned)nb) block_cnt[q * nb + threadIdx.x] = base + ex;
        if (threadIdx.x == 0) {
            d.ct->class_n[q] = tot;
            d.ct->static_off[q] = base;
        }
        base += tot;
    }
    if (threadIdx.x == 0) d.ct->static_off[kNumClasses] = base;
    (void)nhigh;
}

// Every resident node, grouped by class in ascending order (same spans as the scan).
__global__ __launch_bounds__(kSrvBlock) void k_srv_static_fill(SDev d, int64_t nhigh, int32_t span,
                                                              const int32_t *block_off) {
    __shared__ int s_pos[kNumClasses];
    const int b = blockIdx.x, nb = gridDim.x;
    if (threadIdx.x < kNumClasses) s_pos[threadIdx.x] = block_off[threadIdx.x * nb + b];
    __syncthreads();
    const int64_t lo = (int64_t)b * span, hi = min<int64_t>(lo + span, nhigh);
    for (int64_t c0 = lo; c0 < hi; c0 += blockDim.x) {
        const int64_t v = c0 + threadIdx.x;
        const int k = v < hi ? d.cls[v] : kNoNode;
        for (int q = 0; q < kNumClasses; ++q) {
            const int p = block_append(k == q, &s_pos[q]);
            if (k == q) d.static_list[p] = (int32_t)v;
        }
    }
}

// ------------------------------------------------------------------ host

// First-fit allocator over [0, cap).
struct RangeAlloc {
    int64_t cap = 0;
    std::map<int64_t, int64_t> free_;  // start -> length

    void init(int64_t c) {
        cap = c;
        free_.clear();
        if (c > 0) free_[0] = c;
    }
    int64_t alloc(int64_t len) {
        if (len <= 0) return 0;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const int64_t s = it->first, l = it->second;
            free_.erase(it);
            if (l > len) free_[s + len] = l - len;
            return s;
        }
        return -1;
    }
    void release(int64_t s, int64_t len) {
        if (len <= 0) return;
        auto next = free_.lower_bound(s);
        if (next != free_.end() && next->first == s + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == s) {
                prev->second += len;
                return;
            }
        }
        free_[s] = len;
    }
    // one past the highest allocated position
    int64_t high() const {
        if (free_.empty()) return cap;
        auto last = std::prev(free_.end());
        return last->first + last->second == cap ? last->first : cap;
    }
};

struct Job {
    int64_t id = 0;
    const int32_t *rp = nullptr, *ci = nullptr;
    int32_t *out = nullptr;
    int64_t n = 0, m = 0;
    int32_t slot = -1;
    int64_t v0 = 0, e0 = 0, f0 = 0;
    int32_t r_adm = 0;
    int64_t stage = 0;      // its row pointers' offset in the staging buffer
    bool admitted = false;  // its admission kernels have been issued
};

struct Server {
    int dev = 0;
    hipStream_t s = nullptr;   // every kernel
    hipStream_t cs = nullptr;  // uploads of the next jobs, overlapping the rounds on s
    hipEvent_t ev_uploaded = nullptr, ev_stage_free = nullptr;
    Params P;
    int quantum = kDefaultQuantum;
    int grid = 1;
    int64_t ncap = 0, ecap = 0, fcap = 0;
    int32_t max_jobs = 0;
    int32_t seg_cap = 0;

    DBuf<int64_t> growptr, gend, gfshift, seg_deg, units;
    DBuf<int32_t> colidx, gbase, gidx, c, lower, lstart, llen, static_list, seg0, seg1, seg_cnt, block_cnt, stage;
    DBuf<uint64_t> mask;
    DBuf<uint32_t> pend;
    DBuf<int32_t> grounds, gleft, gerr;
    DBuf<int8_t> cls;
    DBuf<uint8_t> F;
    DBuf<HubRec> hub_won;
    DBuf<Barrier> bar;
    DBuf<Counters> ctb;
    Counters *ct = nullptr, *host_ct = nullptr;
    uint64_t bar_limit = 0;

    RangeAlloc nodes, edges, fbytes;
    std::vector<int32_t> free_slots;
    std::vector<Job> slot_job;
    std::vector<int32_t> h_gleft, h_grounds, h_gerr;
    std::deque<Job> queue;         // submitted, no room yet
    std::vector<int32_t> staged;   // slots reserved and uploaded (or uploading), not yet admitted
    int64_t stage_used = 0;
    std::vector<ipgc_job_result> done;
    int64_t next_id = 0;
    int32_t next_round = 2;  // round numbers start at 2 so that every round reads a segmented list
    bool static_dirty = true;
    ipgc_server_stats st{};

    int create(const ipgc_server_config &cfg);
    void destroy();
    int cancel(int64_t job_id);
    int wait(int64_t job_id, ipgc_job_result *out);
    bool pending(int64_t job_id) const;
    SDev dev_view(int64_t nhigh, int64_t threshold);
    int reserve_and_upload();
    int admit_staged();
    int retire(const std::vector<int32_t> &slots, int status);
    int step();
};

int cooperative_grid(int dev, int want, int *out) {
    int coop = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(IPGC_EHIP, "the device cannot launch cooperatively");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_rounds<SDev>),
                                                         kRoundBlock, 0));
    const int cap = std::min(kMaxRoundBlocks, std::max(1, cus * per_cu));
    *out = std::max(1, std::min(want > 0 ? want : cap, cap));
    return IPGC_OK;
}

int Server::create(const ipgc_server_config &cfg) {
    if (cfg.node_capacity < 2 || cfg.edge_capacity < 0 || cfg.max_jobs < 1 || cfg.rounds_per_step < 0 ||
        cfg.reserved != 0)
        return fail(IPGC_EINVAL, "bad server config (node_capacity >= 2, edge_capacity >= 0, max_jobs >= 1)");
    if (cfg.node_capacity >= INT32_MAX) return fail(IPGC_ETOOBIG, "node_capacity must be below 2^31 - 1");
    TRY(parse_options(&cfg.options, cfg.mode, &P));
    if (!P.check_ids) return fail(IPGC_EINVAL, "a server checks every job: validate must not be NONE");
    if (P.stepped || P.prof) return fail(IPGC_EINVAL, "a server takes no profile and no IPGC_FLAG_STEPPED");
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ev_uploaded, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&ev_stage_free, hipEventDisableTiming));
    quantum = cfg.rounds_per_step > 0 ? cfg.rounds_per_step : kDefaultQuantum;
    TRY(cooperative_grid(dev, P.workgroups, &grid));
    ncap = cfg.node_capacity;
    ecap = cfg.edge_capacity;
    fcap = ecap + ncap + 8 * (int64_t)cfg.max_jobs;
    max_jobs = cfg.max_jobs;
    seg_cap = (int32_t)((ncap + grid - 1) / grid) + kRoundBlock;
    const int64_t seg = (int64_t)kNumClasses * grid * seg_cap;
    // hubs committing in one round: at most one per hub_min + 1 entries
    const int64_t hubs = ecap / (P.hub_min + 1) + max_jobs + 1;

    TRY(growptr.reserve(ncap + 1));
    TRY(gbase.reserve(ncap));
    TRY(gidx.reserve(ncap));
    TRY(c.reserve(ncap));
    TRY(mask.reserve(ncap));
    TRY(pend.reserve(ncap));
    TRY(cls.reserve(ncap));
    TRY(lstart.reserve(ncap));
    TRY(llen.reserve(ncap));
    TRY(static_list.reserve(ncap));
    TRY(stage.reserve(ncap + 1));
    TRY(colidx.reserve(std::max<int64_t>(ecap, 1)));
    TRY(lower.reserve(std::max<int64_t>(ecap, 1)));
    TRY(F.reserve(fcap + 2 * kFPad));
    TRY(seg0.reserve(seg));
    TRY(seg1.reserve(seg));
    TRY(seg_cnt.reserve(2 * kNumClasses * (int64_t)kMaxRoundBlocks));
    TRY(seg_deg.reserve(2 * kNumClasses * (int64_t)kMaxRoundBlocks));
    TRY(block_cnt.reserve(kNumClasses * (int64_t)kMaxRoundBlocks));
    TRY(units.reserve((int64_t)kNumUnits * kMaxRoundBlocks));
    TRY(hub_won.reserve(hubs));
    TRY(gend.reserve(max_jobs));
    TRY(gfshift.reserve(max_jobs));
    TRY(grounds.reserve(max_jobs));
    TRY(gleft.reserve(max_jobs));
    TRY(gerr.reserve(max_jobs));
    TRY(bar.reserve(1));
    TRY(ctb.reserve(1));
    ct = ctb.p;
    HIP_TRY(hipHostMalloc(&host_ct, sizeof(Counters), hipHostMallocDefault));
    TRY(barrier_limit_ticks(dev, P.barrier_ms, &bar_limit));

    HIP_TRY(hipMemsetAsync(cls.p, 0xff, ncap, s));  // every slot kNoNode
    HIP_TRY(hipMemsetAsync(gleft.p, 0, sizeof(int32_t) * max_jobs, s));
    HIP_TRY(hipMemsetAsync(units.p, 0, sizeof(int64_t) * kNumUnits * kMaxRoundBlocks, s));
    HIP_TRY(hipMemsetAsync(F.p, 0, fcap + 2 * kFPad, s));
    Counters h{};
    for (int k = 0; k <= kNumClasses; ++k) h.seg_off[k] = (int64_t)k * grid * seg_cap;
    for (int k = 0; k < kNumClasses; ++k) h.seg_cap[k] = seg_cap;
    *host_ct = h;
    HIP_TRY(hipMemcpyAsync(ct, host_ct, sizeof(Counters), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ev_stage_free, s));
    HIP_TRY(hipStreamSynchronize(s));

    nodes.init(ncap);
    edges.init(ecap);
    fbytes.init(fcap);
    free_slots.clear();
    for (int32_t j = max_jobs - 1; j >= 0; --j) free_slots.push_back(j);
    slot_job.assign(max_jobs, Job());
    h_gleft.assign(max_jobs, 0);
    h_grounds.assign(max_jobs, 0);
    h_gerr.assign(max_jobs, 0);
    st.arena_bytes = (int64_t)(sizeof(int64_t) * (ncap + 1) + sizeof(int32_t) * ncap * 7 + ncap +
                               sizeof(int32_t) * (ncap + 1) + sizeof(int32_t) * 2 * std::max<int64_t>(ecap, 1) +
                               fcap + 2 * kFPad + sizeof(int32_t) * 2 * seg + sizeof(HubRec) * hubs);
    return IPGC_OK;
}

void Server::destroy() {
    growptr.release(); gend.release(); gfshift.release(); seg_deg.release(); units.release();
    colidx.release(); gbase.release(); gidx.release(); c.release(); lower.release(); lstart.release();
    llen.release(); static_list.release(); seg0.release(); seg1.release(); seg_cnt.release();
    block_cnt.release(); stage.release(); grounds.release(); gleft.release(); gerr.release(); cls.release();
    F.release(); mask.release(); pend.release(); hub_won.release(); bar.release(); ctb.release();
    if (host_ct) (void)hipHostFree(host_ct);
    if (s) (void)hipStreamDestroy(s);
    if (cs) (void)hipStreamDestroy(cs);
    if (ev_uploaded) (void)hipEventDestroy(ev_uploaded);
    if (ev_stage_free) (void)hipEventDestroy(ev_stage_free);
    ct = host_ct = nullptr;
    s = cs = nullptr;
    ev_uploaded = ev_stage_free = nullptr;
}

SDev Server::dev_view(int64_t nhigh, int64_t threshold) {
    SDev d{};
    d.rowptr = growptr.p;
    d.colidx = colidx.p;
    d.gbase = gbase.p;
    d.gidx = gidx.p;
    d.gend = gend.p;
    d.grounds = grounds.p;
    d.gleft = gleft.p;
    d.gfshift = gfshift.p;
    d.c = c.p;
    d.cls = cls.p;
    d.F = F.p + kFPad;
    d.mask = mask.p;
    d.pend = pend.p;
    d.lower = lower.p;
    d.lstart = lstart.p;
    d.llen = llen.p;
    d.static_list = static_list.p;
    d.seg_list[0] = seg0.p;
    d.seg_list[1] = seg1.p;
    d.seg_cnt[0] = seg_cnt.p;
    d.seg_cnt[1] = seg_cnt.p + kNumClasses * kMaxRoundBlocks;
    d.seg_deg[0] = seg_deg.p;
    d.seg_deg[1] = seg_deg.p + kNumClasses * kMaxRoundBlocks;
    d.hub_won = hub_won.p;
    d.block_cnt = block_cnt.p;
    d.block_deg = nullptr;
    d.units = units.p;
    d.ct = ct;
    d.bar = bar.p;
    d.trace = nullptr;
    d.trace_deg = nullptr;
    d.trace_cap = 0;
    d.ticks = nullptr;
    d.tick_cap = 0;
    d.threshold = threshold;
    d.m = ecap;
    d.n = (int32_t)nhigh;
    d.light_max = P.light_max;
    d.hub_min = P.hub_min;
    d.sorted = 0;
    d.grid = grid;
    d.light_pull = P.light == 1 ? kPullLight : kPushAll;  // jobs of any class may arrive later
    d.racy = P.racy ? 1 : 0;
    d.tail_groups = P.tail_groups;
    d.discard = P.mode == IPGC_MODE_REBUILD ? 1 : 0;
    d.bar_limit = bar_limit;
    return d;
}

// Retires the jobs in `slots` (copying out the colors of successful ones) and frees their ranges.
int Server::retire(const std::vector<int32_t> &slots, int status) {
    if (slots.empty()) return IPGC_OK;
    for (int32_t slot : slots) {
        const Job &j = slot_job[slot];
        if (status == IPGC_OK)
            HIP_TRY(hipMemcpyAsync(j.out, c.p + j.v0, sizeof(int32_t) * j.n, hipMemcpyDeviceToHost, s));
        k_srv_retire<<<(int)std::min<int64_t>(1024, (j.n + 1 + 255) / 256), 256, 0, s>>>(cls.p, (int32_t)j.v0,
                                                                                         j.n + 1);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t slot : slots) {
        Job &j = slot_job[slot];
        nodes.release(j.v0, j.n + 1);
        edges.release(j.e0, j.m);
        fbytes.release(j.f0, j.m + j.n + 8);
        done.push_back(ipgc_job_result{j.id, status, status == IPGC_OK ? h_grounds[slot] - j.r_adm : -1});
        st.resident -= 1;
        st.resident_nodes -= j.n;
        st.resident_edges -= j.m;
        st.completed += 1;
        free_slots.push_back(slot);
        j = Job();
    }
    static_dirty = true;
    return IPGC_OK;
}

// Reserves arena ranges and a slot for queued jobs in FIFO order while they fit,
// and uploads their CSR on the copy stream (the caller's arrays are pageable,
// so each copy returns once its data is on its way; the rounds of the running
// step continue meanwhile).  Their admission kernels run at the next step.
int Server::reserve_and_upload() {
    if (queue.empty() || free_slots.empty()) return IPGC_OK;
    // the admission kernels of the previous step read the staging buffer
    HIP_TRY(hipStreamWaitEvent(cs, ev_stage_free, 0));
    while (!queue.empty() && !free_slots.empty()) {
        Job j = queue.front();
        if (stage_used + j.n + 1 > ncap + 1) break;
        const int64_t v0 = nodes.alloc(j.n + 1);
        if (v0 < 0) break;
        const int64_t e0 = edges.alloc(j.m);
        if (e0 < 0) {
            nodes.release(v0, j.n + 1);
            break;
        }
        const int64_t f0 = fbytes.alloc(j.m + j.n + 8);
        if (f0 < 0) {
            nodes.release(v0, j.n + 1);
            edges.release(e0, j.m);
            break;
        }
        queue.pop_front();
        const int32_t slot = free_slots.back();
        free_slots.pop_back();
        j.slot = slot;
        j.v0 = v0;
        j.e0 = e0;
        j.f0 = f0;
        j.stage = stage_used;
        stage_used += j.n + 1;
        slot_job[slot] = j;
        HIP_TRY(hipMemcpyAsync(stage.p + j.stage, j.rp, sizeof(int32_t) * (j.n + 1), hipMemcpyHostToDevice, cs));
        if (j.m > 0) HIP_TRY(hipMemcpyAsync(colidx.p + e0, j.ci, sizeof(int32_t) * j.m, hipMemcpyHostToDevice, cs));
        HIP_TRY(hipMemsetAsync(gerr.p + slot, 0, sizeof(int32_t), cs));
        HIP_TRY(hipMemsetAsync(F.p + kFPad + f0, 0, j.m + j.n + 8, cs));
        staged.push_back(slot);
        st.admitted += 1;
        st.resident += 1;
        st.resident_nodes += j.n;
        st.resident_edges += j.m;
        st.peak_resident = std::max(st.peak_resident, st.resident);
    }
    HIP_TRY(hipEventRecord(ev_uploaded, cs));
    st.queued = (int64_t)queue.size();
    return IPGC_OK;
}

// Admission kernels of the staged jobs (after their uploads): rows, classes, state,
// id checks and rings; a job that fails its checks leaves the union at once and is
// reported after the step.
int Server::admit_staged() {
    if (staged.empty()) return IPGC_OK;
    HIP_TRY(hipStreamWaitEvent(s, ev_uploaded, 0));
    for (int32_t slot : staged) {
        Job &j = slot_job[slot];
        j.r_adm = next_round - 1;
        const int64_t v0 = j.v0, e0 = j.e0, f0 = j.f0;
        const AdmitJob aj{stage.p + j.stage, j.n, j.m, e0, f0 - (e0 + v0), (int32_t)v0, slot, j.r_adm};
        const int blocks = (int)std::min<int64_t>(4096, (j.n + 1 + 255) / 256);
        k_srv_admit<<<blocks, 256, 0, s>>>(aj, P.light_max, P.hub_min, growptr.p, gbase.p, gidx.p, cls.p, c.p, mask.p, pend.p,
                                           lstart.p, llen.p, gend.p, gfshift.p, gleft.p, grounds.p, gerr.p);
        SDev d = dev_view(nodes.high(), 0);
        const int pblocks = (int)std::min<int64_t>(8192, (j.n + 3) / 4);
        if (P.full) {
            // sorted rows in the job's ring slots (the rings are built over them next), then the checks
            k_full_sort<<<(int)std::min<int64_t>(j.n, 65536), kSortBlock, 0, s>>>(d, v0, v0 + j.n, lower.p, gerr.p + slot);
            k_full_check<<<std::max(1, pblocks), kPrepBlock, 0, s>>>(d, v0, v0 + j.n, lower.p, gerr.p + slot,
                                                                    gerr.p + slot);
        }
        k_srv_prep<<<std::max(1, pblocks), 256, 0, s>>>(d, (int32_t)v0, j.n, slot, gerr.p);
        k_srv_reject<<<blocks, 256, 0, s>>>(cls.p, (int32_t)v0, j.n + 1, slot, gerr.p);
        HIP_TRY(hipGetLastError());
        j.admitted = true;
    }
    HIP_TRY(hipEventRecord(ev_stage_free, s));
    staged.clear();
    stage_used = 0;
    static_dirty = true;
    return IPGC_OK;
}

int Server::step() {
    if (st.resident == 0 && queue.empty()) return IPGC_OK;
    int64_t active_jobs = 0;
    for (const Job &j : slot_job) active_jobs += j.slot >= 0 && j.admitted;
    // with no rounds to overlap them with, uploads happen now; otherwise during the rounds
    if (active_jobs == 0 && staged.empty()) TRY(reserve_and_upload());
    active_jobs += (int64_t)staged.size();
    TRY(admit_staged());
    if (active_jobs == 0) return IPGC_OK;
    const int64_t nhigh = nodes.high();
    int64_t H;
    if (P.mode == IPGC_MODE_TOPOLOGY) H = -1;
    else if (P.mode == IPGC_MODE_DATA) H = INT64_MAX;
    else H = P.threshold > 0 ? P.threshold : (6 * st.resident_nodes) / 10;
    SDev d = dev_view(nhigh, H);
    const int32_t first = next_round, last = next_round + quantum - 1;
    const int32_t span = (int32_t)((nhigh + grid - 1) / grid);
    k_srv_scan<<<grid, kSrvBlock, 0, s>>>(d, nhigh, span, first & 1, block_cnt.p);
    if (static_dirty) {
        k_srv_static_offsets<<<1, kSrvBlock, 0, s>>>(d, block_cnt.p, (int32_t)nhigh);
        k_srv_static_fill<<<grid, kSrvBlock, 0, s>>>(d, nhigh, span, block_cnt.p);
        static_dirty = false;
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemsetAsync(bar.p, 0, sizeof(Barrier), s));
    HIP_TRY(hipMemsetAsync(reinterpret_cast<char *>(ct) + offsetof(Counters, finished), 0, sizeof(int32_t), s));
    int32_t a_first = first, a_last = last;
    void *args[] = {&d, &a_first, &a_last};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_rounds<SDev>), dim3(grid), dim3(kRoundBlock),
                                       args, 0, s));
    HIP_TRY(hipMemcpyAsync(host_ct, ct, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_gleft.data(), gleft.p, sizeof(int32_t) * max_jobs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_grounds.data(), grounds.p, sizeof(int32_t) * max_jobs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_gerr.data(), gerr.p, sizeof(int32_t) * max_jobs, hipMemcpyDeviceToHost, s));
    // while the rounds run: upload the next jobs that fit now
    TRY(reserve_and_upload());
    HIP_TRY(hipStreamSynchronize(s));
    if (!host_ct->finished) {
        unsigned aborted = 0;
        HIP_TRY(hipMemcpy(&aborted, &bar.p->abort.v, sizeof aborted, hipMemcpyDeviceToHost));
        if (aborted)
            return fail(IPGC_EHIP, "a grid-barrier wait exceeded %d ms: not every workgroup of the cooperative launch "
                        "ran (%d workgroups)", P.barrier_ms, grid);
    }
    if (host_ct->seg_overflow) return fail(IPGC_EHIP, "internal error: a worklist segment overflowed");
    const int32_t ran_to = host_ct->finished ? host_ct->rounds : last;
    st.rounds += ran_to - first + 1;
    st.steps += 1;
    next_round = ran_to + 1;
    std::vector<int32_t> finished, failed;
    for (int32_t slot = 0; slot < max_jobs; ++slot) {
        const Job &j = slot_job[slot];
        if (j.slot < 0 || !j.admitted) continue;
        if (h_gerr[slot]) failed.push_back(slot);
        else if (h_gleft[slot] == 0) finished.push_back(slot);
    }
    TRY(retire(failed, IPGC_EBADCSR));
    return retire(finished, IPGC_OK);
}

// A job that has not finished: queued, staged (upload issued) or resident.
bool Server::pending(int64_t job_id) const {
    for (const Job &j : queue)
        if (j.id == job_id) return true;
    for (const Job &j : slot_job)
        if (j.slot >= 0 && j.id == job_id) return true;
    return false;
}

int Server::cancel(int64_t job_id) {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
        if (it->id != job_id) continue;
        queue.erase(it);
        st.queued = (int64_t)queue.size();
        done.push_back(ipgc_job_result{job_id, IPGC_ECANCELED, -1});
        st.cancelled += 1;
        st.completed += 1;
        return IPGC_OK;
    }
    int32_t slot = -1;
    for (const Job &j : slot_job)
        if (j.slot >= 0 && j.id == job_id) slot = j.slot;
    if (slot < 0) {
        for (const ipgc_job_result &r : done)
            if (r.job_id == job_id) return fail(IPGC_EINVAL, "job %lld has already finished", (long long)job_id);
        return fail(IPGC_EINVAL, "no job %lld is queued or resident", (long long)job_id);
    }
    Job &j = slot_job[slot];
    if (!j.admitted) {
        // its upload reads the caller's arrays: let it end before the job is reported
        HIP_TRY(hipStreamSynchronize(cs));
        staged.erase(std::find(staged.begin(), staged.end(), slot));
    } else {
        // the job's node slots leave the union; the next step rebuilds the worklist and static lists without them
        k_srv_retire<<<(int)std::min<int64_t>(1024, (j.n + 1 + 255) / 256), 256, 0, s>>>(cls.p, (int32_t)j.v0, j.n + 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        static_dirty = true;
    }
    nodes.release(j.v0, j.n + 1);
    edges.release(j.e0, j.m);
    fbytes.release(j.f0, j.m + j.n + 8);
    done.push_back(ipgc_job_result{job_id, IPGC_ECANCELED, -1});
    st.resident -= 1;
    st.resident_nodes -= j.n;
    st.resident_edges -= j.m;
    st.cancelled += 1;
    st.completed += 1;
    free_slots.push_back(slot);
    j = Job();
    return IPGC_OK;
}

int Server::wait(int64_t job_id, ipgc_job_result *out) {
    for (;;) {
        for (auto it = done.begin(); it != done.end(); ++it) {
            if (it->job_id != job_id) continue;
            *out = *it;
            done.erase(it);
            return IPGC_OK;
        }
        if (!pending(job_id)) return fail(IPGC_EINVAL, "no job %lld is pending or unreported", (long long)job_id);
        TRY(step());
    }
}

}  // namespace srv
}  // namespace ipgc

struct ipgc_server {
    ipgc::srv::Server impl;
};

extern "C" {

int ipgc_server_create(const ipgc_server_config *config, ipgc_server **out) {
    IPGC_GUARD(([&]() -> int {
    using namespace ipgc;
    using namespace ipgc::srv;
    if (!config || !out) return fail(IPGC_EINVAL, "null pointer");
    *out = nullptr;
    ipgc_server *sv = new ipgc_server();
    const int rc = sv->impl.create(*config);
    if (rc != IPGC_OK) {
        char msg[sizeof g_err];
        std::memcpy(msg, g_err, sizeof msg);
        sv->impl.destroy();
        delete sv;
        std::memcpy(g_err, msg, sizeof msg);
        return rc;
    }
    *out = sv;
    g_err[0] = 0;
    return IPGC_OK;
    })());
}

int ipgc_server_submit(ipgc_server *server, const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m,
                       int32_t *out_colors, int64_t *job_id) {
    IPGC_GUARD(([&]() -> int {
    using namespace ipgc;
    using namespace ipgc::srv;
    if (!server || !job_id) return fail(IPGC_EINVAL, "null pointer");
    Server &sv = server->impl;
    if (n < 0 || m < 0) return fail(IPGC_EINVAL, "negative n or m");
    if (!rowptr || (n > 0 && !out_colors) || (m > 0 && !colidx)) return fail(IPGC_EINVAL, "null host pointer");
    if (n + 1 > sv.ncap || m > sv.ecap || m >= INT32_MAX)
        return fail(IPGC_ETOOBIG, "a job of %lld nodes and %lld entries never fits this server's arena", (long long)n,
                    (long long)m);
    Job j;
    j.id = sv.next_id++;
    j.rp = rowptr;
    j.ci = colidx;
    j.out = out_colors;
    j.n = n;
    j.m = m;
    *job_id = j.id;
    sv.st.submitted += 1;
    if (n == 0) {  // nothing to color
        sv.done.push_back(ipgc_job_result{j.id, m == 0 && rowptr[0] == 0 ? IPGC_OK : IPGC_EBADCSR, m == 0 ? 0 : -1});
        sv.st.completed += 1;
    } else {
        sv.queue.push_back(j);
        sv.st.queued = (int64_t)sv.queue.size();
    }
    g_err[0] = 0;
    return IPGC_OK;
    })());
}

int ipgc_server_step(ipgc_server *server) {
    using namespace ipgc;
    using namespace ipgc::srv;
    if (!server) return fail(IPGC_EINVAL, "null server");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != server->impl.dev) HIP_TRY(hipSetDevice(server->impl.dev));
    int rc;
    try {
        rc = server->impl.step();
    } catch (const std::bad_alloc &) {
        rc = fail(IPGC_ENOMEM, "host memory allocation failed");
    }
    if (cur != server->impl.dev) (void)hipSetDevice(cur);
    if (rc == IPGC_OK) g_err[0] = 0;
    return rc;
}

int ipgc_server_wait(ipgc_server *server, int64_t job_id, ipgc_job_result *result) {
    using namespace ipgc;
    if (!server || !result) return fail(IPGC_EINVAL, "null pointer");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != server->impl.dev) HIP_TRY(hipSetDevice(server->impl.dev));
    int rc;
    try {
        rc = server->impl.wait(job_id, result);
    } catch (const std::bad_alloc &) {
        rc = fail(IPGC_ENOMEM, "host memory allocation failed");
    }
    if (cur != server->impl.dev) (void)hipSetDevice(cur);
    if (rc == IPGC_OK) g_err[0] = 0;
    return rc;
}

int ipgc_server_cancel(ipgc_server *server, int64_t job_id) {
    using namespace ipgc;
    if (!server) return fail(IPGC_EINVAL, "null server");
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != server->impl.dev) HIP_TRY(hipSetDevice(server->impl.dev));
    int rc;
    try {
        rc = server->impl.cancel(job_id);
    } catch (const std::bad_alloc &) {
        rc = fail(IPGC_ENOMEM, "host memory allocation failed");
    }
    if (cur != server->impl.dev) (void)hipSetDevice(cur);
    if (rc == IPGC_OK) g_err[0] = 0;
    return rc;
}

int ipgc_server_poll(ipgc_server *server, ipgc_job_result *results, int64_t capacity, int64_t *count) {
    using namespace ipgc;
    using namespace ipgc::srv;
    if (!server || !count || (capacity > 0 && !results)) return fail(IPGC_EINVAL, "null pointer");
    Server &sv = server->impl;
    const int64_t k = std::min<int64_t>(std::max<int64_t>(capacity, 0), (int64_t)sv.done.size());
    for (int64_t i = 0; i < k; ++i) results[i] = sv.done[i];
    sv.done.erase(sv.done.begin(), sv.done.begin() + k);
    *count = k;
    g_err[0] = 0;
    return IPGC_OK;
}

int ipgc_server_stats_get(const ipgc_server *server, ipgc_server_stats *stats) {
    using namespace ipgc;
    using namespace ipgc::srv;
    if (!server || !stats) return fail(IPGC_EINVAL, "null pointer");
    const Server &sv = server->impl;
    *stats = sv.st;
    std::vector<int64_t> u((size_t)kNumUnits * kMaxRoundBlocks);
    HIP_TRY(hipMemcpy(u.data(), sv.units.p, sizeof(int64_t) * u.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < kNumUnits; ++k)
        for (int b = 0; b < sv.grid; ++b) stats->units[k] += u[(size_t)k * sv.grid + b];
    g_err[0] = 0;
    return IPGC_OK;
}

void ipgc_server_destroy(ipgc_server *server) {
    if (!server) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(server->impl.dev);
    (void)hipStreamSynchronize(server->impl.s);
    (void)hipStreamSynchronize(server->impl.cs);
    server->impl.destroy();
    (void)hipSetDevice(cur);
    delete server;
}

}  // extern "C"
