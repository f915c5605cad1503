// IPGC graph coloring for MI355X (gfx950): host driver and C ABI.
//
// Method: Section II-C of Rai, M P, Pai, "A Hybrid Graph Coloring Algorithm for
// GPUs" (arXiv 1912.01478); schedule: Section IV (worklist kept in every round,
// topology-driven or data-driven rounds chosen by worklist size against H).
// The device code and its data layout are described in ipgc_device.hpp.
//
// One call (one stream, in order):
//   k_init        initial state, node classes, row-pointer checks (rowptr[0] == 0
//                 and rowptr[n] == m among them), class counts;
//                 column ids in range and sorted rows of the light nodes
//                 (unless validation is off)
//   k_offsets     prefix sums of the class counts, list layouts
//   k_fill_static every node grouped by class, ascending ids (not written when
//                 one class holds every node); the state pushes need
//   k_prep_wide   smaller-neighbour rings of W nodes, with the same checks of
//                 their rows
//   k_prep_hubs   the same for class-M nodes, a row chunk per wavefront (a
//                 counting launch, then a placing launch)
//   k_round1_light  round 1 of a graph of at least 2^20 nodes that are all light
//                 and pull their colors (no state read), before the round kernel
//   k_rounds      every round (from round 2 after k_round1_light), one
//                 cooperative launch with grid barriers (or k_assign_round +
//                 k_conflict_round + k_push_round per round when stepped)
// and read back the round count.  The host synchronizes after k_fill_static
// (class counts decide the launches that follow; a node's row is only read
// through its own checked row pointers), after the ring building when there is
// one (the column checks decide whether to go on) and after the rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ipgc.h"
#include "ipgc_device.hpp"
#include "ipgc_host.hpp"

namespace ipgc {

thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

// ------------------------------------------------------------ device memory

namespace {
std::mutex g_alloc_mutex;
AllocOwner g_alloc;  // the installed hook (null functions: hipMalloc / hipFree)
}  // namespace

int dev_alloc(void **p, size_t bytes, AllocOwner *owner) {
    *p = nullptr;
    AllocOwner o;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mutex);
        o = g_alloc;
    }
    HIP_TRY(hipGetDevice(&o.device));
    if (o.alloc) {
        *p = o.alloc((uint64_t)bytes, o.device, o.user);
        if (!*p) return fail(IPGC_ENOMEM, "device allocation of %llu bytes failed (allocation hook)", (unsigned long long)bytes);
    } else if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(IPGC_ENOMEM, "device allocation of %llu bytes failed", (unsigned long long)bytes);
    }
    *owner = o;
    return IPGC_OK;
}

void dev_free(void *p, size_t bytes, const AllocOwner &owner) {
    if (!p) return;
    if (owner.free) owner.free(p, (uint64_t)bytes, owner.device, owner.user);
    else (void)hipFree(p);
}

namespace {

constexpr int kPrepSpanMin = 2048;  // nodes per preparation workgroup (at least)
constexpr int kMaxPrepBlocks = 65536;

// Profile kernel kinds.
enum Kind { kKindInit = 0, kKindCheck, kKindPrep, kKindRounds, kKindAssign, kKindConflict, kKindPush, kNumKinds };
const char *const kKindNames[kNumKinds] = {"init", "check", "prep", "rounds", "assign_step", "conflict_step", "push_step"};
const char *const kUnitNames[kNumUnits] = {"assign_nodes",   "pull_entries", "map_bytes",    "conflict_nodes",
                                           "conflict_entries", "list_writes", "push_entries", "commits"};

struct Workspace {
    DBuf<int32_t> static_list, seg_list0, seg_list1, seg_cnt, block_cnt, hub_pre, hub_cnt, trace, lstart, llen, lower;
    DBuf<HubRec> hub_won;
    DBuf<int64_t> seg_deg, block_deg, units, trace_deg;
    DBuf<int8_t> cls;
    DBuf<uint8_t> F;
    DBuf<uint64_t> mask;
    DBuf<uint32_t> pend;
    DBuf<int64_t> growptr, node_off, edge_off;  // batches: union row starts, graph offsets
    DBuf<int32_t> gbase, gidx, grounds;         // batches: per-node graph base and index, rounds per graph
    DBuf<int32_t> gthr, gleft, trace_topo;      // per-graph schedules: H_g, uncolored nodes per graph, trace
    DBuf<uint32_t> gsplit;                      // per-graph schedules, stepped launches: each graph's kind
    DBuf<uint64_t> ticks;
    DBuf<Barrier> bar;
    DBuf<Counters> ctb;
    DBuf<int32_t> sorted_rows;  // IPGC_VALIDATE_FULL: every row sorted (m entries)
    Counters *ct = nullptr;       // ctb.p
    Counters *host_ct = nullptr;  // pinned (or &host_local for a carved workspace)
    Counters host_local;
    bool borrowed = false;        // carved from static scratch: nothing here is owned
    std::vector<hipEvent_t> events;
    int coop_blocks = -1;  // co-resident round workgroups on this device (0: no cooperative launch)

    // Every buffer one call of the single-graph or batched path needs, with its entry count, in
    // one fixed order (the batched path adds its union arrays itself).  At most m / (hub_min + 1)
    // nodes have a degree above hub_min, so no more hubs can commit in one round.  Per-graph
    // schedules (split) double the worklist segments: a round may append the losers of two passes.
    template <class Fn>
    int plan(int64_t n, int64_t m, int grid, int prep_grid, int hub_min, bool full, bool split, Fn &&f) {
        const int64_t seg = (n + (int64_t)kNumClasses * grid * (kRoundBlock + 1)) * (split ? 2 : 1);
        TRY(f(ctb, 1));
        TRY(f(bar, 1));
        TRY(f(static_list, n));
        TRY(f(seg_list0, seg));
        TRY(f(seg_list1, seg));
        TRY(f(seg_cnt, 2 * kNumClasses * (int64_t)kMaxRoundBlocks));
        TRY(f(seg_deg, 2 * kNumClasses * (int64_t)kMaxRoundBlocks));
        TRY(f(hub_won, std::min<int64_t>(n, m / ((int64_t)hub_min + 1) + 1)));
        TRY(f(block_cnt, (int64_t)(kNumClasses + 1) * prep_grid));
        // class-M nodes (degree above hub_min) + the total; two counts per row chunk of them
        const int64_t hubs = std::min<int64_t>(n, m / ((int64_t)hub_min + 1));
        TRY(f(hub_pre, hubs + 1));
        TRY(f(hub_cnt, hubs + m / kRingChunk + 1));
        TRY(f(block_deg, (int64_t)kNumClasses * prep_grid));
        TRY(f(units, (int64_t)kNumUnits * kMaxRoundBlocks));
        TRY(f(trace, n));
        TRY(f(trace_deg, n));
        TRY(f(cls, n));
        TRY(f(F, m + n + 64));
        TRY(f(mask, n));
        TRY(f(pend, n));
        TRY(f(lower, std::max<int64_t>(m, 1)));
        TRY(f(lstart, n));
        TRY(f(llen, n));
        if (full) TRY(f(sorted_rows, std::max<int64_t>(m, 1)));
        return IPGC_OK;
    }

    int reserve(int64_t n, int64_t m, int grid, int prep_grid, int hub_min, bool full, bool split = false) {
        TRY(plan(n, m, grid, prep_grid, hub_min, full, split, [](auto &b, int64_t c) { return b.reserve(c); }));
        ct = ctb.p;
        if (!host_ct) HIP_TRY(hipHostMalloc(&host_ct, sizeof(Counters), hipHostMallocDefault));
        return IPGC_OK;
    }

    // Points every buffer of the plan into [base, base + size), 256-byte aligned pieces in plan
    // order, without allocating: the buffers are borrowed, and the counters are read back into
    // host_local.  *used receives the bytes the plan needs; IPGC_ETOOBIG if that exceeds size.
    int carve(unsigned char *base, size_t size, int64_t n, int64_t m, int grid, int prep_grid, int hub_min, bool full,
              size_t *used) {
        size_t off = 0;
        TRY(plan(n, m, grid, prep_grid, hub_min, full, false, [&](auto &b, int64_t c) {
            using T = std::remove_reference_t<decltype(*b.p)>;
            off = (off + 255) & ~(size_t)255;
            const size_t bytes = sizeof(T) * (size_t)c;
            if (off + bytes <= size) b.lend(reinterpret_cast<T *>(base + off), c);
            else b.release();
            off += bytes;
            return IPGC_OK;
        }));
        *used = off;
        if (off > size)
            return fail(IPGC_ETOOBIG, "this graph needs %llu bytes of scratch; the static scratch holds %llu",
                        (unsigned long long)off, (unsigned long long)size);
        ct = ctb.p;
        host_ct = &host_local;
        borrowed = true;
        return IPGC_OK;
    }

    void release() {
        static_list.release(); seg_list0.release(); seg_list1.release(); seg_cnt.release(); hub_won.release();
        hub_pre.release(); hub_cnt.release();
        block_cnt.release(); trace.release(); lstart.release(); llen.release(); lower.release();
        seg_deg.release(); block_deg.release(); units.release(); trace_deg.release(); cls.release();
        F.release(); mask.release(); pend.release(); ticks.release(); bar.release(); growptr.release(); node_off.release(); edge_off.release();
        gbase.release(); gidx.release(); grounds.release(); ctb.release(); sorted_rows.release();
        gthr.release(); gleft.release(); trace_topo.release(); gsplit.release();
        if (host_ct && !borrowed) (void)hipHostFree(host_ct);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        *this = Workspace();
    }

    int event(size_t i, hipEvent_t *out) {
        while (events.size() <= i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            events.push_back(e);
        }
        *out = events[i];
        return IPGC_OK;
    }
};

// Brackets launches of the selected kernel kinds with HIP events.
struct Profiler {
    Workspace &ws;
    hipStream_t s;
    uint32_t mask;
    std::vector<int> kinds;
    size_t used = 0;

    int mark(int kind, bool end) {
        if (!(mask >> kind & 1u)) return IPGC_OK;
        hipEvent_t e;
        TRY(ws.event(used, &e));
        HIP_TRY(hipEventRecord(e, s));
        ++used;
        if (end) kinds.push_back(kind);
        return IPGC_OK;
    }
    int begin(int kind) { return mark(kind, false); }
    int end(int kind) { return mark(kind, true); }
    int collect(ipgc_profile *p) {
        for (size_t k = 0; k < kinds.size(); ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ws.events[2 * k], ws.events[2 * k + 1]));
            p->ms[kinds[k]] += ms;
            p->launches[kinds[k]] += 1;
        }
        return IPGC_OK;
    }
};

std::mutex g_mutex;
std::vector<Workspace> g_ws;

int read_counters(Workspace &ws, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(ws.host_ct, ws.ct, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return IPGC_OK;
}

// Workgroups of the round kernel that fit on the device at once (0: no cooperative launch).
int cooperative_capacity(Workspace &ws, int dev, int *out) {
    if (ws.coop_blocks < 0) {
        int coop = 0, cus = 0, per_cu = 0;
        HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        // the three instantiations (one graph, batches, batches with per-graph schedules) must all fit
        int per_cu64 = 0, per_cu_split = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_rounds<DevT<int32_t>>), kRoundBlock, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu64, reinterpret_cast<const void *>(k_rounds<DevT<int64_t>>), kRoundBlock, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu_split, reinterpret_cast<const void *>(k_rounds<DevT<int64_t, true>>), kRoundBlock, 0));
        per_cu = std::min(per_cu, std::min(per_cu64, per_cu_split));
        ws.coop_blocks = coop ? std::min(kMaxRoundBlocks, std::max(0, cus * per_cu)) : 0;
    }
    *out = ws.coop_blocks;
    return IPGC_OK;
}

}  // namespace

int parse_options(const ipgc_options *opt, int mode, Params *p) {
    if (mode != IPGC_MODE_TOPOLOGY && mode != IPGC_MODE_DATA && mode != IPGC_MODE_HYBRID && mode != IPGC_MODE_REBUILD)
        return fail(IPGC_EINVAL, "unknown mode %d", mode);
    ipgc_options o{};
    if (opt) o = *opt;
    p->mode = mode;
    p->light_max = o.light_max_degree ? o.light_max_degree : kDefaultLightMax;
    p->hub_min = o.hub_min_degree ? o.hub_min_degree : std::max(kDefaultHubMin, p->light_max + 1);
    if (p->light_max < 1 || p->light_max > kLightMaxLimit)
        return fail(IPGC_EINVAL, "light_max_degree %d outside 1..%d", p->light_max, kLightMaxLimit);
    if (p->hub_min <= p->light_max)
        return fail(IPGC_EINVAL, "hub_min_degree %d must exceed light_max_degree %d", p->hub_min, p->light_max);
    if (o.validate < IPGC_VALIDATE_DEFAULT || o.validate > IPGC_VALIDATE_FULL)
        return fail(IPGC_EINVAL, "unknown validate level %d", o.validate);
    if (o.reserved != 0) return fail(IPGC_EINVAL, "ipgc_options.reserved must be 0");
    if (o.barrier_timeout_ms < -1) return fail(IPGC_EINVAL, "barrier_timeout_ms %d below -1", o.barrier_timeout_ms);
    p->barrier_ms = o.barrier_timeout_ms == 0 ? 60000 : o.barrier_timeout_ms;
    p->full = o.validate == IPGC_VALIDATE_FULL;
    if (o.flags & ~(IPGC_FLAG_STEPPED | IPGC_FLAG_LIGHT_PULL | IPGC_FLAG_LIGHT_PUSH | IPGC_FLAG_RACY |
                    IPGC_FLAG_PER_GRAPH))
        return fail(IPGC_EINVAL, "unknown flags 0x%x", o.flags);
    if ((o.flags & IPGC_FLAG_LIGHT_PULL) && (o.flags & IPGC_FLAG_LIGHT_PUSH))
        return fail(IPGC_EINVAL, "IPGC_FLAG_LIGHT_PULL and IPGC_FLAG_LIGHT_PUSH exclude each other");
    p->light = (o.flags & IPGC_FLAG_LIGHT_PULL) ? 1 : (o.flags & IPGC_FLAG_LIGHT_PUSH) ? 0 : -1;
    p->racy = (o.flags & IPGC_FLAG_RACY) != 0;
    p->per_graph = (o.flags & IPGC_FLAG_PER_GRAPH) != 0;
    if (p->racy && p->light < 0) p->light = 1;
    if (o.workgroups < 0) return fail(IPGC_EINVAL, "negative workgroups %d", o.workgroups);
    p->workgroups = o.workgroups;
    p->tail_groups = o.tail_workgroups == 0 ? kDefaultTailGroups : std::max(0, o.tail_workgroups);
    p->check_ids = o.validate != IPGC_VALIDATE_NONE;
    p->stepped = (o.flags & IPGC_FLAG_STEPPED) != 0;
    p->threshold = o.threshold;
    p->prof = o.profile;
    if (p->prof) {  // clear the out fields, keep the in fields
        ipgc_profile *pr = p->prof;
        const uint32_t mask = pr->mask;
        uint64_t *const ticks = pr->phase_ticks;
        const int64_t cap = pr->phase_capacity;
        std::memset(pr, 0, sizeof *pr);
        pr->mask = mask;
        pr->phase_ticks = ticks;
        pr->phase_capacity = cap;
        pr->kinds = kNumKinds;
        pr->unit_kinds = kNumUnits;
    }
    return IPGC_OK;
}

int full_check_verdict(int bits) {
    if (bits & kFullSelfLoop)
        return fail(IPGC_EBADCSR, "a row holds its own node (a self-loop); full validation takes simple graphs");
    if (bits & kFullDuplicate)
        return fail(IPGC_EBADCSR, "a row holds the same id twice (a duplicate entry); full validation takes simple graphs");
    if (bits & kFullAsymmetric)
        return fail(IPGC_EBADCSR, "an entry (v, u) has no reverse entry (u, v): the CSR is not symmetric");
    return IPGC_OK;
}

// IPGC_OK, or IPGC_EBADCSR for the CSR ends or row pointers k_init found bad.
int row_verdict(const Counters &c, int64_t m) {
    if (c.bad_ends)
        return fail(IPGC_EBADCSR, "rowptr[0]=%lld rowptr[n]=%lld, expected 0 and m=%lld", (long long)c.ends[0],
                    (long long)c.ends[1], (long long)m);
    if (c.bad_rows) return fail(IPGC_EBADCSR, "rowptr is decreasing or outside [0, m]");
    return IPGC_OK;
}

int barrier_limit_ticks(int dev, int barrier_ms, uint64_t *ticks) {
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *ticks = barrier_ms < 0 ? 0 : (uint64_t)barrier_ms * (uint64_t)std::max(khz, 1);
    return IPGC_OK;
}

namespace {

Workspace &workspace(int dev) {
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    return g_ws[dev];
}

// Round grid: enough workgroups for the first round, at most what is co-resident.
int round_grid(Workspace &ws, int dev, const Params &P, int64_t n, int *grid, int *coop) {
    *coop = 0;
    if (!P.stepped) TRY(cooperative_capacity(ws, dev, coop));
    const int64_t want = P.workgroups > 0 ? P.workgroups : (n + 4 * kRoundBlock - 1) / (4 * kRoundBlock);
    *grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, *coop > 0 ? *coop : kMaxRoundBlocks));
    return IPGC_OK;
}

// Preparation kernels: workgroup b covers nodes [b * span, (b + 1) * span).
void prep_layout(int64_t n, int64_t *span, int *prep_grid) {
    *span = std::max<int64_t>(kPrepSpanMin, (n + kMaxPrepBlocks - 1) / kMaxPrepBlocks);
    *prep_grid = (int)((n + *span - 1) / *span);
}

// IPGC_VALIDATE_FULL on a graph whose row pointers and ids have passed their
// checks: sorted copies of the rows in the workspace, then self-loops,
// repeated ids and missing reverse entries.
template <class D>
int check_full(Workspace &ws, hipStream_t s, const D &d, int64_t n, int64_t m) {
    TRY(ws.sorted_rows.reserve(std::max<int64_t>(m, 1)));  // in the plan when full validation is on
    TRY(clear(&ws.ct->bad_full, sizeof(int32_t), s));
    const int sort_grid = (int)std::min<int64_t>(n, 65536);
    k_full_sort<<<sort_grid, kSortBlock, 0, s>>>(d, 0, n, ws.sorted_rows.p, nullptr);
    k_full_check<<<(int)std::min<int64_t>(16384, (n + 3) / 4), kPrepBlock, 0, s>>>(d, 0, n, ws.sorted_rows.p,
                                                                                   &ws.ct->bad_full, nullptr);
    HIP_TRY(hipGetLastError());
    TRY(read_counters(ws, s));
    return full_check_verdict(ws.host_ct->bad_full);
}

// Everything after the input is in place: d.rowptr, d.colidx, d.c and (for a
// batch) d.gbase / d.gidx / d.node_off / d.grounds are set by the caller.
template <class D>
int run(Workspace &ws, int dev, hipStream_t s, const Params &P, D d, int64_t n, int64_t m, int grid,
        int coop, int32_t *out_rounds, ipgc_trace *trace) {
    using Off = typename D::OffT;
    int64_t span = 0;
    int prep_grid = 0;
    prep_layout(n, &span, &prep_grid);
    TRY(ws.reserve(n, m, grid, prep_grid, P.hub_min, P.full, d.gthr != nullptr));
    ipgc_profile *prof = P.prof;
    Profiler pf{ws, s, prof ? prof->mask : 0u, {}, 0};

    int64_t H;
    if (P.mode == IPGC_MODE_TOPOLOGY) H = -1;          // |WL| > -1 always holds
    else if (P.mode == IPGC_MODE_DATA) H = INT64_MAX;  // never
    else H = P.threshold > 0 ? P.threshold : (6 * n) / 10;  // HYBRID and REBUILD

    d.cls = ws.cls.p;
    d.F = ws.F.p;
    d.mask = ws.mask.p;
    d.pend = ws.pend.p;
    d.lower = ws.lower.p;
    d.lstart = ws.lstart.p;
    d.llen = ws.llen.p;
    d.static_list = ws.static_list.p;
    d.seg_list[0] = ws.seg_list0.p;
    d.seg_list[1] = ws.seg_list1.p;
    d.seg_cnt[0] = ws.seg_cnt.p;
    d.seg_cnt[1] = ws.seg_cnt.p + kNumClasses * kMaxRoundBlocks;
    d.seg_deg[0] = ws.seg_deg.p;
    d.seg_deg[1] = ws.seg_deg.p + kNumClasses * kMaxRoundBlocks;
    d.hub_won = ws.hub_won.p;
    d.block_cnt = ws.block_cnt.p;
    d.hub_pre = ws.hub_pre.p;
    d.hub_cnt = ws.hub_cnt.p;
    d.block_deg = ws.block_deg.p;
    d.units = ws.units.p;
    d.ct = ws.ct;
    d.bar = ws.bar.p;
    d.trace = ws.trace.p;
    d.trace_deg = ws.trace_deg.p;
    d.trace_cap = n;
    d.ticks = nullptr;
    d.tick_cap = 0;
    d.threshold = H;
    d.n = (int32_t)n;
    d.m = m;
    d.light_max = P.light_max;
    d.hub_min = P.hub_min;
    d.sorted = 0;
    d.grid = grid;
    TRY(barrier_limit_ticks(dev, P.barrier_ms, &d.bar_limit));
    if (prof && prof->phase_ticks && prof->phase_capacity > 0) {
        TRY(ws.ticks.reserve(prof->phase_capacity));
        TRY(clear(ws.ticks.p, sizeof(uint64_t) * prof->phase_capacity, s));
        d.ticks = ws.ticks.p;
        d.tick_cap = prof->phase_capacity;
    }

    TRY(clear(ws.bar.p, sizeof(Barrier), s));
    TRY(clear(ws.units.p, sizeof(int64_t) * kNumUnits * grid, s));
    TRY(pf.begin(kKindInit));
    k_init<<<prep_grid, kPrepBlock, 0, s>>>(d, ws.cls.p, (int32_t)span, P.check_ids ? 1 : 0);
    k_offsets<<<1, 1024, 0, s>>>(d, prep_grid);
    k_fill_static<<<prep_grid, kPrepBlock, 0, s>>>(d, (int32_t)span, P.light);
    TRY(pf.end(kKindInit));
    HIP_TRY(hipGetLastError());
    TRY(read_counters(ws, s));
    TRY(row_verdict(*ws.host_ct, m));
    const int64_t n_wide = (int64_t)ws.host_ct->class_n[kW] + ws.host_ct->class_n[kM];
    // byte maps hold colors above 64, which only W/M nodes (degree above 63) can need: every map
    // starts empty when such nodes exist, and none is read otherwise
    if (n_wide > 0) TRY(clear(ws.F.p, (size_t)(m + n + 64), s));
    if (P.light == 0 || (P.light < 0 && n_wide > 0)) d.light_pull = kPushAll;
    else d.light_pull = n_wide > 0 ? kPullLight : kPullOnly;
    d.racy = P.racy ? 1 : 0;
    d.tail_groups = P.tail_groups;
    d.discard = P.mode == IPGC_MODE_REBUILD ? 1 : 0;
    if (n_wide > 0) {  // also checks the ids of the wide rows
        const int64_t n_w = ws.host_ct->class_n[kW], n_hub = ws.host_ct->class_n[kM];
        const int64_t hub_chunks = ws.host_ct->hub_chunks;
        TRY(pf.begin(kKindPrep));
        // a wavefront per W node, or a quarter wavefront per node while their rows hold at most 1024 entries
        const int64_t per_wave = P.hub_min <= 1024 ? 4 : 1;
        if (n_w > 0)
            k_prep_wide<<<(int)std::min<int64_t>(8192, (n_w + 4 * per_wave - 1) / (4 * per_wave)), kPrepBlock, 0, s>>>(d);
        if (n_hub > 0) {
            const int blocks = (int)std::min<int64_t>(8192, (hub_chunks + 3) / 4);
            k_prep_hubs<false><<<blocks, kPrepBlock, 0, s>>>(d);
            k_prep_hubs<true><<<blocks, kPrepBlock, 0, s>>>(d);
        }
        TRY(pf.end(kKindPrep));
        HIP_TRY(hipGetLastError());
    }
    if (P.check_ids) {
        // the ring building of W/M rows checks their ids; with none, k_init's checks of the light
        // rows were all, and the counters read above hold them
        if (n_wide > 0) TRY(read_counters(ws, s));
        if (ws.host_ct->bad_ids) return fail(IPGC_EBADCSR, "a column id is outside [0, n)");
    }
    d.sorted = P.check_ids && !ws.host_ct->unsorted;
    if (P.full) TRY(check_full(ws, s, d, n, m));

    // Rounds: at most n (the worklist shrinks every round), plus the start of the one that finds it empty.
    if (coop > 0) {
        int32_t first = 1, last = (int32_t)std::min<int64_t>(n + 1, INT32_MAX - 2);
        void *args[] = {&d, &first, &last};
        TRY(pf.begin(kKindRounds));
        // one graph whose nodes all pull: round 1 needs no state reads, in a launch of its own so
        // that the round kernel does not carry that code
        if constexpr (!D::kSplit && std::is_same<Off, int32_t>::value) {
            if (n >= (1 << 20) && d.light_pull == kPullOnly && ws.host_ct->class_n[kL] == n && !d.racy && !d.discard) {
                k_round1_light<<<grid, kRoundBlock, 0, s>>>(d);
                HIP_TRY(hipGetLastError());
                first = 2;
            }
        }
        HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_rounds<D>), dim3(grid),
                                           dim3(kRoundBlock), args, 0, s));
        TRY(pf.end(kKindRounds));
        TRY(read_counters(ws, s));
        if constexpr (D::kSplit) {
            // per-graph schedules: from resume_round on every graph runs data-driven, which the plain
            // batch kernel does with fewer registers (same layout, every round data-driven)
            if (!ws.host_ct->finished && ws.host_ct->resume_round > 0) {
                static_assert(sizeof(DevT<Off, false>) == sizeof(D), "the two instantiations share one layout");
                DevT<Off, false> d2;
                std::memcpy(static_cast<void *>(&d2), &d, sizeof d2);
                d2.threshold = INT64_MAX;
                d2.gleft = nullptr;
                d2.gthr = nullptr;
                int32_t first2 = ws.host_ct->resume_round;
                void *args2[] = {&d2, &first2, &last};
                TRY(clear(ws.bar.p, sizeof(Barrier), s));
                TRY(pf.begin(kKindRounds));
                HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_rounds<DevT<Off, false>>),
                                                   dim3(grid), dim3(kRoundBlock), args2, 0, s));
                TRY(pf.end(kKindRounds));
                TRY(read_counters(ws, s));
            }
        }
    } else {
        for (int32_t r = 1; r <= n + 1; ++r) {
            if (d.discard) k_rebuild_round<<<grid, kRoundBlock, 0, s>>>(d, r);
            TRY(pf.begin(kKindAssign));
            k_assign_round<<<grid, kRoundBlock, 0, s>>>(d, r);
            TRY(pf.end(kKindAssign));
            TRY(pf.begin(kKindConflict));
            k_conflict_round<<<grid, kRoundBlock, 0, s>>>(d, r);
            TRY(pf.end(kKindConflict));
            TRY(pf.begin(kKindPush));
            k_push_round<<<grid, kRoundBlock, 0, s>>>(d);
            TRY(pf.end(kKindPush));
            HIP_TRY(hipGetLastError());
            TRY(read_counters(ws, s));
            if (ws.host_ct->finished || ws.host_ct->bad_ids) break;
        }
    }
    if (ws.host_ct->bad_ids) return fail(IPGC_EBADCSR, "a column id is outside [0, n)");
    if (!ws.host_ct->finished) {
        unsigned aborted = 0;
        HIP_TRY(hipMemcpy(&aborted, &ws.bar.p->abort.v, sizeof aborted, hipMemcpyDeviceToHost));
        if (aborted)
            return fail(IPGC_EHIP, "a grid-barrier wait exceeded %d ms: not every workgroup of the cooperative "
                        "launch ran (%d workgroups)", P.barrier_ms, grid);
        return fail(IPGC_ELIMIT, "rounds did not finish");
    }
    if (ws.host_ct->seg_overflow) return fail(IPGC_EHIP, "internal error: a worklist segment overflowed");
    const int32_t rounds = ws.host_ct->rounds;
    if (trace) {
        const int64_t k = std::min<int64_t>(trace->capacity, rounds);
        if (k > 0 && trace->wl_size)
            HIP_TRY(hipMemcpyAsync(trace->wl_size, ws.trace.p, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
        if (k > 0 && trace->wl_degree)
            HIP_TRY(hipMemcpyAsync(trace->wl_degree, ws.trace_deg.p, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (d.trace_topo) {  // per-graph schedules: the device counted the graphs of each kind
            const int64_t kt = std::min<int64_t>(k, d.topo_cap);
            std::vector<int32_t> tg((size_t)std::max<int64_t>(kt, 1));
            if (kt > 0) HIP_TRY(hipMemcpy(tg.data(), d.trace_topo, sizeof(int32_t) * kt, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < kt; ++i) {
                if (trace->topo_graphs) trace->topo_graphs[i] = tg[i];
                if (trace->topology) trace->topology[i] = (int8_t)(tg[i] > 0);
            }
        } else if (k > 0 && trace->topology && trace->wl_size) {
            for (int64_t i = 0; i < k; ++i) trace->topology[i] = (int8_t)((int64_t)trace->wl_size[i] > H);
        }
        trace->recorded = k;
    }
    if (prof) {
        HIP_TRY(hipStreamSynchronize(s));
        TRY(pf.collect(prof));
        std::vector<int64_t> u((size_t)kNumUnits * grid);
        HIP_TRY(hipMemcpy(u.data(), ws.units.p, sizeof(int64_t) * u.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < kNumUnits; ++k)
            for (int b = 0; b < grid; ++b) prof->units[k] += u[(size_t)k * grid + b];
        if (d.ticks) {
            const int64_t k = std::min<int64_t>(prof->phase_capacity, 3 * (int64_t)rounds + 1);
            HIP_TRY(hipMemcpy(prof->phase_ticks, ws.ticks.p, sizeof(uint64_t) * k, hipMemcpyDeviceToHost));
            prof->phase_recorded = k;
        }
        int khz = 0;
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        prof->tick_khz = khz;
    }
    *out_rounds = rounds;
    return IPGC_OK;
}

int color_impl(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m, int mode, const ipgc_options *opt,
               hipStream_t s, int32_t *out_colors, int32_t *out_rounds, ipgc_trace *trace) {
    if (!out_rounds) return fail(IPGC_EINVAL, "out_rounds is NULL");
    *out_rounds = -1;
    if (n < 0 || m < 0) return fail(IPGC_EINVAL, "negative size (n=%lld, m=%lld)", (long long)n, (long long)m);
    if (n >= INT32_MAX || m >= INT32_MAX)
        return fail(IPGC_ETOOBIG, "n=%lld or m=%lld exceeds the int32 CSR", (long long)n, (long long)m);
    Params P;
    TRY(parse_options(opt, mode, &P));
    if (trace) trace->recorded = 0;
    if (n == 0) {
        *out_rounds = 0;
        g_err[0] = 0;
        return IPGC_OK;
    }
    if (!rowptr || !out_colors || (m > 0 && !colidx)) return fail(IPGC_EINVAL, "null device pointer");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace &ws = workspace(dev);
    if (!ws.ct) TRY(ws.reserve(0, 0, 1, 1, kDefaultHubMin, false));

    // rowptr[0] == 0 and rowptr[n] == m are checked by k_init, before any row is read
    int grid = 1, coop = 0;
    TRY(round_grid(ws, dev, P, n, &grid, &coop));
    DevT<int32_t> d{};
    d.rowptr = rowptr;
    d.colidx = colidx;
    d.c = out_colors;
    TRY(clear(ws.ct, sizeof(Counters), s));
    TRY(run(ws, dev, s, P, d, n, m, grid, coop, out_rounds, trace));
    g_err[0] = 0;
    return IPGC_OK;
}

int batch_impl(int64_t graphs, const int64_t *node_off, const int64_t *edge_off, const int32_t *rowptr_packed,
               const int32_t *colidx_packed, int mode, const ipgc_options *opt, hipStream_t s,
               int32_t *out_colors_packed, int32_t *out_rounds, ipgc_trace *trace) {
    if (graphs < 0) return fail(IPGC_EINVAL, "negative graph count");
    if (graphs > 0 && (!node_off || !edge_off || !out_rounds)) return fail(IPGC_EINVAL, "null host pointer");
    for (int64_t g = 0; g < graphs; ++g) out_rounds[g] = -1;
    if (graphs == 0) return IPGC_OK;
    if (node_off[0] != 0 || edge_off[0] != 0) return fail(IPGC_EINVAL, "node_off[0] and edge_off[0] must be 0");
    for (int64_t g = 0; g < graphs; ++g) {
        const int64_t ng = node_off[g + 1] - node_off[g], mg = edge_off[g + 1] - edge_off[g];
        if (ng < 0 || mg < 0) return fail(IPGC_EINVAL, "graph %lld has negative size", (long long)g);
        if (mg >= INT32_MAX) return fail(IPGC_ETOOBIG, "graph %lld has %lld entries, more than int32", (long long)g, (long long)mg);
    }
    const int64_t n = node_off[graphs], m = edge_off[graphs];
    if (n >= INT32_MAX) return fail(IPGC_ETOOBIG, "the batch has %lld nodes, more than int32 ids allow", (long long)n);
    Params P;
    TRY(parse_options(opt, mode, &P));
    if (P.per_graph && P.mode == IPGC_MODE_REBUILD)
        return fail(IPGC_EINVAL, "IPGC_FLAG_PER_GRAPH does not combine with IPGC_MODE_REBUILD");
    if (P.per_graph && graphs > kMaxSplitGraphs)
        return fail(IPGC_EINVAL, "IPGC_FLAG_PER_GRAPH takes at most %d graphs (%lld given)", kMaxSplitGraphs,
                    (long long)graphs);
    if (n == 0) {
        for (int64_t g = 0; g < graphs; ++g) out_rounds[g] = 0;
        g_err[0] = 0;
        return IPGC_OK;
    }
    if (!rowptr_packed || !out_colors_packed || (m > 0 && !colidx_packed)) return fail(IPGC_EINVAL, "null device pointer");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mutex);
    Workspace &ws = workspace(dev);
    if (!ws.ct) TRY(ws.reserve(0, 0, 1, 1, kDefaultHubMin, false));
    TRY(ws.growptr.reserve(n + 1));
    TRY(ws.gbase.reserve(n));
    TRY(ws.gidx.reserve(n));
    TRY(ws.grounds.reserve(graphs));
    TRY(ws.node_off.reserve(graphs + 1));
    TRY(ws.edge_off.reserve(graphs + 1));
    HIP_TRY(hipMemcpyAsync(ws.node_off.p, node_off, sizeof(int64_t) * (graphs + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ws.edge_off.p, edge_off, sizeof(int64_t) * (graphs + 1), hipMemcpyHostToDevice, s));
    TRY(clear(ws.grounds.p, sizeof(int32_t) * graphs, s));
    TRY(clear(ws.ct, sizeof(Counters), s));
    k_batch_union<<<(int)std::min<int64_t>(graphs, 16384), kPrepBlock, 0, s>>>(
        ws.node_off.p, ws.edge_off.p, rowptr_packed, graphs, ws.growptr.p, ws.gbase.p, ws.gidx.p, ws.ct);
    HIP_TRY(hipGetLastError());

    int grid = 1, coop = 0;
    TRY(round_grid(ws, dev, P, n, &grid, &coop));
    auto setup = [&](auto &d) {
        d.rowptr = ws.growptr.p;
        d.colidx = colidx_packed;
        d.gbase = ws.gbase.p;
        d.gidx = ws.gidx.p;
        d.gend = ws.node_off.p + 1;
        d.grounds = ws.grounds.p;
        d.c = out_colors_packed;
    };
    // a workgroup's out segment per class holds (its share + a workgroup) entries, twice that with
    // per-graph schedules, counted in int32
    if (((n + grid - 1) / grid + kRoundBlock) * (P.per_graph ? 2 : 1) > INT32_MAX)
        return fail(IPGC_ETOOBIG, "%lld nodes over %d workgroups overflow a worklist segment; use more workgroups",
                    (long long)n, grid);
    int32_t rounds = -1;
    std::vector<int32_t> h_thr, h_left;  // per-graph schedules (alive until the call has synchronized)
    if (P.per_graph) {
        // H_g per graph, and every graph's worklist (its uncolored nodes) at the start of round 1
        h_thr.resize((size_t)graphs);
        h_left.resize((size_t)graphs);
        const int64_t Hc = std::min<int64_t>(P.threshold, n);  // H >= N: no graph is ever above it
        for (int64_t g = 0; g < graphs; ++g) {
            const int64_t ng = node_off[g + 1] - node_off[g];
            h_left[g] = (int32_t)ng;
            if (P.mode == IPGC_MODE_TOPOLOGY) h_thr[g] = -1;
            else if (P.mode == IPGC_MODE_DATA) h_thr[g] = INT32_MAX;
            else h_thr[g] = (int32_t)(P.threshold > 0 ? Hc * ng / n : (6 * ng) / 10);
        }
        TRY(ws.gthr.reserve(graphs));
        TRY(ws.gleft.reserve(graphs));
        TRY(ws.gsplit.reserve((graphs + 63) / 64 * 2));
        HIP_TRY(hipMemcpyAsync(ws.gthr.p, h_thr.data(), sizeof(int32_t) * graphs, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ws.gleft.p, h_left.data(), sizeof(int32_t) * graphs, hipMemcpyHostToDevice, s));
        DevT<int64_t, true> d{};
        setup(d);
        d.gthr = ws.gthr.p;
        d.gleft = ws.gleft.p;
        d.gsplit = ws.gsplit.p;
        d.ngraphs = (int32_t)graphs;
        const int64_t tcap = trace ? std::min<int64_t>(n, std::max<int64_t>(trace->capacity, 0)) : 0;
        if (tcap > 0) {  // cleared: rounds left to the plain kernel have no topology-driven graph
            TRY(ws.trace_topo.reserve(tcap));
            TRY(clear(ws.trace_topo.p, sizeof(int32_t) * tcap, s));
            d.trace_topo = ws.trace_topo.p;
            d.topo_cap = tcap;
        }
        TRY(run(ws, dev, s, P, d, n, m, grid, coop, &rounds, trace));
    } else {
        DevT<int64_t> d{};
        setup(d);
        TRY(run(ws, dev, s, P, d, n, m, grid, coop, &rounds, trace));
    }
    HIP_TRY(hipMemcpyAsync(out_rounds, ws.grounds.p, sizeof(int32_t) * graphs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g_err[0] = 0;
    return IPGC_OK;
}

// ------------------------------------------------------------ static scratch (no allocation)
//
// ipgc_color_graph_noalloc carves its workspace out of one file-scope device
// array instead of allocating it.  In host code `scratch` is only the host-side
// stand-in of the array: its device address on each GPU comes from
// hipGetSymbolAddress, once per device, and only that address reaches kernels.

constexpr size_t kStaticScratchBytes = IPGC_NOALLOC_SCRATCH_BYTES;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void *g_scratch_ptr[kStaticMaxDevices];          // device address of `scratch` per device (null: not yet looked up)
Workspace g_static_ws[kStaticMaxDevices];        // the carved workspace per device (borrowed buffers only)

// The device address of this device's copy of `scratch` (caller holds g_mutex, dev is current).
int static_scratch(int dev, unsigned char **out) {
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(IPGC_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return IPGC_OK;
}

int color_noalloc_impl(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m, int mode,
                       const ipgc_options *opt, hipStream_t s, int32_t *out_colors, int32_t *out_rounds,
                       ipgc_trace *trace) {
    if (!out_rounds) return fail(IPGC_EINVAL, "out_rounds is NULL");
    *out_rounds = -1;
    if (n < 0 || m < 0) return fail(IPGC_EINVAL, "negative size (n=%lld, m=%lld)", (long long)n, (long long)m);
    if (n >= INT32_MAX || m >= INT32_MAX)
        return fail(IPGC_ETOOBIG, "n=%lld or m=%lld exceeds the int32 CSR", (long long)n, (long long)m);
    Params P;
    TRY(parse_options(opt, mode, &P));
    // a profile records HIP events and a device tick buffer, which would have to be created
    if (P.prof) return fail(IPGC_EINVAL, "ipgc_color_graph_noalloc takes no profile (it would need allocations)");
    if (trace) trace->recorded = 0;
    if (n == 0) {
        *out_rounds = 0;
        g_err[0] = 0;
        return IPGC_OK;
    }
    if (!rowptr || !out_colors || (m > 0 && !colidx)) return fail(IPGC_EINVAL, "null device pointer");

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(IPGC_EINVAL, "device %d past the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_mutex);
    unsigned char *base = nullptr;
    TRY(static_scratch(dev, &base));
    Workspace &ws = g_static_ws[dev];
    int grid = 1, coop = 0;
    TRY(round_grid(ws, dev, P, n, &grid, &coop));
    int64_t span = 0;
    int prep_grid = 0;
    prep_layout(n, &span, &prep_grid);
    size_t used = 0;
    TRY(ws.carve(base, kStaticScratchBytes, n, m, grid, prep_grid, P.hub_min, P.full, &used));

    DevT<int32_t> d{};
    d.rowptr = rowptr;
    d.colidx = colidx;
    d.c = out_colors;
    TRY(clear(ws.ct, sizeof(Counters), s));  // the array keeps the previous call's contents
    TRY(run(ws, dev, s, P, d, n, m, grid, coop, out_rounds, trace));
    g_err[0] = 0;
    return IPGC_OK;
}

}  // namespace
}  // namespace ipgc

extern "C" {

int ipgc_color_graph(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                     int32_t *out_colors, int32_t *out_rounds) {
    IPGC_GUARD(ipgc::color_impl(csr_rowptr, csr_colidx, n, m, mode, nullptr, nullptr, out_colors, out_rounds, nullptr));
}

int ipgc_color_graph_ex(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                        const ipgc_options *options, void *stream, int32_t *out_colors, int32_t *out_rounds,
                        ipgc_trace *trace) {
    IPGC_GUARD(ipgc::color_impl(csr_rowptr, csr_colidx, n, m, mode, options, (hipStream_t)stream, out_colors,
                                out_rounds, trace));
}

int ipgc_color_graphs_batched(int64_t num_graphs, const int64_t *node_off, const int64_t *edge_off,
                              const int32_t *rowptr_packed, const int32_t *colidx_packed, int mode,
                              const ipgc_options *options, void *stream, int32_t *out_colors_packed,
                              int32_t *out_rounds, ipgc_trace *trace) {
    IPGC_GUARD(ipgc::batch_impl(num_graphs, node_off, edge_off, rowptr_packed, colidx_packed, mode, options,
                                (hipStream_t)stream, out_colors_packed, out_rounds, trace));
}

int ipgc_color_graph_noalloc(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                             const ipgc_options *options, void *stream, int32_t *out_colors, int32_t *out_rounds,
                             ipgc_trace *trace) {
    IPGC_GUARD(ipgc::color_noalloc_impl(csr_rowptr, csr_colidx, n, m, mode, options, (hipStream_t)stream, out_colors,
                                        out_rounds, trace));
}

const char *ipgc_last_error(void) { return ipgc::g_err; }

const char *ipgc_kernel_name(int kind) { return kind >= 0 && kind < ipgc::kNumKinds ? ipgc::kKindNames[kind] : ""; }

const char *ipgc_unit_name(int kind) { return kind >= 0 && kind < ipgc::kNumUnits ? ipgc::kUnitNames[kind] : ""; }

int ipgc_version(void) { return (2 << 16) | 1; }

void ipgc_release_workspaces(void) {
    std::lock_guard<std::mutex> lock(ipgc::g_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < ipgc::g_ws.size(); ++d) {
        if (hipSetDevice((int)d) == hipSuccess) ipgc::g_ws[d].release();
    }
    (void)hipSetDevice(cur);
    ipgc::g_ws.clear();
    ipgc::release_bfs_workspaces();
}

int ipgc_set_allocator(ipgc_alloc_fn alloc, ipgc_free_fn free_fn, void *user) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return ipgc::fail(IPGC_EINVAL, "ipgc_set_allocator takes both functions or neither");
    std::lock_guard<std::mutex> lock(ipgc::g_alloc_mutex);
    ipgc::g_alloc.alloc = alloc;
    ipgc::g_alloc.free = free_fn;
    ipgc::g_alloc.user = alloc ? user : nullptr;
    ipgc::g_err[0] = 0;
    return IPGC_OK;
}

}  // extern "C"
